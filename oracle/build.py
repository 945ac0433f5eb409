"""Build the CPU oracle's shared library (test infrastructure).

    python oracle/build.py

Compiles fw_oracle.c with gcc into oracle/liboracle.so.  No fast-math: the
oracle's fp32 adds must be IEEE binary32 round-to-nearest, and its min must
be the plain compare-select.  The target is x86-64-v3 (AVX2) so that a library
built on one host still runs on another x86 server.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fw_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-std=c11", "-O3", "-march=x86-64-v3", "-fno-fast-math",
        "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall",
        "-Wextra", "-o", OUT + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
