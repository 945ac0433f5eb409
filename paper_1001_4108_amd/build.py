"""Build libfwapsp.so (HIP, gfx950) in-tree.

    python paper_1001_4108_amd/build.py

Every source under csrc/ is compiled by hipcc for gfx950 and linked into
paper_1001_4108_amd/libfwapsp.so.  Packed-FP32 instruction selection is
switched off for the device code (the kernels use scalar fp32 adds).  The
vector-ALU issue-rate probe (probe/valu_probe.hip, measurement only) is built
beside it as libfwprobe.so.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.environ.get("FWAPSP_OUT") or os.path.join(HERE, "libfwapsp.so")
BUILD = os.environ.get("FWAPSP_BUILD_DIR") or os.path.join(ROOT, "_build")
PROBE_SRC = os.path.join(HERE, "probe", "valu_probe.hip")
PROBE_OUT = os.path.join(HERE, "libfwprobe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("FWAPSP_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"),
] + os.environ.get("FWAPSP_EXTRA_FLAGS", "").split()


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    noisy = [l for l in (r.stdout + r.stderr).splitlines()
             if "packed-fp32-ops" not in l and l.strip()]
    if noisy and verbose:
        print("\n".join(noisy))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", OUT + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    build_probe(verbose)
    return OUT


def build_probe(verbose: bool = False) -> str:
    cmd = [HIPCC, *COMMON, "-shared", PROBE_SRC, "-o", PROBE_OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on the probe")
    os.replace(PROBE_OUT + ".tmp", PROBE_OUT)
    return PROBE_OUT


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
