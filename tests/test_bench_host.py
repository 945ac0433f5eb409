"""Host-side parts of the benchmark contract (no GPU): the one-GPU refusal,
the committed profile's traffic figures and the CPU-oracle baseline leg."""
import os
import subprocess
import sys

import numpy as np

import oracle
from paper_1001_4108_amd import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_profile_traffic_figures_parse():
    # the committed summary carries the hash of the kernel sources it was
    # taken from and the scaled FETCH/WRITE bytes per bulk launch
    text = open(bench.PROFILE).read()
    fields = {}
    for line in text.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    for key in ("kernel_source_sha256", "bulk_fetch_bytes_per_launch",
                "bulk_write_bytes_per_launch", "bulk_avg_launch_us"):
        assert key in fields, key
    assert len(fields["kernel_source_sha256"]) == 64
    fetch = float(fields["bulk_fetch_bytes_per_launch"])
    write = float(fields["bulk_write_bytes_per_launch"])
    # at least the algorithmic C read + write of one n=16384, tile-128 launch
    algorithmic_c = 16256 ** 2 * 4
    assert fetch >= algorithmic_c and write >= 0.9 * algorithmic_c
    t = bench.measured_traffic()
    assert t is None or abs(t - (fetch + write)) < 1.0


def test_bits_profile_traffic_figures_parse(tmp_path):
    # the bit-packed reachability summary: the same fields, bytes at least the
    # bulk words read and written once at n=16384; a different source hash
    # turns the figure off
    text = open(bench.BITS_PROFILE).read()
    fields = {}
    for line in text.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    assert len(fields["kernel_source_sha256"]) == 64
    fetch = float(fields["bulk_fetch_bytes_per_launch"])
    write = float(fields["bulk_write_bytes_per_launch"])
    words = 16128 * 504 * 4
    assert fetch >= words and write >= words
    t = bench.measured_traffic(bench.BITS_PROFILE, bench.BITS_SOURCES)
    assert t is None or abs(t - (fetch + write)) < 1.0
    stale = tmp_path / "stale.md"
    stale.write_text(text.replace(fields["kernel_source_sha256"], "0" * 64))
    assert bench.measured_traffic(str(stale), bench.BITS_SOURCES) is None


def test_cpu_baseline_leg_matches_the_oracle_prefix():
    W = gen.dense_graph(96, 0.3, 1, 1000, seed=3)
    out = bench.cpu_baseline(W, 40, 8)
    assert out["kind"] == "oracle" and out["unit"] == "cell-updates/s"
    assert out["cores"] >= 1 and out["value"] > 0
    assert out["one_core"]["cores"] == 1 and out["one_core"]["value"] > 0
    assert out["cpu_model"] is None or isinstance(out["cpu_model"], str)
    # the leg runs the first 40 k-iterations of the plain loop: compare with
    # the same prefix computed directly
    ref = np.array(W, copy=True)
    oracle.fw_inplace(ref, nthreads=1, k_begin=0, k_end=40)
    work = np.array(W, copy=True)
    oracle.fw_inplace(work, nthreads=oracle.max_threads(), k_begin=0, k_end=40)
    assert np.array_equal(work, ref)
