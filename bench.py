#!/usr/bin/env python3
"""Benchmark: blocked Floyd-Warshall APSP on one MI355X.

    python bench.py [--steps K] [--warmup W] [--n 16384]

One step = one whole solve of the n=16384 fp32 graph (edge prob 0.3, integer
weights in [1, 1000]): every stage and phase of the blocked sweep.  The input
is generated once; one resident copy per timed step is filled in HBM before
the timed region starts.

Prints ONE JSON line with the metric (n^3 cell updates per second), the bulk
kernel's roofline figures (HIP events around every phase launch inside the
timed region) and the CPU oracle timed on the host on a bounded sample of the
same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X's published fp32 vector peak, 157.3 TFLOP/s = 256 CUs x 2.4 GHz x
# 256 flops per clock per CU, an FMA counting two flops: 7.86e13 32-bit
# lane-operations per second.  A cell update is two operations (one add, one
# min), so the roofline's "achieved" is 2 x updates/s in TFLOP/s against this
# peak.  The ceiling of the bulk's own instruction mix (two v_add_f32 and one
# v_minimum3_f32 per two updates: 1.5 lane-instructions per update; packed
# fp32 is not used) is reported beside it, from the issue-rate probe run in
# the same process (bench_valu_probe).
FP32_VECTOR_PEAK_FLOPS = 157.3e12
OPS_PER_UPDATE = 2
VALU_LANE_OPS_PER_S = FP32_VECTOR_PEAK_FLOPS / 2
MIX_INSTR_PER_UPDATE = 1.5
CUS, CLOCK_HZ = 256, 2.4e9


PROFILE = os.path.join(ROOT, "profiles", "bulk_dma_kernel_f32_t128_n16384.md")
KERNEL_SOURCES = ("paper_1001_4108_amd/csrc/fw_tiles.h", "paper_1001_4108_amd/csrc/fw_kernels.hip")
BITS_PROFILE = os.path.join(ROOT, "profiles", "bits_kernels_reachability_n16384.md")
BITS_SOURCES = ("paper_1001_4108_amd/csrc/fw_bits.hip",)
# Bit-packed reachability: the bulk needs 1.125 lane-instructions per 32-cell
# word-update (one v_and_or_b32, plus one v_bfe_i32 per 8 words); its peak is
# the published lane-operation rate at that count
BITS_INSTR_PER_WORD = 1.125
BITS_WORD_PEAK = VALU_LANE_OPS_PER_S / BITS_INSTR_PER_WORD


def measured_traffic(profile=PROFILE, sources=KERNEL_SOURCES):
    """HBM bytes per bulk launch from a committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (already scaled by the copy-kernel calibration), or
    None when the kernel sources changed since the counters were taken."""
    import hashlib
    try:
        text = open(profile).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.split(":", 1)[0].strip() in (
                "kernel_source_sha256", "bulk_fetch_bytes_per_launch",
                "bulk_write_bytes_per_launch"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if vals.get("kernel_source_sha256") != h.hexdigest():
        return None
    try:
        return float(vals["bulk_fetch_bytes_per_launch"]) + float(vals["bulk_write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--cpu-ksteps", type=int, default=2048,
                    help="k-iterations of the oracle timed for the CPU baseline")
    ap.add_argument("--cpu-ksteps-one-core", type=int, default=96,
                    help="k-iterations of the oracle timed on one thread")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-pred-f32", action="store_true",
                    help="skip the fp32 n=8192 solve with predecessors")
    ap.add_argument("--no-captured", action="store_true",
                    help="skip timing the solve as one captured-graph launch")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the vector-ALU issue-rate probe")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the n=512 latency / per-phase bandwidth leg")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the per-phase HIP events (plain timed region)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-ladder", action="store_true",
                    help="skip the ablation-ladder leg (rungs 0-4 at n=4096)")
    ap.add_argument("--no-maxmin", action="store_true",
                    help="skip the n=16384 widest-path (max, min) solve")
    ap.add_argument("--no-closure", action="store_true",
                    help="skip the n=16384 bit-packed reachability leg")
    ap.add_argument("--no-negative", action="store_true",
                    help="skip the n=8192 int32 negative-weight solve with predecessors")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="arrival window of the serving trace at the configured rate")
    ap.add_argument("--serve-uncapped-seconds", type=float, default=4.0,
                    help="arrival window of the same trace replayed without the queue cap")
    ap.add_argument("--serve-point-seconds", type=float, default=10.0,
                    help="arrival window of the 0.5x / 0.9x capacity load points")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--batched-reps", type=int, default=5)
    ap.add_argument("--batched-modes", default="graph,kernel,per_graph",
                    help="batch-plan launch modes to time (comma-separated)")
    ap.add_argument("--batched-tiles", default="",
                    help="tiles of the size buckets 16-32,33-64,65-128,129-256,257-512 "
                         "(comma-separated) instead of autotuning them; 9 values split "
                         "129-512 into buckets 64 vertices wide")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


PROBE_FORMS = {0: "v_add_f32", 1: "fp32 min-plus (2 v_add_f32 + v_minimum3_f32)",
               2: "int32 min-plus (2 v_add_u32 + v_min3_i32)", 3: "v_fma_f32",
               4: "v_and_or_b32", 5: "v_add_u32", 6: "v_min3_i32", 7: "v_minimum3_f32",
               8: "2 v_add_u32 + v_minimum3_f32",
               9: "fp32 max-min (2 v_minimum3_f32 as two-input minima + v_maximum3_f32)",
               10: "v_min_f32", 11: "v_min_i32"}


def bench_valu_probe(torch, dev):
    """Issue rates of the kernels' instruction mixes (probe/valu_probe.hip):
    register-only loops, 2048 workgroups of 256 threads, timed by HIP events
    on the current stream.  Lane-instructions per second, and per clock per CU
    at the 2.4 GHz nominal clock."""
    import ctypes
    from paper_1001_4108_amd import build as libbuild
    L = ctypes.CDLL(libbuild.PROBE_OUT)
    L.fw_probe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]
    blocks = 2048
    src = torch.rand(4096, device=dev) * 100
    dst = torch.empty(blocks * 256 * 64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    out = {"what": "register-only loops of one instruction mix, 2048 x 256 threads; "
                   "lanes per clock per CU at the 2.4 GHz nominal clock",
           "published_lane_ops_per_clk_per_cu": VALU_LANE_OPS_PER_S / (CUS * CLOCK_HZ),
           "forms": {}}
    for form, what in PROBE_FORMS.items():
        per_step = L.fw_probe_valu_instr_per_step(form)
        iters = 20000 if per_step > 64 else 60000
        ms = ctypes.c_float(0)
        rc = L.fw_probe_valu(form, blocks, iters, src.data_ptr(), dst.data_ptr(),
                             ctypes.c_void_p(stream), ctypes.byref(ms))
        if rc != 0:
            raise RuntimeError(f"valu probe form {form} failed ({rc})")
        lane_instr = float(blocks) * 256 * iters * per_step
        rate = lane_instr / (ms.value / 1e3)
        out["forms"][what] = {"lane_instr_per_s": rate, "ms": ms.value,
                              "lanes_per_clk_per_cu": rate / (CUS * CLOCK_HZ)}
    mix = out["forms"][PROBE_FORMS[1]]["lane_instr_per_s"]
    out["fp32_minplus_update_ceiling"] = mix / MIX_INSTR_PER_UPDATE
    out["int32_minplus_update_ceiling"] = out["forms"][PROBE_FORMS[2]]["lane_instr_per_s"] / 1.5
    out["fp32_maxmin_update_ceiling"] = out["forms"][PROBE_FORMS[9]]["lane_instr_per_s"] / 1.5
    return out


def bench_small(torch, fw, gen, dev, reps=50):
    """n=512 fp32 (edge prob 0.5, weights [1,100]): solve latency as eager
    launches and as one captured-graph launch (solve plan), per-phase time
    and achieved HBM bandwidth over each phase's algorithmic bytes, and the
    whole result against the oracle."""
    import numpy as np
    import oracle
    W = gen.single_graph_512()
    n = W.shape[0]
    pristine = torch.from_numpy(W).to(dev)
    work = torch.empty_like(pristine)
    tile = fw.plan_tile(torch.float32, n)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    plan = fw.SolvePlan(work)
    out = {"workload": f"single dense directed graph n={n} fp32, edge prob 0.5, integer "
                       f"weights [1,100]", "tile": tile}
    for mode in ("eager", "graph"):
        times = []
        for r in range(reps + 3):
            work.copy_(pristine)
            ev0.record()
            plan.launch(mode)
            ev1.record()
            torch.cuda.synchronize(dev)
            if r >= 3:
                times.append(ev0.elapsed_time(ev1))
        ms = float(np.median(times))
        out[mode] = {"ms": ms, "updates_per_s": float(n) ** 3 / (ms / 1e3)}
    ok = bool(np.array_equal(work.cpu().numpy().view(np.uint32), oracle.fw(W).view(np.uint32)))
    # phase times of eager solves (HIP events around every launch)
    fw.profile_read()
    fw.profile_enable(True)
    for _ in range(reps):
        work.copy_(pristine)
        plan.launch("eager")
    torch.cuda.synchronize(dev)
    fw.profile_enable(False)
    prof = fw.profile_read()
    s, m = tile, n - tile
    nb = n // tile
    # algorithmic bytes per launch (n a multiple of the tile): the diagonal
    # tile read and written; both panels read and written plus the diagonal
    # tile read; the bulk read and written plus both panels read (plus the
    # next diagonal tile closed by the launch, read and written)
    per_launch = {"diag": 2 * s * s * 4, "panel": (4 * m * s + s * s) * 4,
                  "bulk": (2 * m * m + 2 * m * s) * 4 + 2 * s * s * 4}
    phases = {}
    for k, b in per_launch.items():
        ms, cnt, upd = prof[k]
        if cnt:
            us = ms * 1e3 / cnt
            phases[k] = {"launches_per_solve": cnt / reps, "us_per_launch": us,
                         "bytes_per_launch": b, "gb_per_s": b / (us * 1e-6) / 1e9}
    out["phases"] = phases
    out["stages"] = nb
    out["check"] = "ok" if ok else "mismatch"
    plan.destroy()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(W, ksteps, ksteps_one_core):
    """Oracle (plain triple loop) on the same matrix, first `ksteps`
    k-iterations on all host threads, then `ksteps_one_core` on one thread
    (the paper's CPU column is one core)."""
    import numpy as np
    import oracle
    n = W.shape[0]
    work = np.array(W, copy=True)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.fw_inplace(work, nthreads=threads, k_begin=0, k_end=ksteps)
    dt = time.perf_counter() - t0
    upd = float(ksteps) * n * n
    work = np.array(W, copy=True)
    t0 = time.perf_counter()
    oracle.fw_inplace(work, nthreads=1, k_begin=0, k_end=ksteps_one_core)
    dt1 = time.perf_counter() - t0
    upd1 = float(ksteps_one_core) * n * n
    return {"value": upd / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"first {ksteps} of {n} k-iterations of the plain triple loop on the "
                      f"same n={n} fp32 matrix ({upd:.3e} updates, {dt:.1f} s)",
            "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "one_core": {"value": upd1 / dt1, "unit": "cell-updates/s", "cores": 1,
                         "sample": f"first {ksteps_one_core} k-iterations, one thread "
                                   f"({upd1:.3e} updates, {dt1:.1f} s)"}}


def pack_graphs(graphs, torch, dev):
    """One device pool; graph g is an n x n view (ld = n rounded up to 4,
    16-byte aligned origin) so every graph takes the vectorised path."""
    import numpy as np
    lds = [(w.shape[0] + 3) // 4 * 4 for w in graphs]
    offs = np.concatenate([[0], np.cumsum([w.shape[0] * l for w, l in zip(graphs, lds)])])
    host = np.full(int(offs[-1]) + 4, np.inf, dtype=np.float32)
    for w, l, o in zip(graphs, lds, offs):
        n = w.shape[0]
        host[o:o + n * l].reshape(n, l)[:, :n] = w
    pool = torch.from_numpy(host).to(dev)
    views = [pool[o:o + w.shape[0] * l].view(w.shape[0], l)[:, :w.shape[0]]
             for w, l, o in zip(graphs, lds, offs)]
    return pool, views


def bench_maxmin(torch, fw, W, dev, reps=3):
    """Widest paths over the (max, min) semiring on the same n=16384 edges
    (absent = -INF, diagonal +INF): the same kernels, another semiring."""
    import numpy as np
    import oracle
    from paper_1001_4108_amd import gen
    n = W.shape[0]
    Wm = np.where(np.isinf(W), np.float32(-np.inf), W).astype(np.float32)
    np.fill_diagonal(Wm, np.inf)
    pristine = torch.from_numpy(Wm).to(dev)
    work = torch.empty_like(pristine)
    work.copy_(pristine)
    fw.fw_apsp_semiring(work, "maxmin")
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(reps):
        work.copy_(pristine)
        fw.fw_apsp_semiring(work, "maxmin")
    torch.cuda.synchronize(dev)
    ms = (time.perf_counter() - t0) * 1e3 / reps
    srcs = gen.dijkstra_sources_16384(n, 2) if n >= 2 else np.arange(n)
    rows = work[torch.from_numpy(srcs).to(dev)].cpu().numpy()
    ok = bool(np.array_equal(rows.view(np.uint32),
                             oracle.widest_rows(Wm, srcs).astype(np.float32).view(np.uint32)))
    return {"workload": f"widest paths, n={n} fp32 (the same edges, absent -INF)", "ms": ms,
            "updates_per_s": float(n) ** 3 / (ms / 1e3), "check": "ok" if ok else "mismatch"}


def bench_closure(torch, fw, gen, dev, n=16384, reps=5):
    """Reachability (reflexive transitive closure) of an n=16384 digraph with
    edge probability 1.2/n (long paths, many unreachable pairs), bit-packed:
    the closure timed on resident packed words; packing the int32 0/1 matrix
    and unpacking the result timed once each; one closure more with phase
    events for the bulk kernel's roofline; the int32 (max, min) closure of
    the same 0/1 matrix timed once beside it; rows checked against BFS."""
    import numpy as np
    import oracle
    W = gen.dense_graph(n, 1.2 / n, 1, 1, seed=19, dtype=np.int32)
    A = np.where(W == gen.I32_INF, 0, 1).astype(np.int32)
    adj = torch.from_numpy(A).to(dev)
    del A
    pristine = fw.pack_bits(adj)
    torch.cuda.synchronize(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    pristine = fw.pack_bits(adj)
    ev1.record()
    torch.cuda.synchronize(dev)
    ms_pack = ev0.elapsed_time(ev1)
    bits = pristine.clone()
    fw.fw_transitive_closure_bits(bits, n)
    torch.cuda.synchronize(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        bits.copy_(pristine)
        ev0.record()
        fw.fw_transitive_closure_bits(bits, n)
        ev1.record()
        torch.cuda.synchronize(dev)
        times.append(ev0.elapsed_time(ev1))
    ms = float(np.median(times))
    srcs = [0, n // 3, n - 1]
    full = torch.empty((n, n), dtype=torch.int32, device=dev)
    ev0.record()
    fw.unpack_bits(bits, n, out=full)
    ev1.record()
    torch.cuda.synchronize(dev)
    ms_unpack = ev0.elapsed_time(ev1)
    rows = full[torch.tensor(srcs, device=dev)].cpu().numpy()
    del full
    # one more closure with the library's phase events: the bulk kernel's
    # average launch time on its own stream, for the roofline
    fw.profile_read()
    fw.profile_enable(True)
    work = pristine.clone()
    fw.fw_transitive_closure_bits(work, n)
    torch.cuda.synchronize(dev)
    prof = fw.profile_read()
    fw.profile_enable(False)
    del work
    bulk_ms, bulk_launches, _ = prof["bits_bulk"]
    nw = fw.words_per_row(n)
    kb = min(256, n)
    words_per_launch = float(n - kb) * (nw - (kb + 31) // 32) * kb  # every stage: one block out
    avg_us = bulk_ms * 1e3 / max(bulk_launches, 1)
    achieved = words_per_launch / (avg_us * 1e-6) if avg_us > 0 else 0.0
    roofline = {"bound": "alu", "kernel": "bits_bulk_kernel (bulk tiles + next diagonal block)",
                "achieved": achieved / 1e12, "peak": BITS_WORD_PEAK / 1e12,
                "unit": "T word-updates/s (32 cells each)", "frac": achieved / BITS_WORD_PEAK,
                "traffic": measured_traffic(BITS_PROFILE, BITS_SOURCES),
                "traffic_unit": "bytes per bulk launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "avg_launch_us": avg_us, "word_updates_per_launch": words_per_launch,
                "launches": int(bulk_launches),
                "phase_ms": {k: prof[k][0] for k in ("bits_diag", "bits_panel", "bits_bulk")}}
    ok = all(np.array_equal(rows[q].astype(bool), oracle.reach_row(W, s)) for q, s in enumerate(srcs))
    # the same closure through the int32 (max, min) semiring, one cell per int
    adj.fill_diagonal_(1)
    ev0.record()
    fw.fw_apsp_semiring(adj, "maxmin")
    ev1.record()
    torch.cuda.synchronize(dev)
    ms_int = ev0.elapsed_time(ev1)
    ok &= bool(np.array_equal(adj[torch.tensor(srcs, device=dev)].cpu().numpy(), rows))
    del adj
    return {"workload": f"reachability, n={n} digraph, edge prob 1.2/n, bit-packed "
                        f"({n} x {fw.words_per_row(n)} words)",
            "ms": ms, "cell_updates_per_s": float(n) ** 3 / (ms / 1e3),
            "int32_maxmin_ms": ms_int, "speedup_vs_int32_maxmin": ms_int / ms,
            "pack_ms": ms_pack, "unpack_ms": ms_unpack, "roofline": roofline,
            "check": "ok" if ok else "mismatch"}


# The paper's Table 1 at n=4096 (Tesla C1060, seconds): per-task threads,
# 32-wide blocked with tiles in shared memory, its instruction-optimised
# version, and the staged-load kernel.  Context for the ratios only.
PAPER_TABLE1_N4096 = {"per_k": 26.05, "blocked_tiles_in_shared": 4.62,
                      "optimised_blocked": 2.06, "staged_load": 0.934}


def bench_ladder(torch, fw, gen, dev, n=4096, reps=3):
    """The ablation ladder (fw_apsp_ladder rungs 0-4) on one n=4096 fp32 graph
    (edge prob 0.3, integer weights [1,1000]); every rung's result is
    compared bit for bit with rung 4's, which is checked on Dijkstra rows."""
    import numpy as np
    import oracle
    W = gen.dense_graph(n, 0.3, 1, 1000, seed=6)
    pristine = torch.from_numpy(W).to(dev)
    work = torch.empty_like(pristine)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    out = {"workload": f"single dense directed graph n={n} fp32, edge prob 0.3, integer "
                       f"weights [1,1000]", "rungs": {}}
    ref = None
    ok = True
    for rung in (4, 3, 2, 1, 0):
        times = []
        for r in range(reps + 1):
            work.copy_(pristine)
            torch.cuda.synchronize(dev)
            ev0.record()
            fw.fw_apsp_ladder(work, rung)
            ev1.record()
            torch.cuda.synchronize(dev)
            if r:
                times.append(ev0.elapsed_time(ev1))
        got = work.cpu().numpy()
        if ref is None:
            ref = got
            srcs = np.array([0, n // 3, n - 1])
            ok &= bool(np.array_equal(got[srcs], oracle.dijkstra_rows(W, srcs).astype(np.float32)))
        else:
            ok &= bool(np.array_equal(got.view(np.uint32), ref.view(np.uint32)))
        ms = float(np.median(times))
        out["rungs"][str(rung)] = {"what": fw.LADDER_RUNGS[rung], "ms": ms,
                                   "updates_per_s": float(n) ** 3 / (ms / 1e3)}
    r = {k: v["ms"] for k, v in out["rungs"].items()}
    out["ratios"] = {"per_k/blocked_lds": r["0"] / r["1"],
                     "blocked_lds/registers_whole_tiles": r["1"] / r["2"],
                     "registers_whole_tiles/staged_slices": r["2"] / r["3"],
                     "staged_slices/tile128_direct_copy": r["3"] / r["4"],
                     "blocked_lds/best_of_3_4": r["1"] / min(r["3"], r["4"])}
    p = PAPER_TABLE1_N4096
    out["paper_ratios_n4096"] = {
        "per_task/blocked_in_shared": p["per_k"] / p["blocked_tiles_in_shared"],
        "blocked_in_shared/optimised": p["blocked_tiles_in_shared"] / p["optimised_blocked"],
        "optimised/staged_load": p["optimised_blocked"] / p["staged_load"]}
    out["check"] = "ok" if ok else "mismatch"
    return out


def bench_negative(torch, fw, gen, dev, reps=3):
    """n=8192 int32 with negative weights (potential-reweighted), distances plus
    predecessors, and the same solve without predecessors.  Each timed solve
    runs on its own pre-filled copy of the input (the refresh is not timed);
    one more solve with predecessors is timed per phase."""
    import numpy as np
    import oracle
    g = gen.negative_graph_8192()
    n = g.w.shape[0]
    pristine = torch.from_numpy(g.w).to(dev)
    bufs = [torch.empty_like(pristine) for _ in range(reps)]
    P = torch.empty((n, n), dtype=torch.int32, device=dev)
    out = {"workload": "single graph n=8192 int32, edge prob 0.2, base weights [1,1000] "
                       "reweighted by potentials in [-500,500], INT32_MAX/2 absent",
           "n": n, "tile": {"with_pred": fw.plan_tile(torch.int32, n, pred=True),
                            "distances_only": fw.plan_tile(torch.int32, n)}}
    fb0 = fw.pred_fallbacks()
    for mode, pp in (("with_pred", P), ("distances_only", None)):
        bufs[0].copy_(pristine)
        fw.fw_apsp_pred(bufs[0], pp)  # warm-up
        for b in bufs:
            b.copy_(pristine)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for b in bufs:
            fw.fw_apsp_pred(b, pp)
        torch.cuda.synchronize(dev)
        ms = (time.perf_counter() - t0) * 1e3 / reps
        out[mode] = {"ms": ms, "updates_per_s": float(n) ** 3 / (ms / 1e3)}
    # every solve with predecessors took the keyed sweep (its gated 64-bit
    # form stayed closed)
    out["with_pred"]["fallbacks"] = fw.pred_fallbacks() - fb0
    work = bufs[0]
    work.copy_(pristine)
    torch.cuda.synchronize(dev)
    fw.profile_read()
    fw.profile_enable(True)
    fw.fw_apsp_pred(work, P)
    torch.cuda.synchronize(dev)
    fw.profile_enable(False)
    prof = fw.profile_read()
    out["with_pred"]["phases"] = {k: {"ms": v[0], "launches": v[1]} for k, v in prof.items() if v[1]}
    srcs = np.array([17, 4321, 8000])
    idx = torch.from_numpy(srcs).to(dev)
    rows = work[idx].cpu().numpy()
    base = oracle.dijkstra_rows(g.base, srcs)
    ref = (base.astype(np.int64) + g.pot[srcs][:, None] - g.pot[None, :]).astype(np.int32)
    ok = bool(np.array_equal(rows, ref)) and bool(np.array_equal(
        P[idx].cpu().numpy(), oracle.canonical_pred(ref, g.w, rows=srcs)))
    out["check"] = "ok" if ok else "mismatch"
    return out


def bench_pred_f32(torch, fw, gen, dev, reps=3):
    """n=8192 fp32 (edge prob 0.3, integer weights [1,1000]) with predecessors:
    the keyed sweep (integer weights), and for contrast the same graph with
    every weight raised by 0.5, which the keyed sweep hands to the fp32
    canonical path (the distances at tile 64, then every last hop from its
    definition).  Each timed solve on its own pre-filled copy; rows checked
    against the oracle."""
    import numpy as np
    import oracle
    n = 8192
    W = gen.single_graph_16384(n)
    Wh = W.copy()
    Wh[np.isfinite(Wh)] += 0.5
    np.fill_diagonal(Wh, 0)
    P = torch.empty((n, n), dtype=torch.int32, device=dev)
    srcs = np.array([5, 4097, 8000])
    out = {"workload": "single graph n=8192 fp32, edge prob 0.3, integer weights [1,1000], +INF "
                       "absent, with predecessors; canonical path: the same graph + 0.5 per weight",
           "n": n, "tile": {"keyed_sweep": fw.plan_tile(torch.float32, n),
                            "canonical_path_distances": 64}}
    ok = True
    for mode, w, r in (("keyed", W, reps), ("canonical_path", Wh, reps)):
        pristine = torch.from_numpy(w).to(dev)
        bufs = [torch.empty_like(pristine) for _ in range(r)]
        bufs[0].copy_(pristine)
        fw.fw_apsp_pred(bufs[0], P)  # warm-up
        for b in bufs:
            b.copy_(pristine)
        fb0 = fw.pred_fallbacks()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for b in bufs:
            fw.fw_apsp_pred(b, P)
        torch.cuda.synchronize(dev)
        ms = (time.perf_counter() - t0) * 1e3 / r
        out[mode] = {"ms": ms, "updates_per_s": float(n) ** 3 / (ms / 1e3),
                     "fallbacks": fw.pred_fallbacks() - fb0}
        idx = torch.from_numpy(srcs).to(dev)
        rows = bufs[-1][idx].cpu().numpy()
        ref = oracle.dijkstra_rows(w, srcs).astype(np.float32)
        ok &= bool(np.array_equal(rows.view(np.uint32), ref.view(np.uint32)))
        ok &= bool(np.array_equal(P[idx].cpu().numpy(), oracle.canonical_pred(ref, w, rows=srcs)))
        del bufs, pristine
    out["check"] = "ok" if ok else "mismatch"
    return out


def bench_batched(torch, fw, gen, dev, reps, modes=("graph", "kernel", "per_graph"), tiles=None):
    """Ragged batch: 4096 graphs, n log-uniform in [16, 512], fp32."""
    import numpy as np
    import oracle
    graphs = gen.ragged_batch()
    sizes = np.array([w.shape[0] for w in graphs], dtype=np.float64)
    # tile per size bucket, picked by the library's autotuner for the batched
    # launch (installed into the plan table the batch plan reads)
    buckets = [(16, 32), (33, 64), (65, 128), (129, 256), (257, 512)]
    if tiles is not None and len(tiles) == 9:  # buckets 64 vertices wide above 128
        buckets = buckets[:3] + [(lo + 1, lo + 64) for lo in range(128, 512, 64)]
    if tiles is not None and len(tiles) != len(buckets):
        raise SystemExit("--batched-tiles takes 5 tiles (or 9: 16-32, 33-64, 65-128, then "
                         "129-512 in buckets 64 vertices wide)")
    counts = {(lo, hi): int(((sizes >= lo) & (sizes <= hi)).sum()) for lo, hi in buckets}
    batch_tuned = None
    if tiles is None:
        # each bucket tuned on as many graphs as this batch holds in it, then
        # the whole batch's plan launch tuned over buckets 64 vertices wide
        # above 128 (the tile groups share the GPU, which per-bucket timing
        # cannot see)
        tuned = {}
        for lo, hi in buckets:
            tuned.update(fw.autotune(torch.float32, [(lo, hi)], objective="batched",
                                     batch=max(counts[(lo, hi)], 16), reps=3))
        fine = buckets[:3] + [(lo + 1, lo + 64) for lo in range(128, 512, 64)]
        batch_tuned = fw.autotune_batch(torch.float32, [int(v) for v in sizes], fine,
                                        mode="graph", reps=9, passes=2)
    else:  # given tiles (profiling runs: counters distort the autotuner's timings)
        tuned = {}
        for (lo, hi), t in zip(buckets, tiles):
            fw.plan_set(torch.float32, lo, hi, t)
            tuned[(lo, hi)] = {"tile": t, "ms": {}}
    pool, views = pack_graphs(graphs, torch, dev)
    pristine = pool.clone()
    plan = fw.BatchPlan(views)
    out = {"workload": "ragged batch of 4096 fp32 graphs, n log-uniform in [16,512], edge "
                       "prob 0.4, integer weights [1,100]",
           "graphs": len(graphs), "updates": float((sizes ** 3).sum()), "grid": plan.grid,
           "autotuned_tiles": {f"{lo}-{hi}": {"tile": v["tile"], "graphs": counts[(lo, hi)],
                                              "ms_by_tile": {str(t): round(m, 4)
                                                             for t, m in v["ms"].items()}}
                               for (lo, hi), v in tuned.items()}}
    if batch_tuned is not None:
        out["batch_tuned_tiles"] = {f"{lo}-{hi}": {"tile": v["tile"],
                                                   "ms_by_tile": {str(t): round(m, 4)
                                                                  for t, m in v["ms"].items()}}
                                    for (lo, hi), v in batch_tuned.items()}
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # warm-up launches per mode: the first replays of a fresh graph run a few
    # percent slower than the steady state (3.30 vs 3.21 ms measured)
    for mode, nrep, warm in (("graph", reps, 3), ("kernel", reps, 3),
                             ("per_graph", max(1, reps // 2), 1)):
        if mode not in modes:
            continue
        times = []
        for r in range(nrep + warm):
            pool.copy_(pristine)
            torch.cuda.synchronize(dev)
            ev0.record()
            plan.launch(mode)
            ev1.record()
            torch.cuda.synchronize(dev)
            if r >= warm:
                times.append(ev0.elapsed_time(ev1))
        ms = float(np.median(times))
        out[mode] = {"ms": ms, "graphs_per_s": len(graphs) / (ms / 1e3),
                     "updates_per_s": out["updates"] / (ms / 1e3)}
    # spot check 32 graphs against the oracle
    idx = np.linspace(0, len(graphs) - 1, 32).astype(int)
    ok = all(np.array_equal(views[g].cpu().numpy().view(np.uint32),
                            oracle.fw(graphs[g]).view(np.uint32)) for g in idx)
    out["check"] = "ok" if ok else "mismatch"
    if "per_graph" in out and "graph" in out:
        out["speedup_vs_per_graph"] = out["per_graph"]["ms"] / out["graph"]["ms"]
    plan.destroy()
    return out


FW_ERR_BUSY = 5
QUEUE_CAP = 256


def run_trace(torch, fw, srv, bases, tr, limit_s):
    """Open-loop replay: submit each request at its arrival time, then drain."""
    import threading
    import numpy as np
    ids = {}
    t0 = time.perf_counter_ns()
    sub_err = []
    refused = [0]  # requests the server refused at submission (queue cap)

    def submitter():
        try:
            for r in range(len(tr.t)):
                due = t0 + int(tr.t[r] * 1e9)
                while True:
                    now = time.perf_counter_ns()
                    if now >= due:
                        break
                    if due - now > 200_000:
                        time.sleep((due - now - 100_000) / 1e9)
                n, o, b = int(tr.n[r]), int(tr.o[r]), int(tr.b[r])
                try:
                    ids[srv.submit(bases[b][o:o + n, o:o + n])] = r
                except fw.FwError as e:
                    if e.status != FW_ERR_BUSY:
                        raise
                    refused[0] += 1
        except Exception as e:  # surfaced after the join
            sub_err.append(e)

    th = threading.Thread(target=submitter)
    th.start()
    recs = []
    next_report = time.perf_counter() + 15.0
    while th.is_alive():
        recs += srv.poll(timeout_us=20000)
        if time.perf_counter() >= next_report:
            log(f"serving: {len(recs)} completed, {len(ids)} accepted, {refused[0]} refused")
            next_report += 15.0
    th.join()
    if sub_err:
        raise sub_err[0]
    srv.drain(timeout_s=limit_s)
    while len(recs) < len(tr.t) - refused[0]:
        got = srv.poll(timeout_us=100000)
        if not got:
            break
        recs += got
    lat = np.array([(c[6] - c[4]) / 1e6 for c in recs if c[2] == 0])
    first = min(c[4] for c in recs)
    last = max(c[6] for c in recs)
    span = (last - first) / 1e9
    upd = float(sum(float(c[1]) ** 3 for c in recs if c[2] == 0))
    st = srv.stats()
    return {"requests": len(tr.t), "refused": refused[0],
            "completed": int((np.array([c[2] for c in recs]) == 0).sum()),
            "offered_per_s": len(tr.t) / float(tr.t[-1]) if len(tr.t) > 1 else 0.0,
            "solves_per_s": len(lat) / span, "updates_per_s": upd / span, "span_s": span,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "mean_group": float(np.mean([c[3] for c in recs])),
            "batched_groups": st["batched_groups"], "single_groups": st["single_groups"],
            "deferrals": st["deferrals"], "peak_bytes": st["peak_bytes"]}


def bench_serving(torch, fw, gen, dev, seconds, rate, uncapped_seconds, point_seconds):
    """Poisson arrivals, n log-uniform in [64, 8192], fp32 windows of resident
    base graphs; footprint admission into a 32 GiB budget, 4 worker streams.

    The offered load (2000 req/s) is about 2.5x the GPU's capacity, so the
    full trace runs with admission control: at most QUEUE_CAP requests may
    wait for admission and later submissions are refused (FW_ERR_BUSY, counted);
    p50/p99 are over the accepted requests.  The same arrivals without the cap
    are replayed for a shorter prefix (an unbounded queue grows for as long as
    the trace lasts, so its p99 measures the trace length).  Load points at
    0.5x and 0.9x of the capacity measured under the cap follow."""
    import numpy as np
    tr_full = gen.serving_trace(rate=rate, duration=seconds)
    bases = [torch.from_numpy(tr_full.base_graph(b)).to(dev) for b in range(tr_full.nbase)]
    cfg = dict(budget_bytes=32 << 30, streams=4, small_n=512, max_batch=2048)
    out = {"workload": f"Poisson arrivals at {rate:.0f} req/s for {seconds:.1f} s, n log-uniform "
                       "in [64,8192], fp32, edge prob 0.3, integer weights [1,1000] (principal "
                       "windows of 2 resident 8192-vertex base graphs); admission: at most "
                       f"{QUEUE_CAP} requests waiting, later ones refused", "config": cfg}

    def warm(srv):
        for n in (64, 300, 700, 2000):
            srv.submit(bases[0][:n, :n])
        srv.drain(timeout_s=60)
        srv.poll()

    with fw.Server(torch.float32, queue_cap=QUEUE_CAP, **cfg) as srv:
        warm(srv)
        out["at_rate"] = run_trace(torch, fw, srv, bases, tr_full, 600)
    cap = out["at_rate"]["solves_per_s"]
    out["capacity_solves_per_s"] = cap
    with fw.Server(torch.float32, **cfg) as srv:
        warm(srv)
        tr = gen.serving_trace(rate=rate, duration=uncapped_seconds)
        out[f"at_rate_uncapped_first_{uncapped_seconds:g}s"] = run_trace(torch, fw, srv, bases,
                                                                          tr, 600)
        for frac in (0.5, 0.9):
            tr = gen.serving_trace(rate=cap * frac, duration=point_seconds,
                                   seed=50 + int(frac * 10))
            out[f"at_{frac:.1f}x_capacity"] = run_trace(torch, fw, srv, bases, tr, 600)
    # correctness: a few requests of the trace solved through the server with
    # copy-back, compared with the oracle
    import oracle
    rng = np.random.default_rng(9)
    picks = [r for r in rng.permutation(len(tr_full.n)) if tr_full.n[r] <= 700][:6]
    ok = True
    with fw.Server(torch.float32, budget_bytes=1 << 30, streams=2, small_n=512) as srv:
        dsts = []
        for r in picks:
            n, o, b = int(tr_full.n[r]), int(tr_full.o[r]), int(tr_full.b[r])
            dst = torch.empty((n, n), dtype=torch.float32).pin_memory()
            srv.submit(bases[b][o:o + n, o:o + n], dst_host=dst)
            dsts.append((r, dst))
        srv.drain(timeout_s=60)
        for r, dst in dsts:
            ok &= bool(np.array_equal(dst.numpy().view(np.uint32),
                                      oracle.fw(tr_full.request_graph(r)).view(np.uint32)))
    out["check"] = "ok" if ok else "mismatch"
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "this library has no multi-GPU path to time", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1001_4108_amd as fw
    from paper_1001_4108_amd import gen

    n = args.n
    log(f"generating n={n} fp32 graph")
    W = gen.single_graph_16384(n)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pristine = torch.from_numpy(W).to(dev)
    work = torch.empty_like(pristine)
    stream = torch.cuda.current_stream(dev)
    tile = fw.plan_tile(torch.float32, n)
    log(f"tile={tile}; warmup {args.warmup}")

    for _ in range(args.warmup):
        work.copy_(pristine)
        fw.fw_apsp(work)
    torch.cuda.synchronize(dev)

    # one resident copy of the input per timed step, filled before the timed
    # region: a step is the solve alone (the refresh is not timed)
    need = (args.steps - 1) * pristine.numel() * pristine.element_size()
    free = torch.cuda.mem_get_info(dev)[0]
    if need > 0.8 * free:
        sys.exit(f"--steps {args.steps} needs {need / 2**30:.1f} GiB of resident input copies; "
                 f"{free / 2**30:.1f} GiB free")
    inputs = [work] + [torch.empty_like(pristine) for _ in range(args.steps - 1)]

    def refill():
        for buf in inputs:
            buf.copy_(pristine)
        torch.cuda.synchronize(dev)

    refill()
    fw.profile_read()  # drop anything accumulated so far
    if not args.no_profile:
        fw.profile_enable(True)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for i in range(args.steps):
        fw.fw_apsp(inputs[i])
    torch.cuda.synchronize(dev)
    t1 = time.perf_counter()
    fw.profile_enable(False)
    prof = fw.profile_read()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = float(n) ** 3 / (ms_per_step / 1e3)

    # correctness spot check outside the timed region: 4 Dijkstra rows of
    # every solved copy
    import oracle
    srcs = gen.dijkstra_sources_16384(n, 4) if n >= 4 else np.arange(n)
    ref = oracle.dijkstra_rows(W, srcs).astype(np.float32)
    ok = all(np.array_equal(buf[torch.from_numpy(srcs).to(dev)].cpu().numpy().view(np.uint32),
                            ref.view(np.uint32)) for buf in inputs)
    log(f"spot check vs Dijkstra rows: {'ok' if ok else 'MISMATCH'}")

    phases = {}
    roof = None
    if prof:
        for k, (ms, cnt, upd) in prof.items():
            if cnt:
                phases[k] = {"ms_per_step": ms / args.steps, "launches_per_step": cnt / args.steps,
                             "updates_per_step": upd / args.steps}
        if "bulk" in phases and phases["bulk"]["ms_per_step"] > 0:
            b = phases["bulk"]
            per_launch_upd = b["updates_per_step"] / b["launches_per_step"]
            per_launch_s = b["ms_per_step"] / b["launches_per_step"] / 1e3
            ach = per_launch_upd / per_launch_s
            roof = {"bound": "alu", "kernel": "bulk_dma_kernel (bulk tiles + next diagonal closure)",
                    "achieved": ach * OPS_PER_UPDATE / 1e12, "peak": FP32_VECTOR_PEAK_FLOPS / 1e12,
                    "unit": "TFLOP/s", "frac": ach * OPS_PER_UPDATE / FP32_VECTOR_PEAK_FLOPS,
                    "traffic": measured_traffic(),
                    "ops_per_update": OPS_PER_UPDATE,
                    "traffic_unit": "bytes per bulk launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                    "copy-calibrated)",
                    "avg_launch_us": per_launch_s * 1e6,
                    "updates_per_launch": per_launch_upd,
                    "updates_per_s": ach}
        if "panel" in phases and phases["panel"]["ms_per_step"] > 0:
            p = phases["panel"]
            s_ = tile
            pbytes = (4.0 * (n - s_) * s_ + s_ * s_) * 4
            us = p["ms_per_step"] / p["launches_per_step"] * 1e3
            phases["panel"]["bytes_per_launch"] = pbytes
            phases["panel"]["gb_per_s"] = pbytes / (us * 1e-6) / 1e9

    # the same solves as one captured-graph launch of a solve plan each (the
    # stage loop captured once per buffer; inputs refilled before timing)
    captured = None
    if not args.no_captured:
        plans = [fw.SolvePlan(buf) for buf in inputs]
        for plan in plans:  # the first launch captures (and solves)
            plan.launch("graph")
        refill()
        t0 = time.perf_counter()
        for plan in plans:
            plan.launch("graph")
        torch.cuda.synchronize(dev)
        cms = (time.perf_counter() - t0) * 1e3 / args.steps
        captured = {"ms_per_step": cms, "updates_per_s": float(n) ** 3 / (cms / 1e3),
                    "launches_per_graph": 2 * ((n + tile - 1) // tile)}
        ok &= all(np.array_equal(buf[torch.from_numpy(srcs).to(dev)].cpu().numpy().view(np.uint32),
                                 ref.view(np.uint32)) for buf in inputs)
        for plan in plans:
            plan.destroy()
        log(f"captured stage loop: {cms:.2f} ms per step (eager {ms_per_step:.2f})")
    del inputs[1:]

    probe = None
    if not args.no_probe:
        log("vector-ALU issue-rate probe")
        probe = bench_valu_probe(torch, dev)
        if roof:
            ceil = probe["fp32_minplus_update_ceiling"]
            roof["instruction_mix_ceiling"] = {
                "updates_per_s": ceil, "frac": roof["updates_per_s"] / ceil,
                "basis": "measured issue rate of the bulk's instruction mix (2 v_add_f32 + "
                         "1 v_minimum3_f32 per two updates) on this GPU, this run"}

    small = None
    if not args.no_small:
        log("n=512 solve latency and per-phase bandwidth")
        small = bench_small(torch, fw, gen, dev)
        log(f"n=512: {small['eager']['ms']:.3f} ms eager, {small['graph']['ms']:.3f} ms graph")

    maxmin = None
    if not args.no_maxmin:
        log("widest paths (max, min) n=16384")
        maxmin = bench_maxmin(torch, fw, W, dev)
        if probe is not None:  # the issue-rate ceiling of its own instruction mix
            maxmin["mix_ceiling_updates_per_s"] = probe["fp32_maxmin_update_ceiling"]
            maxmin["of_mix_ceiling"] = maxmin["updates_per_s"] / probe["fp32_maxmin_update_ceiling"]

    closure = None
    if not args.no_closure:
        log("reachability (bit-packed) n=16384")
        closure = bench_closure(torch, fw, gen, dev)
        log(f"reachability: {closure['ms']:.2f} ms (int32 max-min {closure['int32_maxmin_ms']:.0f} ms)")

    ladder = None
    if not args.no_ladder:
        log("ablation ladder n=4096 (rungs 4..0)")
        ladder = bench_ladder(torch, fw, gen, dev)
        log("ladder ms: " + ", ".join(f"{k}: {v['ms']:.1f}" for k, v in ladder["rungs"].items()))

    negative = None
    if not args.no_negative:
        log("negative-weight int32 n=8192 with predecessors")
        negative = bench_negative(torch, fw, gen, dev)
        log(f"negative: {negative['with_pred']['ms']:.1f} ms with predecessors, "
            f"{negative['distances_only']['ms']:.1f} ms distances only")

    pred_f32 = None
    if not args.no_pred_f32:
        log("fp32 n=8192 with predecessors (keyed, and the canonical path)")
        pred_f32 = bench_pred_f32(torch, fw, gen, dev)
        log(f"fp32 predecessors: {pred_f32['keyed']['ms']:.1f} ms keyed, "
            f"{pred_f32['canonical_path']['ms']:.1f} ms canonical path")

    batched = None
    if not args.no_batched:
        log("batched: 4096 ragged graphs")
        tiles = [int(t) for t in args.batched_tiles.split(",")] if args.batched_tiles else None
        batched = bench_batched(torch, fw, gen, dev, args.batched_reps,
                                tuple(args.batched_modes.split(",")), tiles)
        log("batched: " + ", ".join(f"{m} {batched[m]['graphs_per_s']:.0f} graphs/s"
                                    for m in ("graph", "kernel", "per_graph") if m in batched))

    serving = None
    if not args.no_serving:
        log(f"serving: {args.serve_rate:.0f} req/s for {args.serve_seconds:.1f} s")
        serving = bench_serving(torch, fw, gen, dev, args.serve_seconds, args.serve_rate,
                                args.serve_uncapped_seconds, args.serve_point_seconds)
        a = serving["at_rate"]
        log(f"serving, queue cap {QUEUE_CAP}: {a['solves_per_s']:.0f} solves/s, "
            f"{a['refused']} of {a['requests']} refused, p50 {a['p50_ms']:.1f} ms, "
            f"p99 {a['p99_ms']:.1f} ms at {args.serve_rate:.0f} req/s offered")
        for k in ("at_0.5x_capacity", "at_0.9x_capacity"):
            c = serving[k]
            log(f"serving {k}: p50 {c['p50_ms']:.1f} ms, p99 {c['p99_ms']:.1f} ms")

    cpu = None
    if not args.no_cpu:
        log(f"cpu baseline: {args.cpu_ksteps} oracle k-iterations")
        cpu = cpu_baseline(W, min(args.cpu_ksteps, n), min(args.cpu_ksteps_one_core, n))

    out = {
        "metric": "n^3 cell-updates/s at n=16384 fp32 (% VALU peak); batched graphs/s; p99 latency",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"single dense directed graph n={n} fp32, edge prob 0.3, "
                               f"integer weights [1,1000], +INF absent",
                   "n": n, "tile": tile, "global_batch": 1, "parallelism": "single-gpu"},
        "frac_of_fp32_vector_peak": value * OPS_PER_UPDATE / FP32_VECTOR_PEAK_FLOPS,
        "check": "ok" if ok else "mismatch",
        "phases": phases, "captured_graph": captured, "roofline": roof, "cpu_baseline": cpu,
        "valu_probe": probe,
        "small_n512": small, "negative_int32_pred": negative, "pred_f32": pred_f32,
        "maxmin": maxmin,
        "transitive_closure": closure, "ladder": ladder,
        "batched": batched,
        "serving": serving,
        "paper_context": {"tesla_c1060_s_n16384": 53.06,
                          "speedup_vs_paper": 53.06 / (ms_per_step / 1e3) if n == 16384 else None},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
