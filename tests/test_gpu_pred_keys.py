"""Solves with predecessors: the 32-bit keyed sweep and its fallback.

fw_apsp_pred first sweeps (distance, last hop) pairs packed into 32-bit
integer keys and falls back (queued behind it, gated on a device flag) when
an entry is not an integer with |w| < 2^14, a distance met during the sweep
has |d| >= 2^14 or a diagonal entry ends negative: int32 to the pair form
with 64-bit keys; fp32 to the canonical path, or to the compare form after a
negative diagonal.  Both must give the oracle's d and canonical P
bit for bit; fw.pred_fallbacks() tells which one ran.

* in-range graphs take the keyed path (no fallback) at every tile;
* the exact range edge: an edge of weight +-(2^14 - 1) stays keyed, +-2^14
  falls back; on a weight-4 cycle the distances cross 2^14 mid-sweep between
  n = 4096 (max 16380) and n = 4097 (max 16384);
* unreachable pairs: the keyed unpack writes the value the int32 sweep over
  the complete graph reaches (FW_I32_INF + row minimum + column minimum);
* differential: appending two isolated vertices joined by one edge of weight
  20000 forces the fallback without changing any result on the original
  vertices, so keyed and 64-bit results are compared on graphs the oracle's
  canonical reading does not cover (absent and positive diagonal entries);
* negative cycles fall back; captured solve plans replay both paths;
  a side stream gets the same bits;
* fp32: integer weights keyed (also n=5000, tile 128); fractional and large
  weights take the canonical path (the distances, then every last hop from
  its definition over the saved weights), a negative diagonal the compare
  form; unreachable pairs stay +INF; keyed vs fallback differential, plan
  replays of both paths.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1001_4108_amd as fw
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu

INF = gen.I32_INF


def _solve(w, tile=None, stream=None):
    n = w.shape[0]
    d = torch.from_numpy(np.ascontiguousarray(w)).cuda()
    P = torch.full((n, n), -77, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()  # inputs in place before another stream reads them
    if tile is None:
        fw.fw_apsp_pred(d, P, stream=stream)
    else:
        fw.fw_apsp_plan(d, tile, P, stream=stream)
    torch.cuda.synchronize()
    return d.cpu().numpy(), P.cpu().numpy()


def _check_oracle(w, d, P):
    ref = oracle.fw(w)
    assert np.array_equal(d, ref)
    assert np.array_equal(P, oracle.canonical_pred(ref, w))


def _forced(w):
    """w plus vertices n, n+1 (isolated from w) with the edge n -> n+1 of
    weight 20000: the keyed sweep gives up, nothing on w's vertices changes."""
    n = w.shape[0]
    f = np.full((n + 2, n + 2), INF, dtype=np.int32)
    f[:n, :n] = w
    f[n, n] = f[n + 1, n + 1] = 0
    f[n, n + 1] = 20000
    return f


@pytest.mark.parametrize("n,tile", [(2000, None), (777, None), (300, 32), (300, 64), (300, 128),
                                    (129, 128), (64, 64)])
def test_keyed_path_taken_and_exact(n, tile):
    g = gen.reweighted_graph(n, 0.2, 1, 1000, -500, 500, seed=100 + n)
    print(f"[pred keys] keyed n={n} tile={tile}", flush=True)
    before = fw.pred_fallbacks()
    d, P = _solve(g.w, tile)
    assert fw.pred_fallbacks() == before
    _check_oracle(g.w, d, P)


def test_large_weights_fall_back_exact():
    g = gen.reweighted_graph(700, 0.1, 1, 30000, -500, 500, seed=7)
    print("[pred keys] large weights n=700", flush=True)
    before = fw.pred_fallbacks()
    d, P = _solve(g.w)
    assert fw.pred_fallbacks() == before + 1
    _check_oracle(g.w, d, P)


@pytest.mark.parametrize("wt,falls", [(16383, False), (16384, True), (-16383, False),
                                      (-16384, True)])
def test_range_edge_on_one_edge(wt, falls):
    n = 300
    w = gen.dense_graph(n, 0.3, 1, 100, seed=11, dtype=np.int32)
    a, b = 5, 200
    w[:, a] = INF          # nothing enters a: no cycle through the heavy edge
    w[a, a] = 0
    w[a, b] = wt
    print(f"[pred keys] edge weight {wt}", flush=True)
    before = fw.pred_fallbacks()
    d, P = _solve(w)
    assert fw.pred_fallbacks() == before + (1 if falls else 0)
    _check_oracle(w, d, P)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n,falls", [(4096, False), (4097, True)])
def test_range_crossed_mid_sweep(n, falls):
    # weight-4 cycle over a seeded permutation: d_ij = 4 ((pos_j - pos_i) mod n),
    # built up stage by stage; n = 4097 reaches 16384 only on the longest paths
    perm = gen.cycle_permutation(n, seed=n)
    pos = np.empty(n, np.int64)
    pos[perm] = np.arange(n)
    w = np.full((n, n), INF, dtype=np.int32)
    np.fill_diagonal(w, 0)
    w[perm, np.roll(perm, -1)] = 4
    print(f"[pred keys] weight-4 cycle n={n}", flush=True)
    before = fw.pred_fallbacks()
    d, P = _solve(w)
    assert fw.pred_fallbacks() == before + (1 if falls else 0)
    dist = 4 * ((pos[None, :] - pos[:, None]) % n)
    assert np.array_equal(d, dist.astype(np.int32))
    last = np.broadcast_to(perm[(pos - 1) % n].astype(np.int32), (n, n)).copy()
    np.fill_diagonal(last, -1)
    assert np.array_equal(P, last)


@pytest.mark.parametrize("n,p,seed", [(1500, 0.003, 1), (600, 0.01, 2), (333, 0.0, 3)])
def test_unreachable_pairs_keyed(n, p, seed):
    # small weights: long sparse paths stay far inside |d| < 2^14
    g = gen.reweighted_graph(n, p, 1, 100, -100, 100, seed=seed)
    print(f"[pred keys] sparse n={n} p={p}", flush=True)
    before = fw.pred_fallbacks()
    d, P = _solve(g.w)
    assert fw.pred_fallbacks() == before
    ref = oracle.fw(g.w)
    assert (ref > INF // 2).any()          # the case under test is there
    assert np.array_equal(d, ref)
    assert np.array_equal(P, oracle.canonical_pred(ref, g.w))


def _differential(w):
    n = w.shape[0]
    before = fw.pred_fallbacks()
    d, P = _solve(w)
    mid = fw.pred_fallbacks()
    fd, fP = _solve(_forced(w))
    assert fw.pred_fallbacks() == mid + 1
    assert mid == before                   # the graph itself stays keyed
    assert np.array_equal(d, fd[:n, :n])
    assert np.array_equal(P, fP[:n, :n])
    _check_oracle(w, d, P)


@pytest.mark.parametrize("seed", range(8))
def test_keyed_equals_fallback_random(seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(40, 900))
    p = float(rng.choice([0.002, 0.02, 0.2, 0.6]))
    # edges of at most 300: a path needs over 50 hops to reach |d| = 2^14
    g = gen.reweighted_graph(n, p, 1, int(rng.integers(2, 100)), -100, 100, seed=seed)
    w = g.w
    # some absent and some positive diagonal entries (allowed by the contract)
    k = rng.choice(n, size=min(n, 7), replace=False)
    w[k[:3], k[:3]] = INF
    w[k[3:], k[3:]] = rng.integers(1, 50, size=len(k[3:]))
    print(f"[pred keys] differential seed={seed} n={n} p={p}", flush=True)
    _differential(w)


def test_negative_cycle_falls_back():
    w, cyc = gen.planted_negative_cycle(400, 0.2, 5, seed=21)
    print("[pred keys] planted negative cycle", flush=True)
    before = fw.pred_fallbacks()
    d, P = _solve(w)
    assert fw.pred_fallbacks() == before + 1
    neg = np.flatnonzero(np.diag(d) < 0)
    assert set(neg.tolist()) == set(int(c) for c in cyc)


@pytest.mark.parametrize("heavy", [False, True])
def test_solve_plan_replays(heavy):
    hi = 30000 if heavy else 1000
    g = gen.reweighted_graph(1000, 0.2, 1, hi, -500, 500, seed=33)
    n = g.w.shape[0]
    print(f"[pred keys] solve plan heavy={heavy}", flush=True)
    ref_d, ref_P = _solve(g.w)
    src = torch.from_numpy(g.w).cuda()
    d = src.clone()
    P = torch.empty((n, n), dtype=torch.int32, device="cuda")
    plan = fw.SolvePlan(d, P)
    try:
        for rep in range(3):
            d.copy_(src)
            P.fill_(-77)
            before = fw.pred_fallbacks()
            plan.launch("graph")
            torch.cuda.synchronize()
            assert fw.pred_fallbacks() == before + (1 if heavy else 0), rep
            assert np.array_equal(d.cpu().numpy(), ref_d), rep
            assert np.array_equal(P.cpu().numpy(), ref_P), rep
    finally:
        plan.destroy()


def test_side_stream_same_bits():
    g = gen.reweighted_graph(900, 0.2, 1, 1000, -500, 500, seed=44)
    print("[pred keys] side stream", flush=True)
    ref_d, ref_P = _solve(g.w)
    s = torch.cuda.Stream()
    d, P = _solve(g.w, stream=s)
    assert np.array_equal(d, ref_d) and np.array_equal(P, ref_P)


# ---------------------------------------------------------------------------
# fp32: integer weights with |w| < 2^14 take the same keyed sweep (fp32
# arithmetic on them is exact); anything else takes the fp32 canonical path,
# or the compare form after a negative diagonal.  Unreachable pairs stay +INF.
# ---------------------------------------------------------------------------
def _f32(g_w):
    w = g_w.astype(np.float32)
    w[g_w == INF] = np.inf
    return w


@pytest.mark.parametrize("n,tile", [(2000, None), (777, None), (300, 32), (300, 64), (300, 128),
                                    (5000, None)])
def test_f32_keyed_path_taken_and_exact(n, tile):
    g = gen.reweighted_graph(n, 0.2, 1, 1000, -500, 500, seed=300 + n)
    w = _f32(g.w)
    print(f"[pred keys] f32 keyed n={n} tile={tile}", flush=True)
    before = fw.pred_fallbacks()
    d, P = _solve(w, tile)
    assert fw.pred_fallbacks() == before
    ref = oracle.fw(w)
    assert np.array_equal(d.view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(P, oracle.canonical_pred(ref, w))


@pytest.mark.parametrize("what", ["half", "large", "sparse"])
def test_f32_fallbacks_and_unreachable(what):
    n = 600
    if what == "half":     # fractional weights: the canonical path (exact: multiples of 1/2)
        w = gen.dense_graph(n, 0.2, 1, 100, seed=31, dtype=np.float32)
        w[np.isfinite(w)] += 0.5
        np.fill_diagonal(w, 0)
        falls = True
    elif what == "large":  # integer, but beyond the key range
        w = gen.dense_graph(n, 0.2, 1, 40000, seed=32, dtype=np.float32)
        falls = True
    else:                  # unreachable pairs: +INF, keyed
        w = gen.dense_graph(n, 0.004, 1, 100, seed=33, dtype=np.float32)
        falls = False
    print(f"[pred keys] f32 {what}", flush=True)
    before = fw.pred_fallbacks()
    d, P = _solve(w)
    assert fw.pred_fallbacks() == before + (1 if falls else 0)
    ref = oracle.fw(w)
    if what == "sparse":
        assert np.isinf(ref).any()
    assert np.array_equal(d.view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(P, oracle.canonical_pred(ref, w))


@pytest.mark.parametrize("n,p,tile", [(2, 1.0, None), (37, 0.3, None), (64, 0.3, None),
                                      (1100, 0.05, 128), (1500, 0.001, None),
                                      (2100, 0.03, None)])
def test_f32_canonical_path(n, p, tile):
    """Fractional weights leave the keyed sweep for the fp32 canonical path:
    the distances, then each last hop from its definition, in strips of up to
    1024 columns.  One and several strips, ragged tiles and strips, a
    2-vertex graph, unreachable pairs (p=0.001), a 128-wide keyed sweep."""
    w = gen.dense_graph(n, p, 1, 100, seed=900 + n, dtype=np.float32)
    w[np.isfinite(w)] += 0.25
    np.fill_diagonal(w, 0)
    print(f"[pred keys] f32 canonical path n={n} p={p} tile={tile}", flush=True)
    before = fw.pred_fallbacks()
    d, P = _solve(w, tile)
    assert fw.pred_fallbacks() == before + 1
    ref = oracle.fw(w)
    if p <= 0.001:
        assert np.isinf(ref).any()
    assert np.array_equal(d.view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(P, oracle.canonical_pred(ref, w))


def test_f32_canonical_path_negative_weights():
    """Negative fractional weights (a reweighted graph, every real edge
    raised by 0.25: cycles stay positive) through the canonical path: the
    distances and every last hop against the oracle."""
    n = 700
    g = gen.reweighted_graph(n, 0.1, 1, 200, -100, 100, seed=808)
    w = _f32(g.w)
    off = np.isfinite(w) & ~np.eye(n, dtype=bool)
    w[off] += 0.25
    assert (w[off] < 0).any()
    print("[pred keys] f32 canonical path, negative weights", flush=True)
    before = fw.pred_fallbacks()
    d, P = _solve(w)
    assert fw.pred_fallbacks() == before + 1
    ref = oracle.fw(w)
    assert (ref < 0).any()
    assert np.array_equal(d.view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(P, oracle.canonical_pred(ref, w))


def test_f32_canonical_path_beyond_the_keys_plan_replays():
    """The canonical path beyond the keys captured in a solve plan (its
    scratch the plan's): two graph replays, each after fresh input, give the
    eager solve's bits."""
    n = 16390
    w = gen.dense_graph(n, 0.002, 1, 100, seed=515, dtype=np.float32)
    w[np.isfinite(w)] += 0.5
    np.fill_diagonal(w, 0)
    print(f"[pred keys] f32 canonical path beyond the keys, plan replays n={n}", flush=True)
    src = torch.from_numpy(w).cuda()
    d = src.clone()
    P = torch.empty((n, n), dtype=torch.int32, device="cuda")
    fw.fw_apsp_pred(d, P)
    torch.cuda.synchronize()
    ref_d, ref_P = d.clone(), P.clone()
    plan = fw.SolvePlan(d, P)
    try:
        for rep in range(2):
            d.copy_(src)
            P.fill_(-77)
            plan.launch("graph")
            torch.cuda.synchronize()
            assert torch.equal(d.view(torch.int32), ref_d.view(torch.int32)), rep
            assert torch.equal(P, ref_P), rep
    finally:
        plan.destroy()
    srcs = np.array([3, 9000])
    ref = oracle.dijkstra_rows(w, srcs).astype(np.float32)
    idx = torch.from_numpy(srcs).cuda()
    assert np.array_equal(ref_d[idx].cpu().numpy().view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(ref_P[idx].cpu().numpy(), oracle.canonical_pred(ref, w, rows=srcs))


def test_f32_canonical_path_side_stream():
    """The canonical path on a side stream: its scratch, gate and strips are
    ordered on the caller's stream like the rest of the solve."""
    n = 1300
    w = gen.dense_graph(n, 0.05, 1, 100, seed=77, dtype=np.float32)
    w[np.isfinite(w)] += 0.5
    np.fill_diagonal(w, 0)
    print("[pred keys] f32 canonical path, side stream", flush=True)
    ref_d, ref_P = _solve(w)
    s = torch.cuda.Stream()
    d, P = _solve(w, stream=s)
    assert np.array_equal(d.view(np.uint32), ref_d.view(np.uint32))
    assert np.array_equal(P, ref_P)


def test_f32_canonical_path_beyond_the_keys():
    """fp32 with predecessors on 16400 vertices (beyond the keys' 16383): no
    keyed sweep, the canonical path directly -- the 128-wide distances sweep,
    then 17 strips of last hops (the last one 16 columns wide).  Sampled rows
    of d against Dijkstra and of P against the oracle's canonical
    predecessors; no fallback is counted."""
    n = 16400
    w = gen.dense_graph(n, 0.002, 1, 100, seed=4242, dtype=np.float32)
    srcs = np.array([0, 5, 8191, 16383, 16399])
    print(f"[pred keys] f32 canonical path beyond the keys n={n}", flush=True)
    d = torch.from_numpy(w).cuda()
    P = torch.full((n, n), -77, dtype=torch.int32, device="cuda")
    before = fw.pred_fallbacks()
    fw.fw_apsp_pred(d, P)
    torch.cuda.synchronize()
    assert fw.pred_fallbacks() == before
    idx = torch.from_numpy(srcs).cuda()
    rows, prow = d[idx].cpu().numpy(), P[idx].cpu().numpy()
    del d, P
    ref = oracle.dijkstra_rows(w, srcs).astype(np.float32)
    assert np.isfinite(ref).sum() > len(srcs) * n // 2
    assert np.array_equal(rows.view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(prow, oracle.canonical_pred(ref, w, rows=srcs))


def test_f32_negative_cycle_beyond_the_keys():
    """Beyond the keys, a negative diagonal after the distances sweep sends
    the solve to the compare form (from the weights saved in P; counted as a
    fallback); the planted cycle is listed and recovered."""
    n = 16390
    w, cyc = gen.planted_negative_cycle(n, 0.001, 3, seed=97, dtype=np.float32)
    print(f"[pred keys] f32 negative cycle beyond the keys n={n}", flush=True)
    d = torch.from_numpy(w).cuda()
    P = torch.empty((n, n), dtype=torch.int32, device="cuda")
    before = fw.pred_fallbacks()
    fw.fw_apsp_pred(d, P)
    torch.cuda.synchronize()
    assert fw.pred_fallbacks() == before + 1
    listed = fw.fw_negative_cycle_vertices(d)
    assert listed == sorted(cyc.tolist())
    v = listed[0]
    Pv = P.cpu().numpy()
    del d, P
    found, _ = fw.fw_negative_cycle_find(w, v, Pv)
    assert sorted(found) == sorted(cyc.tolist())


def test_f32_nan_entry_leaves_the_keyed_sweep():
    """A NaN is outside the contract, but the keyed sweep's input check must
    still see it (a NaN is not an integer) and hand the solve on."""
    n = 200
    w = gen.dense_graph(n, 0.2, 1, 100, seed=71, dtype=np.float32)
    w[3, 7] = np.nan
    print("[pred keys] f32 NaN entry", flush=True)
    before = fw.pred_fallbacks()
    _solve(w)
    assert fw.pred_fallbacks() == before + 1


@pytest.mark.parametrize("seed", range(4))
def test_f32_keyed_equals_fallback_random(seed):
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(40, 700))
    p = float(rng.choice([0.003, 0.03, 0.3]))
    g = gen.reweighted_graph(n, p, 1, int(rng.integers(2, 100)), -100, 100, seed=50 + seed)
    w = _f32(g.w)
    k = rng.choice(n, size=min(n, 6), replace=False)
    w[k[:3], k[:3]] = np.inf
    w[k[3:], k[3:]] = rng.integers(1, 50, size=len(k[3:]))
    # forced fallback: two isolated extra vertices joined by an edge of weight 0.5
    f = np.full((n + 2, n + 2), np.inf, dtype=np.float32)
    f[:n, :n] = w
    f[n, n] = f[n + 1, n + 1] = 0
    f[n, n + 1] = 0.5
    print(f"[pred keys] f32 differential seed={seed} n={n} p={p}", flush=True)
    before = fw.pred_fallbacks()
    d, P = _solve(w)
    mid = fw.pred_fallbacks()
    fd, fP = _solve(f)
    assert mid == before and fw.pred_fallbacks() == mid + 1
    assert np.array_equal(d.view(np.uint32), fd[:n, :n].view(np.uint32))
    assert np.array_equal(P, fP[:n, :n])
    ref = oracle.fw(w)
    assert np.array_equal(d.view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(P, oracle.canonical_pred(ref, w))


def test_f32_solve_plan_replays_both_paths():
    n = 800
    for frac in (False, True):
        w = gen.dense_graph(n, 0.2, 1, 100, seed=61, dtype=np.float32)
        if frac:
            w[np.isfinite(w)] += 0.25
            np.fill_diagonal(w, 0)
        print(f"[pred keys] f32 solve plan frac={frac}", flush=True)
        ref_d, ref_P = _solve(w)
        src = torch.from_numpy(w).cuda()
        d = src.clone()
        P = torch.empty((n, n), dtype=torch.int32, device="cuda")
        plan = fw.SolvePlan(d, P)
        try:
            for rep in range(3):
                d.copy_(src)
                P.fill_(-77)
                before = fw.pred_fallbacks()
                plan.launch("graph")
                torch.cuda.synchronize()
                assert fw.pred_fallbacks() == before + (1 if frac else 0), rep
                assert np.array_equal(d.cpu().numpy().view(np.uint32), ref_d.view(np.uint32)), rep
                assert np.array_equal(P.cpu().numpy(), ref_P), rep
        finally:
            plan.destroy()
