"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar: bit-exact distances and predecessors.  Every input uses integer-valued
weights whose path sums are exact in the matrix dtype, so every correct
evaluation order yields the same bits (blocked and plain Floyd-Warshall
differ only in the association of the path sums, section 3.2).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1001_4108_amd as fw
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu

I32_INF = gen.I32_INF
SIZES = [1, 2, 3, 15, 16, 17, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512]
TILES = [32, 64, 128]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def graph(n, dtype, seed, p=0.3, hi=100):
    if dtype == "f32":
        return gen.dense_graph(n, p, 1, hi, seed)
    return gen.reweighted_graph(n, p, 1, hi, -hi // 2, hi // 2, seed).w


def solve(W, tile=None, pred=False, ld_extra=0, fill=None):
    n = W.shape[0]
    buf = np.empty((n, n + ld_extra), W.dtype)
    if fill is not None:
        buf[:] = fill
    buf[:, :n] = W
    d = dev(buf)
    view = d[:, :n]
    P = None
    if pred:
        P = torch.full((n, n + ld_extra), -77, dtype=torch.int32, device="cuda")[:, :n]
    if tile is None:
        fw.fw_apsp_pred(view, P)
    else:
        fw.fw_apsp_plan(view, tile, P)
    torch.cuda.synchronize()
    out = d.cpu().numpy()
    return out, (P.cpu().numpy() if pred else None)


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("dtype", ["f32", "i32"])
@pytest.mark.parametrize("n", SIZES)
def test_distances_bit_exact(n, dtype, tile):
    W = graph(n, dtype, seed=31 * n + tile)
    ref = oracle.fw(W)
    got, _ = solve(W, tile)
    assert np.array_equal(bits(got), bits(ref)), (n, dtype, tile)


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("dtype", ["f32", "i32"])
@pytest.mark.parametrize("n", [2, 17, 33, 64, 65, 129, 200, 257])
def test_predecessors_bit_exact(n, dtype, tile):
    # weights in [1, 3] make shortest-path ties dense
    W = graph(n, dtype, seed=17 * n + tile, p=0.2, hi=3 if dtype == "f32" else 4)
    ref = oracle.fw(W)
    Pref = oracle.canonical_pred(ref, W)
    got, P = solve(W, tile, pred=True)
    assert np.array_equal(bits(got), bits(ref))
    assert np.array_equal(P, Pref)


@pytest.mark.parametrize("dtype", ["f32", "i32"])
def test_sparse_graph_with_unreachable_pairs_pred(dtype):
    n = 150
    W = graph(n, dtype, seed=5, p=0.01, hi=20)
    ref = oracle.fw(W)
    Pref = oracle.canonical_pred(ref, W)
    assert (Pref == -1).sum() > n  # some unreachable pairs exist
    for tile in TILES:
        got, P = solve(W, tile, pred=True)
        assert np.array_equal(bits(got), bits(ref))
        assert np.array_equal(P, Pref)


@pytest.mark.parametrize("extra", [3, 4, 7, 64])
@pytest.mark.parametrize("dtype", ["f32", "i32"])
def test_leading_dimension_padding_untouched(dtype, extra):
    n = 131
    W = graph(n, dtype, seed=extra)
    fill = np.float32(-7.5) if dtype == "f32" else np.int32(-12345)
    ref = oracle.fw(W)
    for tile in TILES:
        out, _ = solve(W, tile, ld_extra=extra, fill=fill)
        assert np.array_equal(bits(out[:, :n]), bits(ref))
        assert (out[:, n:] == fill).all()


def test_empty_and_single_vertex():
    for dtype in (torch.float32, torch.int32):
        d = torch.zeros((0, 0), dtype=dtype, device="cuda")
        fw.fw_apsp_pred(d)
        d1 = torch.zeros((1, 1), dtype=dtype, device="cuda")
        P = torch.full((1, 1), 5, dtype=torch.int32, device="cuda")
        fw.fw_apsp_pred(d1, P)
        torch.cuda.synchronize()
        assert d1.item() == 0 and P.item() == -1


def test_default_plan_matches_oracle_single_graph_512():
    """n=512 fp32, edge prob 0.5, weights in [1, 100]: the whole matrix."""
    W = gen.single_graph_512()
    ref = oracle.fw(W)
    d = dev(W)
    fw.fw_apsp(d)
    torch.cuda.synchronize()
    assert np.array_equal(bits(d.cpu().numpy()), bits(ref))


def test_repeat_runs_are_deterministic_and_idempotent():
    W = graph(700, "f32", seed=3)
    a, _ = solve(W, 64)
    b, _ = solve(W, 64)
    assert np.array_equal(bits(a), bits(b))
    c, _ = solve(a, 128)
    assert np.array_equal(bits(c), bits(a))


def test_negative_cycle_flag():
    W = graph(90, "i32", seed=8)
    d = dev(W)
    fw.fw_apsp_i32(d)
    assert not fw.fw_negative_cycle(d)
    bad = W.copy()
    bad[3, 4] = -5
    bad[4, 3] = 2  # cycle 3 -> 4 -> 3 of weight -3
    d = dev(bad)
    fw.fw_apsp_i32(d)
    assert fw.fw_negative_cycle(d)


def test_signed_zero_inputs_equal_as_values():
    """-0 weights: either zero may come back, values equal the oracle's."""
    W = graph(70, "f32", seed=12)
    W[W == 1.0] = -0.0
    ref = oracle.fw(W)
    got, _ = solve(W, 32)
    assert np.array_equal(got, ref)  # == treats +0 and -0 as equal


def test_single_graph_16384_dijkstra_rows():
    """n=16384 fp32 (p=0.3, weights [1,1000]): 64 seeded sources checked
    bit-exactly against float64 Dijkstra (exact for these integers)."""
    W = gen.single_graph_16384()
    srcs = gen.dijkstra_sources_16384()
    d = dev(W)
    fw.fw_apsp(d)
    rows = d[torch.from_numpy(srcs).cuda()].cpu().numpy()
    ref = oracle.dijkstra_rows(W, srcs).astype(np.float32)
    assert np.array_equal(bits(rows), bits(ref))
    # sampled-k triangle inequality on the sampled rows
    for k in srcs[:8]:
        dk = d[int(k)].cpu().numpy()
        assert (rows <= rows[:, [int(k)]] + dk[None, :]).all()


def test_negative_graph_8192_johnson_rows_with_pred():
    """n=8192 int32 with negative weights and predecessors: sampled rows
    checked against Dijkstra on the base weights plus the potential identity
    d'(u,v) = d(u,v) + p(u) - p(v), and the canonical predecessors."""
    g = gen.negative_graph_8192()
    n = g.w.shape[0]
    d = dev(g.w)
    P = torch.empty((n, n), dtype=torch.int32, device="cuda")
    fw.fw_apsp_pred(d, P)
    srcs = np.sort(np.random.default_rng(3003).choice(n, 24, replace=False))
    idx = torch.from_numpy(srcs).cuda()
    rows = d[idx].cpu().numpy()
    prow = P[idx].cpu().numpy()
    base = oracle.dijkstra_rows(g.base, srcs)
    assert np.isfinite(base).all()  # strongly connected
    ref = (base.astype(np.int64) + g.pot[srcs][:, None] - g.pot[None, :]).astype(np.int32)
    assert np.array_equal(rows, ref)
    Pref = oracle.canonical_pred(ref, g.w, rows=srcs)
    assert np.array_equal(prow, Pref)
