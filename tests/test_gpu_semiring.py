"""GPU parity of the (max, min) semiring: bit-exact for any input, every tile."""
import numpy as np
import pytest
import torch

import oracle
import paper_1001_4108_amd as fw
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu

TILES = [32, 64, 128]


def widths(n, p, seed, dtype):
    rng = np.random.default_rng(seed)
    if dtype == "f32":
        w = rng.uniform(0.5, 1000.0, size=(n, n)).astype(np.float32)  # arbitrary reals
        absent, top = np.float32(-np.inf), np.float32(np.inf)
    else:
        w = rng.integers(-100000, 100000, size=(n, n)).astype(np.int32)
        absent, top = np.int32(np.iinfo(np.int32).min), np.int32(np.iinfo(np.int32).max)
    w = np.where(rng.random((n, n)) < p, w, absent)
    np.fill_diagonal(w, top)
    return w


@pytest.fixture(autouse=True)
def reset_plan():
    yield
    fw.plan_reset()


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("dtype", ["f32", "i32"])
@pytest.mark.parametrize("n", [1, 2, 31, 33, 64, 65, 127, 129, 200, 257, 390])
def test_maxmin_bit_exact(n, dtype, tile):
    W = widths(n, 0.05, 100 * n + tile, dtype)
    ref = oracle.fw_maxmin(W)
    torch_dt = torch.float32 if dtype == "f32" else torch.int32
    fw.plan_set(torch_dt, 0, 1 << 20, tile)
    buf = np.full((n, n + 5), 7, W.dtype)
    buf[:, :n] = W
    d = torch.from_numpy(buf).cuda()
    fw.fw_apsp_semiring(d[:, :n], "maxmin")
    torch.cuda.synchronize()
    out = d.cpu().numpy()
    assert np.array_equal(out[:, :n].view(np.uint32), ref.view(np.uint32))
    assert (out[:, n:] == 7).all()


def test_transitive_closure_matches_bfs():
    n = 1000
    W = gen.dense_graph(n, 0.002, 1, 1, seed=17, dtype=np.int32)
    A = torch.from_numpy(np.where(W == gen.I32_INF, 0, 1).astype(np.int32)).cuda()
    fw.fw_transitive_closure(A)
    R = A.cpu().numpy()
    assert set(np.unique(R)) <= {0, 1}
    for s in range(0, n, 37):
        assert np.array_equal(R[s].astype(bool), oracle.reach_row(W, s))


def test_minplus_through_semiring_entry_equals_fw_apsp():
    W = gen.dense_graph(300, 0.2, 1, 50, seed=9)
    a = torch.from_numpy(W).cuda()
    b = a.clone()
    fw.fw_apsp(a)
    fw.fw_apsp_semiring(b, "minplus")
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_widest_paths_16384_rows():
    """n=16384 fp32 widest paths on the benchmark graph's edges (absent = -INF),
    8 rows against the bottleneck Dijkstra."""
    W = gen.single_graph_16384()
    W = np.where(np.isinf(W), np.float32(-np.inf), W).astype(np.float32)
    np.fill_diagonal(W, np.inf)
    d = torch.from_numpy(W).cuda()
    fw.fw_apsp_semiring(d, "maxmin")
    srcs = gen.dijkstra_sources_16384(count=8)
    rows = d[torch.from_numpy(srcs).cuda()].cpu().numpy()
    ref = oracle.widest_rows(W, srcs).astype(np.float32)
    assert np.array_equal(rows.view(np.uint32), ref.view(np.uint32))
