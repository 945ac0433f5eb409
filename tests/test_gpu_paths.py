"""Path reconstruction and negative-cycle reports from the GPU's outputs.

* Walks of the GPU's predecessor matrix (fw_path) for seeded pairs: every
  hop is an edge and the hop weights sum, exactly, to the oracle's distance.
* Negative cycles (outside section 3.1's problem statement): the device list
  of vertices with d_ii < 0 equals a host scan of the GPU's diagonal, and the
  cycle recovered from the GPU's predecessor matrix (and by the Bellman-Ford
  fallback without it) is the one planted cycle, the only negative simple
  cycle by construction.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1001_4108_amd as fw
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu


def _edge_sum(W, path):
    return sum(float(W[path[t], path[t + 1]]) for t in range(len(path) - 1))


@pytest.mark.parametrize("n,dtype", [(700, "f32"), (2048, "i32"), (1300, "i32")])
def test_predecessor_walks_sum_to_oracle_distances(n, dtype):
    if dtype == "f32":
        W = gen.dense_graph(n, 0.05, 1, 1000, seed=n)
    else:
        W = gen.reweighted_graph(n, 0.1, 1, 1000, -500, 500, seed=n).w
    d = torch.from_numpy(W).cuda()
    P = torch.empty((n, n), dtype=torch.int32, device="cuda")
    fw.fw_apsp_pred(d, P)
    torch.cuda.synchronize()
    Ph = P.cpu().numpy()
    ref = oracle.fw(W)
    absent = np.inf if dtype == "f32" else gen.I32_INF
    rng = np.random.default_rng(n + 1)
    pairs = rng.integers(0, n, size=(400, 2))
    hops = 0
    for i, j in pairs:
        path = fw.fw_path(Ph, int(i), int(j))
        if i == j:
            assert path == [i]
            continue
        assert path[0] == i and path[-1] == j
        assert all(W[path[t], path[t + 1]] != absent for t in range(len(path) - 1))
        assert _edge_sum(W, path) == float(ref[i, j])
        hops += len(path) - 1
    assert hops > 400  # multi-hop paths were walked


@pytest.mark.parametrize("n,dtype,length,tile", [
    (90, "i32", 3, 32), (300, "i32", 5, 64), (1000, "f32", 4, 64), (520, "i32", 2, 128),
    (2100, "i32", 6, None), (700, "f32", 7, 32)])
def test_planted_negative_cycle_found(n, dtype, length, tile):
    np_dtype = np.float32 if dtype == "f32" else np.int32
    W, cyc = gen.planted_negative_cycle(n, 0.05, length, seed=n + length, dtype=np_dtype)
    d = torch.from_numpy(W).cuda()
    P = torch.empty((n, n), dtype=torch.int32, device="cuda")
    if tile is None:
        fw.fw_apsp_pred(d, P)
    else:
        fw.fw_apsp_plan(d, tile, P)
    torch.cuda.synchronize()
    diag = torch.diagonal(d).cpu().numpy()
    listed = fw.fw_negative_cycle_vertices(d)
    assert listed == np.flatnonzero(diag < 0).tolist()
    assert listed == sorted(cyc.tolist())  # exactly the cycle's vertices
    assert fw.fw_negative_cycle(d)
    Ph = P.cpu().numpy()
    want = sorted(cyc.tolist())
    for v in listed:
        found, from_pred = fw.fw_negative_cycle_find(W, v, Ph)
        assert sorted(found) == want, (v, found)
        m = len(found)
        assert sum(float(W[found[t], found[(t + 1) % m]]) for t in range(m)) == -length
    found, from_pred = fw.fw_negative_cycle_find(W, listed[0])  # Bellman-Ford only
    assert not from_pred and sorted(found) == want


def test_no_negative_cycle_lists_nothing():
    g = gen.reweighted_graph(600, 0.1, 1, 100, -50, 50, seed=6)
    d = torch.from_numpy(g.w).cuda()
    fw.fw_apsp_i32(d)
    assert fw.fw_negative_cycle_vertices(d) == []
    assert not fw.fw_negative_cycle(d)


@pytest.mark.parametrize("n", [1, 1023, 1024, 1025, 3001])
def test_negative_vertex_list_spans_chunks(n):
    """The scan on its own, on a matrix whose diagonal is set directly: a
    seeded half of the vertices negative, ascending order across the
    1024-vertex chunks of the one workgroup."""
    rng = np.random.default_rng(n)
    diag = np.where(rng.random(n) < 0.5, -rng.integers(1, 9, n), rng.integers(0, 9, n))
    d = torch.zeros((n, n + 5), dtype=torch.int32, device="cuda")[:, :n]
    d.diagonal().copy_(torch.from_numpy(diag.astype(np.int32)).cuda())
    assert fw.fw_negative_cycle_vertices(d) == np.flatnonzero(diag < 0).tolist()
    df = d.float()
    assert fw.fw_negative_cycle_vertices(df) == np.flatnonzero(diag < 0).tolist()
