"""Solve plans: the stage loop of one matrix captured once into a hipGraph.

Every graph replay must give the eager launches' bits (and the oracle's):
each case replays the graph several times, with unrelated eager work and
synchronisations between the replays, and compares every replay."""
import numpy as np
import pytest
import torch

import oracle
import paper_1001_4108_amd as fw
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


@pytest.mark.parametrize("n,tile,dtype,pred,ld_extra", [
    (300, 64, "f32", False, 3), (300, 64, "i32", True, 0), (700, 64, "f32", True, 1),
    (1000, 128, "f32", False, 0), (1000, 128, "i32", False, 4), (333, 32, "i32", True, 3),
    (1536, 0, "f32", False, 0), (512, 0, "f32", False, 0), (2, 0, "i32", True, 0),
    (1, 0, "f32", True, 0), (0, 0, "f32", False, 0)])
def test_graph_replays_match_eager_and_oracle(n, tile, dtype, pred, ld_extra):
    if dtype == "f32":
        W = gen.dense_graph(n, 0.2, 1, 100, seed=n + 7)
    else:
        W = gen.reweighted_graph(n, 0.2, 1, 100, -40, 40, seed=n + 7).w
    buf = np.full((n, n + ld_extra), -5, W.dtype)
    buf[:, :n] = W
    pristine = torch.from_numpy(buf).cuda()
    work = pristine.clone()
    d = work[:, :n]
    P = torch.full((n, n + ld_extra), -9, dtype=torch.int32, device="cuda")[:, :n] if pred else None
    plan = fw.SolvePlan(d, P, tile=tile)
    if tile:
        assert plan.tile == tile
    plan.launch("eager")
    torch.cuda.synchronize()
    eager = work.cpu().numpy()
    eagerP = P.cpu().numpy() if pred else None
    ref = oracle.fw(W) if n else W
    assert np.array_equal(bits(eager[:, :n]), bits(ref))
    assert (eager[:, n:] == -5).all()
    if pred and n:
        assert np.array_equal(eagerP, oracle.canonical_pred(ref, W))
    for rep in range(4):
        work.copy_(pristine)
        if pred:
            P.fill_(-9)
        x = torch.randn(8192, device="cuda")
        y = (x * 2).sum()  # unrelated eager work between replays
        plan.launch("graph")
        torch.cuda.synchronize()
        assert float(y) == float(y)
        assert np.array_equal(bits(work.cpu().numpy()), bits(eager)), rep
        if pred:
            assert np.array_equal(P.cpu().numpy(), eagerP), rep
    plan.destroy()
    with pytest.raises(RuntimeError):
        plan.launch("graph")


def test_graph_replay_on_a_side_stream():
    n = 1500
    W = gen.dense_graph(n, 0.3, 1, 1000, seed=21)
    pristine = torch.from_numpy(W).cuda()
    d = pristine.clone()
    plan = fw.SolvePlan(d)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    for rep in range(3):
        with torch.cuda.stream(s):
            d.copy_(pristine)
            plan.launch("graph", stream=s)
        s.synchronize()
        srcs = np.array([0, 777, 1499])
        rows = d[torch.from_numpy(srcs).cuda()].cpu().numpy()
        assert np.array_equal(rows, oracle.dijkstra_rows(W, srcs).astype(np.float32)), rep
    plan.destroy()
