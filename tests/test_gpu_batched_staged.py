"""Stage-batched part of batch plans: graphs of 257 vertices and more run as
per-stage launches shared by all graphs of one tile size.  Checked bit for bit
against the oracle with tiles 32, 64 and 128 in one batch, predecessors on
some graphs, both dtypes, unaligned leading dimensions and small graphs
(persistent kernel) in the same batch."""
import numpy as np
import pytest
import torch

import oracle
import paper_1001_4108_amd as fw
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu

SIZES = [257, 300, 385, 450, 511, 640, 700, 1000, 1100, 3, 40, 100, 200]


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def graph(n, dtype, seed):
    if dtype == np.float32:
        return gen.dense_graph(n, 0.25, 1, 50, seed)
    return gen.reweighted_graph(n, 0.25, 1, 50, -20, 20, seed).w


@pytest.fixture(autouse=True)
def mixed_tiles():
    for dt in ("f32", "i32"):
        for pred in (False, True):
            fw.plan_set(dt, 257, 400, 32, pred=pred)
            fw.plan_set(dt, 401, 700, 64, pred=pred)
            fw.plan_set(dt, 701, 4096, 128, pred=pred)
    yield
    fw.plan_reset()


@pytest.mark.parametrize("dtype", [np.float32, np.int32])
@pytest.mark.parametrize("ld_pad", [0, 1])
def test_staged_distances_and_predecessors(dtype, ld_pad):
    graphs = [graph(n, dtype, 100 + g) for g, n in enumerate(SIZES)]
    fill = dtype(-7)
    bufs, views, preds = [], [], []
    for g, w in enumerate(graphs):
        n = w.shape[0]
        ld = (n + 3) // 4 * 4 + ld_pad  # ld_pad 1: rows not 16-byte aligned
        host = np.full((n, ld), fill, dtype)
        host[:, :n] = w
        t = torch.from_numpy(host).cuda()
        bufs.append(t)
        views.append(t[:, :n])
        preds.append(torch.full((n, n), -9, dtype=torch.int32, device="cuda") if g % 2 == 0
                     else None)
    fw.fw_apsp_batched(views, preds)
    torch.cuda.synchronize()
    for w, t, p in zip(graphs, bufs, preds):
        n = w.shape[0]
        ref = oracle.fw(w)
        got = t.cpu().numpy()
        assert np.array_equal(bits(got[:, :n]), bits(ref)), n
        assert (got[:, n:] == fill).all(), n
        if p is not None:
            assert np.array_equal(p.cpu().numpy(), oracle.canonical_pred(ref, w)), n


def test_staged_plan_graph_replays():
    graphs = [graph(n, np.float32, 200 + g) for g, n in enumerate(SIZES)]
    ts = [torch.from_numpy(w).cuda() for w in graphs]
    pristine = [t.clone() for t in ts]
    refs = [oracle.fw(w) for w in graphs]
    plan = fw.BatchPlan(ts)
    for rep, mode in enumerate(["graph", "kernel", "graph", "graph"]):
        for t, p0 in zip(ts, pristine):
            t.copy_(p0)
        torch.cuda.synchronize()
        _ = torch.randn(1000, device="cuda").sum().item()  # unrelated eager work
        plan.launch(mode)
        torch.cuda.synchronize()
        for t, r in zip(ts, refs):
            assert np.array_equal(bits(t.cpu().numpy()), bits(r)), (rep, mode, t.shape)
    plan.destroy()
