"""The autotuner installs a measured tile per bucket; results stay bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import paper_1001_4108_amd as fw
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("objective", ["single", "batched"])
def test_autotune_installs_fastest_tile(objective, tmp_path):
    fw.plan_reset()
    buckets = [(20, 40), (100, 300)]
    res = fw.autotune(torch.float32, buckets, objective=objective, batch=32, reps=2)
    tiles = fw.plan_tiles()
    for (lo, hi), v in res.items():
        assert v["tile"] in tiles
        assert all(ms > 0 for ms in v["ms"].values())
        assert v["ms"][v["tile"]] == min(v["ms"].values())
        for n in (lo, hi, (lo + hi) // 2):
            assert fw.plan_tile(torch.float32, n) == v["tile"]
    path = tmp_path / "plan.json"
    fw.save_plan(res, str(path), objective=objective)
    fw.plan_reset()
    fw.load_plan(str(path))
    for (lo, hi), v in res.items():
        assert fw.plan_tile(torch.float32, lo) == v["tile"]
    W = gen.dense_graph(173, 0.2, 1, 9, seed=4)
    d = torch.from_numpy(W).cuda()
    fw.fw_apsp(d)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy().view(np.uint32), oracle.fw(W).view(np.uint32))
    fw.plan_reset()


@pytest.mark.parametrize("objective", ["single", "batched"])
def test_autotune_predecessor_table(objective, tmp_path):
    """Tuning with predecessors writes the FW_PLAN_PRED part only, and a
    solve with predecessors at the tuned tile is still bit-exact."""
    fw.plan_reset()
    before = {n: fw.plan_tile(torch.int32, n) for n in (150, 250)}
    res = fw.autotune(torch.int32, [(129, 300)], objective=objective, batch=16, reps=2, pred=True)
    v = res[(129, 300)]
    assert v["tile"] in fw.plan_tiles() and v["ms"][v["tile"]] == min(v["ms"].values())
    for n in (150, 250):
        assert fw.plan_tile(torch.int32, n, pred=True) == v["tile"]
        assert fw.plan_tile(torch.int32, n) == before[n]
    path = tmp_path / "plan_pred.json"
    fw.save_plan(res, str(path), dtype="i32", objective=objective, pred=True)
    fw.plan_reset()
    fw.load_plan(str(path))
    assert fw.plan_tile(torch.int32, 200, pred=True) == v["tile"]
    g = gen.reweighted_graph(211, 0.2, 1, 40, -10, 10, seed=8)
    d = torch.from_numpy(g.w).cuda()
    P = torch.empty((211, 211), dtype=torch.int32, device="cuda")
    fw.fw_apsp_pred(d, P)
    torch.cuda.synchronize()
    ref = oracle.fw(g.w)
    assert np.array_equal(d.cpu().numpy(), ref)
    assert np.array_equal(P.cpu().numpy(), oracle.canonical_pred(ref, g.w))
    fw.plan_reset()


def test_autotune_batch_installs_tiles_and_stays_exact():
    """Whole-batch tuning (eager and graph launches) installs one of the
    plan's tiles per used bucket, the fastest it timed, skips the unused
    bucket, and batched solves afterwards stay bit-exact."""
    rng = np.random.default_rng(11)
    sizes = [int(v) for v in rng.integers(20, 300, size=48)]
    buckets = [(16, 64), (65, 200), (201, 300), (301, 400)]
    tiles = set(fw.plan_tiles())
    try:
        for mode in ("kernel", "graph"):
            res = fw.autotune_batch(torch.float32, sizes, buckets, mode=mode, reps=2, passes=1)
            for (lo, hi), v in res.items():
                assert v["tile"] in tiles
                used = any(lo <= n <= hi for n in sizes)
                assert bool(v["ms"]) == used
                if used:
                    assert fw.plan_tile(torch.float32, (lo + hi) // 2) == v["tile"]
                    assert min(v["ms"], key=v["ms"].get) == v["tile"]
        graphs = [gen.dense_graph(n, 0.3, 1, 9, 900 + g) for g, n in enumerate(sizes[:12])]
        ts = [torch.from_numpy(w).cuda() for w in graphs]
        fw.fw_apsp_batched(ts)
        torch.cuda.synchronize()
        for w, t in zip(graphs, ts):
            assert np.array_equal(t.cpu().numpy().view(np.uint32), oracle.fw(w).view(np.uint32))
    finally:
        fw.plan_reset()


def test_autotune_batch_rejects_bad_arguments():
    with pytest.raises(fw.FwError):
        fw.autotune_batch(torch.float32, [10, 20], [(30, 10)])
    with pytest.raises(fw.FwError):
        fw.autotune_batch(torch.float32, [10, 10 ** 6], [(2, 64)])
    with pytest.raises(fw.FwError):
        fw.autotune_batch(torch.float32, [10], [(2, 64)], reps=0)
    with pytest.raises(ValueError):
        fw.autotune_batch(torch.float32, [10], [(2, 64)], mode="eager")
