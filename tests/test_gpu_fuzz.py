"""Seeded randomized parity sweep: sizes, densities (empty to complete),
dtypes, negative weights, tiles, leading-dimension padding and misalignment,
predecessors and the (max, min) semiring, each case bit-exact against the
oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_1001_4108_amd as fw
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu

CASES = 400


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def draw(rng):
    n = int(rng.choice([int(rng.integers(1, 70)), int(rng.integers(70, 300)),
                        int(rng.integers(300, 700))]))
    p = float(rng.choice([0.0, 0.03, 0.2, 0.6, 1.0]))
    dtype = str(rng.choice(["f32", "i32"]))
    negative = dtype == "i32" and bool(rng.integers(0, 2))
    tile = [None, 32, 64, 128][int(rng.integers(0, 4))]
    ld_extra = int(rng.choice([0, 0, 1, 4, 7]))
    pred = bool(rng.integers(0, 3) == 0)
    maxmin = (not pred) and bool(rng.integers(0, 6) == 0)
    return n, p, dtype, negative, tile, ld_extra, pred, maxmin


def test_randomized_cases():
    rng = np.random.default_rng(20260101)
    failures = []
    for case in range(CASES):
        n, p, dtype, negative, tile, ld_extra, pred, maxmin = draw(rng)
        seed = 1000 + case
        if dtype == "f32":
            W = gen.dense_graph(n, p, 1, 500, seed)
        elif negative:
            W = gen.reweighted_graph(n, p, 1, 500, -200, 200, seed).w
        else:
            W = gen.dense_graph(n, p, 1, 500, seed, dtype=np.int32)
        if maxmin:
            absent = np.float32(-np.inf) if dtype == "f32" else np.int32(np.iinfo(np.int32).min)
            present = np.isfinite(W) if dtype == "f32" else W != gen.I32_INF
            W = np.where(present, W, absent).astype(W.dtype)
            ref = oracle.fw_maxmin(W)
        else:
            ref = oracle.fw(W)
        fill = W.dtype.type(-3)
        buf = np.full((n, n + ld_extra), fill, W.dtype)
        buf[:, :n] = W
        d = torch.from_numpy(buf).cuda()
        view = d[:, :n]
        P = None
        if pred:
            P = torch.full((n, n + 3), -9, dtype=torch.int32, device="cuda")[:, :n]
        if maxmin:
            fw.fw_apsp_semiring(view, "maxmin")
        elif tile is None:
            fw.fw_apsp_pred(view, P)
        else:
            fw.fw_apsp_plan(view, tile, P)
        torch.cuda.synchronize()
        out = d.cpu().numpy()
        ok = np.array_equal(bits(out[:, :n]), bits(ref)) and bool((out[:, n:] == fill).all())
        if ok and pred:
            ok = np.array_equal(P.cpu().numpy(), oracle.canonical_pred(ref, W))
        if not ok:
            failures.append((case, n, p, dtype, negative, tile, ld_extra, pred, maxmin))
    assert not failures, failures[:5]


def test_randomized_batches():
    """Random batch compositions through batch plans (persistent and
    stage-batched parts, random tile per size bucket, predecessors on random
    graphs, padded rows), every graph bit-exact against the oracle."""
    rng = np.random.default_rng(777)
    try:
        for rep in range(6):
            dtype = [np.float32, np.int32][rep % 2]
            code = "f32" if dtype == np.float32 else "i32"
            fw.plan_reset()
            for lo, hi in ((2, 32), (33, 64), (65, 128), (129, 256), (257, 700)):
                tile = int(rng.choice([32, 64, 128]))
                fw.plan_set(code, lo, hi, tile)
                fw.plan_set(code, lo, hi, tile, pred=True)
            count = int(rng.integers(20, 120))
            graphs, bufs, views, preds = [], [], [], []
            for g in range(count):
                n = int(rng.choice([int(rng.integers(1, 40)), int(rng.integers(40, 260)),
                                    int(rng.integers(260, 700))]))
                if dtype == np.float32:
                    W = gen.dense_graph(n, float(rng.choice([0.05, 0.3, 0.9])), 1, 300, (rep, g))
                else:
                    W = gen.reweighted_graph(n, float(rng.choice([0.05, 0.3, 0.9])), 1, 300,
                                             -100, 100, (rep, g)).w
                ld = n + int(rng.choice([0, 3, 4]))
                host = np.full((n, ld), dtype(-5), dtype)
                host[:, :n] = W
                t = torch.from_numpy(host).cuda()
                graphs.append(W)
                bufs.append(t)
                views.append(t[:, :n])
                preds.append(torch.full((n, n), -9, dtype=torch.int32, device="cuda")
                             if rng.integers(0, 3) == 0 else None)
            plan = fw.BatchPlan(views, preds)
            plan.launch("graph" if rep % 3 else "kernel")
            torch.cuda.synchronize()
            for g, (W, t, P) in enumerate(zip(graphs, bufs, preds)):
                n = W.shape[0]
                out = t.cpu().numpy()
                ref = oracle.fw(W)
                assert np.array_equal(bits(out[:, :n]), bits(ref)), (rep, g, n)
                assert (out[:, n:] == dtype(-5)).all(), (rep, g, n)
                if P is not None:
                    assert np.array_equal(P.cpu().numpy(), oracle.canonical_pred(ref, W)), (rep, g)
            plan.destroy()
    finally:
        fw.plan_reset()
