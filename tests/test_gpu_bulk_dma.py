"""Bulk phase at tile 128 over many tiles: the direct global->LDS copy kernel
(full tiles, 16-byte aligned rows), the edge-tile launch of a partial last
block, and the register-staged kernel for unaligned rows, all bit-exact
against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_1001_4108_amd as fw
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def run(W, ld_extra, fill, semiring="minplus"):
    n = W.shape[0]
    buf = np.empty((n, n + ld_extra), W.dtype)
    buf[:] = fill
    buf[:, :n] = W
    d = torch.from_numpy(buf).cuda()
    if semiring == "minplus":
        fw.fw_apsp_plan(d[:, :n], 128)
    else:
        code = "f32" if W.dtype == np.float32 else "i32"
        fw.plan_set(code, n, n, 128)
        try:
            fw.fw_apsp_semiring(d[:, :n], semiring)
        finally:
            fw.plan_reset()
    torch.cuda.synchronize()
    return d.cpu().numpy()


# 16-byte aligned rows (ld % 4 == 0) take the copy kernel; ld_extra 3 does not
@pytest.mark.parametrize("ld_extra", [0, 4, 3])
@pytest.mark.parametrize("dtype", ["f32", "i32"])
@pytest.mark.parametrize("n", [256, 384, 640, 700, 1000, 1151])
def test_minplus_bulk_bit_exact(n, dtype, ld_extra):
    if dtype == "f32":
        W = gen.dense_graph(n, 0.25, 1, 1000, seed=7 * n + ld_extra)
        fill = np.float32(-3.25)
    else:
        W = gen.reweighted_graph(n, 0.25, 1, 1000, -500, 500, seed=7 * n + ld_extra).w
        fill = np.int32(-999)
    ref = oracle.fw(W)
    out = run(W, ld_extra, fill)
    assert np.array_equal(bits(out[:, :n]), bits(ref)), (n, dtype, ld_extra)
    assert (out[:, n:] == fill).all()


@pytest.mark.parametrize("dtype", ["f32", "i32"])
@pytest.mark.parametrize("n", [512, 700])
def test_maxmin_bulk_bit_exact(n, dtype):
    rng = np.random.default_rng(n)
    if dtype == "f32":
        W = np.where(rng.random((n, n)) < 0.2, rng.integers(1, 1000, (n, n)), -np.inf)
        W = W.astype(np.float32)
    else:
        W = np.where(rng.random((n, n)) < 0.2, rng.integers(1, 1000, (n, n)),
                     np.iinfo(np.int32).min).astype(np.int32)
    ref = oracle.fw_maxmin(W)
    out = run(W, 0, W.dtype.type(0), semiring="maxmin")
    assert np.array_equal(bits(out[:, :n]), bits(ref))
