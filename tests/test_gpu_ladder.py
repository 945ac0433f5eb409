"""Ablation ladder: every rung gives the oracle's bits (ragged sizes,
padded and unaligned leading dimensions, both dtypes)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1001_4108_amd as fw
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


@pytest.mark.parametrize("rung", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("dtype", ["f32", "i32"])
@pytest.mark.parametrize("n,ld_extra", [(1, 0), (2, 3), (31, 0), (33, 1), (64, 0), (100, 4),
                                        (129, 0), (257, 3), (300, 0)])
def test_rung_bit_exact(rung, dtype, n, ld_extra):
    if dtype == "f32":
        W = gen.dense_graph(n, 0.3, 1, 200, seed=n + 17 * rung)
        fill = np.float32(-2.5)
    else:
        W = gen.reweighted_graph(n, 0.3, 1, 200, -80, 80, seed=n + 17 * rung).w
        fill = np.int32(-31)
    buf = np.full((n, n + ld_extra), fill, W.dtype)
    buf[:, :n] = W
    d = torch.from_numpy(buf).cuda()
    fw.fw_apsp_ladder(d[:, :n], rung)
    torch.cuda.synchronize()
    out = d.cpu().numpy()
    assert np.array_equal(bits(out[:, :n]), bits(oracle.fw(W))), (rung, dtype, n)
    assert (out[:, n:] == fill).all()


def test_bad_rung():
    d = torch.zeros((4, 4), device="cuda")
    with pytest.raises(fw.FwError):
        fw.fw_apsp_ladder(d, 5)
