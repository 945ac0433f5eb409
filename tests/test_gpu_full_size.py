"""Full-size parity: every element at the sizes the benchmark runs.

* The n=8192 int32 negative-weight workload with predecessors: all of d and
  all of the canonical predecessor matrix against the oracle (no sampling).
* Long paths: a unit-weight directed cycle over a seeded permutation pi of the
  vertices has d_ij = (pi^-1(j) - pi^-1(i)) mod n and last hop
  P_ij = pi(pi^-1(j) - 1) -- closed forms that need every stage of the
  blocked sweep (and, at n=16384, every fused next-diagonal closure of the
  128-wide bulk launches), since each path runs through up to n - 1 hops.
  Every element is compared, in row chunks on the GPU.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1001_4108_amd as fw
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_negative_graph_8192_full_distances_and_predecessors():
    g = gen.negative_graph_8192()
    n = g.w.shape[0]
    print(f"[full parity] n={n} int32 with predecessors", flush=True)
    d = torch.from_numpy(g.w).cuda()
    P = torch.full((n, n), -77, dtype=torch.int32, device="cuda")
    fw.fw_apsp_pred(d, P)
    torch.cuda.synchronize()
    got, gotP = d.cpu().numpy(), P.cpu().numpy()
    del d, P
    torch.cuda.empty_cache()
    ref = oracle.fw(g.w)
    assert np.array_equal(got, ref)
    Pref = oracle.canonical_pred(ref, g.w)
    assert (Pref >= 0).sum() == n * (n - 1)  # strongly connected: every i != j reached
    assert np.array_equal(gotP, Pref)


def _cycle_graph(n, perm, dtype, ld):
    inf = float("inf") if dtype == torch.float32 else gen.I32_INF
    buf = torch.full((n, ld), inf, dtype=dtype, device="cuda")
    d = buf[:, :n]
    d.fill_diagonal_(0)
    src = torch.from_numpy(perm).cuda()
    d[src, torch.roll(src, -1)] = 1
    return buf, d


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,dtype,ld_extra,pred", [
    (16384, torch.float32, 0, False),   # the benchmark's size: 128 stages of tile 128
    (12345, torch.float32, 3, False),   # partial last block, padded unaligned rows
    (8192, torch.int32, 0, False),
    (8192, torch.int32, 0, True),       # the predecessor kernels on long paths
    (3000, torch.float32, 1, True),
])
def test_long_cycle_closed_form(n, dtype, ld_extra, pred):
    print(f"[full parity] cycle n={n} {dtype} ld+{ld_extra} pred={pred}", flush=True)
    perm = gen.cycle_permutation(n, seed=n)
    pos = np.empty(n, np.int64)
    pos[perm] = np.arange(n)
    buf, d = _cycle_graph(n, perm, dtype, n + ld_extra)
    P = None
    if pred:
        P = torch.full((n, n), -77, dtype=torch.int32, device="cuda")
        fw.fw_apsp_pred(d, P)
    elif dtype == torch.float32:
        fw.fw_apsp(d)
    else:
        fw.fw_apsp_i32(d)
    torch.cuda.synchronize()
    pos_t = torch.from_numpy(pos).cuda()
    perm_t = torch.from_numpy(perm).cuda()
    inf = float("inf") if dtype == torch.float32 else gen.I32_INF
    for r0 in range(0, n, 1024):
        r1 = min(n, r0 + 1024)
        dist = (pos_t[None, :] - pos_t[r0:r1, None]) % n
        assert torch.equal(d[r0:r1], dist.to(dtype)), r0
        if pred:
            last = perm_t[(pos_t - 1) % n].to(torch.int32)[None, :].expand(r1 - r0, n).clone()
            rows = torch.arange(r0, r1, device="cuda")
            last[rows - r0, rows] = -1
            assert torch.equal(P[r0:r1], last), r0
    if ld_extra:
        assert bool((buf[:, n:] == inf).all())  # padding untouched
    del buf, d, P
    torch.cuda.empty_cache()
