"""fw_apsp_batched_noalloc -- the batched entry point for callers that cannot
allocate -- against fw_apsp_batched: bit-identical distances and
predecessors on two calls in a row, the second with a smaller batch, both
through the C ABI; a batch whose tables exceed the static array is refused
before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1001_4108_amd import _binding as B
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu


def _declare(L):
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    P64 = ctypes.POINTER(ctypes.c_int64)
    L.fw_apsp_batched_noalloc.argtypes = [ctypes.POINTER(vp), P64, P64, i64, ci,
                                          ctypes.POINTER(vp), P64, vp]
    L.fw_apsp_batched_noalloc.restype = ci
    L.fw_batched_noalloc_max_bytes.argtypes = []
    L.fw_batched_noalloc_max_bytes.restype = i64


def _batch(sizes, dtype, seed):
    out = []
    for g, n in enumerate(sizes):
        if dtype == torch.float32:
            out.append(gen.dense_graph(int(n), 0.3, 1, 100, seed=(seed, g)))
        else:
            out.append(gen.reweighted_graph(int(n), 0.3, 1, 100, -40, 40, seed=(seed, g)).w)
    return out


def _arrays(mats, preds):
    count = len(mats)
    ptrs = (ctypes.c_void_p * count)(*[m.data_ptr() for m in mats])
    ns = (ctypes.c_int64 * count)(*[m.shape[0] for m in mats])
    lds = (ctypes.c_int64 * count)(*[max(m.stride(0), m.shape[0]) for m in mats])
    pp = (ctypes.c_void_p * count)(*[p.data_ptr() if p is not None else None for p in preds])
    pl = (ctypes.c_int64 * count)(*[p.stride(0) if p is not None else 0 for p in preds])
    return ptrs, ns, lds, pp, pl


def _run(call, graphs, with_pred, dtype):
    mats, preds = [], []
    for g, W in enumerate(graphs):
        n = W.shape[0]
        buf = torch.full((n, n + (g % 3)), -3, dtype=dtype, device="cuda")
        buf[:, :n] = torch.from_numpy(W).cuda()
        mats.append(buf[:, :n])
        preds.append(torch.full((n, n), -7, dtype=torch.int32, device="cuda")
                     if with_pred[g] else None)
    ptrs, ns, lds, pp, pl = _arrays(mats, preds)
    code = B.FW_F32 if dtype == torch.float32 else B.FW_I32
    s = torch.cuda.current_stream().cuda_stream
    rc = call(ptrs, ns, lds, len(mats), code, pp, pl, ctypes.c_void_p(s))
    assert rc == 0, B.lib().fw_status_string(rc)
    torch.cuda.synchronize()
    return ([m.cpu().numpy() for m in mats],
            [p.cpu().numpy() if p is not None else None for p in preds])


@pytest.mark.parametrize("dtype", [torch.float32, torch.int32])
def test_noalloc_matches_batched_on_two_calls(dtype):
    L = B.lib()
    _declare(L)
    rng = np.random.default_rng(11 if dtype == torch.float32 else 12)
    for call_no, count in enumerate((700, 90)):  # the second call is smaller
        sizes = np.clip(np.rint(np.exp(rng.uniform(np.log(1), np.log(600), count))), 1, 600)
        graphs = _batch(sizes.astype(int), dtype, seed=(call_no, count))
        with_pred = rng.random(count) < 0.3
        ref_d, ref_p = _run(L.fw_apsp_batched, graphs, with_pred, dtype)
        got_d, got_p = _run(L.fw_apsp_batched_noalloc, graphs, with_pred, dtype)
        for g in range(count):
            assert np.array_equal(got_d[g].view(np.uint32), ref_d[g].view(np.uint32)), (call_no, g)
            if with_pred[g]:
                assert np.array_equal(got_p[g], ref_p[g]), (call_no, g)
        for g in rng.choice(count, 8, replace=False):  # and a sample against the oracle
            assert np.array_equal(got_d[g].view(np.uint32),
                                  oracle.fw(graphs[g]).view(np.uint32)), (call_no, g)


def test_noalloc_refuses_tables_beyond_the_array():
    L = B.lib()
    _declare(L)
    cap = L.fw_batched_noalloc_max_bytes()
    assert cap == 16 << 20
    # nine 8192-vertex graphs: 2 MiB of stage-batched work entries
    # each at tile 128, 18 MiB together -- refused on the host, nothing runs
    n, k = 8192, 9
    mats = [torch.empty((n, n), dtype=torch.float32, device="cuda") for _ in range(k)]
    ptrs, ns, lds, pp, pl = _arrays(mats, [None] * k)
    rc = L.fw_apsp_batched_noalloc(ptrs, ns, lds, k, B.FW_F32, None, None, None)
    assert rc == 4  # FW_ERR_UNSUPPORTED
    del mats
    torch.cuda.empty_cache()
    # the array still serves a batch afterwards
    graphs = _batch([40, 300, 7], torch.float32, seed=5)
    got_d, _ = _run(L.fw_apsp_batched_noalloc, graphs, [False] * 3, torch.float32)
    for g, W in enumerate(graphs):
        assert np.array_equal(got_d[g].view(np.uint32), oracle.fw(W).view(np.uint32))
