"""Calls made on a side stream: temporaries and outputs are allocated on the
stream the kernels run on, so work on the current stream cannot reuse their
memory while those kernels still run."""
import numpy as np
import pytest
import torch

import oracle
import paper_1001_4108_amd as fw
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu


def test_transitive_closure_on_a_side_stream():
    n = 3000
    W = gen.dense_graph(n, 1.5 / n, 1, 1, seed=5, dtype=np.int32)
    A = np.where(W == gen.I32_INF, 0, 1).astype(np.int32)
    s = torch.cuda.Stream()
    adj = torch.from_numpy(A).cuda()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pass
    fw.fw_transitive_closure(adj, stream=s)
    # the current stream allocates and writes while the side stream works
    junk = [torch.full((1 << 20,), 7, dtype=torch.int32, device="cuda") for _ in range(8)]
    s.synchronize()
    torch.cuda.synchronize()
    got = adj.cpu().numpy()
    for src in (0, 1234, n - 1):
        assert np.array_equal(got[src].astype(bool), oracle.reach_row(W, src)), src
    assert all(int(j[0]) == 7 for j in junk)


def test_pack_unpack_on_a_side_stream():
    n = 1000
    rng = np.random.default_rng(4)
    A = (rng.random((n, n)) < 0.1).astype(np.int32)
    adj = torch.from_numpy(A).cuda()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    bits = fw.pack_bits(adj, stream=s)
    out = fw.unpack_bits(bits, n, stream=s)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), A)
