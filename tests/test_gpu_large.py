"""Largest size exercised: n=32768 fp32 (a 4 GiB matrix, 256 stages of the
128-wide schedule, 255^2 bulk tiles per stage), checked on seeded Dijkstra
rows and a sampled triangle inequality."""
import numpy as np
import pytest
import torch

import oracle
from paper_1001_4108_amd import gen
import paper_1001_4108_amd as fw

pytestmark = pytest.mark.gpu


def test_n32768_fp32_dijkstra_rows():
    n = 32768
    W = gen.dense_graph(n, 0.05, 1, 1000, seed=32768)
    d = torch.from_numpy(W).cuda()
    fw.fw_apsp(d)
    torch.cuda.synchronize()
    rng = np.random.default_rng(327)
    srcs = np.sort(rng.choice(n, 3, replace=False))
    rows = d[torch.from_numpy(srcs).cuda()].cpu().numpy()
    ref = oracle.dijkstra_rows(W, srcs).astype(np.float32)
    assert np.array_equal(rows.view(np.uint32), ref.view(np.uint32))
    # triangle inequality d_ij <= d_ik + d_kj on sampled triples
    i, j, k = (torch.from_numpy(rng.integers(0, n, 4096)).cuda() for _ in range(3))
    assert bool((d[i, j] <= d[i, k] + d[k, j]).all())
    del d
    torch.cuda.empty_cache()
