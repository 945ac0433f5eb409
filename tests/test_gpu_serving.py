"""GPU tests of the serving loop: each result is the same alone and in the mix,
admission never exceeds the memory budget, queue limits and cancellation."""
import numpy as np
import pytest
import torch

import oracle
import paper_1001_4108_amd as fw
from paper_1001_4108_amd import gen

pytestmark = pytest.mark.gpu


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def windows(count, base_n, nlo, nhi, seed):
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(nlo), np.log(nhi), count))).astype(int)
    os_ = np.array([rng.integers(0, base_n - k + 1) for k in ns])
    return list(zip(ns, os_))


def test_results_same_alone_and_in_mix():
    base_n = 1400
    W = gen.dense_graph(base_n, 0.3, 1, 1000, seed=77)
    base = torch.from_numpy(W).cuda()
    reqs = windows(48, base_n, 16, base_n, seed=5)
    # a budget far below the total footprint forces admission to wait
    total = sum(n * ((n + 3) // 4 * 4) * 4 for n, _ in reqs)
    budget = max(total // 6, base_n * 1400 * 4 + 4096)
    with fw.Server(torch.float32, budget_bytes=budget, streams=3, small_n=512,
                   max_batch=64) as srv:
        ids = [srv.submit(base[o:o + n, o:o + n], keep=True) for n, o in reqs]
        by_id = dict(zip(ids, reqs))
        results = {}
        done = {}
        # kept results hold their memory: fetch and release each one as it
        # completes so the waiting requests can be admitted
        while len(done) < len(reqs):
            got = srv.poll(timeout_us=200000)
            assert got, "server made no progress"
            for c in got:
                done[c[0]] = c
                n, o = by_id[c[0]]
                out = torch.empty((n, n), dtype=torch.float32, device="cuda")
                srv.fetch(c[0], out)
                torch.cuda.synchronize()
                results[c[0]] = out.cpu().numpy()
                srv.release(c[0])
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0
        assert st["peak_bytes"] <= budget and st["deferrals"] >= 1
        assert st["batched_groups"] >= 1 and st["single_groups"] >= 1
        assert st["bytes_in_use"] == 0
    for rid, (n, o) in zip(ids, reqs):
        _, cn, status, group, t_sub, t_adm, t_done = done[rid]
        assert status == 0 and cn == n and t_sub <= t_adm <= t_done
        alone = base[o:o + n, o:o + n].clone()
        fw.fw_apsp(alone)
        torch.cuda.synchronize()
        got = results[rid]
        assert np.array_equal(bits(got), bits(alone.cpu().numpy())), (n, o, group)
        if n <= 400:
            assert np.array_equal(bits(got), bits(oracle.fw(np.ascontiguousarray(
                W[o:o + n, o:o + n])))), (n, o)


def test_int32_server_and_host_copy_back():
    g = gen.reweighted_graph(300, 0.3, 1, 50, -20, 20, seed=3)
    base = torch.from_numpy(g.w).cuda()
    dst = torch.full((300, 300), -1, dtype=torch.int32).pin_memory()
    with fw.Server(torch.int32, budget_bytes=16 << 20, streams=2, small_n=128) as srv:
        rid = srv.submit(base, dst_host=dst)
        srv.drain(timeout_s=60)
        (c,) = srv.poll(timeout_us=100000)
        assert c[0] == rid and c[2] == 0
    assert np.array_equal(dst.numpy(), oracle.fw(g.w))


def test_queue_cap_memory_hold_and_cancellation():
    n = 256
    W = gen.dense_graph(n, 0.3, 1, 9, seed=4)
    a = torch.from_numpy(W).cuda()
    fp = n * n * 4
    srv = fw.Server(torch.float32, budget_bytes=fp + 1024, streams=2, small_n=64, queue_cap=2)
    with pytest.raises(fw.FwError):
        srv.submit(torch.zeros((400, 400), device="cuda"))  # larger than the whole budget
    first = srv.submit(a, keep=True)
    srv.drain(timeout_s=60)          # done, but its memory stays held
    srv.submit(a)                    # waits for memory
    srv.submit(a)                    # waits for memory
    with pytest.raises(fw.FwError):  # queue_cap = 2 waiting requests
        srv.submit(a)
    assert srv.stats()["waiting"] == 2
    srv.release(first)               # memory frees -> both run
    srv.drain(timeout_s=60)
    st = srv.stats()
    assert st["completed"] == 3 and st["rejected"] == 1 and st["deferrals"] >= 1
    # requests still waiting at shutdown are cancelled, not lost
    hold = srv.submit(a, keep=True)
    srv.drain(timeout_s=60)
    srv.submit(a)
    srv.close()
    assert hold > 0
