"""CPU pins of the 32-bit (distance, last hop) key reading.

The library sweeps predecessors as keys key = d * 2^14 + p (p = 2^14 - 1:
no last hop), the candidate through k being (key_ik with its hop field
cleared) + key_kj, values at or above 2^29 settled to K = 2^30 - 2^14, and
an unreachable pair's int32 distance written as M + (row i's minimum) +
(column j's minimum) over the finite distances (0 included).  This module
restates that reading in numpy, runs it in the plain triple-loop order (the
result is order-free), and checks it against the oracle's distances and
canonical predecessors, raw unreachable int32 values included.  It shares
nothing with the GPU kernels; it pins the arithmetic the kernels follow.
"""
import numpy as np
import pytest

import oracle
from paper_1001_4108_amd import gen

M = gen.I32_INF
BITS = 14
HOP = (1 << BITS) - 1
K = (1 << 30) - (1 << BITS)
REAL = 1 << 28
LOW = -REAL + (1 << BITS)
INF_FLOOR = 1 << 29


def key_sweep(W):
    """Keyed Floyd-Warshall of int32 W: returns (keys, in_range)."""
    n = W.shape[0]
    absent = W == M
    i = np.arange(n)
    hop = np.where(i[:, None] == i[None, :], HOP, i[:, None]).astype(np.int64)
    key = np.where(absent, K, W.astype(np.int64) * (1 << BITS) + hop)
    ok = bool(((W[~absent] > -(1 << BITS)) & (W[~absent] < (1 << BITS))).all())
    for k in range(n):
        a = key[:, k] & ~np.int64(HOP)
        cand = a[:, None] + key[k, :][None, :]
        assert cand.max() < 2 ** 31 and cand.min() >= -(2 ** 31)  # the int32 sums never wrap
        key = np.minimum(key, cand)
        inf = key >= INF_FLOOR
        real = key[~inf]
        ok &= bool(((real >= LOW) & (real < REAL)).all())
        key = np.where(inf, K, key)
    return key, ok


def decode(key):
    n = key.shape[0]
    real = key < INF_FLOOR
    d = np.where(real, key >> BITS, 0)
    rowmin = np.minimum(d.min(axis=1), 0)
    colmin = np.minimum(d.min(axis=0), 0)
    dist = np.where(real, d, M + rowmin[:, None] + colmin[None, :]).astype(np.int32)
    h = key & HOP
    i = np.arange(n)
    P = np.where(real & (h != HOP) & (i[:, None] != i[None, :]), h, -1).astype(np.int32)
    return dist, P


@pytest.mark.parametrize("seed", range(12))
def test_keys_give_oracle_distances_and_predecessors(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 48))
    p = float(rng.choice([0.0, 0.03, 0.1, 0.3, 0.8]))
    g = gen.reweighted_graph(n, p, 1, int(rng.integers(1, 300)), -200, 200, seed=seed)
    W = g.w.copy()
    if seed % 3 == 0 and n > 4:  # absent and positive diagonal entries
        W[1, 1] = M
        W[2, 2] = 7
    key, ok = key_sweep(W)
    assert ok
    dist, P = decode(key)
    ref = oracle.fw(W)
    assert np.array_equal(dist, ref)            # raw unreachable values included
    assert np.array_equal(P, oracle.canonical_pred(ref, W))


def test_unreachable_values_are_present_and_reproduced():
    W = gen.reweighted_graph(40, 0.02, 1, 100, -100, 100, seed=3).w
    dist, _ = decode(key_sweep(W)[0])
    ref = oracle.fw(W)
    unreach = ref > M // 2
    assert unreach.sum() > 100 and (ref[unreach] != M).any()  # values other than M occur
    assert np.array_equal(dist, ref)


def test_range_check_rejects_large_distances():
    n = 30
    W = np.full((n, n), M, dtype=np.int32)
    np.fill_diagonal(W, 0)
    perm = gen.cycle_permutation(n, seed=4)
    W[perm, np.roll(perm, -1)] = 600  # longest distance 29 * 600 = 17400 >= 2^14
    assert not key_sweep(W)[1]
    W[perm, np.roll(perm, -1)] = 560  # longest distance 16240 < 2^14
    key, ok = key_sweep(W)
    assert ok
    assert np.array_equal(decode(key)[0], oracle.fw(W))


def test_key_constants():
    # finite keys and the infinite class never meet and nothing overflows
    assert 2 * REAL <= INF_FLOOR <= K - REAL
    assert 2 * K < 2 ** 31 and K % (1 << BITS) == 0
    # the hop value "none" orders after every vertex of a graph of at most 2^14 - 1 vertices
    assert HOP == (1 << BITS) - 1
