"""Pins for the widest-path (max, min) oracle: brute force over simple paths,
closed forms, transitive closure against breadth-first search, invariants and
a planted mistake."""
import numpy as np
import pytest

import oracle
from paper_1001_4108_amd import gen

NEG = np.float32(-np.inf)


def random_widths(n, p, rng, dtype=np.float32):
    w = rng.uniform(0.5, 100.0, size=(n, n)).astype(np.float32)  # non-integer widths
    if dtype == np.int32:
        w = rng.integers(1, 50, size=(n, n)).astype(np.int32)
    absent = NEG if dtype == np.float32 else np.int32(np.iinfo(np.int32).min)
    w = np.where(rng.random((n, n)) < p, w, absent).astype(dtype)
    top = np.float32(np.inf) if dtype == np.float32 else np.int32(np.iinfo(np.int32).max)
    np.fill_diagonal(w, top)
    return w, absent, top


def brute_widest(w, absent):
    n = w.shape[0]
    best = np.full((n, n), absent, dtype=w.dtype)
    for i in range(n):
        def dfs(u, width, seen):
            for v in range(n):
                if v == u or v in seen or w[u, v] == absent:
                    continue
                nw = min(width, w[u, v]) if width is not None else w[u, v]
                if nw > best[i, v]:
                    best[i, v] = nw
                dfs(v, nw, seen | {v})
        dfs(i, None, {i})
        best[i, i] = max(best[i, i], w[i, i])
    return best


@pytest.mark.parametrize("seed", range(30))
@pytest.mark.parametrize("dtype", [np.float32, np.int32])
def test_maxmin_matches_brute_force(seed, dtype):
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(1, 8))
    w, absent, top = random_widths(n, float(rng.uniform(0.1, 0.9)), rng, dtype)
    got = oracle.fw_maxmin(w)
    ref = brute_widest(w, absent)
    # a cycle through i can never be wider than the +INF / INT32_MAX diagonal
    assert np.array_equal(got, ref)


def test_maxmin_path_graph_closed_form():
    n = 40
    rng = np.random.default_rng(3)
    wts = rng.uniform(1, 10, n - 1).astype(np.float32)
    w = np.full((n, n), NEG, np.float32)
    np.fill_diagonal(w, np.inf)
    w[np.arange(n - 1), np.arange(1, n)] = wts
    got = oracle.fw_maxmin(w)
    for i in range(n):
        for j in range(n):
            if i < j:
                assert got[i, j] == wts[i:j].min()
            elif i > j:
                assert got[i, j] == NEG


@pytest.mark.parametrize("p", [0.01, 0.03, 0.2])
def test_transitive_closure_matches_bfs(p):
    n = 200
    W = gen.dense_graph(n, p, 1, 1, seed=int(p * 1000), dtype=np.int32)
    A = np.where(W == gen.I32_INF, 0, 1).astype(np.int32)
    np.fill_diagonal(A, 1)
    R = oracle.fw_maxmin(A)
    for s in range(0, n, 7):
        assert np.array_equal(R[s].astype(bool), oracle.reach_row(W, s))


def test_maxmin_invariants_and_idempotence():
    rng = np.random.default_rng(11)
    w, absent, top = random_widths(150, 0.05, rng)
    d = oracle.fw_maxmin(w)
    assert (d >= w).all()
    for k in range(0, 150, 5):
        assert (d >= np.minimum(d[:, k:k + 1], d[k:k + 1, :])).all()
    assert np.array_equal(oracle.fw_maxmin(d), d)


def test_pins_reject_swapped_semiring():
    """Computing min over paths of the max edge (a plausible swap) fails."""
    caught = False
    for seed in range(20):
        rng = np.random.default_rng(900 + seed)
        n = int(rng.integers(3, 7))
        w, absent, top = random_widths(n, 0.6, rng)
        d = w.astype(np.float64).copy()
        for k in range(n):
            for i in range(n):
                for j in range(n):
                    d[i, j] = min(d[i, j], max(d[i, k], d[k, j]))
        if not np.array_equal(d.astype(np.float32), brute_widest(w, absent)):
            caught = True
            break
    assert caught


@pytest.mark.parametrize("seed", range(6))
def test_widest_rows_match_maxmin_loop(seed):
    rng = np.random.default_rng(1200 + seed)
    n = int(rng.integers(2, 120))
    w, absent, top = random_widths(n, float(rng.uniform(0.02, 0.5)), rng)
    d = oracle.fw_maxmin(w)
    srcs = np.arange(n)
    r = oracle.widest_rows(w, srcs).astype(np.float32)
    off = ~np.eye(n, dtype=bool)
    assert np.array_equal(r[off], d[off])
