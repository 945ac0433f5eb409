"""Properties of the seeded input generators (shared by tests and benchmark)."""
import numpy as np

from paper_1001_4108_amd import gen


def test_dense_graph_shape_density_range_and_determinism():
    W = gen.dense_graph(600, 0.3, 1, 1000, seed=2)
    assert W.dtype == np.float32 and W.shape == (600, 600)
    assert (np.diag(W) == 0).all()
    off = ~np.eye(600, dtype=bool)
    real = np.isfinite(W) & off
    assert abs(real.sum() / off.sum() - 0.3) < 0.01
    vals = W[real]
    assert vals.min() >= 1 and vals.max() <= 1000 and (vals == np.rint(vals)).all()
    assert np.isposinf(W[off & ~real]).all()
    assert np.array_equal(W, gen.dense_graph(600, 0.3, 1, 1000, seed=2))
    assert not np.array_equal(W, gen.dense_graph(600, 0.3, 1, 1000, seed=3))


def test_int32_graph_uses_sentinel():
    W = gen.dense_graph(100, 0.2, 1, 10, seed=1, dtype=np.int32)
    off = ~np.eye(100, dtype=bool)
    assert set(np.unique(W[off])) <= set(range(1, 11)) | {gen.I32_INF}
    assert (np.diag(W) == 0).all()


def test_reweighted_graph_keeps_cycle_weights():
    g = gen.reweighted_graph(50, 0.5, 1, 1000, -500, 500, seed=3)
    edge = (g.base != gen.I32_INF) & ~np.eye(50, dtype=bool)
    assert np.array_equal(edge, (g.w != gen.I32_INF) & ~np.eye(50, dtype=bool))
    w = g.w.astype(np.int64)
    assert w[edge].min() >= -999 and w[edge].max() <= 2000
    # every 2-cycle and 3-cycle keeps its base weight
    for u in range(10):
        for v in range(10):
            if u != v and edge[u, v] and edge[v, u]:
                assert w[u, v] + w[v, u] == int(g.base[u, v]) + int(g.base[v, u])


def test_ragged_sizes_are_log_uniform_in_range():
    s = gen.ragged_sizes()
    assert len(s) == 4096 and s.min() >= 16 and s.max() <= 512
    counts = [((s >= a) & (s <= b)).sum() for a, b in [(16, 32), (33, 64), (65, 128),
                                                      (129, 256), (257, 512)]]
    assert all(700 < c < 950 for c in counts)


def test_serving_trace_statistics():
    tr = gen.serving_trace()
    assert 118000 < len(tr.t) < 122000
    assert (np.diff(tr.t) > 0).all() and tr.t[-1] < 60.0
    assert tr.n.min() >= 64 and tr.n.max() <= 8192
    assert ((tr.o >= 0) & (tr.o + tr.n <= tr.base_n)).all()
    small = gen.serving_trace(rate=100, duration=1.0, nhi=256)
    g = small.request_graph(0)
    assert g.shape == (small.n[0], small.n[0]) and (np.diag(g) == 0).all()
