"""Seeded synthetic graph generators.

This module only draws inputs.  It holds none of the shortest-path
arithmetic and is shared, unchanged, by the tests, the benchmark and the
oracle checks.  All randomness comes from numpy's PCG64 (`default_rng`), so a
(seed, size) pair always gives the same bytes on any host.

Graph model (the paper times "any graph" with n vertices, since the run time
of Floyd-Warshall does not depend on the data; section 1 and section 5): a
dense directed graph with an edge on each ordered pair i != j independently
with probability ``p``, integer-valued weights drawn uniformly from
``[lo, hi]`` (inclusive), weight 0 on the diagonal and "infinity" for the
absent pairs (+INF for float32, ``I32_INF`` for int32; section 3.1).

Rows are drawn in blocks of ``CHUNK_ROWS``: per block, first the edge
coin-flips (float32 uniforms) then the weights, so large matrices need not be
materialised twice in float64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

I32_INF = 1073741823  # INT32_MAX // 2, "no edge" for int32 matrices
CHUNK_ROWS = 1024


def dense_graph(n: int, p: float, lo: int, hi: int, seed, dtype=np.float32) -> np.ndarray:
    """Dense directed Bernoulli(p) graph with integer weights in [lo, hi]."""
    dtype = np.dtype(dtype)
    rng = np.random.default_rng(seed)
    inf = np.float32(np.inf) if dtype == np.float32 else np.int32(I32_INF)
    out = np.empty((n, n), dtype=dtype)
    for r0 in range(0, n, CHUNK_ROWS):
        r1 = min(n, r0 + CHUNK_ROWS)
        edge = rng.random((r1 - r0, n), dtype=np.float32) < np.float32(p)
        wts = rng.integers(lo, hi + 1, size=(r1 - r0, n), dtype=np.int32)
        out[r0:r1] = np.where(edge, wts.astype(dtype), inf)
    np.fill_diagonal(out, 0)
    return out


@dataclass
class Reweighted:
    """A graph with negative edges obtained by potential reweighting."""
    w: np.ndarray      # int32 reweighted matrix w'(u,v) = w(u,v) + pot(u) - pot(v)
    base: np.ndarray   # int32 non-negative original weights (I32_INF absent)
    pot: np.ndarray    # int64 potentials, one per vertex


def reweighted_graph(n: int, p: float, lo: int, hi: int, pot_lo: int, pot_hi: int,
                     seed) -> Reweighted:
    """int32 graph with negative weights and no negative cycle.

    Base weights as in :func:`dense_graph` (stream 0 of ``SeedSequence(seed)``),
    potentials uniform integers in [pot_lo, pot_hi] (stream 1).  Reweighting
    adds pot(u) - pot(v) to every real edge, which leaves the weight of every
    cycle unchanged, so the graph keeps its (positive) cycle weights.
    """
    ss = np.random.SeedSequence(seed)
    s_mat, s_pot = ss.spawn(2)
    base = dense_graph(n, p, lo, hi, s_mat, dtype=np.int32)
    pot = np.random.default_rng(s_pot).integers(pot_lo, pot_hi + 1, size=n, dtype=np.int64)
    edge = base != I32_INF
    np.fill_diagonal(edge, False)
    w64 = base.astype(np.int64) + pot[:, None] - pot[None, :]
    w = np.where(edge, w64, I32_INF).astype(np.int32)
    np.fill_diagonal(w, 0)
    return Reweighted(w=w, base=base, pot=pot)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def single_graph_512() -> np.ndarray:
    """n=512 fp32, edge prob 0.5, weights integer in [1, 100] (seed 1)."""
    return dense_graph(512, 0.5, 1, 100, seed=1)


def single_graph_16384(n: int = 16384) -> np.ndarray:
    """n=16384 fp32 (1 GiB), edge prob 0.3, weights integer in [1, 1000] (seed 2)."""
    return dense_graph(n, 0.3, 1, 1000, seed=2)


def dijkstra_sources_16384(n: int = 16384, count: int = 64) -> np.ndarray:
    """The 64 seeded source vertices checked on the n=16384 solve."""
    return np.sort(np.random.default_rng(2002).choice(n, count, replace=False)).astype(np.int64)


def negative_graph_8192(n: int = 8192) -> Reweighted:
    """n=8192 int32, edge prob 0.2, base weights [1,1000], potentials [-500,500] (seed 3)."""
    return reweighted_graph(n, 0.2, 1, 1000, -500, 500, seed=3)


def ragged_sizes(count: int = 4096, lo: int = 16, hi: int = 512, seed: int = 4) -> np.ndarray:
    """Log-uniform sizes n = round(exp(U(ln lo, ln hi))) for a ragged batch."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return np.clip(np.rint(np.exp(u)), lo, hi).astype(np.int64)


def ragged_batch(count: int = 4096, lo: int = 16, hi: int = 512, seed: int = 4,
                 p: float = 0.4, wlo: int = 1, whi: int = 100):
    """Ragged batch: sizes from :func:`ragged_sizes`, graph g from child g of
    ``SeedSequence((seed, 1))``; fp32, edge prob 0.4, weights [1, 100]."""
    sizes = ragged_sizes(count, lo, hi, seed)
    kids = np.random.SeedSequence((seed, 1)).spawn(count)
    return [dense_graph(int(n), p, wlo, whi, kids[g]) for g, n in enumerate(sizes)]


@dataclass
class ServingTrace:
    """Arrival schedule of the serving workload.

    Request r arrives at ``t[r]`` seconds and asks for APSP on the principal
    window ``base[b[r]][o[r]:o[r]+n[r], o[r]:o[r]+n[r]]`` of one of the
    ``nbase`` base graphs (each ``dense_graph(base_n, p, wlo, whi, (seed, b))``).
    A principal window of an i.i.d. Bernoulli graph is itself such a graph, so
    every request is a correctly distributed n-vertex graph while the payload
    pool stays small enough to keep resident in device memory.
    """
    t: np.ndarray
    n: np.ndarray
    b: np.ndarray
    o: np.ndarray
    base_n: int
    nbase: int
    p: float
    wlo: int
    whi: int
    seed: int

    def base_graph(self, b: int) -> np.ndarray:
        return dense_graph(self.base_n, self.p, self.wlo, self.whi, (self.seed, int(b)))

    def request_graph(self, r: int, bases=None) -> np.ndarray:
        base = bases[self.b[r]] if bases is not None else self.base_graph(self.b[r])
        o, n = int(self.o[r]), int(self.n[r])
        return np.ascontiguousarray(base[o:o + n, o:o + n])


def serving_trace(rate: float = 2000.0, duration: float = 60.0, nlo: int = 64,
                  nhi: int = 8192, seed: int = 5, nbase: int = 2, p: float = 0.3,
                  wlo: int = 1, whi: int = 1000) -> ServingTrace:
    """Poisson arrivals at ``rate``/s for ``duration`` s; n log-uniform [nlo, nhi]."""
    rng = np.random.default_rng(seed)
    expect = int(rate * duration * 1.2 + 100)
    gaps = rng.exponential(1.0 / rate, size=expect)
    t = np.cumsum(gaps)
    t = t[t < duration]
    m = len(t)
    u = rng.uniform(math.log(nlo), math.log(nhi), size=m)
    n = np.clip(np.rint(np.exp(u)), nlo, nhi).astype(np.int64)
    b = rng.integers(0, nbase, size=m)
    o = rng.integers(0, nhi - n + 1).astype(np.int64) if m else np.zeros(0, np.int64)
    return ServingTrace(t=t, n=n, b=b.astype(np.int64), o=o, base_n=nhi, nbase=nbase,
                        p=p, wlo=wlo, whi=whi, seed=seed)


def cycle_permutation(n: int, seed) -> np.ndarray:
    """A seeded random order of the n vertices: the directed cycle
    perm[0] -> perm[1] -> ... -> perm[n-1] -> perm[0] is a graph whose
    shortest paths run up to n - 1 hops (the long-path parity input)."""
    return np.random.default_rng(seed).permutation(n)


def planted_negative_cycle(n: int, p: float, length: int, seed, dtype=np.int32):
    """A graph with exactly one negative simple cycle: Bernoulli(p) edges with
    integer weights in [length, length + 99] and, on `length` seeded distinct
    vertices c_0 .. c_{L-1}, the edges c_t -> c_{t+1 mod L} of weight -1.
    No other edge enters a cycle vertex (edges leave it freely), so no other
    vertex lies on a closed walk through the cycle and only c_0 .. c_{L-1}
    reach themselves at negative cost; every other simple cycle avoids the
    cycle vertices and weighs at least L.  Floyd-Warshall's values then stay
    above -L * 2^L (each cycle vertex at most doubles the negative part).
    Returns (matrix, cycle vertices in order)."""
    ss = np.random.SeedSequence(seed)
    s_mat, s_cyc = ss.spawn(2)
    w = dense_graph(n, p, length, length + 99, s_mat, dtype=dtype)
    cyc = np.random.default_rng(s_cyc).choice(n, length, replace=False)
    absent = np.float32(np.inf) if np.dtype(dtype) == np.float32 else np.int32(I32_INF)
    w[:, cyc] = absent
    w[cyc, cyc] = 0
    for t in range(length):
        w[cyc[t], cyc[(t + 1) % length]] = -1
    return w, cyc
