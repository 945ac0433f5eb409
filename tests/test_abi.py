"""The C-ABI library loads, exports every declared symbol, and validates
arguments on the host (no GPU needed: every call here returns before any HIP
call is made)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1001_4108_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fwapsp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fw_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name


def test_status_strings():
    L = B.lib()
    for code, name in B.STATUS.items():
        assert L.fw_status_string(code).decode().startswith(name)
    assert L.fw_status_string(999).decode() == "FW_ERR_UNKNOWN"
    assert b"gfx950" in L.fw_version()


def test_argument_validation_without_gpu():
    L = B.lib()
    null = None
    assert L.fw_apsp(null, 5, 5, null) == 1           # NULL matrix
    assert L.fw_apsp(ctypes.c_void_p(16), -1, 5, null) == 1
    assert L.fw_apsp(ctypes.c_void_p(16), 6, 5, null) == 1   # ld < n
    assert L.fw_apsp(ctypes.c_void_p(16), 2**40, 2**40, null) == 1  # n too large
    assert L.fw_apsp_i32(null, 3, 3, null) == 1
    assert L.fw_apsp(null, 0, 0, null) == 0            # empty graph: no-op
    assert L.fw_apsp(ctypes.c_void_p(16), 1, 1, null) == 0   # one vertex: no-op
    assert L.fw_apsp_pred(ctypes.c_void_p(16), 7, 4, 4, null, 0, null) == 1  # dtype
    assert L.fw_apsp_pred(ctypes.c_void_p(16), 0, 4, 4, ctypes.c_void_p(32), 3, null) == 1
    assert L.fw_apsp_plan(ctypes.c_void_p(16), 0, 64, 64, null, 0, 48, null) == 1  # tile
    assert L.fw_negative_cycle(ctypes.c_void_p(16), 0, 4, 4, null, null) == 1
    assert L.fw_apsp_batched(None, None, None, 0, 0, None, None, null) == 0
    assert L.fw_apsp_ladder(ctypes.c_void_p(16), 0, 8, 8, 7, null) == 1   # rung
    assert L.fw_apsp_ladder(ctypes.c_void_p(16), 0, 8, 4, 0, null) == 1   # ld < n
    assert L.fw_apsp_ladder(null, 0, 0, 0, 2, null) == 0                  # empty graph


def test_bit_packed_closure_argument_validation():
    L = B.lib()
    null = ctypes.c_void_p(0)
    some = ctypes.c_void_p(16)
    assert L.fw_transitive_closure_bits(null, 5, 1, 1, null) == 1      # NULL bits
    assert L.fw_transitive_closure_bits(some, -1, 1, 1, null) == 1     # n < 0
    assert L.fw_transitive_closure_bits(some, 33, 1, 1, null) == 1     # ldw < 2 words
    assert L.fw_transitive_closure_bits(null, 0, 0, 1, null) == 0      # empty graph
    assert L.fw_transitive_closure_bits(some, (1 << 21) + 1, 1 << 17, 1, null) == 4  # too large
    assert L.fw_pack_bits(some, 40, 39, some, 2, null) == 1            # ld < n
    assert L.fw_pack_bits(some, 40, 40, some, 1, null) == 1            # ldw < 2
    assert L.fw_unpack_bits(null, 40, 2, some, 40, null) == 1          # NULL bits
    assert L.fw_unpack_bits(some, 0, 0, null, 0, null) == 0
    assert B.words_per_row(0) == 0 and B.words_per_row(32) == 1 and B.words_per_row(33) == 2


def test_plan_table():
    tiles = B.plan_tiles()
    assert tiles == sorted(tiles) and set(tiles) <= {32, 64, 128, 256}
    B.plan_reset()
    assert B.plan_tile("f32", 0) == 0 and B.plan_tile("f32", 1) == 0
    for n in (2, 100, 512, 5000, 16384):
        assert B.plan_tile("f32", n) in tiles
        assert B.plan_tile("i32", n) in tiles
    assert B.lib().fw_plan_tile(5, 10) == -1
    B.plan_set("f32", 100, 200, tiles[-1])
    assert B.plan_tile("f32", 150) == tiles[-1]
    with pytest.raises(B.FwError):
        B.plan_set("f32", 10, 5, tiles[0])
    with pytest.raises(B.FwError):
        B.plan_set("f32", 1, 5, 48)
    B.plan_reset()


def test_plan_table_predecessor_key():
    # the solves that compute predecessors have their own part of the table
    B.plan_reset()
    assert B.FW_PLAN_PRED == 2
    for dt, code in (("f32", 0), ("i32", 1)):
        for n in (2, 100, 512, 5000, 16384):
            assert B.plan_tile(dt, n, pred=True) == B.lib().fw_plan_tile(code | 2, n)
            assert B.plan_tile(dt, n, pred=True) in B.plan_tiles()
    # built-in defaults: with predecessors tile 32 for small blocked solves and
    # 64 above (int32 above 4096: 128, the keyed sweep's tile), without 64 then
    # 128 for large solves
    assert B.plan_tile("i32", 8192, pred=True) == 128  # the keyed sweep's tile
    assert B.plan_tile("i32", 3000, pred=True) == 64
    assert B.plan_tile("i32", 500, pred=True) == 32 and B.plan_tile("f32", 1500, pred=True) == 32
    assert B.plan_tile("f32", 16384) == 128 and B.plan_tile("i32", 8192) == 128
    assert B.plan_tile("f32", 1024) == 64
    B.plan_set("i32", 1000, 2000, 32, pred=True)
    assert B.plan_tile("i32", 1500, pred=True) == 32
    assert B.plan_tile("i32", 1500) == 64 and B.plan_tile("i32", 2500, pred=True) == 64
    assert B.lib().fw_plan_tile(4, 10) == -1 and B.lib().fw_plan_tile(-1, 10) == -1
    assert B.lib().fw_plan_set(6, 1, 2, 64) == 1
    B.plan_reset()
    assert B.plan_tile("i32", 1500, pred=True) == 64


def test_fw_path_host_reconstruction():
    # 0 -> 2 -> 1 -> 3, 4 unreachable
    P = np.array([[-1, 2, 0, 1, -1],
                  [-1, -1, -1, 1, -1],
                  [-1, 2, -1, 1, -1],
                  [-1, -1, -1, -1, -1],
                  [-1, -1, -1, -1, -1]], np.int32)
    assert B.fw_path(P, 0, 3) == [0, 2, 1, 3]
    assert B.fw_path(P, 0, 0) == [0]
    assert B.fw_path(P, 0, 4) == []
    bad = P.copy()
    bad[0, 1] = 3  # 3 -> 1 -> 3 ... never returns to 0
    bad[0, 3] = 1
    with pytest.raises(B.FwError):
        B.fw_path(bad, 0, 3)


def test_solve_plan_and_negative_cycle_argument_validation():
    L = B.lib()
    null = None
    some = ctypes.c_void_p(16)
    h = ctypes.c_void_p()
    assert L.fw_solve_plan_create(null, 0, 5, 5, null, 0, 0, ctypes.byref(h)) == 1
    assert L.fw_solve_plan_create(some, 0, 5, 4, null, 0, 0, ctypes.byref(h)) == 1   # ld < n
    assert L.fw_solve_plan_create(some, 0, 64, 64, null, 0, 48, ctypes.byref(h)) == 1  # tile
    assert L.fw_solve_plan_create(some, 0, 64, 64, null, 0, 0, null) == 1
    assert L.fw_solve_plan_launch(null, 1, null) == 1
    assert L.fw_solve_plan_destroy(null) == 1
    assert L.fw_solve_plan_tile(null) == -1
    assert L.fw_negative_cycle_vertices(some, 0, 4, 4, null, some, null) == 1  # no list
    assert L.fw_negative_cycle_vertices(some, 0, 4, 4, some, null, null) == 1  # no count
    assert L.fw_negative_cycle_vertices(some, 9, 4, 4, some, some, null) == 1  # dtype
    buf = (ctypes.c_int64 * 4)()
    W = np.zeros((4, 4), np.int32)
    f = L.fw_negative_cycle_find
    assert f(null, 1, 4, 4, null, 0, 0, buf, 4, null) == -1          # no weights
    assert f(W.ctypes.data, 1, 4, 4, null, 0, 4, buf, 4, null) == -1  # v out of range
    assert f(W.ctypes.data, 1, 4, 3, null, 0, 0, buf, 4, null) == -1  # ld < n
    assert f(W.ctypes.data, 1, 4, 4, W.ctypes.data, 3, 0, buf, 4, null) == -1  # ld_pred < n


def _cycle_weight(W, cyc):
    return sum(int(W[cyc[t], cyc[(t + 1) % len(cyc)]]) for t in range(len(cyc)))


def test_negative_cycle_find_on_host():
    """Cycle extraction from a predecessor row and by the Bellman-Ford
    fallback, on hand-built inputs (host only)."""
    M = B.I32_INF
    # 0 -> 1 -> 2 -> 0 weighs -3; 3 -> 0 and 2 -> 4 hang off it
    W = np.full((5, 5), M, np.int32)
    np.fill_diagonal(W, 0)
    W[0, 1] = W[1, 2] = W[2, 0] = -1
    W[3, 0] = 5
    W[2, 4] = 2
    # a predecessor row 0 whose last hops follow the cycle
    P = np.full((5, 5), -1, np.int32)
    P[0, 0], P[0, 1], P[0, 2], P[0, 4] = 2, 0, 1, 2
    cyc, from_pred = B.fw_negative_cycle_find(W, 0, P)
    assert from_pred and cyc == [0, 1, 2] and _cycle_weight(W, cyc) == -3
    # without predecessors: Bellman-Ford from 1 finds the same cycle (a rotation)
    cyc, from_pred = B.fw_negative_cycle_find(W, 1)
    assert not from_pred and sorted(cyc) == [0, 1, 2] and _cycle_weight(W, cyc) == -3
    # a predecessor row whose walk closes a non-negative cycle is not trusted
    P2 = P.copy()
    W2 = W.copy()
    W2[1, 0] = 7            # 0 -> 1 -> 0 weighs 6
    P2[0, 0], P2[0, 1] = 1, 0
    cyc, from_pred = B.fw_negative_cycle_find(W2, 0, P2)
    assert not from_pred and _cycle_weight(W2, cyc) < 0 and sorted(cyc) == [0, 1, 2]
    # no negative cycle reachable from 4: empty
    assert B.fw_negative_cycle_find(W, 4) == ([], False)
    # fp32 weights
    Wf = np.where(W == M, np.float32(np.inf), W.astype(np.float32)).astype(np.float32)
    cyc, _ = B.fw_negative_cycle_find(Wf, 2)
    assert sorted(cyc) == [0, 1, 2]


def test_autotune_argument_validation():
    import ctypes
    L = B.lib()
    lo = (ctypes.c_int64 * 1)(64)
    hi = (ctypes.c_int64 * 1)(32)   # hi < lo
    out = (ctypes.c_int * 1)()
    assert L.fw_autotune(0, lo, hi, 1, 0, 1, 1, out, None) == 1
    hi[0] = 128
    assert L.fw_autotune(5, lo, hi, 1, 0, 1, 1, out, None) == 1   # dtype
    assert L.fw_autotune(0, lo, hi, 1, 2, 1, 1, out, None) == 1   # objective
    assert L.fw_autotune(0, lo, hi, 1, 1, 0, 1, out, None) == 1   # empty batch
    assert L.fw_autotune(0, lo, hi, 0, 0, 1, 1, out, None) == 1   # no buckets


def test_negative_cycle_find_on_random_graphs():
    """On random graphs with negative cycles (host only): for every vertex v
    whose oracle distance d_vv is negative (a negative closed walk through v),
    Bellman-Ford from v returns a simple cycle of real edges with negative
    weight.  Graphs stay small enough (n <= 12, weights >= -4) that the
    oracle's values cannot overflow int32."""
    import oracle
    rng = np.random.default_rng(77)
    M = B.I32_INF
    found_any = 0
    for trial in range(80):
        n = int(rng.integers(3, 13))
        W = np.where(rng.random((n, n)) < rng.uniform(0.1, 0.5),
                     rng.integers(-4, 20, (n, n)), M).astype(np.int32)
        np.fill_diagonal(W, 0)
        D = oracle.fw(W)
        for v in range(n):
            cyc, _ = B.fw_negative_cycle_find(W, v)
            if D[v, v] < 0:
                assert cyc, (trial, v)
                m = len(cyc)
                assert all(W[cyc[t], cyc[(t + 1) % m]] != M and cyc[t] != cyc[(t + 1) % m]
                           for t in range(m))
                assert _cycle_weight(W, cyc) < 0
                assert len(set(cyc)) == m  # a simple cycle
                found_any += 1
    assert found_any > 20
