"""CPU oracle for blocked Floyd-Warshall APSP.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package; the library in
``paper_1001_4108_amd`` never does, and shares no code with it.

Everything here is a thin numpy front end over ``fw_oracle.c`` (plain C,
built by ``oracle/build.py``):

* ``fw(w)``                 -- Floyd-Warshall, section 3.1 / Fig. FW-Alg, in the
                               matrix's own dtype (fp32 or int32).
* ``canonical_pred(D, W)``  -- smallest-index last hop over all shortest
                               paths (the library's predecessor reading).
* ``dijkstra_rows(W, srcs)``-- textbook dense Dijkstra in float64, for rows
                               of solves too large for ``fw``.
* ``reach_row(W, src)``     -- breadth-first reachability over the edges.
* ``fw_maxmin(w)``          -- the same loop over the (max, min) semiring
                               (widest paths; transitive closure on {0, 1}).
* ``widest_rows(W, srcs)``  -- bottleneck Dijkstra, rows of large widest-path
                               solves.

Parity status: every function here is pinned by ``tests/test_oracle_pins.py``
(brute-force path enumeration, closed forms, library routines, invariants).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

I32_INF = 1073741823  # "no edge" for int32 matrices (INT32_MAX // 2)

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    i64, vp, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
    lib.oracle_fw_f32.argtypes = [vp, i64, i64, i64, i64, ci]
    lib.oracle_fw_i32.argtypes = [vp, i64, i64, i64, i64, ci]
    lib.oracle_reach_row.argtypes = [vp, ci, i64, i64, i64, vp]
    lib.oracle_canonical_pred_rows.argtypes = [vp, i64, vp, i64, ci, i64, vp, i64, vp, i64, ci]
    lib.oracle_dijkstra_rows.argtypes = [vp, ci, i64, i64, vp, i64, vp, i64, ci]
    lib.oracle_dijkstra_rows.restype = ci
    lib.oracle_max_threads.restype = ci
    lib.oracle_fw_maxmin_f32.argtypes = [vp, i64, i64, ci]
    lib.oracle_fw_maxmin_i32.argtypes = [vp, i64, i64, ci]
    lib.oracle_widest_rows_f32.argtypes = [vp, i64, i64, vp, i64, vp, i64, ci]
    _lib = lib
    return lib


def max_threads() -> int:
    """OpenMP threads the oracle uses by default."""
    return int(_load().oracle_max_threads())


def _dtype_code(a: np.ndarray) -> int:
    if a.dtype == np.float32:
        return 0
    if a.dtype == np.int32:
        return 1
    raise TypeError(f"oracle supports float32 and int32, got {a.dtype}")


def _square_rowmajor(a: np.ndarray):
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("expected a square matrix")
    if a.strides[1] != a.itemsize or a.strides[0] % a.itemsize:
        raise ValueError("expected row-major storage with unit column stride")
    return a.shape[0], a.strides[0] // a.itemsize


def fw(w: np.ndarray, nthreads: int = 0, k_begin: int = 0, k_end=None) -> np.ndarray:
    """Floyd-Warshall (Fig. FW-Alg) on a copy of ``w``; returns the distances.

    ``k_begin``/``k_end`` restrict the outer k loop (a prefix of it is what the
    CPU timing leg measures); the default is the whole algorithm.
    """
    code = _dtype_code(w)
    d = np.array(w, copy=True, order="C")
    fw_inplace(d, nthreads, k_begin, k_end)
    return d


def fw_inplace(d: np.ndarray, nthreads: int = 0, k_begin: int = 0, k_end=None) -> None:
    """In-place form of :func:`fw` (``d`` may be a row-major view with ld > n)."""
    code = _dtype_code(d)
    n, ld = _square_rowmajor(d)
    if k_end is None:
        k_end = n
    if not (0 <= k_begin <= k_end <= n):
        raise ValueError("bad k range")
    lib = _load()
    fn = lib.oracle_fw_f32 if code == 0 else lib.oracle_fw_i32
    fn(d.ctypes.data, n, ld, k_begin, k_end, nthreads)


def fw_maxmin(w: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """Widest-path (max, min) closure of Fig. FW-Alg's loop on a copy of ``w``.

    Absent edges must hold -INF (float32) or INT32_MIN (int32).
    """
    code = _dtype_code(w)
    d = np.array(w, copy=True, order="C")
    n, ld = _square_rowmajor(d)
    lib = _load()
    fn = lib.oracle_fw_maxmin_f32 if code == 0 else lib.oracle_fw_maxmin_i32
    fn(d.ctypes.data, n, ld, nthreads)
    return d


def widest_rows(W: np.ndarray, srcs, nthreads: int = 0) -> np.ndarray:
    """float64 widest-path widths from each source (bottleneck Dijkstra), fp32
    input with -INF for absent edges; the source's own entry is +inf."""
    if W.dtype != np.float32:
        raise TypeError("widest_rows takes float32")
    n, ld = _square_rowmajor(W)
    srcs = np.ascontiguousarray(srcs, dtype=np.int64)
    out = np.empty((len(srcs), n), dtype=np.float64)
    _load().oracle_widest_rows_f32(W.ctypes.data, n, ld, srcs.ctypes.data, len(srcs),
                                   out.ctypes.data, n, nthreads)
    return out


def reach_row(w: np.ndarray, src: int) -> np.ndarray:
    """Boolean row: which vertices ``src`` reaches over the edges of ``w``."""
    code = _dtype_code(w)
    n, ld = _square_rowmajor(w)
    out = np.zeros(n, dtype=np.uint8)
    _load().oracle_reach_row(w.ctypes.data, code, n, ld, int(src), out.ctypes.data)
    return out.astype(bool)


def canonical_pred(D: np.ndarray, W: np.ndarray, rows=None, nthreads: int = 0) -> np.ndarray:
    """Canonical predecessors from final distances ``D`` and original weights ``W``.

    With ``rows=None`` ``D`` is the full n x n distance matrix and the result
    is n x n.  With ``rows`` (source indices) ``D`` holds only those rows, in
    that order, and the result has one row per listed source.
    """
    code = _dtype_code(W)
    n, ldw = _square_rowmajor(W)
    if D.dtype != W.dtype:
        raise TypeError("D and W must share a dtype")
    if rows is None:
        rows = np.arange(n, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    D = np.ascontiguousarray(D)
    if D.shape != (len(rows), n):
        raise ValueError("D must hold one full row per listed source")
    P = np.empty((len(rows), n), dtype=np.int32)
    _load().oracle_canonical_pred_rows(D.ctypes.data, n, W.ctypes.data, ldw, code, n,
                                       rows.ctypes.data, len(rows), P.ctypes.data, n,
                                       nthreads)
    return P


def dijkstra_rows(W: np.ndarray, srcs, nthreads: int = 0) -> np.ndarray:
    """float64 distances from each source in ``srcs`` (rows), +inf unreachable."""
    code = _dtype_code(W)
    n, ld = _square_rowmajor(W)
    srcs = np.ascontiguousarray(srcs, dtype=np.int64)
    out = np.empty((len(srcs), n), dtype=np.float64)
    rc = _load().oracle_dijkstra_rows(W.ctypes.data, code, n, ld, srcs.ctypes.data,
                                      len(srcs), out.ctypes.data, n, nthreads)
    if rc != 0:
        raise ValueError("dijkstra_rows needs non-negative edge weights")
    return out
