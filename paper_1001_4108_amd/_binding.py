"""ctypes binding of libfwapsp.so (the C ABI in include/fwapsp.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  The library
is loaded on first use and its absence is an error (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch  # imported first so the process uses torch's HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
# FWAPSP_LIB selects another build of the same library (e.g. to compare kernel
# variants); the default is the in-tree build.
LIB_PATH = os.environ.get("FWAPSP_LIB") or os.path.join(HERE, "libfwapsp.so")

I32_INF = 1073741823
FW_F32, FW_I32 = 0, 1
STATUS = {0: "FW_OK", 1: "FW_ERR_INVALID", 2: "FW_ERR_HIP", 3: "FW_ERR_NOMEM",
          4: "FW_ERR_UNSUPPORTED", 5: "FW_ERR_BUSY", 6: "FW_ERR_NOT_FOUND"}

_lib = None
_lock = threading.Lock()


class FwError(RuntimeError):
    """A non-OK status returned by the library."""

    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {lib().fw_status_string(status).decode()}")


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python paper_1001_4108_amd/build.py` "
                "(or __graft_entry__.build()); there is no non-HIP fallback")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


class ServerConfig(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("streams", ctypes.c_int),
                ("budget_bytes", ctypes.c_int64), ("small_n", ctypes.c_int64),
                ("max_batch", ctypes.c_int), ("queue_cap", ctypes.c_int64)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("n", ctypes.c_int64), ("status", ctypes.c_int),
                ("group_size", ctypes.c_int), ("t_submit_ns", ctypes.c_int64),
                ("t_admit_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "submitted", "admitted", "completed", "failed", "rejected", "deferrals",
        "batched_groups", "single_groups", "max_group", "waiting", "bytes_in_use",
        "peak_bytes", "budget_bytes")]


def _declare(L):
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    P64 = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "fw_status_string": ([ci], ctypes.c_char_p),
        "fw_version": ([], ctypes.c_char_p),
        "fw_apsp": ([vp, i64, i64, vp], ci),
        "fw_apsp_i32": ([vp, i64, i64, vp], ci),
        "fw_apsp_pred": ([vp, ci, i64, i64, vp, i64, vp], ci),
        "fw_apsp_plan": ([vp, ci, i64, i64, vp, i64, ci, vp], ci),
        "fw_plan_tiles": ([ctypes.POINTER(ci), ci], ci),
        "fw_apsp_semiring": ([vp, ci, ci, i64, i64, vp], ci),
        "fw_apsp_ladder": ([vp, ci, i64, i64, ci, vp], ci),
        "fw_transitive_closure_bits": ([vp, i64, i64, ci, vp], ci),
        "fw_pack_bits": ([vp, i64, i64, vp, i64, vp], ci),
        "fw_unpack_bits": ([vp, i64, i64, vp, i64, vp], ci),
        "fw_plan_tile": ([ci, i64], ci),
        "fw_plan_set": ([ci, i64, i64, ci], ci),
        "fw_plan_reset": ([], None),
        "fw_autotune": ([ci, P64, P64, ci, ci, ci, ci, ctypes.POINTER(ci),
                         ctypes.POINTER(ctypes.c_double)], ci),
        "fw_autotune_batch": ([ci, P64, i64, P64, P64, ci, ci, ci, ci, ctypes.POINTER(ci),
                               ctypes.POINTER(ctypes.c_double)], ci),
        "fw_apsp_batched": ([ctypes.POINTER(vp), P64, P64, i64, ci, ctypes.POINTER(vp), P64, vp],
                            ci),
        "fw_batched_max_n": ([ci, ci], i64),
        "fw_apsp_batched_noalloc": ([ctypes.POINTER(vp), P64, P64, i64, ci, ctypes.POINTER(vp),
                                     P64, vp], ci),
        "fw_batched_noalloc_max_bytes": ([], i64),
        "fw_batch_plan_create": ([ctypes.POINTER(vp), P64, P64, i64, ci, ctypes.POINTER(vp), P64,
                                  ctypes.POINTER(vp)], ci),
        "fw_batch_plan_launch": ([vp, ci, vp], ci),
        "fw_batch_plan_destroy": ([vp], ci),
        "fw_batch_plan_grid": ([vp], i64),
        "fw_negative_cycle": ([vp, ci, i64, i64, vp, vp], ci),
        "fw_negative_cycle_vertices": ([vp, ci, i64, i64, vp, vp, vp], ci),
        "fw_pred_fallbacks": ([], i64),
        "fw_negative_cycle_find": ([vp, ci, i64, i64, vp, i64, i64, P64, i64,
                                    ctypes.POINTER(ci)], i64),
        "fw_solve_plan_create": ([vp, ci, i64, i64, vp, i64, ci, ctypes.POINTER(vp)], ci),
        "fw_solve_plan_launch": ([vp, ci, vp], ci),
        "fw_solve_plan_tile": ([vp], ci),
        "fw_solve_plan_destroy": ([vp], ci),
        "fw_server_create": ([ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)], ci),
        "fw_server_submit": ([vp, vp, i64, i64, vp, i64, ci, P64], ci),
        "fw_server_poll": ([vp, ctypes.POINTER(Completion), ci, i64], ci),
        "fw_server_fetch": ([vp, i64, vp, i64, vp], ci),
        "fw_server_release": ([vp, i64], ci),
        "fw_server_drain": ([vp, i64], ci),
        "fw_server_get_stats": ([vp, ctypes.POINTER(ServerStats)], ci),
        "fw_server_destroy": ([vp], ci),
        "fw_path": ([vp, i64, i64, i64, i64, P64, i64], i64),
        "fw_profile_enable": ([ci], ci),
        "fw_profile_read": ([ctypes.POINTER(ctypes.c_double), P64, ci], ci),
        "fw_profile_updates": ([ctypes.POINTER(ctypes.c_double), ci], ci),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res


def _check(status: int, where: str):
    if status != 0:
        raise FwError(status, where)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return FW_F32
    if t.dtype == torch.int32:
        return FW_I32
    raise TypeError(f"distance matrices are float32 or int32, got {t.dtype}")


def _matrix(t: torch.Tensor, name: str):
    """(pointer, n, ld) of a square row-major device matrix view."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise ValueError(f"{name} must be square, got {tuple(t.shape)}")
    n = t.shape[0]
    if n > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} needs unit column stride (row-major)")
    ld = t.stride(0) if n > 0 else 0
    if n > 0 and ld < n:
        raise ValueError(f"{name} rows overlap (stride {ld} < n {n})")
    return t.data_ptr(), n, max(ld, n)


def _stream(t: torch.Tensor, stream):
    if stream is None:
        stream = torch.cuda.current_stream(t.device)
    return ctypes.c_void_p(stream.cuda_stream)


def _empty_on(stream, device, *shape, dtype=torch.int32):
    """A new device tensor for work enqueued on ``stream``: allocated while
    that stream is current, so the caching allocator ties the block to it and
    does not hand it out again before the stream's work on it is done."""
    if stream is None:
        return torch.empty(shape, dtype=dtype, device=device)
    with torch.cuda.stream(stream):
        return torch.empty(shape, dtype=dtype, device=device)


def fw_apsp(d: torch.Tensor, stream=None) -> torch.Tensor:
    """All-pairs shortest paths in place on a float32 device matrix view."""
    if d.dtype != torch.float32:
        raise TypeError("fw_apsp takes float32; use fw_apsp_i32 for int32")
    p, n, ld = _matrix(d, "d")
    with torch.cuda.device(d.device):
        _check(lib().fw_apsp(p, n, ld, _stream(d, stream)), "fw_apsp")
    return d


def fw_apsp_i32(d: torch.Tensor, stream=None) -> torch.Tensor:
    """All-pairs shortest paths in place on an int32 device matrix view."""
    if d.dtype != torch.int32:
        raise TypeError("fw_apsp_i32 takes int32")
    p, n, ld = _matrix(d, "d")
    with torch.cuda.device(d.device):
        _check(lib().fw_apsp_i32(p, n, ld, _stream(d, stream)), "fw_apsp_i32")
    return d


def _pred_args(d, pred):
    if pred is None:
        return None, 0
    if pred.dtype != torch.int32 or pred.device != d.device:
        raise ValueError("pred must be an int32 tensor on d's device")
    pp, pn, pld = _matrix(pred, "pred")
    if pn != d.shape[0]:
        raise ValueError("pred must have d's shape")
    return pp, pld


def fw_apsp_pred(d: torch.Tensor, pred: torch.Tensor | None = None, stream=None):
    """Distances in place plus, when ``pred`` is given, the canonical predecessors."""
    code = _dtype_code(d)
    p, n, ld = _matrix(d, "d")
    pp, pld = _pred_args(d, pred)
    with torch.cuda.device(d.device):
        _check(lib().fw_apsp_pred(p, code, n, ld, pp, pld, _stream(d, stream)), "fw_apsp_pred")
    return d, pred


def fw_apsp_plan(d: torch.Tensor, tile: int, pred: torch.Tensor | None = None, stream=None):
    """fw_apsp_pred with an explicit tile size (one of :func:`plan_tiles`)."""
    code = _dtype_code(d)
    p, n, ld = _matrix(d, "d")
    pp, pld = _pred_args(d, pred)
    with torch.cuda.device(d.device):
        _check(lib().fw_apsp_plan(p, code, n, ld, pp, pld, int(tile), _stream(d, stream)),
               "fw_apsp_plan")
    return d, pred


SEMIRINGS = {"minplus": 0, "maxmin": 1}


def fw_apsp_semiring(d: torch.Tensor, semiring: str = "maxmin", stream=None) -> torch.Tensor:
    """In-place closure of ``d`` over "minplus" (shortest paths) or "maxmin"
    (widest paths; transitive closure over int32 {0, 1})."""
    code = _dtype_code(d)
    p, n, ld = _matrix(d, "d")
    with torch.cuda.device(d.device):
        _check(lib().fw_apsp_semiring(p, code, SEMIRINGS[semiring], n, ld, _stream(d, stream)),
               "fw_apsp_semiring")
    return d


LADDER_RUNGS = {
    0: "one launch per k, one thread per cell",
    1: "blocked, 32x32 tiles in LDS, one cell per thread",
    2: "blocked, 64x64 tiles, 4x4 register sub-tiles, whole tiles in LDS",
    3: "blocked, 64x64 tiles, 4x4 register sub-tiles, staged 16-deep LDS slices",
    4: "tile 128, direct global->LDS copies, 8x8 register sub-tiles (the large-n path)",
}


def fw_apsp_ladder(d: torch.Tensor, rung: int, stream=None) -> torch.Tensor:
    """In-place shortest paths by one rung of the ablation ladder (see
    ``LADDER_RUNGS``); every rung gives the same bits as ``fw_apsp``."""
    code = _dtype_code(d)
    p, n, ld = _matrix(d, "d")
    with torch.cuda.device(d.device):
        _check(lib().fw_apsp_ladder(p, code, n, ld, int(rung), _stream(d, stream)),
               "fw_apsp_ladder")
    return d


def words_per_row(n: int) -> int:
    """32-bit words per row of the bit-packed adjacency layout."""
    return (int(n) + 31) // 32


def _bits(bits: torch.Tensor, n: int, name: str):
    """(pointer, ldw) of an n x >= ceil(n/32) int32 device tensor holding the
    packed words (int32 is uint32 reinterpreted)."""
    if not isinstance(bits, torch.Tensor) or not bits.is_cuda or bits.dtype != torch.int32:
        raise ValueError(f"{name} must be an int32 device tensor of packed words")
    if bits.dim() != 2 or bits.shape[0] != n or bits.shape[1] < words_per_row(n):
        raise ValueError(f"{name} must be {n} x >= {words_per_row(n)} words")
    if n > 1 and bits.stride(1) != 1:
        raise ValueError(f"{name} needs unit column stride")
    return bits.data_ptr(), max(bits.stride(0), words_per_row(n)) if n else 0


def pack_bits(adj: torch.Tensor, stream=None) -> torch.Tensor:
    """Bit-packed copy (n x ceil(n/32) int32 words) of an int32 matrix whose
    non-zero entries are edges."""
    if adj.dtype != torch.int32:
        raise TypeError("pack_bits takes an int32 0/1 matrix")
    p, n, ld = _matrix(adj, "adj")
    out = _empty_on(stream, adj.device, n, words_per_row(n))
    with torch.cuda.device(adj.device):
        _check(lib().fw_pack_bits(p, n, ld, out.data_ptr(), words_per_row(n),
                                  _stream(adj, stream)), "fw_pack_bits")
    return out


def unpack_bits(bits: torch.Tensor, n: int, out: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
    """The n x n int32 0/1 matrix of a bit-packed one (into ``out`` if given)."""
    bp, ldw = _bits(bits, n, "bits")
    if out is None:
        out = _empty_on(stream, bits.device, n, n)
    if out.dtype != torch.int32:
        raise TypeError("unpack_bits writes an int32 matrix")
    p, m, ld = _matrix(out, "out")
    if m != n:
        raise ValueError("out must be n x n")
    with torch.cuda.device(bits.device):
        _check(lib().fw_unpack_bits(bp, n, ldw, p, ld, _stream(bits, stream)), "fw_unpack_bits")
    return out


def fw_transitive_closure_bits(bits: torch.Tensor, n: int, reflexive: bool = True,
                               stream=None) -> torch.Tensor:
    """Reachability in place on a bit-packed adjacency matrix (see pack_bits)."""
    bp, ldw = _bits(bits, n, "bits")
    with torch.cuda.device(bits.device):
        _check(lib().fw_transitive_closure_bits(bp, int(n), ldw, 1 if reflexive else 0,
                                                _stream(bits, stream)),
               "fw_transitive_closure_bits")
    return bits


def fw_transitive_closure(adj: torch.Tensor, stream=None) -> torch.Tensor:
    """Reachability in place on an int32 0/1 adjacency matrix (non-zero =
    edge; every vertex reaches itself): packed to bits, closed by the
    bit-packed kernels, unpacked into ``adj``."""
    if adj.dtype != torch.int32:
        raise TypeError("transitive closure takes an int32 0/1 matrix")
    n = adj.shape[0]
    # the packed temporary is allocated on `stream` (see _empty_on): freed on
    # return, its block is reused only by later work of that stream
    bits = pack_bits(adj, stream)
    fw_transitive_closure_bits(bits, n, True, stream)
    return unpack_bits(bits, n, adj, stream)


def plan_tiles() -> list[int]:
    buf = (ctypes.c_int * 16)()
    k = lib().fw_plan_tiles(buf, 16)
    return [buf[i] for i in range(k)]


FW_PLAN_PRED = 2


def _plan_key(dtype, pred: bool) -> int:
    code = FW_F32 if dtype in (torch.float32, "f32", FW_F32) else FW_I32
    return code | (FW_PLAN_PRED if pred else 0)


def plan_tile(dtype, n: int, pred: bool = False) -> int:
    """Tile of the plan table for (dtype, n); ``pred``: the table of solves
    that also compute predecessors."""
    return int(lib().fw_plan_tile(_plan_key(dtype, pred), int(n)))


def plan_set(dtype, n_lo: int, n_hi: int, tile: int, pred: bool = False) -> None:
    _check(lib().fw_plan_set(_plan_key(dtype, pred), int(n_lo), int(n_hi), int(tile)),
           "fw_plan_set")


def plan_reset() -> None:
    lib().fw_plan_reset()


def autotune(dtype, buckets, objective: str = "single", batch: int = 256, reps: int = 3,
             device=None, pred: bool = False) -> dict:
    """Time every tile per size bucket on the device and install the fastest.

    ``buckets`` is a list of (lo, hi) sizes; ``objective`` is "single" (one
    solve) or "batched" (one persistent launch of ``batch`` graphs); with
    ``pred`` the solves compute predecessors and that table is tuned.
    Returns {(lo, hi): {"tile": t, "ms": {tile: median_ms}}}.
    """
    code = _plan_key(dtype, pred)
    k = len(buckets)
    lo = (ctypes.c_int64 * k)(*[int(b[0]) for b in buckets])
    hi = (ctypes.c_int64 * k)(*[int(b[1]) for b in buckets])
    tiles = plan_tiles()
    out = (ctypes.c_int * k)()
    ms = (ctypes.c_double * (k * len(tiles)))()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    with torch.cuda.device(dev):
        _check(lib().fw_autotune(code, lo, hi, k, 1 if objective == "batched" else 0, int(batch),
                                 int(reps), out, ms), "fw_autotune")
    return {(int(buckets[i][0]), int(buckets[i][1])):
            {"tile": out[i], "ms": {t: ms[i * len(tiles) + j] for j, t in enumerate(tiles)}}
            for i in range(k)}


def autotune_batch(dtype, sizes, buckets, mode: str = "graph", reps: int = 5, passes: int = 2,
                   device=None, pred: bool = False) -> dict:
    """Tune the plan table for one batch as a whole (``fw_autotune_batch``).

    ``sizes`` are the batch's graph sizes, ``buckets`` a list of (lo, hi),
    ``mode`` the launch mode to tune for ("graph" or "kernel", as
    ``BatchPlan.launch``); each pass times every tile of every bucket that
    holds some of the graphs on the whole batch plan, the other buckets
    fixed, and installs the fastest.  Returns {(lo, hi): {"tile": t, "ms": {tile: median_ms}}} (the
    last pass's times; empty for buckets the batch does not use).
    """
    code = _plan_key(dtype, pred)
    k = len(buckets)
    ns = (ctypes.c_int64 * max(len(sizes), 1))(*[int(v) for v in sizes])
    lo = (ctypes.c_int64 * k)(*[int(b[0]) for b in buckets])
    hi = (ctypes.c_int64 * k)(*[int(b[1]) for b in buckets])
    tiles = plan_tiles()
    out = (ctypes.c_int * k)()
    ms = (ctypes.c_double * (k * len(tiles)))()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    with torch.cuda.device(dev):
        if mode not in ("graph", "kernel"):
            raise ValueError("mode is 'graph' or 'kernel'")
        _check(lib().fw_autotune_batch(code, ns, len(sizes), lo, hi, k,
                                       1 if mode == "graph" else 0, int(reps), int(passes), out,
                                       ms), "fw_autotune_batch")
    return {(int(buckets[i][0]), int(buckets[i][1])):
            {"tile": out[i], "ms": {t: ms[i * len(tiles) + j] for j, t in enumerate(tiles)
                                    if ms[i * len(tiles) + j] > 0}}
            for i in range(k)}


def save_plan(result: dict, path: str, dtype="f32", objective="single", pred: bool = False) -> None:
    """Persist an autotune result as JSON."""
    import json
    rows = [{"lo": lo, "hi": hi, "tile": v["tile"], "ms": {str(t): m for t, m in v["ms"].items()}}
            for (lo, hi), v in result.items()]
    with open(path, "w") as f:
        json.dump({"dtype": str(dtype), "pred": bool(pred), "objective": objective,
                   "buckets": rows}, f, indent=1)


def load_plan(path: str) -> None:
    """Install a saved autotune result into the plan table."""
    import json
    spec = json.load(open(path))
    dt = "i32" if "int32" in spec["dtype"] or spec["dtype"] == "i32" else "f32"
    for row in spec["buckets"]:
        plan_set(dt, row["lo"], row["hi"], row["tile"], pred=bool(spec.get("pred", False)))


def fw_apsp_batched(mats, preds=None, stream=None) -> None:
    """Solve a list of independent square device matrices (one dtype) together."""
    if len(mats) == 0:
        return
    code, dev, ptrs, ns, lds, pptr, pld = _batch_arrays(mats, preds)
    with torch.cuda.device(dev):
        _check(lib().fw_apsp_batched(ptrs, ns, lds, len(mats), code, pptr, pld,
                                     _stream(mats[0], stream)), "fw_apsp_batched")


def fw_apsp_batched_noalloc(mats, preds=None, stream=None) -> None:
    """fw_apsp_batched with the plan's tables in the library's static device
    array: no device allocation; synchronises ``stream`` after the upload."""
    if len(mats) == 0:
        return
    code, dev, ptrs, ns, lds, pptr, pld = _batch_arrays(mats, preds)
    with torch.cuda.device(dev):
        _check(lib().fw_apsp_batched_noalloc(ptrs, ns, lds, len(mats), code, pptr, pld,
                                             _stream(mats[0], stream)),
               "fw_apsp_batched_noalloc")


def _batch_arrays(mats, preds):
    count = len(mats)
    code = _dtype_code(mats[0])
    dev = mats[0].device
    ptrs = (ctypes.c_void_p * count)()
    ns = (ctypes.c_int64 * count)()
    lds = (ctypes.c_int64 * count)()
    for g, m in enumerate(mats):
        if m.dtype != mats[0].dtype or m.device != dev:
            raise ValueError("batched matrices must share dtype and device")
        p, n, ld = _matrix(m, f"mats[{g}]")
        ptrs[g], ns[g], lds[g] = p, n, ld
    pptr = pld = None
    if preds is not None:
        if len(preds) != count:
            raise ValueError("preds must match mats")
        pptr = (ctypes.c_void_p * count)()
        pld = (ctypes.c_int64 * count)()
        for g, (m, q) in enumerate(zip(mats, preds)):
            if q is None:
                pptr[g], pld[g] = None, 0
            else:
                pptr[g], pld[g] = _pred_args(m, q)
    return code, dev, ptrs, ns, lds, pptr, pld


class BatchPlan:
    """A reusable batch (fw_batch_plan_*): the descriptor table is built once;
    ``launch("graph")`` replays one captured hipGraph per call.  The
    matrices are solved in place on every launch and must outlive the plan."""

    def __init__(self, mats, preds=None):
        if not mats:
            raise ValueError("empty batch")
        code, dev, ptrs, ns, lds, pptr, pld = _batch_arrays(mats, preds)
        self.device = dev
        self._mats = list(mats)
        self._preds = list(preds) if preds is not None else None
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            _check(lib().fw_batch_plan_create(ptrs, ns, lds, len(mats), code, pptr, pld,
                                              ctypes.byref(h)), "fw_batch_plan_create")
        self._h = h

    @property
    def grid(self) -> int:
        return int(lib().fw_batch_plan_grid(self._h))

    MODES = {"kernel": 0, "graph": 1, "per_graph": 2}

    def launch(self, mode: str = "graph", stream=None) -> None:
        """mode: "graph" (captured persistent launch), "kernel" (eager
        persistent launch) or "per_graph" (single-graph launches, baseline)."""
        if self._h is None:
            raise RuntimeError("plan destroyed")
        with torch.cuda.device(self.device):
            _check(lib().fw_batch_plan_launch(self._h, self.MODES[mode],
                                              _stream(self._mats[0], stream)),
                   "fw_batch_plan_launch")

    def destroy(self) -> None:
        if self._h is not None:
            with torch.cuda.device(self.device):
                lib().fw_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class SolvePlan:
    """One matrix's solve (fw_solve_plan_*): ``launch("graph")`` replays the
    stage loop captured once into a hipGraph, ``launch("eager")`` enqueues the
    same launches one by one.  The matrices are solved in place on every
    launch and must outlive the plan."""

    MODES = {"eager": 0, "graph": 1}

    def __init__(self, d: torch.Tensor, pred: torch.Tensor | None = None, tile: int = 0):
        code = _dtype_code(d)
        p, n, ld = _matrix(d, "d")
        pp, pld = _pred_args(d, pred)
        self.device = d.device
        self._d, self._pred = d, pred
        h = ctypes.c_void_p()
        with torch.cuda.device(d.device):
            _check(lib().fw_solve_plan_create(p, code, n, ld, pp, pld, int(tile),
                                              ctypes.byref(h)), "fw_solve_plan_create")
        self._h = h

    @property
    def tile(self) -> int:
        return int(lib().fw_solve_plan_tile(self._h))

    def launch(self, mode: str = "graph", stream=None) -> None:
        if self._h is None:
            raise RuntimeError("plan destroyed")
        with torch.cuda.device(self.device):
            _check(lib().fw_solve_plan_launch(self._h, self.MODES[mode], _stream(self._d, stream)),
                   "fw_solve_plan_launch")

    def destroy(self) -> None:
        if self._h is not None:
            with torch.cuda.device(self.device):
                lib().fw_solve_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def batched_max_n(dtype, with_pred: bool = False) -> int:
    code = FW_F32 if dtype in (torch.float32, "f32", FW_F32) else FW_I32
    return int(lib().fw_batched_max_n(code, int(bool(with_pred))))


def fw_negative_cycle(d: torch.Tensor, stream=None) -> bool:
    """True when some d_ii < 0 after a solve (a negative cycle).  Synchronises."""
    code = _dtype_code(d)
    p, n, ld = _matrix(d, "d")
    flag = _empty_on(stream, d.device, 1)
    with torch.cuda.device(d.device):
        s = _stream(d, stream)
        _check(lib().fw_negative_cycle(p, code, n, ld, flag.data_ptr(), s), "fw_negative_cycle")
    (stream if stream is not None else torch.cuda.current_stream(d.device)).synchronize()
    return bool(flag.item())


def fw_negative_cycle_vertices(d: torch.Tensor, stream=None) -> list[int]:
    """Vertices i with d_ii < 0 after a solve, ascending (device scan).  Synchronises."""
    code = _dtype_code(d)
    p, n, ld = _matrix(d, "d")
    out = _empty_on(stream, d.device, max(n, 1) + 1)
    with torch.cuda.device(d.device):
        s = _stream(d, stream)
        _check(lib().fw_negative_cycle_vertices(p, code, n, ld, out[1:].data_ptr(),
                                                out.data_ptr(), s),
               "fw_negative_cycle_vertices")
    (stream if stream is not None else torch.cuda.current_stream(d.device)).synchronize()
    host = out.cpu().tolist()
    return host[1:1 + host[0]]


def fw_negative_cycle_find(w_host, v: int, pred_host=None):
    """One negative cycle through the walk from ``v`` (a vertex with d_vv < 0),
    from the original host weights ``w_host`` and optionally the solve's host
    predecessor matrix: ``(cycle, from_pred)`` with cycle = [c_0, ..., c_{m-1}]
    (edges c_t -> c_t+1 and c_{m-1} -> c_0), or ``([], False)`` if none."""
    import numpy as np
    W = np.ascontiguousarray(w_host)
    code = FW_F32 if W.dtype == np.float32 else FW_I32 if W.dtype == np.int32 else None
    if code is None:
        raise TypeError("weights are float32 or int32")
    n = W.shape[0]
    pp, pld = None, 0
    if pred_host is not None:
        P = np.ascontiguousarray(pred_host, dtype=np.int32)
        pp, pld = P.ctypes.data, P.strides[0] // 4
    buf = (ctypes.c_int64 * max(n, 1))()
    fp = ctypes.c_int(0)
    m = lib().fw_negative_cycle_find(W.ctypes.data, code, n, W.strides[0] // W.itemsize, pp,
                                     pld, int(v), buf, max(n, 1), ctypes.byref(fp))
    if m < 0:
        raise FwError(1, "fw_negative_cycle_find")
    return [buf[t] for t in range(m)], bool(fp.value)


def fw_path(pred_host, i: int, j: int) -> list[int]:
    """Shortest path i -> j from a host predecessor matrix ([] if unreachable)."""
    import numpy as np
    P = np.ascontiguousarray(pred_host, dtype=np.int32)
    n = P.shape[0]
    buf = (ctypes.c_int64 * max(n, 1))()
    k = lib().fw_path(P.ctypes.data, n, P.strides[0] // 4, int(i), int(j), buf, max(n, 1))
    if k < 0:
        raise FwError(1, "fw_path")
    return [buf[t] for t in range(k)]


def profile_enable(on: bool = True) -> None:
    lib().fw_profile_enable(1 if on else 0)


KINDS = ("diag", "panel", "bulk", "pred", "batched", "bits_diag", "bits_panel", "bits_bulk",
         "pred_fallback")


def pred_fallbacks() -> int:
    """Number of solves with predecessors on the current device whose 32-bit
    keyed sweep gave up and ran the pair-form sweep (synchronises)."""
    v = lib().fw_pred_fallbacks()
    if v < 0:
        raise FwError(2, "fw_pred_fallbacks")
    return int(v)


def profile_read():
    """{kind: (ms, launches, updates)} accumulated since the last read."""
    cap = len(KINDS)
    ms = (ctypes.c_double * cap)()
    cnt = (ctypes.c_int64 * cap)()
    k = lib().fw_profile_read(ms, cnt, cap)
    if k < 0:
        raise FwError(-k, "fw_profile_read")
    upd = (ctypes.c_double * cap)()
    lib().fw_profile_updates(upd, cap)
    return {KINDS[i]: (ms[i], cnt[i], upd[i]) for i in range(k)}


class Server:
    """Continuous-batching APSP server (fw_server_*): footprint admission into a
    device budget, persistent batched launches for small requests, single-graph
    stage loops for large ones, overlapped on several worker streams."""

    def __init__(self, dtype=torch.float32, budget_bytes: int = 8 << 30, streams: int = 4,
                 small_n: int = 512, max_batch: int = 1024, queue_cap: int = 1 << 20,
                 device=None):
        self.dtype = dtype
        self.device = torch.device(device) if device is not None else \
            torch.device("cuda", torch.cuda.current_device())
        code = FW_F32 if dtype == torch.float32 else FW_I32
        cfg = ServerConfig(code, streams, int(budget_bytes), int(small_n), int(max_batch),
                           int(queue_cap))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().fw_server_create(ctypes.byref(cfg), ctypes.byref(h)), "fw_server_create")
        self._h = h
        self._buf = (Completion * 4096)()

    def submit(self, src: torch.Tensor, keep: bool = False, dst_host=None) -> int:
        """Queue APSP on the square matrix view ``src`` (device or host)."""
        if src.dtype != self.dtype:
            raise TypeError("request dtype differs from the server's")
        if src.dim() != 2 or src.shape[0] != src.shape[1]:
            raise ValueError("square matrix expected")
        n = src.shape[0]
        if n > 1 and src.stride(1) != 1:
            raise ValueError("row-major matrix expected")
        ld = max(src.stride(0), n) if n else 0
        dptr, dld = None, 0
        if dst_host is not None:
            dptr, dld = dst_host.data_ptr(), max(dst_host.stride(0), n)
        rid = ctypes.c_int64()
        _check(lib().fw_server_submit(self._h, src.data_ptr() if n else None, n, ld, dptr, dld,
                                      1 if keep else 0, ctypes.byref(rid)), "fw_server_submit")
        return rid.value

    def poll(self, timeout_us: int = 0):
        k = lib().fw_server_poll(self._h, self._buf, len(self._buf), int(timeout_us))
        if k < 0:
            raise FwError(-k, "fw_server_poll")
        return [(c.id, c.n, c.status, c.group_size, c.t_submit_ns, c.t_admit_ns, c.t_done_ns)
                for c in self._buf[:k]]

    def fetch(self, rid: int, dst: torch.Tensor, stream=None) -> torch.Tensor:
        with torch.cuda.device(self.device):
            _check(lib().fw_server_fetch(self._h, int(rid), dst.data_ptr(),
                                         max(dst.stride(0), dst.shape[0]),
                                         _stream(dst, stream) if dst.is_cuda else None),
                   "fw_server_fetch")
        return dst

    def release(self, rid: int) -> None:
        _check(lib().fw_server_release(self._h, int(rid)), "fw_server_release")

    def drain(self, timeout_s: float = -1.0) -> None:
        us = -1 if timeout_s < 0 else int(timeout_s * 1e6)
        _check(lib().fw_server_drain(self._h, us), "fw_server_drain")

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().fw_server_get_stats(self._h, ctypes.byref(st)), "fw_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self) -> None:
        if self._h is not None:
            lib().fw_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
