"""MI355X-native blocked Floyd-Warshall all-pairs shortest paths.

The compute runs in ``libfwapsp.so`` (hand-written HIP kernels for gfx950,
C ABI in ``include/fwapsp.h``); this package is its thin Python binding plus
the seeded input generators (:mod:`.gen`).  The binding loads the library on
first use and raises if it is missing: there is no CPU fallback.
"""
from . import gen  # noqa: F401  (inputs only; no shortest-path arithmetic)

I32_INF = gen.I32_INF

_EXPORTS = {
    "fw_apsp", "fw_apsp_i32", "fw_apsp_pred", "fw_apsp_plan", "fw_apsp_batched",
    "fw_apsp_batched_noalloc",
    "fw_negative_cycle", "fw_negative_cycle_vertices", "fw_negative_cycle_find",
    "fw_apsp_semiring", "fw_apsp_ladder", "LADDER_RUNGS", "fw_transitive_closure",
    "fw_transitive_closure_bits", "pack_bits", "unpack_bits", "words_per_row", "fw_path",
    "plan_tiles", "plan_tile", "plan_set", "plan_reset", "autotune", "autotune_batch",
    "save_plan", "load_plan",
    "batched_max_n", "BatchPlan", "SolvePlan", "Server", "profile_enable", "profile_read",
    "pred_fallbacks",
    "FwError", "lib", "LIB_PATH",
}


def __getattr__(name):
    # the binding imports torch; load it only when a library call is wanted
    if name in _EXPORTS:
        from . import _binding
        return getattr(_binding, name)
    raise AttributeError(name)
