// C ABI and host driver of libfwapsp (declared in include/fwapsp.h).
//
// The host side runs the stage loop of the blocked algorithm (section 3.2,
// Fig. BFW-Alg): for every k-block b, stream-ordered launches of the diagonal
// tile, the panels and the bulk -- where the bulk kernel can, it also closes
// the next stage's diagonal tile, and stages after the first are two launches.
// It validates every argument before enqueueing anything, picks the tile size
// from a plan table keyed by (dtype, with predecessors or not, n), and can
// bracket each launch with HIP events for per-phase timing.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/fwapsp.h"
#include "fw_internal.h"

namespace fw {
namespace {

// ---------------------------------------------------------------------------
// Plan table: tile size per (dtype, size bucket).
// ---------------------------------------------------------------------------
struct PlanEntry {
    int64_t n_lo, n_hi;
    int tile;
};

const int kTiles[] = {32, 64, 128};

std::mutex g_plan_mu;
// one table per plan key: dtype, | FW_PLAN_PRED for solves with predecessors
std::vector<PlanEntry> g_plan[4];

void default_plan_locked() {
    for (int key = 0; key < 4; ++key) {
        std::vector<PlanEntry> &t = g_plan[key];
        t.clear();
        // n <= tile: one closure over the whole graph (the plain algorithm)
        t.push_back({0, 32, 32});
        t.push_back({33, 64, 64});
        t.push_back({65, 128, 128});
        // blocked (measured with fw_apsp_plan / fw_autotune on one MI355X):
        // below ~4.6k (fp32) / ~4.1k (int32) vertices a stage's 128-wide bulk
        // fills the GPU too few times and the 128-step diagonal closure
        // weighs more, and tile 64 solves faster (n=1024: 1.7x, n=4096:
        // 1.15x); above, tile 128's lower traffic per update wins (n=12288:
        // 1.4x).  With the (distance, last hop) pair forms tile 128 never won
        // (int32 with 64-bit keys at n=8192: 69 vs 82 ms at tile 64), and
        // tile 32 wins below ~2k (fp32) / ~1k (int32) vertices (fp32 n~1448:
        // 4.0 vs 4.6 ms; int32 n~724: 0.78 vs 0.83).  These entries pick the
        // pair forms' tile: batched solves with predecessors, and the gated
        // sweep behind the keyed one of a single solve, whose own tile is the
        // distances-only entry's (it runs those kernels).  Above 4k int32
        // vertices the gated 64-bit sweep takes tile 128: when it runs it is
        // slower than at 64 (82 vs 69 ms at n=8192), but it has half the
        // launches to skip when its gate stays closed, the usual case.
        if (key & FW_PLAN_PRED) {
            const bool i32 = (key & 1) == FW_I32;
            const int64_t hi32 = i32 ? 1024 : 2048;
            t.push_back({129, hi32, 32});
            if (i32) {
                t.push_back({hi32 + 1, 4096, 64});
                t.push_back({4097, INT64_MAX, 128});
            } else {
                t.push_back({hi32 + 1, INT64_MAX, 64});
            }
        } else {
            const int64_t hi64 = (key & 1) == FW_F32 ? 4608 : 4096;
            t.push_back({129, hi64, 64});
            t.push_back({hi64 + 1, INT64_MAX, 128});
        }
    }
}

int plan_tile(int key, int64_t n) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (g_plan[0].empty()) default_plan_locked();
    // the most recently installed entry covering n wins
    for (auto it = g_plan[key].rbegin(); it != g_plan[key].rend(); ++it)
        if (n >= it->n_lo && n <= it->n_hi) return it->tile;
    return 128;
}

int plan_key(int dtype, const int32_t *pred) { return dtype | (pred ? FW_PLAN_PRED : 0); }

bool plan_key_ok(int key) {
    const int dt = key & ~FW_PLAN_PRED;
    return dt == FW_F32 || dt == FW_I32;
}

bool tile_supported(int tile) {
    for (int t : kTiles)
        if (t == tile) return true;
    return false;
}

// ---------------------------------------------------------------------------
// Phase timing.
// ---------------------------------------------------------------------------
struct TimedLaunch {
    int kind;
    hipEvent_t start, stop;
    double updates;
};

std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<TimedLaunch> g_prof_pending;
std::vector<hipEvent_t> g_event_pool;
double g_last_updates[kNumKinds];

hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs `launch` (a callable returning hipError_t), timed when profiling is on.
template <typename F>
hipError_t timed(int kind, double updates, hipStream_t st, F &&launch) {
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        on = g_prof_on;
    }
    if (!on) return launch();
    hipEvent_t a, b;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        a = take_event();
        b = take_event();
    }
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, st);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, st);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back({kind, a, b, updates});
    return hipSuccess;
}

int status_of(hipError_t e) {
    if (e == hipSuccess) return FW_OK;
    if (e == hipErrorOutOfMemory) return FW_ERR_NOMEM;
    return FW_ERR_HIP;
}

bool mul_overflows(int64_t a, int64_t b) {
    if (a <= 0 || b <= 0) return false;
    return a > INT64_MAX / b;
}

int validate(const void *d, int dtype, int64_t n, int64_t ld, const int32_t *pred,
             int64_t ldp) {
    if (dtype != FW_F32 && dtype != FW_I32) return FW_ERR_INVALID;
    if (n < 0 || n > 0x7fffffffLL) return FW_ERR_INVALID;
    if (ld < n || ld < 0) return FW_ERR_INVALID;
    if (n > 0 && d == nullptr) return FW_ERR_INVALID;
    if (mul_overflows(n, ld)) return FW_ERR_INVALID;
    if (pred) {
        if (ldp < n || mul_overflows(n, ldp)) return FW_ERR_INVALID;
    }
    return FW_OK;
}

// Enqueue the whole blocked solve of one graph on `st`.  Arguments already
// validated; n > 1.  Per stage: the panels and the bulk; the diagonal tile has
// its own launch only where the previous bulk launch did not close it.
// `capturing`: the launches are being recorded into a hipGraph, so no phase
// events are recorded around them (an event recorded during a capture belongs
// to that capture and is not reused outside it).  `flag`: the keyed sweep's
// range flag (sr == kKey).  `gate`: every launch runs only if *gate != 0 (the
// 64-bit predecessor sweep behind a keyed one; timed as kPredFallback).
int enqueue_solve(void *d, int dtype, int n, int64_t ld, int32_t *pred, int64_t ldp, int tile,
                  hipStream_t st, bool capturing, int sr = kMinPlus, int32_t *flag = nullptr,
                  const int32_t *gate = nullptr) {
    const int nb = (n + tile - 1) / tile;
    hipError_t e;
    auto run = [&](int kind, double upd, auto &&launch) -> hipError_t {
        if (capturing) return launch();
        if (gate) return timed(kPredFallback, 0.0, st, launch);
        return timed(kind, upd, st, launch);
    };
    if (pred) {
        e = run(kPredFix, 0.0,
                [&] { return launch_pred_init(dtype, d, pred, n, ld, ldp, st, gate); });
        if (e != hipSuccess) return status_of(e);
    }
    // algorithmic updates of each launch: the n^3 tasks split by where the
    // (i, j) cell lies relative to block b (real cells only, padding excluded)
    const double nn = (double)n;
    auto real = [&](int blk) { return std::max(0.0, std::min<double>(tile, nn - (double)blk * tile)); };
    bool closed = false;  // the previous bulk launch closed this stage's diagonal tile
    for (int b = 0; b < nb; ++b) {
        const double kb = real(b);
        if (!closed) {
            e = run(kDiag, kb * kb * kb, [&] {
                return launch_diag(dtype, sr, tile, d, pred, n, ld, ldp, b, st, flag, gate);
            });
            if (e != hipSuccess) return status_of(e);
        }
        closed = false;
        if (nb == 1) break;
        e = run(kPanel, 2.0 * kb * kb * (nn - kb), [&] {
            return launch_panels(dtype, sr, tile, d, pred, n, ld, ldp, b, nb, st, flag, gate);
        });
        if (e != hipSuccess) return status_of(e);
        // close_next: the bulk launch also closes the next diagonal tile (its
        // updates are counted with the bulk's, the launch that does them)
        const bool close_next = bulk_closes_next_diag(sr, tile, d, pred, n, ld, b);
        const double r1 = real(b + 1), rest = nn - kb;
        const double upd = kb * rest * rest + (close_next ? r1 * r1 * r1 : 0.0);
        e = run(kBulk, upd, [&] {
            return launch_bulk(dtype, sr, tile, d, pred, n, ld, ldp, b, nb, close_next, st, flag,
                               gate);
        });
        if (e != hipSuccess) return status_of(e);
        closed = close_next;
    }
    if (pred) {
        e = run(kPredFix, 0.0,
                [&] { return launch_pred_fix(dtype, d, pred, n, ld, ldp, st, gate); });
        if (e != hipSuccess) return status_of(e);
    }
    return FW_OK;
}

// The last hops of the fp32 canonical path (fw_internal.h), strip by strip
// from the final distances in d and the weights saved in P, every launch
// gated on `gate`.
int enqueue_canon_hops(const float *d, int n, int64_t ld, int32_t *pred, int64_t ldp,
                       float *strip, const int32_t *gate, hipStream_t st, bool capturing) {
    auto run = [&](auto &&launch) -> hipError_t {
        if (capturing) return launch();
        return timed(kPredFallback, 0.0, st, launch);
    };
    hipError_t e = hipSuccess;
    const int w = canon_strip_cols(n);
    for (int j0 = 0; j0 < n && e == hipSuccess; j0 += w) {
        const int wc = std::min(w, n - j0);
        e = run([&] { return launch_canon_strip(pred, n, ldp, j0, wc, strip, gate, st); });
        if (e == hipSuccess)
            e = run([&] {
                return launch_canon_pred(d, n, ld, strip, j0, wc, pred, ldp, gate, st);
            });
    }
    return status_of(e);
}

// The fp32 canonical path behind a keyed sweep, every launch gated on
// scratch[3]: the weights saved in P, the distances by the distances-only
// sweep at tile 64 (the register-staged tiles take a gate), then P.
int enqueue_canon(float *d, int n, int64_t ld, int32_t *pred, int64_t ldp, hipStream_t st,
                  bool capturing, int32_t *scratch) {
    const int32_t *gate = scratch + 3;
    auto run = [&](auto &&launch) -> hipError_t {
        if (capturing) return launch();
        return timed(kPredFallback, 0.0, st, launch);
    };
    hipError_t e = run([&] { return launch_canon_gate(scratch, false, st); });
    if (e == hipSuccess) e = run([&] { return launch_canon_save(d, pred, n, ld, ldp, gate, st); });
    if (e != hipSuccess) return status_of(e);
    int s = enqueue_solve(d, FW_F32, n, ld, nullptr, 0, 64, st, capturing, kMinPlus, nullptr, gate);
    if (s != FW_OK) return s;
    return enqueue_canon_hops(d, n, ld, pred, ldp,
                              reinterpret_cast<float *>(scratch + key_scratch_words(n)), gate, st,
                              capturing);
}

// fp32 with predecessors on graphs beyond the keys' vertices: the canonical
// path with no keyed sweep before it.  The weights saved in P; the
// distances-only sweep (tile `tile`, ungated); the negative-diagonal count of
// the distances into scratch[2]; then, gated on no negative diagonal, P from
// the distances -- or, gated on one, d restored from P and the compare form
// (tile `pred_tile`), whose P leads a walk to the cycle.  Scratch as
// canon_scratch_words: `scratch` (a solve plan's), else stream-ordered memory
// of this call; FW_ERR_UNSUPPORTED, nothing enqueued, when none can be had.
int enqueue_canon_direct(float *d, int n, int64_t ld, int32_t *pred, int64_t ldp, int tile,
                         int pred_tile, hipStream_t st, bool capturing, int32_t *scratch) {
    bool own = false;
    if (!scratch) {
        if (capturing) return FW_ERR_UNSUPPORTED;
        void *mem = nullptr;
        if (hipMallocAsync(&mem, (size_t)canon_scratch_words(n) * 4, st) != hipSuccess) {
            (void)hipGetLastError();
            return FW_ERR_UNSUPPORTED;
        }
        scratch = (int32_t *)mem;
        own = true;
    }
    auto run = [&](int kind, auto &&launch) -> hipError_t {
        if (capturing) return launch();
        return timed(kind, 0.0, st, launch);
    };
    int s = FW_OK;
    hipError_t e = run(kPredFix, [&] { return launch_canon_save(d, pred, n, ld, ldp, nullptr, st); });
    if (e != hipSuccess) s = status_of(e);
    if (s == FW_OK) s = enqueue_solve(d, FW_F32, n, ld, nullptr, 0, tile, st, capturing);
    if (s == FW_OK) {
        e = run(kPredFix, [&] {
            const hipError_t e1 = launch_negcycle(FW_F32, d, n, ld, nullptr, scratch + 2, st);
            return e1 != hipSuccess ? e1 : launch_canon_gate(scratch, true, st);
        });
        if (e != hipSuccess) s = status_of(e);
    }
    if (s == FW_OK)
        s = enqueue_canon_hops(d, n, ld, pred, ldp, reinterpret_cast<float *>(scratch + 64),
                               scratch + 3, st, capturing);
    if (s == FW_OK) {
        e = run(kPredFallback, [&] {
            return launch_canon_restore(d, pred, n, ld, ldp, scratch + 2, st);
        });
        if (e != hipSuccess) s = status_of(e);
    }
    if (s == FW_OK)
        s = enqueue_solve(d, FW_F32, n, ld, pred, ldp, pred_tile, st, capturing, kMinPlus,
                          nullptr, scratch + 2);
    if (own) (void)hipFreeAsync(scratch, st);
    return s;
}

// A solve with predecessors as a keyed sweep (fw_internal.h): the pairs
// packed into 32-bit keys in the predecessor matrix, the distances-only
// schedule and int32 arithmetic over them with tile `key_tile`, the keys
// unpacked into d (int32 or fp32) and P.  If an entry is not an integer of
// the key range, a real key leaves its range or a diagonal entry ends
// negative, the unpack leaves d untouched and a form queued behind it, gated
// on the device, solves from the original d; the results are the same either
// way.  int32: the pair-form sweep (tile `tile`, gated on the flag).  fp32:
// the canonical path (enqueue_canon), or, where a diagonal went negative,
// the pair-form sweep (gated on that word), whose predecessors lead a walk to
// the cycle.  Scratch: `scratch` (a solve plan's), else stream-ordered memory
// of this call.  Returns FW_ERR_UNSUPPORTED, nothing enqueued, when no
// scratch can be had (the caller then runs the pair-form sweep).
int enqueue_solve_keyed(void *d, int dtype, int n, int64_t ld, int32_t *pred, int64_t ldp,
                        int tile, int key_tile, hipStream_t st, bool capturing, int32_t *scratch) {
    bool own = false;
    if (!scratch) {
        if (capturing) return FW_ERR_UNSUPPORTED;
        void *mem = nullptr;
        if (hipMallocAsync(&mem, (size_t)key_scratch_words_for(dtype, n) * 4, st) != hipSuccess) {
            (void)hipGetLastError();
            return FW_ERR_UNSUPPORTED;
        }
        scratch = (int32_t *)mem;
        own = true;
    }
    auto run = [&](int kind, auto &&launch) -> hipError_t {
        if (capturing) return launch();
        return timed(kind, 0.0, st, launch);
    };
    int s = FW_OK;
    hipError_t e = run(kPredFix, [&] {
        return launch_key_prepare(dtype, d, pred, n, ld, ldp, scratch, st);
    });
    if (e != hipSuccess) s = status_of(e);
    if (s == FW_OK)
        s = enqueue_solve(pred, FW_I32, n, ldp, nullptr, 0, key_tile, st, capturing, kKey,
                          scratch, nullptr);
    if (s == FW_OK) {
        e = run(kPredFix, [&] {
            return launch_key_finish(dtype, d, pred, n, ld, ldp, scratch, st);
        });
        if (e != hipSuccess) s = status_of(e);
    }
    if (s == FW_OK && dtype == FW_F32)
        s = enqueue_canon(static_cast<float *>(d), n, ld, pred, ldp, st, capturing, scratch);
    if (s == FW_OK)
        s = enqueue_solve(d, dtype, n, ld, pred, ldp, tile, st, capturing, kMinPlus, nullptr,
                          dtype == FW_F32 ? scratch + 2 : scratch);
    if (own) (void)hipFreeAsync(scratch, st);
    return s;
}

bool keyed_solve(const int32_t *pred, int n, int sr) {
    return pred && sr == kMinPlus && n > 1 && n <= kKeyMaxN;
}

bool canon_direct_solve(int dtype, const int32_t *pred, int n, int sr) {
    return pred && dtype == FW_F32 && sr == kMinPlus && n > kKeyMaxN;
}

// Enqueue the whole solve for one graph.  Arguments already valid.  `tile`
// is the tile of the solve (with predecessors: of the pair-form sweep);
// `key_tile` that of a keyed sweep, or of the distances of the fp32
// canonical path beyond the keys' vertices (0: `tile`); `key_scratch` a
// solve plan's scratch for either.
int solve(void *d, int dtype, int n, int64_t ld, int32_t *pred, int64_t ldp, int tile,
          hipStream_t st, bool capturing = false, int sr = kMinPlus,
          int32_t *key_scratch = nullptr, int key_tile = 0) {
    if (n <= 1) {
        if (pred && n == 1) {
            hipError_t e = capturing ? launch_pred_fix(dtype, d, pred, n, ld, ldp, st)
                                     : timed(kPredFix, 0.0, st, [&] {
                                           return launch_pred_fix(dtype, d, pred, n, ld, ldp, st);
                                       });
            return status_of(e);
        }
        return FW_OK;
    }
    if (!tile_supported(tile)) return FW_ERR_INVALID;
    if (keyed_solve(pred, n, sr)) {
        if (key_tile == 0) key_tile = tile;
        if (!tile_supported(key_tile)) return FW_ERR_INVALID;
        const int s = enqueue_solve_keyed(d, dtype, n, ld, pred, ldp, tile, key_tile, st,
                                          capturing, key_scratch);
        if (s != FW_ERR_UNSUPPORTED) return s;
    }
    if (canon_direct_solve(dtype, pred, n, sr)) {
        if (key_tile == 0) key_tile = tile;
        if (!tile_supported(key_tile)) return FW_ERR_INVALID;
        const int s = enqueue_canon_direct(static_cast<float *>(d), n, ld, pred, ldp, key_tile,
                                           tile, st, capturing, key_scratch);
        if (s != FW_ERR_UNSUPPORTED) return s;
    }
    return enqueue_solve(d, dtype, n, ld, pred, ldp, tile, st, capturing, sr);
}

// The plan table's tile for a keyed sweep: the distances-only entry, whose
// kernels it runs (0 for a solve without predecessors).
int key_tile_for(int dtype, const int32_t *pred, int64_t n) {
    return pred ? plan_tile(dtype, n) : 0;
}

}  // namespace

int plan_tile_for(int dtype, int64_t n, bool pred) {
    return plan_tile(dtype | (pred ? FW_PLAN_PRED : 0), n);
}

int solve_single(void *d, int dtype, int64_t n, int64_t ld, int32_t *pred, int64_t ldp,
                 hipStream_t st) {
    return solve(d, dtype, (int)n, ld, pred, ldp, plan_tile(plan_key(dtype, pred), n), st, false,
                 kMinPlus, nullptr, key_tile_for(dtype, pred, n));
}

int solve_with_tile(void *d, int dtype, int n, int64_t ld, int32_t *pred, int64_t ldp, int tile,
                    hipStream_t st) {
    return solve(d, dtype, n, ld, pred, ldp, tile, st);
}

int validate_matrix(const void *d, int dtype, int64_t n, int64_t ld, const int32_t *pred,
                    int64_t ldp) {
    return validate(d, dtype, n, ld, pred, ldp);
}

hipError_t timed_launch(int kind, double updates, hipStream_t st, hipError_t (*launch)(void *),
                        void *ctx) {
    return timed(kind, updates, st, [&] { return launch(ctx); });
}

hipError_t timed_launch_batched(double updates, hipStream_t st, int dtype, bool pred, bool big,
                                BatchHeader *hdr, const BatchItem *items, int grid) {
    return timed(kBatched, updates, st,
                 [&] { return launch_batched_raw(dtype, pred, hdr, items, grid, st, big); });
}

}  // namespace fw

using namespace fw;

extern "C" {

const char *fw_status_string(int status) {
    switch (status) {
    case FW_OK: return "FW_OK";
    case FW_ERR_INVALID: return "FW_ERR_INVALID: invalid argument";
    case FW_ERR_HIP: return "FW_ERR_HIP: a HIP call failed";
    case FW_ERR_NOMEM: return "FW_ERR_NOMEM: out of memory";
    case FW_ERR_UNSUPPORTED: return "FW_ERR_UNSUPPORTED: request not supported";
    case FW_ERR_BUSY: return "FW_ERR_BUSY: admission refused";
    case FW_ERR_NOT_FOUND: return "FW_ERR_NOT_FOUND: unknown request";
    default: return "FW_ERR_UNKNOWN";
    }
}

const char *fw_version(void) { return "fwapsp 0.1 (gfx950)"; }

int fw_apsp(float *d, int64_t n, int64_t ld, void *stream) {
    int s = validate(d, FW_F32, n, ld, nullptr, 0);
    if (s != FW_OK) return s;
    return solve(d, FW_F32, (int)n, ld, nullptr, 0, plan_tile(FW_F32, n), (hipStream_t)stream);
}

int fw_apsp_i32(int32_t *d, int64_t n, int64_t ld, void *stream) {
    int s = validate(d, FW_I32, n, ld, nullptr, 0);
    if (s != FW_OK) return s;
    return solve(d, FW_I32, (int)n, ld, nullptr, 0, plan_tile(FW_I32, n), (hipStream_t)stream);
}

int fw_apsp_pred(void *d, int dtype, int64_t n, int64_t ld, int32_t *pred, int64_t ld_pred,
                 void *stream) {
    int s = validate(d, dtype, n, ld, pred, ld_pred);
    if (s != FW_OK) return s;
    return solve(d, dtype, (int)n, ld, pred, ld_pred, plan_tile(plan_key(dtype, pred), n),
                 (hipStream_t)stream, false, kMinPlus, nullptr, key_tile_for(dtype, pred, n));
}

int fw_apsp_plan(void *d, int dtype, int64_t n, int64_t ld, int32_t *pred, int64_t ld_pred,
                 int tile, void *stream) {
    int s = validate(d, dtype, n, ld, pred, ld_pred);
    if (s != FW_OK) return s;
    if (!tile_supported(tile)) return FW_ERR_INVALID;
    return solve(d, dtype, (int)n, ld, pred, ld_pred, tile, (hipStream_t)stream);
}

int fw_apsp_semiring(void *d, int dtype, int semiring, int64_t n, int64_t ld, void *stream) {
    if (semiring != FW_SR_MINPLUS && semiring != FW_SR_MAXMIN) return FW_ERR_INVALID;
    int s = validate(d, dtype, n, ld, nullptr, 0);
    if (s != FW_OK) return s;
    if (n <= 1) return FW_OK;
    return solve(d, dtype, (int)n, ld, nullptr, 0, plan_tile(dtype, n), (hipStream_t)stream, false,
                 semiring == FW_SR_MAXMIN ? kMaxMin : kMinPlus);
}

int fw_plan_tiles(int *tiles, int cap) {
    const int cnt = (int)(sizeof(kTiles) / sizeof(kTiles[0]));
    for (int i = 0; i < cnt && i < cap && tiles; ++i) tiles[i] = kTiles[i];
    return cnt;
}

int fw_plan_tile(int key, int64_t n) {
    if (!plan_key_ok(key) || n < 0) return -1;
    if (n <= 1) return 0;
    return plan_tile(key, n);
}

int fw_plan_set(int key, int64_t n_lo, int64_t n_hi, int tile) {
    if (!plan_key_ok(key) || n_lo < 0 || n_hi < n_lo || !tile_supported(tile))
        return FW_ERR_INVALID;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (g_plan[0].empty()) default_plan_locked();
    g_plan[key].push_back({n_lo, n_hi, tile});
    return FW_OK;
}

void fw_plan_reset(void) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    default_plan_locked();
}

int fw_negative_cycle(const void *d, int dtype, int64_t n, int64_t ld, int32_t *flag_dev,
                      void *stream) {
    int s = validate(d, dtype, n, ld, nullptr, 0);
    if (s != FW_OK) return s;
    if (!flag_dev) return FW_ERR_INVALID;
    return status_of(
        launch_negcycle(dtype, d, (int)n, ld, nullptr, flag_dev, (hipStream_t)stream));
}

int fw_negative_cycle_vertices(const void *d, int dtype, int64_t n, int64_t ld,
                               int32_t *list_dev, int32_t *count_dev, void *stream) {
    int s = validate(d, dtype, n, ld, nullptr, 0);
    if (s != FW_OK) return s;
    if (!count_dev || (n > 0 && !list_dev)) return FW_ERR_INVALID;
    return status_of(
        launch_negcycle(dtype, d, (int)n, ld, list_dev, count_dev, (hipStream_t)stream));
}

}  // extern "C"

namespace {

// Weight of the edge p -> q of a host weight matrix as a double (exact for
// int32 and for fp32), or +INF when there is no such edge (absent entry or
// the diagonal).
double edge_weight(const void *w, int dtype, int64_t ld, int64_t p, int64_t q) {
    if (p == q) return HUGE_VAL;
    if (dtype == FW_F32) {
        const float x = static_cast<const float *>(w)[p * ld + q];
        return x == HUGE_VALF ? HUGE_VAL : (double)x;
    }
    const int32_t x = static_cast<const int32_t *>(w)[p * ld + q];
    return x == FW_I32_INF ? HUGE_VAL : (double)x;
}

// Weight of the closed walk cyc[0] -> cyc[1] -> ... -> cyc[m-1] -> cyc[0]
// (+INF if some hop is not an edge).
double cycle_weight(const void *w, int dtype, int64_t ld, const int64_t *cyc, int64_t m) {
    double sum = 0.0;
    for (int64_t t = 0; t < m; ++t) {
        const double e = edge_weight(w, dtype, ld, cyc[t], cyc[(t + 1) % m]);
        if (e == HUGE_VAL) return HUGE_VAL;
        sum += e;
    }
    return sum;
}

// The cycle that a chain of last hops x_{t+1} = hop(x_t) runs into, in
// forward edge order (each hop(x) -> x is an edge): written to `out`, its
// length returned; 0 when the chain ends (hop < 0) before repeating.
template <typename Hop>
int64_t chain_cycle(int64_t n, int64_t start, Hop hop, std::vector<int64_t> &out) {
    std::vector<int64_t> pos((size_t)n, -1), seq;
    int64_t cur = start;
    pos[(size_t)cur] = 0;
    seq.push_back(cur);
    while (true) {
        const int64_t p = hop(cur);
        if (p < 0 || p >= n) return 0;
        if (pos[(size_t)p] >= 0) {
            // x_a = p, ..., x_t = cur: edges x_{u+1} -> x_u and p -> cur
            const int64_t a = pos[(size_t)p], t = (int64_t)seq.size() - 1;
            out.clear();
            out.push_back(seq[(size_t)a]);
            for (int64_t u = t; u > a; --u) out.push_back(seq[(size_t)u]);
            return (int64_t)out.size();
        }
        pos[(size_t)p] = (int64_t)seq.size();
        seq.push_back(p);
        cur = p;
    }
}

// Bellman-Ford from `src` over the edges of w (in-place relaxation in vertex
// order), checking the parent graph for a cycle after every pass.  A cycle of
// a Bellman-Ford parent graph has negative weight, and one appears once the
// distances of a negative cycle reachable from src keep falling; with no such
// cycle the relaxation settles within n - 1 passes.  Returns the cycle length
// (written to out) or 0.
int64_t bellman_ford_cycle(const void *w, int dtype, int64_t n, int64_t ld, int64_t src,
                           std::vector<int64_t> &out) {
    std::vector<double> dist((size_t)n, HUGE_VAL);
    std::vector<int64_t> parent((size_t)n, -1);
    std::vector<int32_t> mark((size_t)n, 0);
    dist[(size_t)src] = 0.0;
    for (int64_t pass = 0; pass <= n; ++pass) {
        bool changed = false;
        for (int64_t u = 0; u < n; ++u) {
            const double du = dist[(size_t)u];
            if (du == HUGE_VAL) continue;
            for (int64_t v = 0; v < n; ++v) {
                const double e = edge_weight(w, dtype, ld, u, v);
                if (e == HUGE_VAL) continue;
                if (du + e < dist[(size_t)v]) {
                    dist[(size_t)v] = du + e;
                    parent[(size_t)v] = u;
                    changed = true;
                }
            }
        }
        if (!changed) return 0;
        // look for a cycle in the parent graph: follow parents from every
        // unvisited vertex, marking the walk with its start (+1)
        std::fill(mark.begin(), mark.end(), 0);
        for (int64_t s0 = 0; s0 < n; ++s0) {
            int64_t x = s0;
            while (x >= 0 && mark[(size_t)x] == 0) {
                mark[(size_t)x] = (int32_t)(s0 + 1);
                x = parent[(size_t)x];
            }
            if (x >= 0 && mark[(size_t)x] == (int32_t)(s0 + 1))
                return chain_cycle(n, x, [&](int64_t y) { return parent[(size_t)y]; }, out);
        }
    }
    return 0;
}

}  // namespace

extern "C" {

int64_t fw_negative_cycle_find(const void *w_host, int dtype, int64_t n, int64_t ld,
                               const int32_t *pred_host, int64_t ld_pred, int64_t v,
                               int64_t *cycle, int64_t cap, int *from_pred) {
    if (!w_host || (dtype != FW_F32 && dtype != FW_I32) || n <= 0 || ld < n || v < 0 ||
        v >= n || !cycle || cap <= 0 || (pred_host && ld_pred < n) || n > 0x7fffffffLL)
        return -1;
    if (from_pred) *from_pred = 0;
    std::vector<int64_t> cyc;
    int64_t m = 0;
    if (pred_host) {
        // walk the last hops of row v back from v itself (P_vv is the last
        // hop of the closed walk that made d_vv negative); the result is kept
        // only if its weight over the original edges is negative
        m = chain_cycle(n, v, [&](int64_t x) { return (int64_t)pred_host[v * ld_pred + x]; }, cyc);
        if (m > 0 && !(cycle_weight(w_host, dtype, ld, cyc.data(), m) < 0.0)) m = 0;
        if (m > 0 && from_pred) *from_pred = 1;
    }
    if (m == 0) m = bellman_ford_cycle(w_host, dtype, n, ld, v, cyc);
    if (m == 0) return 0;
    if (m > cap) return -1;
    std::copy(cyc.begin(), cyc.end(), cycle);
    return m;
}

int64_t fw_path(const int32_t *pred, int64_t n, int64_t ldp, int64_t i, int64_t j,
                int64_t *path, int64_t cap) {
    if (!pred || n <= 0 || ldp < n || i < 0 || j < 0 || i >= n || j >= n || !path || cap <= 0)
        return -1;
    if (i == j) {
        path[0] = i;
        return 1;
    }
    if (pred[i * ldp + j] < 0) return 0;
    // walk backwards from j along last hops; a shortest path has at most n vertices
    int64_t len = 0, v = j;
    while (true) {
        if (len >= n || len >= cap) return -1;
        path[len++] = v;
        if (v == i) break;
        const int32_t p = pred[i * ldp + v];
        if (p < 0 || p >= n) return -1;
        v = p;
    }
    std::reverse(path, path + len);
    return len;
}

// ---------------------------------------------------------------------------
// Solve plans: the stage loop of one matrix captured once into a hipGraph.
// ---------------------------------------------------------------------------
}  // extern "C"

struct fw_solve_plan_s {
    void *d = nullptr;
    int dtype = 0;
    int n = 0;
    int64_t ld = 0, ldp = 0;
    int32_t *pred = nullptr;
    int tile = 0, key_tile = 0;
    int32_t *key_scratch = nullptr;  // the keyed predecessor sweep's
    int device = 0;
    // the capture stream lives as long as the plan (and with it the graph
    // captured on it); no event is recorded during the capture
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {
void free_solve_plan(fw_solve_plan_s *pl) {
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    if (pl->key_scratch) (void)hipFree(pl->key_scratch);
    delete pl;
}
}  // namespace

extern "C" {

int fw_solve_plan_create(void *d, int dtype, int64_t n, int64_t ld, int32_t *pred,
                         int64_t ld_pred, int tile, fw_solve_plan *out) {
    if (!out) return FW_ERR_INVALID;
    *out = nullptr;
    int s = validate(d, dtype, n, ld, pred, ld_pred);
    if (s != FW_OK) return s;
    if (tile != 0 && !tile_supported(tile)) return FW_ERR_INVALID;
    auto *pl = new fw_solve_plan_s();
    pl->d = d;
    pl->dtype = dtype;
    pl->n = (int)n;
    pl->ld = ld;
    pl->pred = pred;
    pl->ldp = pred ? ld_pred : 0;
    pl->tile = n <= 1 ? 32 : tile ? tile : plan_tile(plan_key(dtype, pred), n);
    pl->key_tile = n <= 1 ? 0 : tile ? tile : key_tile_for(dtype, pred, n);
    if (hipGetDevice(&pl->device) != hipSuccess) {
        delete pl;
        return FW_ERR_HIP;
    }
    if (keyed_solve(pred, (int)n, kMinPlus) || canon_direct_solve(dtype, pred, (int)n, kMinPlus)) {
        void *mem = nullptr;
        const int64_t words = keyed_solve(pred, (int)n, kMinPlus) ? key_scratch_words_for(dtype, n)
                                                                  : canon_scratch_words(n);
        hipError_t e = hipMalloc(&mem, (size_t)words * 4);
        if (e != hipSuccess) {
            delete pl;
            return status_of(e);
        }
        pl->key_scratch = (int32_t *)mem;
    }
    *out = pl;
    return FW_OK;
}

int fw_solve_plan_launch(fw_solve_plan pl, int mode, void *stream) {
    if (!pl || (mode != 0 && mode != 1)) return FW_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    if (mode == 0 || pl->n <= 1)
        return solve(pl->d, pl->dtype, pl->n, pl->ld, pl->pred, pl->ldp, pl->tile, st, false,
                     kMinPlus, pl->key_scratch, pl->key_tile);
    if (!pl->exec) {
        hipError_t e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            pl->cap_stream = nullptr;
            return status_of(e);
        }
        e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return status_of(e);
        int s = solve(pl->d, pl->dtype, pl->n, pl->ld, pl->pred, pl->ldp, pl->tile,
                      pl->cap_stream, true, kMinPlus, pl->key_scratch, pl->key_tile);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(pl->cap_stream, &g);
        if (s != FW_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return status_of(e);
        pl->graph = g;
        e = hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            pl->exec = nullptr;
            return status_of(e);
        }
    }
    return status_of(hipGraphLaunch(pl->exec, st));
}

int fw_solve_plan_tile(fw_solve_plan pl) { return pl ? pl->tile : -1; }

int fw_solve_plan_destroy(fw_solve_plan pl) {
    if (!pl) return FW_ERR_INVALID;
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipSetDevice(pl->device);
    (void)hipDeviceSynchronize();
    free_solve_plan(pl);
    (void)hipSetDevice(dev);
    return FW_OK;
}

int64_t fw_pred_fallbacks(void) { return pred_fallbacks(); }

int fw_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return FW_OK;
}

int fw_profile_read(double *ms, int64_t *launches, int cap) {
    std::vector<TimedLaunch> pend;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        pend.swap(g_prof_pending);
    }
    double acc[kNumKinds] = {0};
    double upd[kNumKinds] = {0};
    int64_t cnt[kNumKinds] = {0};
    int status = FW_OK;
    for (auto &t : pend) {
        float m = 0.f;
        if (hipEventSynchronize(t.stop) != hipSuccess ||
            hipEventElapsedTime(&m, t.start, t.stop) != hipSuccess)
            status = FW_ERR_HIP;
        acc[t.kind] += m;
        upd[t.kind] += t.updates;
        cnt[t.kind] += 1;
    }
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        for (auto &t : pend) {
            g_event_pool.push_back(t.start);
            g_event_pool.push_back(t.stop);
        }
        for (int k = 0; k < kNumKinds; ++k) g_last_updates[k] = upd[k];
    }
    if (status != FW_OK) return -status;
    const int w = std::min<int>(cap, kNumKinds);
    for (int k = 0; k < w; ++k) {
        if (ms) ms[k] = acc[k];
        if (launches) launches[k] = cnt[k];
    }
    return w;
}

int fw_profile_updates(double *updates, int cap) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    const int w = std::min<int>(cap, kNumKinds);
    for (int k = 0; k < w; ++k)
        if (updates) updates[k] = g_last_updates[k];
    return w;
}

}  // extern "C"
