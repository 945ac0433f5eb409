// C ABI and host driver of libfwapsp (declared in include/fwapsp.h).
//
// The driver runs the stage loop of the blocked algorithm (section 3.2,
// Fig. BFW-Alg): for every k-block b, three stream-ordered launches (diagonal
// tile, panels, bulk).  It validates every argument before enqueueing
// anything, picks the tile size from a plan table keyed by (dtype, n), and can
// bracket each launch with HIP events for per-phase timing.
#include <hip/hip_runtime.h>

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
std::vector<PlanEntry> g_plan[2];

void default_plan_locked() {
    for (int dt = 0; dt < 2; ++dt) {
        g_plan[dt].clear();
        // n <= tile: one closure over the whole graph (the plain algorithm)
        g_plan[dt].push_back({0, 32, 32});
        g_plan[dt].push_back({33, 64, 64});
        g_plan[dt].push_back({65, 128, 128});
        // blocked
        g_plan[dt].push_back({129, 1024, 64});
        g_plan[dt].push_back({1025, INT64_MAX, 128});
    }
}

int plan_tile(int dtype, int64_t n) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (g_plan[0].empty()) default_plan_locked();
    // the most recently installed entry covering n wins
    for (auto it = g_plan[dtype].rbegin(); it != g_plan[dtype].rend(); ++it)
        if (n >= it->n_lo && n <= it->n_hi) return it->tile;
    return 128;
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

// Enqueue the whole blocked solve for one graph.  Arguments already valid.
int solve(void *d, int dtype, int n, int64_t ld, int32_t *pred, int64_t ldp, int tile,
          hipStream_t st) {
    if (n <= 1) {
        if (pred && n == 1) {
            hipError_t e = timed(kPredFix, 0.0, st, [&] {
                return launch_pred_fix(dtype, d, pred, n, ld, ldp, st);
            });
            return status_of(e);
        }
        return FW_OK;
    }
    if (!tile_supported(tile)) return FW_ERR_INVALID;
    const int nb = (n + tile - 1) / tile;
    hipError_t e;
    if (pred) {
        e = timed(kPredFix, 0.0, st, [&] { return launch_pred_init(dtype, d, pred, n, ld, ldp, st); });
        if (e != hipSuccess) return status_of(e);
    }
    // algorithmic updates of each phase: the n^3 tasks split by where the
    // (i, j) cell lies relative to block b (real cells only, padding excluded)
    const double nn = (double)n;
    for (int b = 0; b < nb; ++b) {
        const double kb = std::min<double>(tile, nn - (double)b * tile);  // real k of block b
        const double rb = kb;                                             // real rows of block b
        const double rest = nn - rb;
        e = timed(kDiag, kb * rb * rb, st,
                  [&] { return launch_diag(dtype, tile, d, pred, n, ld, ldp, b, st); });
        if (e != hipSuccess) return status_of(e);
        if (nb > 1) {
            e = timed(kPanel, 2.0 * kb * rb * rest, st, [&] {
                return launch_panels(dtype, tile, d, pred, n, ld, ldp, b, nb, st);
            });
            if (e != hipSuccess) return status_of(e);
            e = timed(kBulk, kb * rest * rest, st, [&] {
                return launch_bulk(dtype, tile, d, pred, n, ld, ldp, b, nb, st);
            });
            if (e != hipSuccess) return status_of(e);
        }
    }
    if (pred) {
        e = timed(kPredFix, 0.0, st, [&] { return launch_pred_fix(dtype, d, pred, n, ld, ldp, st); });
        if (e != hipSuccess) return status_of(e);
    }
    return FW_OK;
}

}  // namespace

int plan_tile_for(int dtype, int64_t n) { return plan_tile(dtype, n); }

int solve_single(void *d, int dtype, int64_t n, int64_t ld, int32_t *pred, int64_t ldp,
                 hipStream_t st) {
    return solve(d, dtype, (int)n, ld, pred, ldp, plan_tile(dtype, n), st);
}

int validate_matrix(const void *d, int dtype, int64_t n, int64_t ld, const int32_t *pred,
                    int64_t ldp) {
    return validate(d, dtype, n, ld, pred, ldp);
}

hipError_t timed_launch_batched(double updates, hipStream_t st, int dtype, bool pred,
                                BatchHeader *hdr, const BatchItem *items, int grid) {
    return timed(kBatched, updates, st,
                 [&] { return launch_batched_raw(dtype, pred, hdr, items, grid, st); });
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
    return solve(d, dtype, (int)n, ld, pred, ld_pred, plan_tile(dtype, n), (hipStream_t)stream);
}

int fw_apsp_plan(void *d, int dtype, int64_t n, int64_t ld, int32_t *pred, int64_t ld_pred,
                 int tile, void *stream) {
    int s = validate(d, dtype, n, ld, pred, ld_pred);
    if (s != FW_OK) return s;
    if (!tile_supported(tile)) return FW_ERR_INVALID;
    return solve(d, dtype, (int)n, ld, pred, ld_pred, tile, (hipStream_t)stream);
}

int fw_plan_tiles(int *tiles, int cap) {
    const int cnt = (int)(sizeof(kTiles) / sizeof(kTiles[0]));
    for (int i = 0; i < cnt && i < cap && tiles; ++i) tiles[i] = kTiles[i];
    return cnt;
}

int fw_plan_tile(int dtype, int64_t n) {
    if ((dtype != FW_F32 && dtype != FW_I32) || n < 0) return -1;
    if (n <= 1) return 0;
    return plan_tile(dtype, n);
}

int fw_plan_set(int dtype, int64_t n_lo, int64_t n_hi, int tile) {
    if ((dtype != FW_F32 && dtype != FW_I32) || n_lo < 0 || n_hi < n_lo || !tile_supported(tile))
        return FW_ERR_INVALID;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (g_plan[0].empty()) default_plan_locked();
    g_plan[dtype].push_back({n_lo, n_hi, tile});
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
    return status_of(launch_negcycle(dtype, d, (int)n, ld, flag_dev, (hipStream_t)stream));
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
