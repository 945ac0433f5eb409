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

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>
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
        // 1.4x).  With predecessors tile 128 never won (int32 n=8192: 69 vs
        // 82 ms at tile 64), and tile 32 wins below ~2k (fp32) / ~1k (int32)
        // vertices (fp32 n~1448: 4.0 vs 4.6 ms; int32 n~724: 0.78 vs 0.83).
        if (key & FW_PLAN_PRED) {
            const int64_t hi32 = (key & 1) == FW_F32 ? 2048 : 1024;
            t.push_back({129, hi32, 32});
            t.push_back({hi32 + 1, INT64_MAX, 64});
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

// ---------------------------------------------------------------------------
// Per-device resources: the look-ahead side stream and a pool of events.
// ---------------------------------------------------------------------------
struct DeviceRes {
    std::mutex mu;                 // serialises eager enqueues that use `side`
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> free_events;
};

std::mutex g_dev_mu;
std::map<int, DeviceRes *> g_dev;

DeviceRes *device_res() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DeviceRes *&r = g_dev[dev];
    if (!r) {
        r = new DeviceRes();
        if (hipStreamCreateWithFlags(&r->side, hipStreamNonBlocking) != hipSuccess) {
            delete r;
            r = nullptr;
        }
    }
    return r;
}

hipError_t take_events(DeviceRes *r, size_t k, std::vector<hipEvent_t> &out) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    while (out.size() < k) {
        if (!r->free_events.empty()) {
            out.push_back(r->free_events.back());
            r->free_events.pop_back();
            continue;
        }
        hipEvent_t e = nullptr;
        hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (err != hipSuccess) return err;
        out.push_back(e);
    }
    return hipSuccess;
}

// Events may be reused as soon as every wait on them has been enqueued.
void give_events(DeviceRes *r, std::vector<hipEvent_t> &ev) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    for (auto e : ev) r->free_events.push_back(e);
    ev.clear();
}

// Library options (fw_set_option).  Both schedules are switched off: a test
// that cycled through them ended in a host-side segmentation fault whose cause
// has not been identified, so they cannot be enabled until it is.
std::atomic<int> g_opt_lookahead{0};
std::atomic<int> g_opt_graphs{0};
constexpr bool kLookaheadAvailable = false;
constexpr bool kGraphsAvailable = false;

// Enqueue the whole blocked solve of one graph on `st` (and, with
// look-ahead, on `side`, joined back into `st` before the last bulk).
// Arguments already validated; n > 1.
//
// Look-ahead (nb >= 3): the bulk of stage b is split into the tiles of row
// and column b+1 ("ahead") and the rest.  The side stream runs ahead(b),
// then stage b+1's diagonal tile and panels, while `st` runs rest(b); the
// two touch disjoint tiles.  Dependencies are events: rest(b) waits for the
// panels of stage b, ahead(b) waits for rest(b-1) (which last wrote row and
// column b+1).
int enqueue_solve(void *d, int dtype, int n, int64_t ld, int32_t *pred, int64_t ldp, int tile,
                  hipStream_t st, hipStream_t side, bool lookahead, std::vector<hipEvent_t> &evs,
                  int sr = kMinPlus) {
    const int nb = (n + tile - 1) / tile;
    hipError_t e;
    if (pred) {
        e = timed(kPredFix, 0.0, st, [&] { return launch_pred_init(dtype, d, pred, n, ld, ldp, st); });
        if (e != hipSuccess) return status_of(e);
    }
    // algorithmic updates of each launch: the n^3 tasks split by where the
    // (i, j) cell lies relative to block b (real cells only, padding excluded)
    const double nn = (double)n;
    auto real = [&](int blk) { return std::max(0.0, std::min<double>(tile, nn - (double)blk * tile)); };
    auto diag = [&](int b, hipStream_t s) {
        const double kb = real(b);
        return timed(kDiag, kb * kb * kb, s,
                     [&] { return launch_diag(dtype, sr, tile, d, pred, n, ld, ldp, b, s); });
    };
    auto panels = [&](int b, hipStream_t s) {
        const double kb = real(b);
        return timed(kPanel, 2.0 * kb * kb * (nn - kb), s, [&] {
            return launch_panels(dtype, sr, tile, d, pred, n, ld, ldp, b, nb, s);
        });
    };
    // close_next: the launch also closes the next diagonal tile (its updates
    // are counted with the bulk's, the launch that does them)
    auto bulk = [&](int b, int part, hipStream_t s, bool close_next = false) {
        const double kb = real(b), r1 = real(b + 1), rest = nn - kb;
        double upd = kb * rest * rest;
        int kind = kBulk;
        if (part == kBulkAheadPart) {
            upd = kb * (r1 * rest + (rest - r1) * r1);
            kind = kBulkAhead;
        } else if (part == kBulkRestPart) {
            upd = kb * (rest - r1) * (rest - r1);
        }
        if (close_next) upd += r1 * r1 * r1;
        return timed(kind, upd, s, [&] {
            return launch_bulk(dtype, sr, tile, d, pred, n, ld, ldp, b, nb, part, close_next, s);
        });
    };

    if (!lookahead || nb < 3) {
        bool closed = false;  // the previous bulk launch closed this stage's diagonal tile
        for (int b = 0; b < nb; ++b) {
            if (!closed && (e = diag(b, st)) != hipSuccess) return status_of(e);
            closed = false;
            if (nb > 1) {
                if ((e = panels(b, st)) != hipSuccess) return status_of(e);
                closed = bulk_closes_next_diag(sr, tile, d, pred, n, ld, b);
                if ((e = bulk(b, kBulkAll, st, closed)) != hipSuccess) return status_of(e);
            }
        }
    } else {
        size_t ei = 0;
        if ((e = diag(0, st)) != hipSuccess) return status_of(e);
        if ((e = panels(0, st)) != hipSuccess) return status_of(e);
        hipEvent_t ev_panels = evs[ei++];  // panels of the current stage are done
        hipEvent_t ev_rest = nullptr;      // rest of the previous stage's bulk is done
        if ((e = hipEventRecord(ev_panels, st)) != hipSuccess) return status_of(e);
        for (int b = 0; b < nb; ++b) {
            if (b == nb - 1) {
                if ((e = hipStreamWaitEvent(st, ev_panels, 0)) != hipSuccess) return status_of(e);
                if ((e = bulk(b, kBulkAll, st)) != hipSuccess) return status_of(e);
                break;
            }
            if ((e = hipStreamWaitEvent(side, ev_panels, 0)) != hipSuccess) return status_of(e);
            if (ev_rest && (e = hipStreamWaitEvent(side, ev_rest, 0)) != hipSuccess)
                return status_of(e);
            if ((e = bulk(b, kBulkAheadPart, side)) != hipSuccess) return status_of(e);
            if ((e = diag(b + 1, side)) != hipSuccess) return status_of(e);
            if ((e = panels(b + 1, side)) != hipSuccess) return status_of(e);
            hipEvent_t ev_next = evs[ei++];
            if ((e = hipEventRecord(ev_next, side)) != hipSuccess) return status_of(e);
            if ((e = hipStreamWaitEvent(st, ev_panels, 0)) != hipSuccess) return status_of(e);
            if (nb > 2 && (e = bulk(b, kBulkRestPart, st)) != hipSuccess) return status_of(e);
            ev_rest = evs[ei++];
            if ((e = hipEventRecord(ev_rest, st)) != hipSuccess) return status_of(e);
            ev_panels = ev_next;
        }
    }
    if (pred) {
        e = timed(kPredFix, 0.0, st, [&] { return launch_pred_fix(dtype, d, pred, n, ld, ldp, st); });
        if (e != hipSuccess) return status_of(e);
    }
    return FW_OK;
}

// ---------------------------------------------------------------------------
// Graph cache: the whole stage loop of one (matrix, plan) captured once and
// replayed with a single graph launch.
// ---------------------------------------------------------------------------
struct GraphKey {
    int dev, dtype, n, tile, lookahead;
    int64_t ld, ldp;
    void *d;
    int32_t *pred;
    bool operator<(const GraphKey &o) const {
        return std::tie(dev, dtype, n, tile, lookahead, ld, ldp, d, pred) <
               std::tie(o.dev, o.dtype, o.n, o.tile, o.lookahead, o.ld, o.ldp, o.d, o.pred);
    }
};
struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};
std::mutex g_graph_mu;
std::map<GraphKey, GraphEntry> g_graphs;
uint64_t g_graph_clock = 0;
constexpr size_t kMaxGraphs = 32;

int capture_solve(void *d, int dtype, int n, int64_t ld, int32_t *pred, int64_t ldp, int tile,
                  bool lookahead, DeviceRes *res, GraphEntry &out) {
    hipStream_t cs = nullptr, cside = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cside, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (cs) hipStreamDestroy(cs);
        return status_of(e);
    }
    const int nb = (n + tile - 1) / tile;
    std::vector<hipEvent_t> evs;
    int s = status_of(take_events(res, 2 * (size_t)nb + 2, evs));
    hipGraph_t g = nullptr;
    if (s == FW_OK) {
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            s = status_of(e);
        } else {
            s = enqueue_solve(d, dtype, n, ld, pred, ldp, tile, cs, cside, lookahead, evs);
            e = hipStreamEndCapture(cs, &g);
            if (s == FW_OK && e != hipSuccess) s = status_of(e);
        }
    }
    if (s == FW_OK) {
        e = hipGraphInstantiate(&out.exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) s = status_of(e);
    }
    if (s == FW_OK) {
        out.graph = g;
    } else if (g) {
        hipGraphDestroy(g);
    }
    give_events(res, evs);
    hipStreamDestroy(cside);
    hipStreamDestroy(cs);
    return s;
}

bool profiling_on() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    return g_prof_on;
}

// Enqueue the whole solve for one graph.  Arguments already valid.
int solve(void *d, int dtype, int n, int64_t ld, int32_t *pred, int64_t ldp, int tile,
          hipStream_t st, bool allow_graph = true, int sr = kMinPlus) {
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
    const bool lookahead = g_opt_lookahead.load() != 0;
    const bool graphs = allow_graph && g_opt_graphs.load() && !profiling_on();
    if ((!lookahead && !graphs) || sr != kMinPlus) {
        // plain schedule on the caller's stream: no side stream, no events
        std::vector<hipEvent_t> none;
        return enqueue_solve(d, dtype, n, ld, pred, ldp, tile, st, nullptr, false, none, sr);
    }
    DeviceRes *res = device_res();
    if (!res) return FW_ERR_HIP;
    if (graphs) {
        int dev = 0;
        hipGetDevice(&dev);
        GraphKey key{dev, dtype, n, tile, lookahead ? 1 : 0, ld, ldp, d, pred};
        std::lock_guard<std::mutex> lk(g_graph_mu);
        auto it = g_graphs.find(key);
        if (it == g_graphs.end()) {
            if (g_graphs.size() >= kMaxGraphs) {
                auto victim = g_graphs.begin();
                for (auto jt = g_graphs.begin(); jt != g_graphs.end(); ++jt)
                    if (jt->second.last_use < victim->second.last_use) victim = jt;
                hipGraphExecDestroy(victim->second.exec);
                hipGraphDestroy(victim->second.graph);
                g_graphs.erase(victim);
            }
            GraphEntry ent;
            int s = capture_solve(d, dtype, n, ld, pred, ldp, tile, lookahead, res, ent);
            if (s != FW_OK) return s;
            it = g_graphs.emplace(key, ent).first;
        }
        it->second.last_use = ++g_graph_clock;
        return status_of(hipGraphLaunch(it->second.exec, st));
    }
    std::lock_guard<std::mutex> lk(res->mu);
    std::vector<hipEvent_t> evs;
    const int nb = (n + tile - 1) / tile;
    int s = status_of(take_events(res, 2 * (size_t)nb + 2, evs));
    if (s == FW_OK) s = enqueue_solve(d, dtype, n, ld, pred, ldp, tile, st, res->side, lookahead, evs);
    give_events(res, evs);
    return s;
}

}  // namespace

int plan_tile_for(int dtype, int64_t n, bool pred) {
    return plan_tile(dtype | (pred ? FW_PLAN_PRED : 0), n);
}

int solve_single(void *d, int dtype, int64_t n, int64_t ld, int32_t *pred, int64_t ldp,
                 hipStream_t st) {
    // eager launches: callers (the per-graph batch baseline, the server) solve
    // many different matrices, which a graph cache would only churn
    return solve(d, dtype, (int)n, ld, pred, ldp, plan_tile(plan_key(dtype, pred), n), st, false);
}

int solve_with_tile(void *d, int dtype, int n, int64_t ld, int32_t *pred, int64_t ldp, int tile,
                    hipStream_t st) {
    return solve(d, dtype, n, ld, pred, ldp, tile, st, false);
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
                 (hipStream_t)stream);
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

int fw_set_option(int option, int64_t value) {
    switch (option) {
    case FW_OPT_LOOKAHEAD:
        if (value && !kLookaheadAvailable) return FW_ERR_UNSUPPORTED;
        g_opt_lookahead.store(value ? 1 : 0);
        return FW_OK;
    case FW_OPT_GRAPHS:
        if (value && !kGraphsAvailable) return FW_ERR_UNSUPPORTED;
        g_opt_graphs.store(value ? 1 : 0);
        return FW_OK;
    default: return FW_ERR_INVALID;
    }
}

int64_t fw_get_option(int option) {
    switch (option) {
    case FW_OPT_LOOKAHEAD: return g_opt_lookahead.load();
    case FW_OPT_GRAPHS: return g_opt_graphs.load();
    default: return -1;
    }
}

int fw_graph_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto &kv : g_graphs) {
        hipGraphExecDestroy(kv.second.exec);
        hipGraphDestroy(kv.second.graph);
    }
    g_graphs.clear();
    return FW_OK;
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
