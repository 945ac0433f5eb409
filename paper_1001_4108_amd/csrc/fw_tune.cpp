// Autotuner for the plan table: for each size bucket, time every tile size on
// the device and install the fastest with fw_plan_set.
//
// Timing uses a matrix of zeros: the sweep is data-oblivious (section 1: the
// run time of Floyd-Warshall does not depend on the graph), so the timings
// hold for every input of that size.  With FW_PLAN_PRED in the dtype argument
// the solves compute predecessors too and the table of such solves is tuned.
// Two objectives:
//   0  one single-graph solve of the bucket's representative size;
//   1  one batch-plan launch of `batch` graphs whose sizes spread
//      log-uniformly over the bucket (persistent or stage-batched, whichever
//      the plan uses for those sizes; batch plans read the same table): in a
//      ragged batch a bucket's graphs span it, and a tile's padding of the
//      last block and its stage count vary across the bucket.
// The single solve takes the geometric middle of the bucket.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/fwapsp.h"
#include "fw_internal.h"

using namespace fw;

namespace {

int status_of(hipError_t e) {
    if (e == hipSuccess) return FW_OK;
    if (e == hipErrorOutOfMemory) return FW_ERR_NOMEM;
    return FW_ERR_HIP;
}

struct TuneScratch {
    void *mat = nullptr;     // device matrices
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneScratch() {
        if (st) (void)hipStreamSynchronize(st);
        if (mat) (void)hipFree(mat);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
    }
};

double median(std::vector<double> v) {
    std::sort(v.begin(), v.end());
    return v.empty() ? 0.0 : v[v.size() / 2];
}

}  // namespace

extern "C" int fw_autotune(int dtype, const int64_t *lo, const int64_t *hi, int nbuckets,
                           int objective, int batch, int reps, int *tile_out, double *ms_out) {
    const int base = dtype & ~FW_PLAN_PRED;
    const bool pred = (dtype & FW_PLAN_PRED) != 0;
    if ((base != FW_F32 && base != FW_I32) || !lo || !hi || nbuckets < 1 || !tile_out ||
        (objective != 0 && objective != 1) || reps < 1 || (objective == 1 && batch < 1))
        return FW_ERR_INVALID;
    for (int k = 0; k < nbuckets; ++k)
        if (lo[k] < 2 || hi[k] < lo[k] || hi[k] > 65536) return FW_ERR_INVALID;
    int tiles[8];
    const int ntiles = fw_plan_tiles(tiles, 8);
    TuneScratch sc;
    hipError_t e = hipStreamCreateWithFlags(&sc.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&sc.e0);
    if (e == hipSuccess) e = hipEventCreate(&sc.e1);
    if (e != hipSuccess) return status_of(e);
    for (int k = 0; k < nbuckets; ++k) {
        const int n = (int)std::llround(std::sqrt((double)lo[k] * (double)hi[k]));
        const int64_t ld = (n + 3) / 4 * 4;
        const int count = objective == 1 ? batch : 1;
        // graph sizes: the middle for a single solve, else log-uniform over
        // the bucket (graph g at quantile (g + 1/2) / count)
        std::vector<int64_t> ns((size_t)count, n), lds((size_t)count, ld);
        std::vector<size_t> offs((size_t)count + 1, 0);
        for (int g = 0; g < count; ++g) {
            if (objective == 1) {
                const double q = (g + 0.5) / count;
                ns[(size_t)g] = std::min<int64_t>(
                    hi[k], std::max<int64_t>(lo[k], std::llround(lo[k] * std::pow((double)hi[k] / lo[k], q))));
                lds[(size_t)g] = (ns[(size_t)g] + 3) / 4 * 4;
            }
            offs[(size_t)g + 1] = offs[(size_t)g] + (size_t)ns[(size_t)g] * (size_t)lds[(size_t)g] * 4;
        }
        const size_t per_set = offs[(size_t)count];
        const size_t total = per_set * (pred ? 2 : 1);  // distances [, predecessors]
        if (sc.mat) (void)hipFree(sc.mat);
        sc.mat = nullptr;
        if ((e = hipMalloc(&sc.mat, total)) != hipSuccess) return status_of(e);
        if ((e = hipMemsetAsync(sc.mat, 0, total, sc.st)) != hipSuccess) return status_of(e);
        std::vector<void *> ptrs((size_t)count);
        std::vector<int32_t *> preds((size_t)count, nullptr);
        for (int g = 0; g < count; ++g) {
            ptrs[(size_t)g] = static_cast<char *>(sc.mat) + offs[(size_t)g];
            if (pred)
                preds[(size_t)g] = reinterpret_cast<int32_t *>(static_cast<char *>(sc.mat) +
                                                               per_set + offs[(size_t)g]);
        }
        double best = 1e300;
        int best_tile = tiles[0];
        for (int t = 0; t < ntiles; ++t) {
            const int tile = tiles[t];
            // the candidate tile is installed for the bucket while it is timed
            // (batch plans read the table when they are built)
            int s = fw_plan_set(dtype, lo[k], hi[k], tile);
            if (s != FW_OK) return s;
            fw_batch_plan plan = nullptr;
            if (objective == 1) {
                s = fw_batch_plan_create(ptrs.data(), ns.data(), lds.data(), count, base,
                                         pred ? preds.data() : nullptr,
                                         pred ? lds.data() : nullptr, &plan);
                if (s != FW_OK) return s;
            }
            std::vector<double> times;
            for (int r = 0; r <= reps && s == FW_OK; ++r) {  // the first run is a warm-up
                if ((e = hipEventRecord(sc.e0, sc.st)) != hipSuccess) s = status_of(e);
                if (s == FW_OK)
                    s = objective == 0 ? solve_with_tile(sc.mat, base, n, ld, preds[0], ld, tile,
                                                         sc.st)
                                       : fw_batch_plan_launch(plan, 0, sc.st);
                if (s == FW_OK && (e = hipEventRecord(sc.e1, sc.st)) != hipSuccess)
                    s = status_of(e);
                if (s == FW_OK && (e = hipEventSynchronize(sc.e1)) != hipSuccess)
                    s = status_of(e);
                float ms = 0.f;
                if (s == FW_OK && (e = hipEventElapsedTime(&ms, sc.e0, sc.e1)) != hipSuccess)
                    s = status_of(e);
                if (s == FW_OK && r) times.push_back(ms);
            }
            if (plan) fw_batch_plan_destroy(plan);
            if (s != FW_OK) return s;
            const double med = median(times);
            if (ms_out) ms_out[(size_t)k * (size_t)ntiles + (size_t)t] = med;
            if (med < best) {
                best = med;
                best_tile = tile;
            }
        }
        tile_out[k] = best_tile;
        int s = fw_plan_set(dtype, lo[k], hi[k], best_tile);
        if (s != FW_OK) return s;
    }
    return FW_OK;
}

// Whole-batch tuning: the buckets' tiles interact inside one batch plan (each
// tile size is its own chain of stage launches, and the chains share the GPU
// through the plan's streams), so a bucket tuned alone can pick a tile that
// is slower for the batch.  Coordinate descent on the plan launch of a batch
// of the given sizes: in each pass, every bucket that holds some of the
// batch's graphs tries every tile with the others fixed and keeps the
// fastest, timing plan launches as the caller will run them (eager launches,
// or replays of the captured graph: the two can favour different tiles, as
// the graph's parallel branches are ordered by the runtime rather than by the
// order of enqueueing).  Zero matrices again (the sweep is data-oblivious).
extern "C" int fw_autotune_batch(int dtype, const int64_t *n, int64_t count, const int64_t *lo,
                                 const int64_t *hi, int nbuckets, int mode, int reps, int passes,
                                 int *tile_out, double *ms_out) {
    const int base = dtype & ~FW_PLAN_PRED;
    const bool pred = (dtype & FW_PLAN_PRED) != 0;
    if ((base != FW_F32 && base != FW_I32) || !n || count < 1 || count > (1 << 20) || !lo ||
        !hi || nbuckets < 1 || !tile_out || reps < 1 || passes < 1 || (mode != 0 && mode != 1))
        return FW_ERR_INVALID;
    for (int k = 0; k < nbuckets; ++k)
        if (lo[k] < 2 || hi[k] < lo[k] || hi[k] > 65536) return FW_ERR_INVALID;
    const int64_t max_n = fw_batched_max_n(base, pred ? 1 : 0);
    for (int64_t g = 0; g < count; ++g)
        if (n[g] < 0) return FW_ERR_INVALID;
        else if (n[g] > max_n) return FW_ERR_UNSUPPORTED;
    int tiles[8];
    const int ntiles = fw_plan_tiles(tiles, 8);
    TuneScratch sc;
    hipError_t e = hipStreamCreateWithFlags(&sc.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&sc.e0);
    if (e == hipSuccess) e = hipEventCreate(&sc.e1);
    if (e != hipSuccess) return status_of(e);
    // zero matrices of the batch's sizes (ld = n rounded up to 4) [and
    // predecessor matrices of the same shape]
    std::vector<int64_t> ns(n, n + count), lds((size_t)count);
    std::vector<size_t> offs((size_t)count + 1, 0);
    for (int64_t g = 0; g < count; ++g) {
        lds[(size_t)g] = std::max<int64_t>(4, (ns[(size_t)g] + 3) / 4 * 4);
        offs[(size_t)g + 1] = offs[(size_t)g] + (size_t)ns[(size_t)g] * (size_t)lds[(size_t)g] * 4;
    }
    const size_t per_set = std::max<size_t>(offs[(size_t)count], 16);
    const size_t total = per_set * (pred ? 2 : 1);
    if ((e = hipMalloc(&sc.mat, total)) != hipSuccess) return status_of(e);
    if ((e = hipMemsetAsync(sc.mat, 0, total, sc.st)) != hipSuccess) return status_of(e);
    std::vector<void *> ptrs((size_t)count);
    std::vector<int32_t *> preds((size_t)count, nullptr);
    for (int64_t g = 0; g < count; ++g) {
        ptrs[(size_t)g] = static_cast<char *>(sc.mat) + offs[(size_t)g];
        if (pred)
            preds[(size_t)g] =
                reinterpret_cast<int32_t *>(static_cast<char *>(sc.mat) + per_set + offs[(size_t)g]);
    }
    // the median time of one plan launch in `mode` with the table as it stands
    // (a graph launch replays the graph the first launch captured)
    auto time_batch = [&](double &out) -> int {
        fw_batch_plan plan = nullptr;
        int s = fw_batch_plan_create(ptrs.data(), ns.data(), lds.data(), count, base,
                                     pred ? preds.data() : nullptr, pred ? lds.data() : nullptr,
                                     &plan);
        if (s != FW_OK) return s;
        std::vector<double> times;
        for (int r = 0; r <= reps && s == FW_OK; ++r) {  // the first launch is a warm-up
            if ((e = hipEventRecord(sc.e0, sc.st)) != hipSuccess) s = status_of(e);
            if (s == FW_OK) s = fw_batch_plan_launch(plan, mode, sc.st);
            if (s == FW_OK && (e = hipEventRecord(sc.e1, sc.st)) != hipSuccess) s = status_of(e);
            if (s == FW_OK && (e = hipEventSynchronize(sc.e1)) != hipSuccess) s = status_of(e);
            float ms = 0.f;
            if (s == FW_OK && (e = hipEventElapsedTime(&ms, sc.e0, sc.e1)) != hipSuccess)
                s = status_of(e);
            if (s == FW_OK && r) times.push_back(ms);
        }
        fw_batch_plan_destroy(plan);
        out = median(times);
        return s;
    };
    for (int k = 0; k < nbuckets; ++k) {
        tile_out[k] = fw_plan_tile(dtype, (int64_t)std::llround(std::sqrt((double)lo[k] * hi[k])));
        if (ms_out)
            for (int t = 0; t < ntiles; ++t) ms_out[(size_t)k * (size_t)ntiles + (size_t)t] = 0.0;
    }
    for (int pass = 0; pass < passes; ++pass) {
        for (int k = 0; k < nbuckets; ++k) {
            const bool held = std::any_of(ns.begin(), ns.end(),
                                          [&](int64_t v) { return v >= lo[k] && v <= hi[k]; });
            if (!held) continue;  // no graph of this batch reads the bucket's tile
            double best = 1e300;
            int best_tile = tile_out[k];
            for (int t = 0; t < ntiles; ++t) {
                int s = fw_plan_set(dtype, lo[k], hi[k], tiles[t]);
                if (s != FW_OK) return s;
                double ms = 0.0;
                if ((s = time_batch(ms)) != FW_OK) return s;
                if (ms_out) ms_out[(size_t)k * (size_t)ntiles + (size_t)t] = ms;
                if (ms < best) {
                    best = ms;
                    best_tile = tiles[t];
                }
            }
            tile_out[k] = best_tile;
            int s = fw_plan_set(dtype, lo[k], hi[k], best_tile);
            if (s != FW_OK) return s;
        }
    }
    return FW_OK;
}
