// Autotuner for the plan table: for each size bucket, time every tile size on
// the device and install the fastest with fw_plan_set.
//
// Timing uses a matrix of zeros: the sweep is data-oblivious (section 1: the
// run time of Floyd-Warshall does not depend on the graph), so the timings
// hold for every input of that size.  Two objectives:
//   0  one single-graph solve of the bucket's representative size;
//   1  one persistent batched launch of `batch` graphs of that size (the
//      batched path's plan comes from the same table).
// The representative size is the geometric middle of the bucket.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/fwapsp.h"
#include "fw_internal.h"

namespace fw {
int solve_with_tile(void *d, int dtype, int n, int64_t ld, int tile, hipStream_t st);
}

using namespace fw;

namespace {

int status_of(hipError_t e) {
    if (e == hipSuccess) return FW_OK;
    if (e == hipErrorOutOfMemory) return FW_ERR_NOMEM;
    return FW_ERR_HIP;
}

struct TuneScratch {
    void *mat = nullptr;     // device matrices
    void *host_tab = nullptr;
    void *dev_tab = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneScratch() {
        if (st) hipStreamSynchronize(st);
        if (mat) hipFree(mat);
        if (dev_tab) hipFree(dev_tab);
        if (host_tab) hipHostFree(host_tab);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        if (st) hipStreamDestroy(st);
    }
};

double median(std::vector<double> v) {
    std::sort(v.begin(), v.end());
    return v.empty() ? 0.0 : v[v.size() / 2];
}

}  // namespace

extern "C" int fw_autotune(int dtype, const int64_t *lo, const int64_t *hi, int nbuckets,
                           int objective, int batch, int reps, int *tile_out, double *ms_out) {
    if ((dtype != FW_F32 && dtype != FW_I32) || !lo || !hi || nbuckets < 1 || !tile_out ||
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
        const size_t per = (size_t)n * (size_t)ld * 4;
        if (sc.mat) hipFree(sc.mat);
        sc.mat = nullptr;
        if ((e = hipMalloc(&sc.mat, per * (size_t)count)) != hipSuccess) return status_of(e);
        if ((e = hipMemsetAsync(sc.mat, 0, per * (size_t)count, sc.st)) != hipSuccess)
            return status_of(e);
        if (objective == 1) {
            const size_t tb = sizeof(BatchHeader) + sizeof(BatchItem) * (size_t)count;
            if (sc.host_tab) hipHostFree(sc.host_tab);
            if (sc.dev_tab) hipFree(sc.dev_tab);
            sc.host_tab = sc.dev_tab = nullptr;
            if ((e = hipHostMalloc(&sc.host_tab, tb, hipHostMallocDefault)) != hipSuccess)
                return status_of(e);
            if ((e = hipMalloc(&sc.dev_tab, tb)) != hipSuccess) return status_of(e);
        }
        double best = 1e300;
        int best_tile = tiles[0];
        for (int t = 0; t < ntiles; ++t) {
            const int tile = tiles[t];
            std::vector<double> times;
            for (int r = 0; r <= reps; ++r) {  // the first run is a warm-up
                const size_t tb = sizeof(BatchHeader) + sizeof(BatchItem) * (size_t)count;
                if (objective == 1) {
                    // the previous launch must be done before its table is rewritten
                    if ((e = hipStreamSynchronize(sc.st)) != hipSuccess) return status_of(e);
                    auto *hdr = static_cast<BatchHeader *>(sc.host_tab);
                    auto *items = reinterpret_cast<BatchItem *>(static_cast<char *>(sc.host_tab) +
                                                                sizeof(BatchHeader));
                    *hdr = BatchHeader{};
                    hdr->count = count;
                    for (int g = 0; g < count; ++g) {
                        fill_batch_item(items[g], static_cast<char *>(sc.mat) + per * (size_t)g,
                                        dtype, n, ld, nullptr, 0);
                        items[g].tile = tile;
                    }
                }
                if ((e = hipEventRecord(sc.e0, sc.st)) != hipSuccess) return status_of(e);
                if (objective == 0) {
                    int s = solve_with_tile(sc.mat, dtype, n, ld, tile, sc.st);
                    if (s != FW_OK) return s;
                } else {
                    if ((e = hipMemcpyAsync(sc.dev_tab, sc.host_tab, tb, hipMemcpyHostToDevice,
                                            sc.st)) != hipSuccess)
                        return status_of(e);
                    const int grid = std::min(count, batched_resident_grid(dtype, false));
                    if (grid <= 0) return FW_ERR_HIP;
                    e = launch_batched_raw(
                        dtype, false, static_cast<BatchHeader *>(sc.dev_tab),
                        reinterpret_cast<const BatchItem *>(static_cast<char *>(sc.dev_tab) +
                                                            sizeof(BatchHeader)),
                        grid, sc.st);
                    if (e != hipSuccess) return status_of(e);
                }
                if ((e = hipEventRecord(sc.e1, sc.st)) != hipSuccess) return status_of(e);
                if ((e = hipEventSynchronize(sc.e1)) != hipSuccess) return status_of(e);
                float ms = 0.f;
                if ((e = hipEventElapsedTime(&ms, sc.e0, sc.e1)) != hipSuccess) return status_of(e);
                if (r) times.push_back(ms);
            }
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
