// Batched solves: many independent graphs in one persistent launch.
//
// Each workgroup repeatedly takes the next graph from a device work counter
// (graphs are ordered largest first) and solves it alone:
//   * n <= tile: closure_tile over the whole graph -- the plain algorithm of
//     section 3.1 with one barrier per k-step;
//   * n >  tile: the blocked schedule of section 3.2 run inside the
//     workgroup (diagonal tile, panel tiles, bulk tiles, workgroup barriers
//     between the phases).
// The tile comes from the same plan table as single-graph solves and the
// per-cell work is the same code (fw_tiles.h), so a graph's bits do not
// depend on whether it was solved alone or in a batch.
//
// No workgroup ever waits for another one, so the grid always drains.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/fwapsp.h"
#include "fw_tiles.h"

namespace fw {

static_assert(sizeof(BatchHeader) == 64, "header keeps items 64-byte aligned");

namespace {

constexpr int kBatchThreads = 256;

template <typename T, bool PRED>
constexpr int batch_smem_bytes() {
    return product_smem_bytes<T, 128, 16, PRED>();
}

template <typename T, int S, int TMC, int TM, bool VEC, bool PRED>
__device__ void blocked_in_wg(T *d, int32_t *p, int n, int64_t ld, int64_t ldp, char *smem) {
    const int nb = (n + S - 1) / S;
    const int m = nb - 1;
    for (int b = 0; b < nb; ++b) {
        closure_tile<T, S, TMC, PRED>(d, p, n, ld, ldp, b * S, smem);
        if (m == 0) break;
        for (int t = 0; t < 2 * m; ++t) {
            int bi, bj;
            panel_coords(t, b, m, bi, bj);
            product_tile<T, S, 16, TM, TM, VEC, PRED>(d, p, n, ld, ldp, bi, bj, b, smem);
        }
        __syncthreads();  // panels complete before the bulk reads them
        for (int t = 0; t < m * m; ++t) {
            int bi, bj;
            bulk_coords(t, b, m, bi, bj);
            product_tile<T, S, 16, TM, TM, VEC, PRED>(d, p, n, ld, ldp, bi, bj, b, smem);
        }
        __syncthreads();  // the next diagonal tile reads this stage's bulk
    }
}

template <typename T, bool PRED>
__device__ void solve_graph(const BatchItem &it, char *smem) {
    T *d = static_cast<T *>(it.d);
    int32_t *p = PRED ? it.p : nullptr;
    const int n = it.n;
    const int64_t ld = it.ld, ldp = it.ldp;
    if constexpr (PRED) {
        for (int64_t c = threadIdx.x; c < (int64_t)n * n; c += kBatchThreads) {
            const int i = (int)(c / n), j = (int)(c - (int64_t)i * n);
            const T w = d[(int64_t)i * ld + j];
            p[(int64_t)i * ldp + j] = (i != j && !Ar<T>::absent(w)) ? i : kPredNone;
        }
        __syncthreads();
    }
    if (n > 1) {
        switch (it.tile) {
        case 32:
            blocked_in_wg<T, 32, 2, 2, false, PRED>(d, p, n, ld, ldp, smem);
            break;
        case 64:
            if (it.vec)
                blocked_in_wg<T, 64, 4, 4, true, PRED>(d, p, n, ld, ldp, smem);
            else
                blocked_in_wg<T, 64, 4, 4, false, PRED>(d, p, n, ld, ldp, smem);
            break;
        default:
            if (it.vec)
                blocked_in_wg<T, 128, 8, 8, true, PRED>(d, p, n, ld, ldp, smem);
            else
                blocked_in_wg<T, 128, 8, 8, false, PRED>(d, p, n, ld, ldp, smem);
            break;
        }
    }
    if constexpr (PRED) {
        for (int64_t c = threadIdx.x; c < (int64_t)n * n; c += kBatchThreads) {
            const int i = (int)(c / n), j = (int)(c - (int64_t)i * n);
            int32_t &q = p[(int64_t)i * ldp + j];
            if (i == j || q == kPredNone || Ar<T>::unreachable(d[(int64_t)i * ld + j])) q = -1;
        }
        __syncthreads();
    }
}

template <typename T, bool PRED>
__global__ void __launch_bounds__(kBatchThreads, PRED ? 2 : 3)
batched_kernel(BatchHeader *hdr, const BatchItem *items) {
    __shared__ __align__(16) char smem[batch_smem_bytes<T, PRED>()];
    __shared__ int cur;
    const int count = hdr->count;
    for (;;) {
        if (threadIdx.x == 0) cur = atomicAdd(&hdr->next, 1);
        __syncthreads();
        const int g = cur;
        __syncthreads();
        if (g >= count) break;
        const BatchItem it = items[g];
        if (PRED && it.p != nullptr)
            solve_graph<T, PRED>(it, smem);
        else
            solve_graph<T, false>(it, smem);
    }
}

int status_of(hipError_t e) {
    if (e == hipSuccess) return FW_OK;
    if (e == hipErrorOutOfMemory) return FW_ERR_NOMEM;
    return FW_ERR_HIP;
}

const void *kernel_ptr(int dtype, bool pred) {
    if (dtype == FW_F32)
        return pred ? (const void *)batched_kernel<float, true>
                    : (const void *)batched_kernel<float, false>;
    return pred ? (const void *)batched_kernel<int32_t, true>
                : (const void *)batched_kernel<int32_t, false>;
}

// Workgroups per CU of each batched kernel, per device.
std::mutex g_occ_mu;
std::map<std::pair<int, int>, int> g_grid;

int resident_grid(int dtype, bool pred) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    const int key2 = dtype * 2 + (pred ? 1 : 0);
    std::lock_guard<std::mutex> lk(g_occ_mu);
    auto it = g_grid.find({dev, key2});
    if (it != g_grid.end()) return it->second;
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel_ptr(dtype, pred), kBatchThreads,
                                                     0) != hipSuccess)
        return -1;
    const int grid = cus * std::max(per, 1);
    g_grid[{dev, key2}] = grid;
    return grid;
}

}  // namespace

int batched_resident_grid(int dtype, bool pred) { return resident_grid(dtype, pred); }

void fill_batch_item(BatchItem &it, void *d, int dtype, int64_t n, int64_t ld, int32_t *p,
                     int64_t ldp) {
    it.d = d;
    it.p = p;
    it.ld = ld;
    it.ldp = p ? ldp : 0;
    it.n = (int32_t)n;
    it.tile = n > 1 ? plan_tile_for(dtype, n) : 32;
    it.vec = vec_ok(d, ld) && (!p || vec_ok(p, ldp)) ? 1 : 0;
    it.pad = 0;
}

hipError_t launch_batched_raw(int dtype, bool pred, BatchHeader *hdr, const BatchItem *items,
                              int grid, hipStream_t st) {
    if (dtype == FW_F32) {
        if (pred)
            batched_kernel<float, true><<<grid, kBatchThreads, 0, st>>>(hdr, items);
        else
            batched_kernel<float, false><<<grid, kBatchThreads, 0, st>>>(hdr, items);
    } else {
        if (pred)
            batched_kernel<int32_t, true><<<grid, kBatchThreads, 0, st>>>(hdr, items);
        else
            batched_kernel<int32_t, false><<<grid, kBatchThreads, 0, st>>>(hdr, items);
    }
    return hipGetLastError();
}

// Defined in fw_api.cpp.
hipError_t timed_launch_batched(double updates, hipStream_t st, int dtype, bool pred,
                                BatchHeader *hdr, const BatchItem *items, int grid);

}  // namespace fw

using namespace fw;

// A batch plan: descriptor table in pinned host memory and on the device,
// plus, once launched through a graph, the captured graph.
struct fw_batch_plan_s {
    int dtype = 0;
    bool pred = false;
    int64_t count = 0;
    int grid = 0;
    int device = 0;
    double updates = 0;
    size_t bytes = 0;
    void *host = nullptr;   // BatchHeader + items (pinned)
    void *dev = nullptr;    // device copy
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int build_plan(void *const *d, const int64_t *n, const int64_t *ld, int64_t count, int dtype,
               int32_t *const *pred, const int64_t *ld_pred, fw_batch_plan_s *pl) {
    if (count < 0 || count > 0x7fffffffLL) return FW_ERR_INVALID;
    if (dtype != FW_F32 && dtype != FW_I32) return FW_ERR_INVALID;
    if (count > 0 && (!d || !n || !ld)) return FW_ERR_INVALID;
    if (pred && !ld_pred) return FW_ERR_INVALID;
    std::vector<BatchItem> items((size_t)count);
    bool any_pred = false;
    double upd = 0;
    for (int64_t g = 0; g < count; ++g) {
        int32_t *pg = pred ? pred[g] : nullptr;
        const int64_t ldp = pg ? ld_pred[g] : 0;
        int s = validate_matrix(d[g], dtype, n[g], ld[g], pg, ldp);
        if (s != FW_OK) return s;
        if (n[g] > fw_batched_max_n(dtype, pg != nullptr)) return FW_ERR_UNSUPPORTED;
        fill_batch_item(items[(size_t)g], d[g], dtype, n[g], ld[g], pg, ldp);
        any_pred |= pg != nullptr;
        upd += (double)n[g] * (double)n[g] * (double)n[g];
    }
    // largest graphs first: the workgroups that take them start earliest
    std::stable_sort(items.begin(), items.end(),
                     [](const BatchItem &a, const BatchItem &b) { return a.n > b.n; });
    pl->dtype = dtype;
    pl->pred = any_pred;
    pl->count = count;
    pl->updates = upd;
    pl->bytes = sizeof(BatchHeader) + sizeof(BatchItem) * (size_t)std::max<int64_t>(count, 1);
    if (hipGetDevice(&pl->device) != hipSuccess) return FW_ERR_HIP;
    const int grid = resident_grid(dtype, any_pred);
    if (grid <= 0) return FW_ERR_HIP;
    pl->grid = (int)std::min<int64_t>(grid, std::max<int64_t>(count, 1));
    if (hipHostMalloc(&pl->host, pl->bytes, hipHostMallocDefault) != hipSuccess)
        return FW_ERR_NOMEM;
    if (hipMalloc(&pl->dev, pl->bytes) != hipSuccess) return FW_ERR_NOMEM;
    auto *hdr = static_cast<BatchHeader *>(pl->host);
    *hdr = BatchHeader{};
    hdr->next = 0;
    hdr->count = (int32_t)count;
    if (count)
        std::copy(items.begin(), items.end(),
                  reinterpret_cast<BatchItem *>(static_cast<char *>(pl->host) + sizeof(BatchHeader)));
    return FW_OK;
}

// Enqueue: refresh the device table (which also resets the work counter) and
// launch the persistent kernel.  Both are plain stream operations, so the
// same sequence can be captured into a graph.
int enqueue_plan(fw_batch_plan_s *pl, hipStream_t st, bool capturing) {
    if (pl->count == 0) return FW_OK;
    hipError_t e = hipMemcpyAsync(pl->dev, pl->host, pl->bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return status_of(e);
    auto *hdr = static_cast<BatchHeader *>(pl->dev);
    auto *items =
        reinterpret_cast<const BatchItem *>(static_cast<char *>(pl->dev) + sizeof(BatchHeader));
    if (capturing)
        return status_of(launch_batched_raw(pl->dtype, pl->pred, hdr, items, pl->grid, st));
    return status_of(
        timed_launch_batched(pl->updates, st, pl->dtype, pl->pred, hdr, items, pl->grid));
}

void free_plan(fw_batch_plan_s *pl) {
    if (pl->exec) hipGraphExecDestroy(pl->exec);
    if (pl->graph) hipGraphDestroy(pl->graph);
    if (pl->cap_stream) hipStreamDestroy(pl->cap_stream);
    if (pl->dev) hipFree(pl->dev);
    if (pl->host) hipHostFree(pl->host);
    delete pl;
}

// One-shot calls keep their plan until the stream has passed the launch.
struct Pending {
    fw_batch_plan_s *plan;
    hipEvent_t done;
};
std::mutex g_pending_mu;
std::vector<Pending> g_pending;

void reap_pending(bool all) {
    std::vector<Pending> keep;
    std::vector<Pending> drop;
    {
        std::lock_guard<std::mutex> lk(g_pending_mu);
        for (auto &p : g_pending) {
            if (all || hipEventQuery(p.done) == hipSuccess)
                drop.push_back(p);
            else
                keep.push_back(p);
        }
        g_pending.swap(keep);
    }
    for (auto &p : drop) {
        hipEventSynchronize(p.done);
        hipEventDestroy(p.done);
        free_plan(p.plan);
    }
}

}  // namespace

extern "C" {

int64_t fw_batched_max_n(int dtype, int with_pred) {
    (void)with_pred;
    if (dtype != FW_F32 && dtype != FW_I32) return -1;
    return 8192;
}

int fw_batch_plan_create(void *const *d, const int64_t *n, const int64_t *ld, int64_t count,
                         int dtype, int32_t *const *pred, const int64_t *ld_pred,
                         fw_batch_plan *out) {
    if (!out) return FW_ERR_INVALID;
    *out = nullptr;
    auto *pl = new fw_batch_plan_s();
    int s = build_plan(d, n, ld, count, dtype, pred, ld_pred, pl);
    if (s != FW_OK) {
        free_plan(pl);
        return s;
    }
    *out = pl;
    return FW_OK;
}

int fw_batch_plan_launch(fw_batch_plan plan, int mode, void *stream) {
    if (!plan || mode < 0 || mode > 2) return FW_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    if (mode == 2) {
        // baseline: every graph through the single-graph stage loop
        const auto *items = reinterpret_cast<const BatchItem *>(static_cast<char *>(plan->host) +
                                                                sizeof(BatchHeader));
        for (int64_t g = 0; g < plan->count; ++g) {
            const BatchItem &it = items[g];
            int s = solve_single(it.d, plan->dtype, it.n, it.ld, it.p, it.ldp, st);
            if (s != FW_OK) return s;
        }
        return FW_OK;
    }
    if (mode == 0 || plan->count == 0) return enqueue_plan(plan, st, false);
    if (!plan->exec) {
        hipError_t e = hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return status_of(e);
        e = hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return status_of(e);
        int s = enqueue_plan(plan, plan->cap_stream, true);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(plan->cap_stream, &g);
        if (s != FW_OK) {
            if (g) hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return status_of(e);
        plan->graph = g;
        e = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) return status_of(e);
    }
    return status_of(hipGraphLaunch(plan->exec, st));
}

int fw_batch_plan_destroy(fw_batch_plan plan) {
    if (!plan) return FW_ERR_INVALID;
    hipDeviceSynchronize();
    free_plan(plan);
    return FW_OK;
}

int64_t fw_batch_plan_grid(fw_batch_plan plan) { return plan ? plan->grid : -1; }

int fw_apsp_batched(void *const *d, const int64_t *n, const int64_t *ld, int64_t count, int dtype,
                    int32_t *const *pred, const int64_t *ld_pred, void *stream) {
    if (count == 0) {
        if (dtype != FW_F32 && dtype != FW_I32) return FW_ERR_INVALID;
        return FW_OK;
    }
    reap_pending(false);
    fw_batch_plan_s *pl = new fw_batch_plan_s();
    int s = build_plan(d, n, ld, count, dtype, pred, ld_pred, pl);
    if (s != FW_OK) {
        free_plan(pl);
        return s;
    }
    hipStream_t st = (hipStream_t)stream;
    s = enqueue_plan(pl, st, false);
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ev, st) != hipSuccess) {
        hipStreamSynchronize(st);
        if (ev) hipEventDestroy(ev);
        free_plan(pl);
        return s != FW_OK ? s : FW_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(g_pending_mu);
    g_pending.push_back({pl, ev});
    return s;
}

}  // extern "C"
