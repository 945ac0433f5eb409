// Ablation ladder: the rungs of the paper's Table 1 comparison, rebuilt as
// in-house gfx950 kernels, so the effect of each design step can be measured
// on this chip.  Every rung computes the same distances (exact arithmetic,
// see fw_tiles.h), so each is checked bit for bit against the plain loop.
//
//   rung 0  one launch per k, one thread per cell: the direct parallel form
//           of Fig. FW-Alg (section 3.1's task-per-thread approach);
//   rung 1  the blocked schedule of section 3.2 with 32 x 32 tiles, all the
//           tiles a phase needs held in LDS, one cell per thread (1024
//           threads), the diagonal and panel phases k-ordered with a barrier
//           per step;
//   rung 2  64 x 64 tiles, 4 x 4 cells per thread in registers with two
//           k-steps fused into a three-input minimum, the whole A and B tiles
//           in LDS (64 KB per workgroup);
//   rung 3  the same with the operands staged through LDS in 16-deep k-slices
//           (16 KB per workgroup): the library's tile-64 path;
//   rung 4  the library's 128-wide path (direct global->LDS slice copies,
//           8 x 8 cells per thread, strip panels, the next diagonal closed in
//           the bulk), which the plan table picks for large solves.
#include <hip/hip_runtime.h>

#include "../../include/fwapsp.h"
#include "fw_tiles.h"

namespace fw {
int solve_with_tile(void *d, int dtype, int n, int64_t ld, int32_t *pred, int64_t ldp, int tile,
                    hipStream_t st);

namespace {

// ---------------------------------------------------------------------------
// Rung 0: d_ij <- min(d_ij, d_ik + d_kj) for one k over the whole matrix.
// Row k and column k do not change in iteration k (d_kk >= 0), so the cells
// of one launch are independent.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
per_k_kernel(T *__restrict__ d, int n, int64_t ld, int k) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const T dkj = d[(int64_t)k * ld + j];
    for (int i = blockIdx.y; i < n; i += gridDim.y) {
        T *row = d + (int64_t)i * ld;
        const T cand = Ar<T>::add(row[k], dkj);
        if (cand < row[j]) row[j] = cand;
    }
}

// ---------------------------------------------------------------------------
// Rung 1: 32 x 32 tiles, one cell per thread, tiles in LDS.
// ---------------------------------------------------------------------------
constexpr int kS1 = 32;

template <typename T>
__device__ __forceinline__ T ld_cell(const T *d, int n, int64_t ld, int i, int j) {
    return (i < n && j < n) ? d[(int64_t)i * ld + j] : Ar<T>::inf();
}

// Diagonal tile (b, b): k-ordered, two barriers per step (read, then write).
template <typename T>
__global__ void __launch_bounds__(kS1 *kS1)
kk_diag_kernel(T *__restrict__ d, int n, int64_t ld, int b) {
    __shared__ T t[kS1][kS1 + 1];
    const int tx = threadIdx.x % kS1, ty = threadIdx.x / kS1;
    const int i = b * kS1 + ty, j = b * kS1 + tx;
    t[ty][tx] = ld_cell(d, n, ld, i, j);
    __syncthreads();
    for (int k = 0; k < kS1; ++k) {
        const T cand = Ar<T>::add(t[ty][k], t[k][tx]);
        __syncthreads();
        if (cand < t[ty][tx]) t[ty][tx] = cand;
        __syncthreads();
    }
    if (i < n && j < n) d[(int64_t)i * ld + j] = t[ty][tx];
}

// Panel tiles of stage b (blockIdx.x < m: row panel (b, j), else column panel
// (i, b)): the singly dependent update, k-ordered as in Fig. BFW-Alg, with the
// finished diagonal tile and the panel tile in LDS.
template <typename T>
__global__ void __launch_bounds__(kS1 *kS1)
kk_panel_kernel(T *__restrict__ d, int n, int64_t ld, int b, int nb) {
    __shared__ T dg[kS1][kS1 + 1];
    __shared__ T p[kS1][kS1 + 1];
    int bi, bj;
    panel_coords(blockIdx.x, b, nb - 1, bi, bj);
    const bool row_panel = bi == b;
    const int tx = threadIdx.x % kS1, ty = threadIdx.x / kS1;
    dg[ty][tx] = ld_cell(d, n, ld, b * kS1 + ty, b * kS1 + tx);
    const int i = bi * kS1 + ty, j = bj * kS1 + tx;
    p[ty][tx] = ld_cell(d, n, ld, i, j);
    __syncthreads();
    for (int k = 0; k < kS1; ++k) {
        // row panel: d_ij <- min(d_ij, D_ik + P_kj); column: P_ik + D_kj
        const T cand = row_panel ? Ar<T>::add(dg[ty][k], p[k][tx]) : Ar<T>::add(p[ty][k], dg[k][tx]);
        __syncthreads();
        if (cand < p[ty][tx]) p[ty][tx] = cand;
        __syncthreads();
    }
    if (i < n && j < n) d[(int64_t)i * ld + j] = p[ty][tx];
}

// Bulk tiles of stage b: the cell, the column-panel tile and the row-panel
// tile in LDS, the cell's value in a register; no barrier in the k loop.
template <typename T>
__global__ void __launch_bounds__(kS1 *kS1)
kk_bulk_kernel(T *__restrict__ d, int n, int64_t ld, int b, int nb) {
    __shared__ T a[kS1][kS1 + 1];
    __shared__ T bt[kS1][kS1 + 1];
    int bi, bj;
    bulk_coords(blockIdx.x, b, nb - 1, bi, bj);
    const int tx = threadIdx.x % kS1, ty = threadIdx.x / kS1;
    const int i = bi * kS1 + ty, j = bj * kS1 + tx;
    a[ty][tx] = ld_cell(d, n, ld, i, b * kS1 + tx);
    bt[ty][tx] = ld_cell(d, n, ld, b * kS1 + ty, j);
    T c = ld_cell(d, n, ld, i, j);
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < kS1; ++k) c = Ar<T>::min2(c, Ar<T>::add(a[ty][k], bt[k][tx]));
    if (i < n && j < n) d[(int64_t)i * ld + j] = c;
}

// ---------------------------------------------------------------------------
// Rung 2: 64 x 64 tiles, 4 x 4 register sub-tiles, whole operand tiles in LDS
// (product_tile with one 64-deep slice).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
whole_diag_kernel(T *__restrict__ d, int n, int64_t ld, int b) {
    __shared__ __align__(16) char smem[closure_smem_bytes<T, 64, false>()];
    closure_tile<T, 64, 4, false>(d, nullptr, n, ld, 0, b * 64, smem);
}

template <typename T, bool VEC>
__global__ void __launch_bounds__(256)
whole_tile_kernel(T *__restrict__ d, int n, int64_t ld, int b, int nb, int mode) {
    extern __shared__ __align__(16) char smem_dyn[];
    int bi, bj;
    if (mode == 0)
        panel_coords(blockIdx.x, b, nb - 1, bi, bj);
    else
        bulk_coords(blockIdx.x, b, nb - 1, bi, bj);
    product_tile<T, 64, 64, 4, 4, VEC, false>(d, nullptr, n, ld, 0, bi, bj, b, smem_dyn);
}

template <typename T, bool VEC>
hipError_t whole_tiles(T *d, int n, int64_t ld, int b, int nb, hipStream_t st) {
    constexpr size_t smem = product_smem_bytes<T, 64, 64, false>();  // 64 KB
    const int m = nb - 1;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&whole_tile_kernel<T, VEC>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    whole_tile_kernel<T, VEC><<<2 * m, 256, smem, st>>>(d, n, ld, b, nb, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    whole_tile_kernel<T, VEC><<<m * m, 256, smem, st>>>(d, n, ld, b, nb, 1);
    return hipGetLastError();
}

int status_of(hipError_t e) {
    if (e == hipSuccess) return FW_OK;
    if (e == hipErrorOutOfMemory) return FW_ERR_NOMEM;
    return FW_ERR_HIP;
}

template <typename T>
hipError_t run_rung(int rung, T *d, int n, int64_t ld, hipStream_t st) {
    if (rung == 0) {
        const dim3 grid((n + 255) / 256, n < 16384 ? n : 16384);
        for (int k = 0; k < n; ++k) {
            per_k_kernel<T><<<grid, 256, 0, st>>>(d, n, ld, k);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const int s = rung == 1 ? kS1 : 64;
    const int nb = (n + s - 1) / s, m = nb - 1;
    const bool vec = vec_ok(d, ld);
    for (int b = 0; b < nb; ++b) {
        hipError_t e;
        if (rung == 1) {
            kk_diag_kernel<T><<<1, kS1 * kS1, 0, st>>>(d, n, ld, b);
            if (m > 0) {
                kk_panel_kernel<T><<<2 * m, kS1 * kS1, 0, st>>>(d, n, ld, b, nb);
                kk_bulk_kernel<T><<<m * m, kS1 * kS1, 0, st>>>(d, n, ld, b, nb);
            }
            e = hipGetLastError();
        } else {
            whole_diag_kernel<T><<<1, 256, 0, st>>>(d, n, ld, b);
            e = hipGetLastError();
            if (e == hipSuccess && m > 0)
                e = vec ? whole_tiles<T, true>(d, n, ld, b, nb, st)
                        : whole_tiles<T, false>(d, n, ld, b, nb, st);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace
}  // namespace fw

using namespace fw;

extern "C" int fw_apsp_ladder(void *d, int dtype, int64_t n, int64_t ld, int rung, void *stream) {
    if (rung < 0 || rung > 4) return FW_ERR_INVALID;
    const int s = validate_matrix(d, dtype, n, ld, nullptr, 0);
    if (s != FW_OK) return s;
    if (n > 65536 || (int64_t)(n + 255) / 256 > 0x7fffffffLL) return FW_ERR_UNSUPPORTED;
    if (n <= 1) return FW_OK;
    hipStream_t st = (hipStream_t)stream;
    if (rung == 3) return solve_with_tile(d, dtype, (int)n, ld, nullptr, 0, 64, st);
    if (rung == 4) return solve_with_tile(d, dtype, (int)n, ld, nullptr, 0, 128, st);
    if (dtype == FW_F32) return status_of(run_rung<float>(rung, (float *)d, (int)n, ld, st));
    return status_of(run_rung<int32_t>(rung, (int32_t *)d, (int)n, ld, st));
}
