// Batched solves: many independent graphs in one batch plan.
//
// Graphs of FW_STAGED_MIN_N vertices and more are stage-batched: per tile
// size, each stage b of the blocked schedule (section 3.2) is a few launches
// shared by every graph that has a stage b -- all their diagonal tiles, all
// their panel tiles, all their bulk tiles -- so a large graph is spread over
// the whole GPU instead of one workgroup.  Where the bulk kernel has the
// closure's geometry, the workgroup of bulk tile (b+1, b+1) also closes it,
// and stages after the first need no diagonal launch; aligned tile-128 graphs
// without predecessors run their panels and bulk on a direct-copy tile
// (staged_tile_dma) and keep a diagonal launch per stage.  The tile groups and
// the persistent part below depend on nothing in each other and run on two
// streams of the plan.  The smaller graphs go through one
// persistent launch in which each workgroup repeatedly takes the next graph
// from a device work counter (largest first) and solves it alone:
//   * n <= tile: the diagonal closure over the whole graph -- the plain
//     algorithm of section 3.1;
//   * n >  tile: the blocked schedule run inside the workgroup (diagonal
//     tile, panel tiles, bulk tiles, workgroup barriers between the phases).
// The tile comes from the same plan table as single-graph solves, and every
// cell takes the same candidates in the same order as there (the same code
// from fw_tiles.h, or staged_tile_dma's same sums), so a graph's bits do not
// depend on whether it was solved alone or in a batch.
//
// No workgroup ever waits for another one, so every grid drains.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/fwapsp.h"
#include "fw_tiles.h"

namespace fw {

static_assert(sizeof(BatchHeader) == 64, "header keeps items 64-byte aligned");

namespace {

constexpr int kBatchThreads = 256;

// The graphs' matrices are reached through pointers read from the plan's
// tables, which the compiler must treat as generic (flat) addresses; flat
// loads also count against the LDS wait counter, so a wait for an LDS read
// also waits for the global prefetch in flight.  Converting through an
// integer to the global address space lets the compiler emit global loads
// (a plain cast pair would be folded away).
template <typename T>
__device__ __forceinline__ T *as_global(T *p) {
    auto *g = (__attribute__((address_space(1))) T *)(uintptr_t)p;
    return (T *)g;
}

// Sets a persistent launch's work counter to 0 before the launch.
__global__ void batch_reset_kernel(BatchHeader *hdr) {
    if (threadIdx.x == 0) hdr->next = 0;
}

// LDS of the persistent kernel whose largest tile is MAXS.
template <typename T, bool PRED, int MAXS>
constexpr int batch_smem_bytes() {
    return product_smem_bytes<T, MAXS, 16, PRED>();
}

template <typename T, int S, int TMC, int TM, bool VEC, bool PRED>
__device__ void blocked_in_wg(T *d, int32_t *p, int n, int64_t ld, int64_t ldp, char *smem) {
    d = as_global(d);
    p = as_global(p);
    const int nb = (n + S - 1) / S;
    const int m = nb - 1;
    for (int b = 0; b < nb; ++b) {
        closure_tile_any<T, S, TMC, PRED>(d, p, n, ld, ldp, b * S, smem);
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

template <typename T, bool PRED, int MAXS>
__device__ void solve_graph(const BatchItem &it, char *smem) {
    T *d = as_global(static_cast<T *>(it.d));
    int32_t *p = PRED ? as_global(it.p) : nullptr;
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
            if constexpr (MAXS == 128) {
                if (it.vec)
                    blocked_in_wg<T, 128, 8, 8, true, PRED>(d, p, n, ld, ldp, smem);
                else
                    blocked_in_wg<T, 128, 8, 8, false, PRED>(d, p, n, ld, ldp, smem);
            }
            break;
        }
    }
    if constexpr (PRED) {
        for (int64_t c = threadIdx.x; c < (int64_t)n * n; c += kBatchThreads) {
            const int i = (int)(c / n), j = (int)(c - (int64_t)i * n);
            int32_t &q = p[(int64_t)i * ldp + j];
            q = final_pred<T>(i, j, d[(int64_t)i * ld + j], q);
        }
        __syncthreads();
    }
}

// MAXS: the largest tile among the graphs of the launch.  Without the
// 128-wide path the kernel needs under 100 VGPRs, so more workgroups share a
// CU.
template <typename T, bool PRED, int MAXS>
__global__ void __launch_bounds__(kBatchThreads, PRED ? 2 : (MAXS == 128 ? 3 : 5))
batched_kernel(BatchHeader *hdr, const BatchItem *items) {
    __shared__ __align__(16) char smem[batch_smem_bytes<T, PRED, MAXS>()];
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
            solve_graph<T, PRED, MAXS>(it, smem);
        else
            solve_graph<T, false, MAXS>(it, smem);
    }
}

// ---------------------------------------------------------------------------
// Stage-batched graphs.  Graphs above a size threshold are not solved by one
// workgroup each: their stages run as launches shared by every such graph of
// one tile size -- for each k-block b, one launch of all diagonal tiles, one
// of all panel tiles and one of all bulk tiles of the graphs that still have
// a stage b (kernel boundaries order the phases, as in a single solve); the
// diagonal launch of stage b > 0 is folded into stage b-1's bulk launch where
// the kernels allow it (staged_can_close), and stays a launch of its own for
// the direct-copy tile-128 path.  A
// launch's workgroups are listed in a table of (graph, tile number) pairs,
// built on the host when the plan is created.
// ---------------------------------------------------------------------------
enum StagedKind { kStagedDiag = 0, kStagedPanel = 1, kStagedBulk = 2, kStagedPredInit = 3,
                  kStagedPredFix = 4, kStagedBulkDma = 5, kStagedPanelDma = 6 };

struct StagedWork {
    int32_t item;   // index into the plan's item array
    int32_t local;  // tile number within the phase (panel_coords / bulk_coords),
                    // | kStagedClose: after the bulk tile (b+1, b+1), close it
};
// Set on the bulk entry of tile (b+1, b+1) when the tile size's kernel has
// the closure's geometry: that workgroup then closes the next stage's
// diagonal tile and the graph needs no diagonal launch for stage b+1.
constexpr int32_t kStagedClose = 0x40000000;

template <typename T, int S, bool PRED>
constexpr bool staged_can_close();

template <typename T, int S, int BK, int TM, int TN, bool VEC, bool PRED>
__device__ void staged_product(const BatchItem &it, int kind, int b, int local, char *smem) {
    T *d = as_global(static_cast<T *>(it.d));
    int32_t *p = PRED ? as_global(it.p) : nullptr;
    const int m = (it.n + S - 1) / S - 1;
    int bi, bj;
    if (kind == kStagedPanel)
        panel_coords(local, b, m, bi, bj);
    else
        bulk_coords(local, b, m, bi, bj);
    product_tile<T, S, BK, TM, TN, VEC, PRED>(d, p, it.n, it.ld, it.ldp, bi, bj, b, smem);
}

// Panels, bulk and predecessor set-up / fix-up of many graphs of tile size S.
// Kinds 3-4 take one workgroup per graph.  Geometry: TM x TM sub-tiles over
// (S/TM)^2 threads, with 4 x 4 over 1024 threads for predecessors at tile
// 128 (as in single solves); the minimum waves per SIMD follow the register
// footprint of each form.
#ifndef FW_STAGED64_TM
#define FW_STAGED64_TM 4
#endif
#ifndef FW_STAGED64_TN
#define FW_STAGED64_TN 4
#endif
#ifndef FW_STAGED64_BK
#define FW_STAGED64_BK 16
#endif
#ifndef FW_STAGED64_WAVES
#define FW_STAGED64_WAVES 6
#endif
template <typename T, int S, bool PRED>
constexpr int staged_tm() {
    return S == 32 ? 2 : S == 64 ? (PRED ? 4 : FW_STAGED64_TM) : (PRED ? 4 : 8);
}
template <typename T, int S, bool PRED>
constexpr int staged_bk() {
    return (PRED && S == 128) ? 32 : (!PRED && S == 64) ? FW_STAGED64_BK : 16;
}
template <typename T, int S, bool PRED>
constexpr int staged_tn() {
    return (S == 64 && !PRED) ? FW_STAGED64_TN : staged_tm<T, S, PRED>();
}
template <typename T, int S, bool PRED>
constexpr int staged_threads() {
    return (S / staged_tm<T, S, PRED>()) * (S / staged_tn<T, S, PRED>());
}
template <typename T, int S, bool PRED>
constexpr int staged_waves() {
    return PRED ? (S == 64 ? 3 : 2)
                : S == 32 ? 8
                : S == 64 ? (staged_tm<T, S, PRED>() * staged_tn<T, S, PRED>() >= 32 ? 4
                                                                                     : FW_STAGED64_WAVES)
                          : 3;
}
template <typename T, int S, bool PRED>
__global__ void __launch_bounds__((staged_threads<T, S, PRED>()), (staged_waves<T, S, PRED>()))
staged_kernel(const BatchItem *items, const StagedWork *work, int kind, int b) {
    constexpr int BK = staged_bk<T, S, PRED>();
    constexpr int NT = staged_threads<T, S, PRED>();
    __shared__ __align__(16) char smem[product_smem_bytes<T, S, BK, PRED>()];
    const StagedWork w = work[blockIdx.x];
    const BatchItem it = items[w.item];
    if (kind == kStagedPredInit || kind == kStagedPredFix) {
        if constexpr (PRED) {
            T *d = as_global(static_cast<T *>(it.d));
            const int n = it.n;
            for (int64_t c = threadIdx.x; c < (int64_t)n * n; c += NT) {
                const int i = (int)(c / n), j = (int)(c - (int64_t)i * n);
                const T v = d[(int64_t)i * it.ld + j];
                int32_t &q = as_global(it.p)[(int64_t)i * it.ldp + j];
                if (kind == kStagedPredInit)
                    q = (i != j && !Ar<T>::absent(v)) ? i : kPredNone;
                else
                    q = final_pred<T>(i, j, v, q);
            }
        }
        return;
    }
    constexpr int TM = staged_tm<T, S, PRED>(), TN = staged_tn<T, S, PRED>();
    constexpr bool V = S != 32;  // 2 x 2 sub-tiles at tile 32 are loaded element-wise
    const int local = w.local & ~kStagedClose;
    const bool with_pred = PRED && it.p != nullptr;
    if (with_pred) {
        if (V && it.vec)
            staged_product<T, S, BK, TM, TN, V, PRED>(it, kind, b, local, smem);
        else
            staged_product<T, S, BK, TM, TN, false, PRED>(it, kind, b, local, smem);
    } else {
        // a graph without predecessors in a plan with some: same geometry
        if (V && it.vec)
            staged_product<T, S, BK, TM, TN, V, false>(it, kind, b, local, smem);
        else
            staged_product<T, S, BK, TM, TN, false, false>(it, kind, b, local, smem);
    }
    if constexpr (staged_can_close<T, S, PRED>()) {
        static_assert(product_smem_bytes<T, S, BK, PRED>() >= closure_smem_bytes<T, S, PRED>() &&
                          product_smem_bytes<T, S, BK, PRED>() >= closure_smem_bytes<T, S, false>(),
                      "closure scratch must fit the product's LDS");
        if (w.local & kStagedClose) {
            __syncthreads();  // the tile's stores before its reloads
            T *d = as_global(static_cast<T *>(it.d));
            if (with_pred)
                closure_tile<T, S, TM, PRED>(d, as_global(it.p), it.n, it.ld, it.ldp, (b + 1) * S, smem);
            else
                closure_tile_any<T, S, TM, false>(d, nullptr, it.n, it.ld, 0, (b + 1) * S, smem);
        }
    }
}

// Tile sizes whose panel/bulk kernel has the closure's geometry (TM x TM
// cells over (S/TM)^2 threads): 32 and 64, and 128 with predecessors.
template <typename T, int S, bool PRED>
constexpr bool staged_can_close() {
    return staged_tm<T, S, PRED>() == staged_tn<T, S, PRED>() && (S <= 64 || PRED);
}

// Diagonal tiles of stage b of many graphs: (S / TMC)^2 threads, the
// geometry of the single-graph phase-1 kernel.
template <int S>
constexpr int staged_diag_tm() {
    return S == 32 ? 2 : 4;
}
template <typename T, int S, bool PRED>
__global__ void __launch_bounds__((S / staged_diag_tm<S>()) * (S / staged_diag_tm<S>()))
staged_diag_kernel(const BatchItem *items, const StagedWork *work, int b) {
    // a plan with predecessors may hold graphs without: room for both forms
    constexpr int kSmem = closure_smem_bytes<T, S, PRED>() > closure_smem_bytes<T, S, false>()
                              ? closure_smem_bytes<T, S, PRED>()
                              : closure_smem_bytes<T, S, false>();
    __shared__ __align__(16) char smem[kSmem];
    const BatchItem it = items[work[blockIdx.x].item];
    T *d = as_global(static_cast<T *>(it.d));
    if (PRED && it.p != nullptr)
        closure_tile<T, S, staged_diag_tm<S>(), PRED>(d, as_global(it.p), it.n, it.ld, it.ldp, b * S, smem);
    else
        closure_tile_any<T, S, staged_diag_tm<S>(), false>(d, nullptr, it.n, it.ld, 0, b * S, smem);
}

// ---------------------------------------------------------------------------
// Bulk tiles of tile-128 graphs without predecessors whose rows are 16-byte
// aligned, edge tiles included: the single-graph bulk's 128 x 128 tile with
// 16-deep k-slices copied global->LDS directly (the same LDS layout, thread
// geometry and candidates as bulk_tile_dma), generalised to tiles that reach
// past the graph's last row, column or k.  Every copy source is clamped into
// the graph -- rows and k-rows to n-1, 16-byte chunks to the one holding
// column n-1, which lies inside the row's ld -- so the clamps are identities
// inside the matrix and each copy reads the graph's own rows.  The k loop
// stops at the last valid k (a single step when an odd count remains); C
// cells outside the graph are neither loaded nor stored, so rows and columns
// beyond n compute values from clamped operands that are never stored, and
// every valid cell gets exactly the candidates of the full form.  Element
// offsets from the graph's base are 32-bit (n * ld < 2^31).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void staged_tile_dma(T *__restrict__ d, int n, int64_t ld, int bi,
                                                int bj, int b) {
    constexpr int S = 128, BK = 16, TM = 8, NS = S / BK;
    __shared__ __align__(16) T A0[S * BK];
    __shared__ __align__(16) T A1[S * BK];
    __shared__ __align__(16) T B0[BK * S];
    __shared__ __align__(16) T B1[BK * S];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tx = tid & 15, ty = tid >> 4;
    const int row0 = bi * S, col0 = bj * S, k0 = b * S;
    const bool inside = row0 + S <= n && col0 + S <= n && k0 + S <= n;  // uniform

    // thread (tx, ty): rows 8*ty .. 8*ty + 7, column groups 4*tx and 64 + 4*tx
    T acc[TM][TM];
    if (inside) {
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const T *row = d + (int64_t)(row0 + ty * TM + i) * ld + col0 + tx * 4;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const typename Vec4<T>::type x =
                    *reinterpret_cast<const typename Vec4<T>::type *>(row + h * 64);
                acc[i][4 * h] = x[0];
                acc[i][4 * h + 1] = x[1];
                acc[i][4 * h + 2] = x[2];
                acc[i][4 * h + 3] = x[3];
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int gi = row0 + ty * TM + i;
#pragma unroll
            for (int e = 0; e < TM; ++e) {
                const int gj = col0 + tx * 4 + (e >> 2) * 64 + (e & 3);
                acc[i][e] = (gi < n && gj < n) ? d[(int64_t)gi * ld + gj] : Ar<T>::inf();
            }
        }
    }

    // copy sources: the wave copies A rows 32*wave + lane/4 (and +16), its
    // 16-byte chunk c at LDS position c ^ ((row / 8) % 4), and B k-rows
    // 4*wave + lane/32 (and +2), 16-byte chunk lane % 32
    const int last = n - 1, cap = (n + 3) / 4 * 4 - 4;
    const uint32_t ldu = (uint32_t)ld;
    const int ar = wave * 32 + (lane >> 2);
    const uint32_t a_row0 = (uint32_t)min(row0 + ar, last) * ldu;
    const uint32_t a_row1 = (uint32_t)min(row0 + ar + 16, last) * ldu;
    const int a_c0 = ((lane & 3) ^ ((ar >> 3) & 3)) << 2;
    const int a_c1 = ((lane & 3) ^ (((ar + 16) >> 3) & 3)) << 2;
    const uint32_t b_col = (uint32_t)min(col0 + ((lane & 31) << 2), cap);
    const int b_r = wave * 4 + (lane >> 5);
    auto issue = [&](int s, T *Ad, T *Bd) {
        const int kc = k0 + s * BK;
        T *a = Ad + wave * 32 * BK;
        T *bb = Bd + wave * 4 * S;
        __builtin_amdgcn_global_load_lds(d + (a_row0 + (uint32_t)min(kc + a_c0, cap)),
                                         (lds_void_t *)a, 16, 0, 0);
        __builtin_amdgcn_global_load_lds(d + (a_row1 + (uint32_t)min(kc + a_c1, cap)),
                                         (lds_void_t *)(a + 16 * BK), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(d + ((uint32_t)min(kc + b_r, last) * ldu + b_col),
                                         (lds_void_t *)bb, 16, 0, 0);
        __builtin_amdgcn_global_load_lds(d + ((uint32_t)min(kc + b_r + 2, last) * ldu + b_col),
                                         (lds_void_t *)(bb + 2 * S), 16, 0, 0);
    };
    // a wave whose 32 rows all lie beyond the graph skips the arithmetic (it
    // still copies its share of every slice and meets every barrier)
    const bool idle = row0 + wave * 32 >= n;
    // kl: the slice's valid k count
    auto compute = [&](const T *Ab, const T *Bb, int kl) {
        if (idle) return;
#pragma unroll 1
        for (int kk = 0; kk < (kl & ~1); kk += 2) {
            const int aoff = ty * (TM * BK) + (((kk >> 2) ^ (ty & 3)) << 2) + (kk & 3);
            T a0[TM], a1[TM], b0[TM], b1[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const typename Pair<T>::type v =
                    *reinterpret_cast<const typename Pair<T>::type *>(Ab + aoff + i * BK);
                a0[i] = v.x;
                a1[i] = v.y;
            }
            // B: the thread's two 4-column groups of rows kk and kk+1, as
            // 16-byte reads
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const typename Vec4<T>::type u0 =
                    *reinterpret_cast<const typename Vec4<T>::type *>(Bb + kk * S + h * 64 + tx * 4);
                const typename Vec4<T>::type u1 = *reinterpret_cast<const typename Vec4<T>::type *>(
                    Bb + (kk + 1) * S + h * 64 + tx * 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    b0[4 * h + e] = u0[e];
                    b1[4 * h + e] = u1[e];
                }
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TM; ++j)
                    acc[i][j] = Ar<T>::min3(acc[i][j], Ar<T>::add(a0[i], b0[j]),
                                            Ar<T>::add(a1[i], b1[j]));
        }
        if (kl & 1) {  // the last valid k alone
            const int kk = kl - 1;
            const int aoff = ty * (TM * BK) + (((kk >> 2) ^ (ty & 3)) << 2) + (kk & 3);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TM; ++j) {
                    const T c =
                        Ar<T>::add(Ab[aoff + i * BK], Bb[kk * S + (j >> 2) * 64 + tx * 4 + (j & 3)]);
                    acc[i][j] = Ar<T>::min3(acc[i][j], c, c);
                }
        }
    };
    auto slice_k = [&](int s) { return max(0, min(BK, n - (k0 + s * BK))); };

    // as bulk_tile_dma: vmcnt(0) and a barrier before each slice is read and
    // before its buffer is refilled
    constexpr int kWaitVm0 = 0x0F70;
    issue(0, A0, B0);
#pragma unroll 1
    for (int s = 0; s < NS; s += 2) {
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        __syncthreads();
        issue(s + 1, A1, B1);
        compute(A0, B0, slice_k(s));
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        __syncthreads();
        if (s + 2 < NS) issue(s + 2, A0, B0);
        compute(A1, B1, slice_k(s + 1));
    }

    if (inside) {
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            T *row = d + (int64_t)(row0 + ty * TM + i) * ld + col0 + tx * 4;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                typename Vec4<T>::type x;
                x[0] = acc[i][4 * h];
                x[1] = acc[i][4 * h + 1];
                x[2] = acc[i][4 * h + 2];
                x[3] = acc[i][4 * h + 3];
                *reinterpret_cast<typename Vec4<T>::type *>(row + h * 64) = x;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int gi = row0 + ty * TM + i;
#pragma unroll
            for (int e = 0; e < TM; ++e) {
                const int gj = col0 + tx * 4 + (e >> 2) * 64 + (e & 3);
                if (gi < n && gj < n) d[(int64_t)gi * ld + gj] = acc[i][e];
            }
        }
    }
}

// Panel or bulk launch of stage b for tile-128 graphs whose rows are 16-byte
// aligned (staged_tile_dma).  A panel tile is the same product with the
// closed diagonal tile as one operand and the tile itself as the other (row
// panel (b, j): D(b,b) x D(b,j); column panel (i, b): D(i,b) x D(b,b)), its
// operand slices copied before its cells are stored.
#ifndef FW_STAGED_DMA_WAVES
#define FW_STAGED_DMA_WAVES 4
#endif
template <typename T>
__global__ void __launch_bounds__(256, FW_STAGED_DMA_WAVES)
staged_dma_kernel(const BatchItem *__restrict__ items, const StagedWork *__restrict__ work,
                  int kind, int b) {
    const StagedWork w = work[blockIdx.x];
    const BatchItem &it = items[w.item];
    const int m = (it.n + 127) / 128 - 1;
    int bi, bj;
    if (kind == kStagedPanelDma)
        panel_coords(w.local, b, m, bi, bj);
    else
        bulk_coords(w.local, b, m, bi, bj);
    staged_tile_dma<T>(as_global(static_cast<T *>(it.d)), it.n, it.ld, bi, bj, b);
}

template <typename T, bool PRED>
hipError_t launch_staged_t(int tile, const BatchItem *items, const StagedWork *work, int kind,
                           int b, unsigned grid, hipStream_t st) {
    if (kind == kStagedBulkDma || kind == kStagedPanelDma) {
        if (PRED || tile != 128) return hipErrorInvalidValue;
        staged_dma_kernel<T><<<grid, 256, 0, st>>>(items, work, kind, b);
        return hipGetLastError();
    }
    if (kind == kStagedDiag) {
        switch (tile) {
        case 32: staged_diag_kernel<T, 32, PRED><<<grid, 256, 0, st>>>(items, work, b); break;
        case 64: staged_diag_kernel<T, 64, PRED><<<grid, 256, 0, st>>>(items, work, b); break;
        case 128: staged_diag_kernel<T, 128, PRED><<<grid, 1024, 0, st>>>(items, work, b); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (tile) {
    case 32:
        staged_kernel<T, 32, PRED>
            <<<grid, staged_threads<T, 32, PRED>(), 0, st>>>(items, work, kind, b);
        break;
    case 64:
        staged_kernel<T, 64, PRED>
            <<<grid, staged_threads<T, 64, PRED>(), 0, st>>>(items, work, kind, b);
        break;
    case 128:
        staged_kernel<T, 128, PRED>
            <<<grid, staged_threads<T, 128, PRED>(), 0, st>>>(items, work, kind, b);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_staged(int dtype, bool pred, int tile, const BatchItem *items,
                         const StagedWork *work, int kind, int b, unsigned grid, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    if (dtype == FW_F32)
        return pred ? launch_staged_t<float, true>(tile, items, work, kind, b, grid, st)
                    : launch_staged_t<float, false>(tile, items, work, kind, b, grid, st);
    return pred ? launch_staged_t<int32_t, true>(tile, items, work, kind, b, grid, st)
                : launch_staged_t<int32_t, false>(tile, items, work, kind, b, grid, st);
}

int status_of(hipError_t e) {
    if (e == hipSuccess) return FW_OK;
    if (e == hipErrorOutOfMemory) return FW_ERR_NOMEM;
    return FW_ERR_HIP;
}

template <typename T>
const void *kernel_ptr_t(bool pred, bool big) {
    if (pred)
        return big ? (const void *)batched_kernel<T, true, 128>
                   : (const void *)batched_kernel<T, true, 64>;
    return big ? (const void *)batched_kernel<T, false, 128>
               : (const void *)batched_kernel<T, false, 64>;
}

const void *kernel_ptr(int dtype, bool pred, bool big) {
    return dtype == FW_F32 ? kernel_ptr_t<float>(pred, big) : kernel_ptr_t<int32_t>(pred, big);
}

// Workgroups per CU of each batched kernel, per device.
std::mutex g_occ_mu;
std::map<std::pair<int, int>, int> g_grid;

// big: the launch holds 128-wide tiles (the kernel with the 128-wide path).
int resident_grid(int dtype, bool pred, bool big = true) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    const int key2 = dtype * 4 + (pred ? 2 : 0) + (big ? 1 : 0);
    std::lock_guard<std::mutex> lk(g_occ_mu);
    auto it = g_grid.find({dev, key2});
    if (it != g_grid.end()) return it->second;
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel_ptr(dtype, pred, big),
                                                     kBatchThreads, 0) != hipSuccess)
        return -1;
    const int grid = cus * std::max(per, 1);
    g_grid[{dev, key2}] = grid;
    return grid;
}

}  // namespace

int batched_resident_grid(int dtype, bool pred) { return resident_grid(dtype, pred, true); }

void fill_batch_item(BatchItem &it, void *d, int dtype, int64_t n, int64_t ld, int32_t *p,
                     int64_t ldp) {
    it.d = d;
    it.p = p;
    it.ld = ld;
    it.ldp = p ? ldp : 0;
    it.n = (int32_t)n;
    it.tile = n > 1 ? plan_tile_for(dtype, n, p != nullptr) : 32;
    it.vec = vec_ok(d, ld) && (!p || vec_ok(p, ldp)) ? 1 : 0;
    it.pad = 0;
}

template <typename T>
void launch_batched_t(bool pred, bool big, BatchHeader *hdr, const BatchItem *items, int grid,
                      hipStream_t st) {
    if (pred) {
        if (big)
            batched_kernel<T, true, 128><<<grid, kBatchThreads, 0, st>>>(hdr, items);
        else
            batched_kernel<T, true, 64><<<grid, kBatchThreads, 0, st>>>(hdr, items);
    } else {
        if (big)
            batched_kernel<T, false, 128><<<grid, kBatchThreads, 0, st>>>(hdr, items);
        else
            batched_kernel<T, false, 64><<<grid, kBatchThreads, 0, st>>>(hdr, items);
    }
}

bool batch_needs_big(const BatchItem *items, int64_t count) {
    for (int64_t g = 0; g < count; ++g)
        if (items[g].n > 1 && items[g].tile > 64) return true;
    return false;
}

hipError_t launch_batched_raw(int dtype, bool pred, BatchHeader *hdr, const BatchItem *items,
                              int grid, hipStream_t st, bool big) {
    if (dtype == FW_F32)
        launch_batched_t<float>(pred, big, hdr, items, grid, st);
    else
        launch_batched_t<int32_t>(pred, big, hdr, items, grid, st);
    return hipGetLastError();
}

// Defined in fw_api.cpp.
hipError_t timed_launch_batched(double updates, hipStream_t st, int dtype, bool pred, bool big,
                                BatchHeader *hdr, const BatchItem *items, int grid);

}  // namespace fw

using namespace fw;

// A batch plan: descriptor table in pinned host memory and on the device,
// plus, once launched through a graph, the captured graph.
// Graphs with at least this many vertices run stage-batched; smaller ones
// are solved one per workgroup by the persistent kernel.
#ifndef FW_STAGED_MIN_N
#define FW_STAGED_MIN_N 33
#endif

struct StagedLaunch {
    int kind, tile, b;
    int64_t offset, count;  // slice of the work table
    // launches of one group depend on each other in plan order; different
    // groups on nothing in each other: the tile size, or minus it for the
    // one-launch closures of a tile group's single-block graphs
    int group;
};

struct fw_batch_plan_s {
    int dtype = 0;
    bool pred = false;
    int64_t count = 0;
    int64_t n_staged = 0;   // items [0, n_staged) are stage-batched
    int grid = 0;           // persistent grid for the other items
    bool big = false;       // some persistent item has a 128-wide tile
    int device = 0;
    double updates = 0;
    size_t bytes = 0;
    void *host = nullptr;   // BatchHeader + items (pinned)
    void *dev = nullptr;    // device copy
    std::vector<StagedLaunch> staged;
    StagedWork *work = nullptr;  // device work table (uploaded at creation)
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // fork / join of the independent launch sequences (see enqueue_plan),
    // created at the first launch that has more than one
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

namespace {

// The workgroups of a launch go to the GPU's XCDs in turn (workgroup w to
// XCD w mod 8) and every XCD has its own L2.  A launch's entries are
// reordered so that all tiles of one graph sit at indices congruent modulo
// the XCD count: the graph's panel tiles, which each of its bulk tiles reads,
// are then fetched into one L2 instead of all eight.  Graphs go to the group
// with the fewest entries so far, largest first; each group keeps the
// launch's order (closing entries first), and the groups are interleaved
// until the shortest runs out, the rest then following in turn.
#ifndef FW_STAGED_DMA
#define FW_STAGED_DMA 1
#endif
#ifndef FW_STAGED_SINGLE_APART
#define FW_STAGED_SINGLE_APART 1
#endif
#ifndef FW_PLAN_MAIN_FIRST
#define FW_PLAN_MAIN_FIRST 1
#endif
#ifndef FW_PLAN_FORK_AFTER_FIRST
#define FW_PLAN_FORK_AFTER_FIRST 1
#endif
#ifndef FW_STAGED_XCD_GROUPS
#define FW_STAGED_XCD_GROUPS 8
#endif
void xcd_group(std::vector<StagedWork> &work, int64_t first, int groups) {
    const int64_t end = (int64_t)work.size();
    std::map<int32_t, int64_t> count;  // graph -> entries in this launch
    std::vector<int32_t> graphs;       // in order of first appearance
    for (int64_t e = first; e < end; ++e)
        if (count[work[(size_t)e].item]++ == 0) graphs.push_back(work[(size_t)e].item);
    std::stable_sort(graphs.begin(), graphs.end(),
                     [&](int32_t a, int32_t b) { return count[a] > count[b]; });
    std::vector<int64_t> load((size_t)groups, 0);
    std::map<int32_t, int> group_of;
    for (int32_t g : graphs) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        group_of[g] = x;
        load[(size_t)x] += count[g];
    }
    std::vector<std::vector<StagedWork>> lists((size_t)groups);
    for (int64_t e = first; e < end; ++e)
        lists[(size_t)group_of[work[(size_t)e].item]].push_back(work[(size_t)e]);
    std::vector<size_t> pos((size_t)groups, 0);
    int64_t out = first;
    while (out < end)
        for (size_t x = 0; x < lists.size(); ++x)
            if (pos[x] < lists[x].size()) work[(size_t)out++] = lists[x][pos[x]++];
}

// Host half of a batch plan: the sorted descriptor table (header + items),
// the stage-batched launches and their work table.  No device memory.
struct HostPlan {
    std::vector<char> table;         // BatchHeader + items
    std::vector<StagedWork> work;
    std::vector<StagedLaunch> staged;
};

int build_host_plan(void *const *d, const int64_t *n, const int64_t *ld, int64_t count,
                    int dtype, int32_t *const *pred, const int64_t *ld_pred,
                    fw_batch_plan_s *pl, HostPlan &hp) {
    if (count < 0 || count > 0x7fffffffLL) return FW_ERR_INVALID;
    if (dtype != FW_F32 && dtype != FW_I32) return FW_ERR_INVALID;
    if (count > 0 && (!d || !n || !ld)) return FW_ERR_INVALID;
    if (pred && !ld_pred) return FW_ERR_INVALID;
    std::vector<BatchItem> items((size_t)count);
    bool any_pred = false;
    for (int64_t g = 0; g < count; ++g) {
        int32_t *pg = pred ? pred[g] : nullptr;
        const int64_t ldp = pg ? ld_pred[g] : 0;
        int s = validate_matrix(d[g], dtype, n[g], ld[g], pg, ldp);
        if (s != FW_OK) return s;
        if (n[g] > fw_batched_max_n(dtype, pg != nullptr)) return FW_ERR_UNSUPPORTED;
        fill_batch_item(items[(size_t)g], d[g], dtype, n[g], ld[g], pg, ldp);
        any_pred |= pg != nullptr;
    }
    // largest graphs first: the stage-batched ones form a prefix, and in the
    // persistent part the workgroups that take the largest start earliest
    std::stable_sort(items.begin(), items.end(),
                     [](const BatchItem &a, const BatchItem &b) { return a.n > b.n; });
    int64_t n_staged = 0;
    while (n_staged < count && items[(size_t)n_staged].n >= FW_STAGED_MIN_N) ++n_staged;
    // the persistent launch's own updates (phase timing attributes them to it)
    double upd = 0;
    for (int64_t g = n_staged; g < count; ++g) {
        const double ng = items[(size_t)g].n;
        upd += ng * ng * ng;
    }
    pl->dtype = dtype;
    pl->pred = any_pred;
    pl->count = count;
    pl->n_staged = n_staged;
    pl->updates = upd;
    pl->bytes = sizeof(BatchHeader) + sizeof(BatchItem) * (size_t)std::max<int64_t>(count, 1);
    if (hipGetDevice(&pl->device) != hipSuccess) return FW_ERR_HIP;
    pl->big = batch_needs_big(items.data() + n_staged, count - n_staged);
    const int grid = resident_grid(dtype, any_pred, pl->big);
    if (grid <= 0) return FW_ERR_HIP;
    pl->grid = (int)std::min<int64_t>(grid, std::max<int64_t>(count - n_staged, 1));
    hp.table.assign(pl->bytes, 0);
    auto *hdr = reinterpret_cast<BatchHeader *>(hp.table.data());
    *hdr = BatchHeader{};
    hdr->next = 0;
    hdr->count = (int32_t)(count - n_staged);  // the persistent part
    if (count)
        std::copy(items.begin(), items.end(),
                  reinterpret_cast<BatchItem *>(hp.table.data() + sizeof(BatchHeader)));
    if (n_staged == 0) return FW_OK;

    // Stage-batched part: per tile size, the launch sequence and its work
    // table.  Within a tile group the graphs stay sorted by size, so the
    // graphs that still have a stage b are a prefix of the group.
    std::vector<StagedWork> &work = hp.work;
    std::map<int, std::vector<int32_t>> groups;
    for (int64_t g = 0; g < n_staged; ++g) groups[items[(size_t)g].tile].push_back((int32_t)g);
    auto add_launch = [&](int kind, int tile, int b, int64_t first, int group = 0) {
        if ((int64_t)work.size() > first) {
            if (FW_STAGED_XCD_GROUPS > 1) xcd_group(work, first, FW_STAGED_XCD_GROUPS);
            hp.staged.push_back(
                {kind, tile, b, first, (int64_t)work.size() - first, group ? group : tile});
        }
    };
    for (auto &kv : groups) {
        const int tile = kv.first;
        const std::vector<int32_t> &gs = kv.second;
        auto blocks = [&](int32_t g) { return (items[(size_t)g].n + tile - 1) / tile; };
        int64_t first = (int64_t)work.size();
        for (int32_t g : gs)
            if (items[(size_t)g].p) work.push_back({g, 0});
        add_launch(kStagedPredInit, tile, 0, first);
        const int nb_max = blocks(gs.front());
        // the bulk launch of stage b closes each graph's tile (b+1, b+1)
        // tile 128 without predecessors: panels and bulk run staged_tile_dma
        // (rows 16-byte aligned in every graph of the group); each stage
        // keeps its diagonal launch, whose 1024-thread workgroups close a
        // tile sooner than a 256-thread bulk workgroup would after its product
        bool dma = tile == 128 && !any_pred && FW_STAGED_DMA;
        for (int32_t g : gs) {
            const BatchItem &it = items[(size_t)g];
            dma = dma && it.vec && (int64_t)it.n * it.ld < (int64_t(1) << 31);
        }
        const bool fuse = tile <= 64 || (tile == 128 && any_pred);
        for (int b = 0; b < nb_max; ++b) {
            first = (int64_t)work.size();
            // without predecessors (no set-up / fix-up launches around them),
            // the single-block graphs' closures -- their whole solve -- form a
            // launch of their own, off the stage chain
            const bool single_apart = !any_pred && FW_STAGED_SINGLE_APART;
            for (int32_t g : gs)
                if (blocks(g) > (single_apart ? std::max(b, 1) : b) && !(fuse && b > 0))
                    work.push_back({g, 0});
            add_launch(kStagedDiag, tile, b, first);
            if (single_apart && b == 0) {
                first = (int64_t)work.size();
                for (int32_t g : gs)
                    if (blocks(g) == 1) work.push_back({g, 0});
                add_launch(kStagedDiag, tile, 0, first, -tile);
            }
            first = (int64_t)work.size();
            for (int32_t g : gs) {
                const int m = blocks(g) - 1;
                if (blocks(g) > b)
                    for (int t = 0; t < 2 * m; ++t) work.push_back({g, t});
            }
            add_launch(dma ? kStagedPanelDma : kStagedPanel, tile, b, first);
            first = (int64_t)work.size();
            if (fuse)  // the closing workgroups first: they run longest
                for (int32_t g : gs)
                    if (blocks(g) > b + 1) {
                        const int m = blocks(g) - 1;
                        work.push_back({g, (b * m + b) | kStagedClose});
                    }
            for (int32_t g : gs) {
                const int m = blocks(g) - 1;
                if (blocks(g) > b)
                    for (int t = 0; t < m * m; ++t)
                        if (!(fuse && blocks(g) > b + 1 && t == b * m + b))
                            work.push_back({g, t});
            }
            add_launch(dma ? kStagedBulkDma : kStagedBulk, tile, b, first);
        }
        first = (int64_t)work.size();
        for (int32_t g : gs)
            if (items[(size_t)g].p) work.push_back({g, 0});
        add_launch(kStagedPredFix, tile, 0, first);
    }
    for (const StagedLaunch &l : hp.staged)
        if (l.count > 0x7fffffffLL) return FW_ERR_UNSUPPORTED;
    return FW_OK;
}

// A reusable plan: the host half, then the tables in pinned host memory and
// on the device, uploaded once on a private stream.
int build_plan(void *const *d, const int64_t *n, const int64_t *ld, int64_t count, int dtype,
               int32_t *const *pred, const int64_t *ld_pred, fw_batch_plan_s *pl) {
    HostPlan hp;
    int s = build_host_plan(d, n, ld, count, dtype, pred, ld_pred, pl, hp);
    if (s != FW_OK) return s;
    if (hipHostMalloc(&pl->host, pl->bytes, hipHostMallocDefault) != hipSuccess)
        return FW_ERR_NOMEM;
    std::copy(hp.table.begin(), hp.table.end(), static_cast<char *>(pl->host));
    if (hipMalloc(&pl->dev, pl->bytes) != hipSuccess) return FW_ERR_NOMEM;
    pl->staged = hp.staged;
    const size_t wbytes = sizeof(StagedWork) * hp.work.size();
    if (wbytes && hipMalloc(&pl->work, wbytes) != hipSuccess) return FW_ERR_NOMEM;
    // the tables never change (only the persistent part's work counter, which
    // each launch resets with a kernel): uploaded once, on a private stream
    hipStream_t up = nullptr;
    if (hipStreamCreateWithFlags(&up, hipStreamNonBlocking) != hipSuccess) return FW_ERR_HIP;
    hipError_t e = hipMemcpyAsync(pl->dev, pl->host, pl->bytes, hipMemcpyHostToDevice, up);
    if (e == hipSuccess && wbytes)
        e = hipMemcpyAsync(pl->work, hp.work.data(), wbytes, hipMemcpyHostToDevice, up);
    if (e == hipSuccess) e = hipStreamSynchronize(up);
    (void)hipStreamDestroy(up);
    return status_of(e);
}

// The launch group whose sequence is longest (the plan's critical path), or
// 0 when the plan has no stage-batched part.
int main_group(const fw_batch_plan_s *pl) {
    std::map<int, int> launches;
    for (const StagedLaunch &l : pl->staged) ++launches[l.group];
    int best = 0, most = 0;
    for (auto &kv : launches)
        if (kv.second > most) best = kv.first, most = kv.second;
    return best;
}

// True when the plan has launch sequences that depend on nothing in each
// other: several tile groups, or stage-batched and persistent parts.
bool has_independent_parts(const fw_batch_plan_s *pl) {
    const int main = main_group(pl);
    for (const StagedLaunch &l : pl->staged)
        if (l.group != main) return true;
    return main != 0 && pl->count > pl->n_staged;
}

// Enqueue: the stage-batched launches, then (if the plan has a persistent
// part) the reset of its work counter and the persistent kernel.  All are
// kernel launches (no copy or memset node), so the same sequence can be
// captured into a graph and replayed.  `untimed`: no phase events (a capture
// is running, or the caller must not create events).  With `side` (a stream
// of the plan, and its `fork` / `join` events), the sequences of different
// graphs run side by side: the longest tile group's stages on `st`, the other
// tile groups and the persistent part on `side`, forked from and joined back
// into `st` by the events (in a capture: parallel branches of the graph).
int enqueue_plan(fw_batch_plan_s *pl, hipStream_t st, bool untimed, hipStream_t side = nullptr,
                 hipEvent_t fork = nullptr, hipEvent_t join = nullptr) {
    if (pl->count == 0) return FW_OK;
    hipError_t e = hipSuccess;
    auto *hdr = static_cast<BatchHeader *>(pl->dev);
    auto *items =
        reinterpret_cast<const BatchItem *>(static_cast<char *>(pl->dev) + sizeof(BatchHeader));
    const bool split = side && has_independent_parts(pl);
    const int main = split ? main_group(pl) : 0;
    hipStream_t other = split ? side : st;
    // The side stream forks from the caller's stream after the main chain's
    // first launch (with FW_PLAN_FORK_AFTER_FIRST), so that the critical
    // chain takes the GPU first also where the launches are replayed from a
    // captured graph, whose parallel branches the runtime orders itself.
    bool forked = false;
    auto do_fork = [&]() -> hipError_t {
        if (!split || forked) return hipSuccess;
        forked = true;
        hipError_t r = hipEventRecord(fork, st);
        return r == hipSuccess ? hipStreamWaitEvent(side, fork, 0) : r;
    };
    if (!FW_PLAN_FORK_AFTER_FIRST || !FW_PLAN_MAIN_FIRST)
        if ((e = do_fork()) != hipSuccess) return status_of(e);
    // pass 0: the side stream's sequences, pass 1: the main chain
    const int order[2] = {FW_PLAN_MAIN_FIRST ? 1 : 0, FW_PLAN_MAIN_FIRST ? 0 : 1};
    for (int oi = split ? 0 : 1; oi < 2; ++oi) {
        const int pass = split ? order[oi] : 1;
        if (pass == 0 && (e = do_fork()) != hipSuccess) return status_of(e);
        for (const StagedLaunch &l : pl->staged) {
            if (split && (pass == 0) == (l.group == main)) continue;
            e = launch_staged(pl->dtype, pl->pred, l.tile, items, pl->work + l.offset, l.kind,
                              l.b, (unsigned)l.count, pass == 0 ? other : st);
            if (e != hipSuccess) return status_of(e);
            if (pass == 1 && (e = do_fork()) != hipSuccess) return status_of(e);
        }
        if (pass == 0 || !split) {
            if (pl->count > pl->n_staged) {
                batch_reset_kernel<<<1, 64, 0, other>>>(hdr);
                if ((e = hipGetLastError()) != hipSuccess) return status_of(e);
                const BatchItem *rest = items + pl->n_staged;
                e = untimed ? launch_batched_raw(pl->dtype, pl->pred, hdr, rest, pl->grid, other,
                                                 pl->big)
                            : timed_launch_batched(pl->updates, other, pl->dtype, pl->pred,
                                                   pl->big, hdr, rest, pl->grid);
                if (e != hipSuccess) return status_of(e);
            }
        }
    }
    if (split) {
        if ((e = hipEventRecord(join, side)) != hipSuccess) return status_of(e);
        if ((e = hipStreamWaitEvent(st, join, 0)) != hipSuccess) return status_of(e);
    }
    return FW_OK;
}

// The plan's side stream and fork / join events, created on first use.
hipError_t plan_side(fw_batch_plan_s *pl) {
    if (pl->side) return hipSuccess;
    hipError_t e = hipStreamCreateWithFlags(&pl->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->join, hipEventDisableTiming);
    return e;
}

void free_plan(fw_batch_plan_s *pl) {
    if (pl->work) (void)hipFree(pl->work);
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    if (pl->side) (void)hipStreamDestroy(pl->side);
    if (pl->fork) (void)hipEventDestroy(pl->fork);
    if (pl->join) (void)hipEventDestroy(pl->join);
    if (pl->dev) (void)hipFree(pl->dev);
    if (pl->host) (void)hipHostFree(pl->host);
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
        (void)hipEventSynchronize(p.done);
        (void)hipEventDestroy(p.done);
        free_plan(p.plan);
    }
}

// ---------------------------------------------------------------------------
// Tables of fw_apsp_batched_noalloc: one static device array per GPU, in
// place of the plan's allocations.  Host code reaches it only through the
// address hipGetSymbolAddress returns for the current device (the array's
// name is a host-side stand-in), looked up once per device.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(16) << 20;
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_ptr;

int scratch_base(int dev, char **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return FW_OK;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) return FW_ERR_HIP;
    g_scratch_ptr[dev] = static_cast<char *>(ptr);
    *out = static_cast<char *>(ptr);
    return FW_OK;
}

}  // namespace

extern "C" {

int fw_apsp_batched_noalloc(void *const *d, const int64_t *n, const int64_t *ld, int64_t count,
                            int dtype, int32_t *const *pred, const int64_t *ld_pred,
                            void *stream) {
    if (count == 0) {
        if (dtype != FW_F32 && dtype != FW_I32) return FW_ERR_INVALID;
        return FW_OK;
    }
    fw_batch_plan_s pl;  // tables in the static array: nothing owned
    HostPlan hp;
    int s = build_host_plan(d, n, ld, count, dtype, pred, ld_pred, &pl, hp);
    if (s != FW_OK) return s;
    const size_t tbytes = (pl.bytes + 255) / 256 * 256;
    const size_t wbytes = sizeof(StagedWork) * hp.work.size();
    if (tbytes + wbytes > kScratchBytes) return FW_ERR_UNSUPPORTED;
    char *base = nullptr;
    s = scratch_base(pl.device, &base);
    if (s != FW_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    // the previous call's kernels on this stream are done with the array
    // before these copies land (stream order); the host tables are freed on
    // return, so the copies are waited for
    hipError_t e = hipMemcpyAsync(base, hp.table.data(), pl.bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && wbytes)
        e = hipMemcpyAsync(base + tbytes, hp.work.data(), wbytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return status_of(e);
    pl.dev = base;
    pl.work = reinterpret_cast<StagedWork *>(base + tbytes);
    pl.staged = hp.staged;
    s = enqueue_plan(&pl, st, true);
    pl.dev = nullptr;
    pl.work = nullptr;
    return s;
}

int64_t fw_batched_noalloc_max_bytes(void) { return (int64_t)kScratchBytes; }

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
    if (plan->count && has_independent_parts(plan)) {
        hipError_t e = plan_side(plan);
        if (e != hipSuccess) return status_of(e);
    }
    if (mode == 0 || plan->count == 0)
        return enqueue_plan(plan, st, false, plan->side, plan->fork, plan->join);
    if (!plan->exec) {
        hipError_t e = hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return status_of(e);
        e = hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return status_of(e);
        int s = enqueue_plan(plan, plan->cap_stream, true, plan->side, plan->fork, plan->join);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(plan->cap_stream, &g);
        if (s != FW_OK) {
            if (g) (void)hipGraphDestroy(g);
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
    (void)hipDeviceSynchronize();
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
        (void)hipStreamSynchronize(st);
        if (ev) (void)hipEventDestroy(ev);
        free_plan(pl);
        return s != FW_OK ? s : FW_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(g_pending_mu);
    g_pending.push_back({pl, ev});
    return s;
}

}  // extern "C"

namespace fw {

int64_t batch_work_entries(int dtype, int64_t n, bool pred) {
    if (n < FW_STAGED_MIN_N) return 0;
    const int tile = plan_tile_for(dtype, n, pred);
    const int64_t nb = (n + tile - 1) / tile, m = nb - 1;
    return nb * (1 + 2 * m + m * m) + 2;  // a diagonal entry every stage, predecessor set-up
}

int enqueue_batch_buffered(void *const *d, const int64_t *n, const int64_t *ld, int64_t count,
                           int dtype, const BatchBuffers &buf, hipStream_t st) {
    if (count == 0) return FW_OK;
    fw_batch_plan_s pl;  // a view of the caller's buffers: nothing owned
    HostPlan hp;
    int s = build_host_plan(d, n, ld, count, dtype, nullptr, nullptr, &pl, hp);
    if (s != FW_OK) return s;
    const size_t wbytes = sizeof(StagedWork) * hp.work.size();
    if (pl.bytes > buf.table_bytes || wbytes > buf.work_bytes) return FW_ERR_UNSUPPORTED;
    std::copy(hp.table.begin(), hp.table.end(), static_cast<char *>(buf.host_table));
    if (wbytes) std::memcpy(buf.host_work, hp.work.data(), wbytes);
    hipError_t e = hipMemcpyAsync(buf.dev_table, buf.host_table, pl.bytes,
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess && wbytes)
        e = hipMemcpyAsync(buf.dev_work, buf.host_work, wbytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return status_of(e);
    pl.dev = buf.dev_table;
    pl.work = static_cast<StagedWork *>(buf.dev_work);
    pl.staged = hp.staged;
    s = enqueue_plan(&pl, st, true);
    pl.dev = nullptr;
    pl.work = nullptr;
    return s;
}

}  // namespace fw

