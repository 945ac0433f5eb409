// Blocked Floyd-Warshall kernels for CDNA4 (gfx950).
//
// The schedule is the blocked algorithm of section 3.2 (Fig. BFW-Alg): the
// matrix is cut into s x s tiles and, for each k-block b, three dependent
// phases run as three kernel launches (a kernel boundary is the global
// barrier between phases):
//
//   1. diag_kernel   -- the "independent block" (b, b): s dependent k-steps
//                       on one tile.
//   2. tile_kernel   -- the "singly dependent" row panel (b, j != b) and
//      (mode 0)         column panel (i != b, b).
//   3. tile_kernel   -- the "doubly dependent" bulk (i != b, j != b), the
//      (mode 1)         phase that sets the speed of the whole algorithm.
//
// Phases 2 and 3 share one kernel because both are the same tile update
//     C(i,j) <- min(C(i,j), min_{k in block b} A(i,k) + B(k,j))
// with A = tile (bi, b) and B = tile (b, bj) read at the moment the phase
// starts.  For the bulk this is the paper's order-free doubly dependent
// update (section 3.2: no dependencies inside the tile).  For a panel tile
// one operand is the finished diagonal tile D and the other is the panel tile
// itself, and the update is D (x) P in the min-plus sense: after phase 1, D
// holds the shortest paths inside block b, so every path from row-block b to
// column j that last leaves block b at vertex k splits into a D part and an
// unchanged P part.  In exact arithmetic this gives the same result as the
// figure's k-ordered panel loop while removing its k-to-k dependency, so the
// panel phase runs at the same register-tiled rate as the bulk.
//
// The workgroup-level bodies (closure_tile, product_tile) live in
// fw_tiles.h.  MFMA is not used: min-plus is not a multiply-add contraction.
#include <type_traits>

#include "fw_tiles.h"

// Build-time switches (variant builds override them with -D): the direct
// global->LDS bulk kernel, keyed int32 predecessor tiles, the next diagonal
// closed inside the bulk launch, strip-split panels, waves per SIMD of the
// bulk kernel.
#ifndef FW_BULK_DMA
#define FW_BULK_DMA 1
#endif
#ifndef FW_PRED_KEYS
#define FW_PRED_KEYS 1
#endif
#ifndef FW_FUSE_DIAG
#define FW_FUSE_DIAG 1
#endif
#ifndef FW_PANEL_STRIPS
#define FW_PANEL_STRIPS 1
#endif
#ifndef FW_BULK_DMA_WAVES
#define FW_BULK_DMA_WAVES 4
#endif

namespace fw {
namespace {

// A gated launch (gate != NULL) does nothing unless *gate != 0: the 64-bit
// predecessor sweep queued behind a keyed one runs only when the keyed one
// gave up.  The gate is uniform, so the whole workgroup leaves at once.
__device__ __forceinline__ bool gated_off(const int32_t *gate) { return gate && *gate == 0; }

// A keyed launch whose solve has already given up (its flag set by an earlier
// launch or the packing) has nothing useful to do: the 64-bit sweep behind it
// starts over from the input.  A flag raised during the launch is only seen
// by later launches.
template <class A>
__device__ __forceinline__ bool given_up(const int32_t *flag) {
    if constexpr (A::kChecked)
        return *flag != 0;
    else
        return false;
}

// Phase 1: closure of the diagonal tile (b, b) -- one workgroup.
template <typename T, int S, int TM, bool PRED, class A>
__global__ void __launch_bounds__((S / TM) * (S / TM))
diag_kernel(T *__restrict__ d, int32_t *__restrict__ P, int n, int64_t ld, int64_t ldp,
            int b, int32_t *flag, const int32_t *gate) {
    __shared__ __align__(16) char smem[closure_smem_bytes<T, S, PRED>()];
    if (gated_off(gate) || given_up<A>(flag)) return;
    closure_tile_any<T, S, TM, PRED, A>(d, P, n, ld, ldp, b * S, smem, flag);
}

// Phases 2 and 3: one tile per workgroup.
//   mode 0: blockIdx.x enumerates the 2(nb-1) panel tiles of stage b;
//   mode 1: blockIdx.x enumerates the (nb-1)^2 bulk tiles;
//   mode 2: the 2(nb-1)-1 bulk tiles in the last block row or column (the
//           part of the bulk that bulk_dma_kernel leaves when the last block
//           is partial).
// int32 with predecessors takes the keyed form (product_tile_key).
template <typename T, int S, int BK, bool PRED, class A>
constexpr bool keyed_tile() {
    return PRED && std::is_same<T, int32_t>::value && std::is_same<A, Ar<int32_t>>::value &&
           FW_PRED_KEYS;
}
template <typename T, int S, int BK, bool PRED, class A>
constexpr int tile_smem_bytes() {
    return keyed_tile<T, S, BK, PRED, A>() ? product_key_smem_bytes<S, BK>()
                                           : product_smem_bytes<T, S, BK, PRED>();
}

// Forms whose geometry is the closure's (4 x 4 cells per thread: tile 64 over
// 256 threads, the 128-wide predecessor form over 1024) can also close the
// next stage's diagonal tile in mode 1, as bulk_dma_kernel does.  (Tile 32
// over 64 threads has it too, but one wave's 32-wide closure is slower than
// the separate four-wave diagonal launch.)
template <int S, int TM, int TN, bool PRED>
constexpr bool tile_can_close() {
    return TM == 4 && TN == 4 && (S == 64 || (PRED && S == 128));
}

template <typename T, int S, int BK, int TM, int TN, bool VEC, bool PRED, class A>
__global__ void __launch_bounds__((S / TM) * (S / TN))
tile_kernel(T *__restrict__ d, int32_t *__restrict__ P, int n, int64_t ld, int64_t ldp, int b,
            int nb, int mode, int close_next, int32_t *flag, const int32_t *gate) {
    __shared__ __align__(16) char smem[tile_smem_bytes<T, S, BK, PRED, A>()];
    if (gated_off(gate) || given_up<A>(flag)) return;
    int idx = blockIdx.x, bi, bj;
    bool close = false;
    if constexpr (tile_can_close<S, TM, TN, PRED>()) {
        // the workgroup of tile (b+1, b+1) takes blockIdx 0 (see bulk_dma_kernel)
        const int dix = b * (nb - 1) + b;
        if (close_next && mode == 1) {
            idx = idx == 0 ? dix : idx == dix ? 0 : idx;
            close = idx == dix;
        }
    }
    switch (mode) {
    case 0: panel_coords(idx, b, nb - 1, bi, bj); break;
    case 1: bulk_coords(idx, b, nb - 1, bi, bj); break;
    default: edge_coords(idx, b, nb - 1, bi, bj); break;
    }
    if constexpr (keyed_tile<T, S, BK, PRED, A>())
        product_tile_key<S, BK, TM, TN, VEC>(d, P, n, ld, ldp, bi, bj, b, smem);
    else
        product_tile<T, S, BK, TM, TN, VEC, PRED, A>(d, P, n, ld, ldp, bi, bj, b, smem, flag);
    if constexpr (tile_can_close<S, TM, TN, PRED>()) {
        static_assert(tile_smem_bytes<T, S, BK, PRED, A>() >= closure_smem_bytes<T, S, PRED>(),
                      "the closure runs in the product's LDS");
        if (close) {
            __syncthreads();  // the tile's stores before its reloads
            closure_tile_any<T, S, TM, PRED, A>(d, P, n, ld, ldp, (b + 1) * S, smem, flag);
        }
    }
}


// Phase 3 for 128-wide tiles without predecessors and with 16-byte aligned
// rows: the bulk tiles among the first nf full blocks (blockIdx.x enumerates
// (nf-1)^2 of them, mf = nf - 1), slices copied into LDS directly
// (bulk_tile_dma); four waves per SIMD.
//
// With close_next (b + 1 < nf), the workgroup of tile (b+1, b+1) -- the next
// stage's diagonal tile, whose stage-b value it alone computes -- also runs
// that tile's closure, which replaces the next stage's phase-1 launch.  It
// takes blockIdx 0 (swapped with the tile enumerated first) so that it is
// dispatched early and its longer run overlaps the rest of the bulk.
template <typename T, class A>
__global__ void __launch_bounds__(256, FW_BULK_DMA_WAVES)
bulk_dma_kernel(T *__restrict__ d, int n, int64_t ld, int b, int mf, int close_next,
                int32_t *flag, const T *acol) {
    if (given_up<A>(flag)) return;
    int idx = blockIdx.x;
    const int dix = b * mf + b;  // enumeration index of tile (b+1, b+1)
    if (close_next) idx = idx == 0 ? dix : idx == dix ? 0 : idx;
    int bi, bj;
    bulk_coords(idx, b, mf, bi, bj);
    bulk_tile_dma<T, A>(d, n, ld, bi, bj, b, close_next && idx == dix, flag, acol);
}

// Phase 2 for 128-wide tiles without predecessors: each panel tile as four
// strips (strip_tile), blockIdx.x = 4 * (panel tile number) + strip.  Row
// panel tiles (b, j) are cut into 32-column strips, column panel tiles
// (i, b) into 32-row strips.
template <typename T, bool VEC, class A>
__global__ void __launch_bounds__(256)
panel_strip_kernel(T *__restrict__ d, int n, int64_t ld, int b, int nb, int32_t *flag,
                   T *acol) {
    constexpr int S = 128, W = 32;
    __shared__ __align__(16) char smem[strip_smem_bytes<T, S, W, S, 16>()];  // R + CW = 160 either way
    if (given_up<A>(flag)) return;
    const int m = nb - 1;
    const int t = blockIdx.x >> 2, q = blockIdx.x & 3;
    int bi, bj;
    panel_coords(t, b, m, bi, bj);
    if (t < m)  // row panel: rows of block b, a 32-column strip of block bj
        strip_tile<T, S, W, S, 16, 4, 4, VEC, A>(d, n, ld, b * S, bj * S + q * W, b * S, smem,
                                                 flag);
    else        // column panel: a 32-row strip of block bi, columns of block b
        strip_tile<T, W, S, S, 16, 4, 4, VEC, A>(d, n, ld, bi * S + q * W, b * S, b * S, smem,
                                                 flag, acol);
}

// ---------------------------------------------------------------------------
// Predecessor initialisation and final fix-up, negative-cycle scan.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
pred_init_kernel(const T *__restrict__ d, int32_t *__restrict__ P, int n, int64_t ld,
                 int64_t ldp, const int32_t *gate) {
    if (gated_off(gate)) return;
    for (int i = blockIdx.y; i < n; i += gridDim.y)
        for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
            const T w = d[(int64_t)i * ld + j];
            P[(int64_t)i * ldp + j] = (i != j && !Ar<T>::absent(w)) ? i : kPredNone;
        }
}

// gated 64-bit sweeps that ran (one count per solve, from its fix-up)
__device__ unsigned long long g_pred_fallbacks;

template <typename T>
__global__ void __launch_bounds__(256)
pred_fix_kernel(const T *__restrict__ d, int32_t *__restrict__ P, int n, int64_t ld,
                int64_t ldp, const int32_t *gate) {
    if (gated_off(gate)) return;
    if (gate && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
        atomicAdd(&g_pred_fallbacks, 1ull);
    for (int i = blockIdx.y; i < n; i += gridDim.y)
        for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
            int32_t &p = P[(int64_t)i * ldp + j];
            p = final_pred<T>(i, j, d[(int64_t)i * ld + j], p);
        }
}

// ---------------------------------------------------------------------------
// The fp32 canonical path (fw_internal.h): the canonical last hops from the
// final distances and the original weights, as the oracle defines them.
// ---------------------------------------------------------------------------
__global__ void canon_gate_kernel(int32_t *__restrict__ flag, int direct) {
    if (threadIdx.x == 0) flag[3] = ((direct || flag[0] != 0) && flag[2] == 0) ? 1 : 0;
}

// A gated save (behind a keyed sweep) counts one fallback.
__global__ void __launch_bounds__(256)
canon_save_kernel(const float *__restrict__ d, int32_t *__restrict__ P, int n, int64_t ld,
                  int64_t ldp, const int32_t *gate) {
    if (gated_off(gate)) return;
    if (gate && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
        atomicAdd(&g_pred_fallbacks, 1ull);
    for (int i = blockIdx.y; i < n; i += gridDim.y)
        for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256)
            P[(int64_t)i * ldp + j] = __float_as_int(d[(int64_t)i * ld + j]);
}

__global__ void __launch_bounds__(256)
canon_restore_kernel(float *__restrict__ d, const int32_t *__restrict__ P, int n, int64_t ld,
                     int64_t ldp, const int32_t *gate) {
    if (gated_off(gate)) return;
    for (int i = blockIdx.y; i < n; i += gridDim.y)
        for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256)
            d[(int64_t)i * ld + j] = __int_as_float(P[(int64_t)i * ldp + j]);
}

__global__ void __launch_bounds__(256)
canon_strip_kernel(const int32_t *__restrict__ P, int n, int64_t ldp, int j0, int w,
                   float *__restrict__ strip, const int32_t *gate) {
    if (gated_off(gate)) return;
    for (int q = blockIdx.y; q < n; q += gridDim.y)
        for (int c = blockIdx.x * 256 + threadIdx.x; c < w; c += gridDim.x * 256)
            strip[(int64_t)q * w + c] = __int_as_float(P[(int64_t)q * ldp + j0 + c]);
}

// One 64 x 64 tile of P (rows i0.., strip columns c0..; global column j0 +
// c) per workgroup, 4 x 4 cells per thread.  The candidates q run downward in
// 32-deep slices staged in LDS, and a cell keeps the last q whose sum equals
// its distance: the smallest.  A cell whose pair has no last hop (i == j,
// or d_ij = +INF) compares against NaN, which equals nothing.  The slice of
// d is staged with 0 at (i, i) (a path from i starts with the empty path)
// and the strip with +INF at (j, j) (q = j is no last hop of j); rows and
// columns beyond the matrix stage +INF, whose sums match no finite
// distance.  No order of the sums matters: each is one fp32 add, compared
// exactly.
constexpr int kCanonTile = 64, kCanonDepth = 32;

// 8 waves per SIMD (at most 64 registers): a 1024-column strip of an
// 8192-vertex graph (16 x 128 workgroups) is then one round of the GPU's
// 2048 workgroup slots instead of 1.33 rounds at 6 waves.
__global__ void __launch_bounds__(256, 8)
canon_pred_kernel(const float *__restrict__ d, int n, int64_t ld, const float *__restrict__ strip,
                  int j0, int w, int32_t *__restrict__ P, int64_t ldp, const int32_t *gate) {
    if (gated_off(gate)) return;
    constexpr int S = kCanonTile, KD = kCanonDepth;
    __shared__ __align__(16) float As[KD][S + 4];  // As[q][r] = d[i0 + r][q0 + q]
    __shared__ __align__(16) float Bs[KD][S + 4];  // Bs[q][c] = w[q0 + q][c0 + c]
    const int i0 = blockIdx.y * S, c0 = blockIdx.x * S;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const float kNaN = __builtin_nanf("");
    float t[4][4];
    int32_t best[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = i0 + ty * 4 + r, cc = c0 + tx * 4 + c, j = j0 + cc;
            float v = kNaN;
            if (i < n && cc < w && i != j) {
                v = d[(int64_t)i * ld + j];
                if (v == __builtin_inff()) v = kNaN;
            }
            t[r][c] = v;
            best[r][c] = -1;
        }
    for (int q0 = (n - 1) / KD * KD; q0 >= 0; q0 -= KD) {
        __syncthreads();  // the previous slice's reads are done
        for (int e = threadIdx.x; e < KD * S; e += 256) {
            const int q = e % KD, r = e / KD, gi = i0 + r, gq = q0 + q;
            float v = __builtin_inff();
            if (gi < n && gq < n) v = gi == gq ? 0.0f : d[(int64_t)gi * ld + gq];
            As[q][r] = v;
        }
        for (int e = threadIdx.x; e < KD * S; e += 256) {
            const int c = e % S, q = e / S, gq = q0 + q, cc = c0 + c;
            float v = __builtin_inff();
            if (gq < n && cc < w && gq != j0 + cc) v = strip[(int64_t)gq * w + cc];
            Bs[q][c] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int q = KD - 1; q >= 0; --q) {
            const float4 a = *reinterpret_cast<const float4 *>(&As[q][ty * 4]);
            const float4 b = *reinterpret_cast<const float4 *>(&Bs[q][tx * 4]);
            const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
            const int32_t gq = q0 + q;
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    best[r][c] = av[r] + bv[c] == t[r][c] ? gq : best[r][c];
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = i0 + ty * 4 + r, cc = c0 + tx * 4 + c;
            if (i < n && cc < w) P[(int64_t)i * ldp + j0 + cc] = best[r][c];
        }
}

// ---------------------------------------------------------------------------
// The keyed int32 predecessor solve (keys as in fw_internal.h).
// ---------------------------------------------------------------------------
// Zero the head of the scratch: the flags, and the row and column minima,
// which start at 0 -- the empty path from a vertex to itself.  (The cleared
// column panel after them is written by each stage's panel launch before
// its bulk reads it.)
__global__ void __launch_bounds__(256)
key_zero_kernel(int32_t *__restrict__ scratch, int64_t words) {
    for (int64_t w = blockIdx.x * 256 + threadIdx.x; w < words; w += (int64_t)gridDim.x * 256)
        scratch[w] = 0;
}

// key_ij = d_ij * 2^kKeyBits + (last hop of the edge: i; none on the
// diagonal), kKeyInf for an absent pair -- the keyed form of the predecessor
// initialisation.  An entry that is not an integer with |d_ij| < 2^14 (fp32:
// also a fraction, a NaN or -INF) raises the flag; within that range fp32
// sums of integers are exact, so the int32 keys compute what the fp32
// compare form does.
template <typename T>
__global__ void __launch_bounds__(256)
key_pack_kernel(const T *__restrict__ d, int32_t *__restrict__ keys, int n, int64_t ld,
                int64_t ldk, int32_t *__restrict__ flag) {
    bool bad = false;
    for (int i = blockIdx.y; i < n; i += gridDim.y)
        for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
            const T w = d[(int64_t)i * ld + j];
            int32_t key = kKeyInf;
            if (!Ar<T>::absent(w)) {
                int32_t v;
                if constexpr (std::is_same<T, float>::value) {
                    bad |= !(w == __builtin_rintf(w)) || !(__builtin_fabsf(w) < (float)(1 << kKeyBits));
                    v = bad ? 0 : (int32_t)w;
                } else {
                    bad |= w <= -(1 << kKeyBits) || w >= (1 << kKeyBits);
                    v = w;
                }
                key = (int32_t)((uint32_t)v << kKeyBits) + (i == j ? kKeyHop : i);
            }
            keys[(int64_t)i * ldk + j] = key;
        }
    if (bad) *flag = 1;
}

// A negative diagonal entry after the keyed sweep (a negative cycle: the
// pair-form sweep then gives its documented result) raises the flag, and
// the negative-diagonal word beside it.
__global__ void __launch_bounds__(256)
key_diag_kernel(const int32_t *__restrict__ keys, int n, int64_t ldk, int32_t *__restrict__ flag) {
    bool bad = false;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const int32_t key = keys[(int64_t)i * ldk + i];
        bad |= key < kKeyInfFloor && (key >> kKeyBits) < 0;
    }
    if (bad) {
        flag[0] = 1;
        flag[2] = 1;
    }
}

__device__ __forceinline__ int32_t wave_min(int32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t u = __shfl_xor(v, o, 64);
        v = u < v ? u : v;
    }
    return v;
}

// Unless the flag is set: every key becomes its distance in d and its last
// hop in the key matrix, now the predecessor matrix as pred_fix_kernel
// leaves it (-1 on the diagonal and for an infinite key).  fp32: an infinite
// key (j not reachable from i) is +INF, as in the fp32 sweep.  int32: it
// leaves FW_I32_INF in d, for key_inf_kernel, and raises the "some pair
// unreachable" word; on the way, the row and column minima of the finite
// distances (starting at 0): a workgroup covers 256 columns of kMinRows
// rows, a column's minimum kept per thread, a row's reduced over each wave
// and then over the four waves in LDS, both folded in with atomicMin.
constexpr int kMinRows = 64;

template <typename T>
__global__ void __launch_bounds__(256)
key_unpack_kernel(T *__restrict__ d, int32_t *__restrict__ keys, int n, int64_t ld, int64_t ldk,
                  int32_t *__restrict__ scratch) {
    constexpr bool I32 = std::is_same<T, int32_t>::value;
    __shared__ int32_t wmin[4][kMinRows];
    if (scratch[0] != 0) return;
    int32_t *rowmin = scratch + 4, *colmin = scratch + 4 + n;
    const int j = blockIdx.x * 256 + threadIdx.x, wave = threadIdx.x >> 6;
    const int r0 = blockIdx.y * kMinRows;
    const int rows = n - r0 < kMinRows ? n - r0 : kMinRows;
    int32_t cmin = 0;
    bool unreachable = false;
    for (int r = 0; r < rows; ++r) {
        const int i = r0 + r;
        int32_t v = 0;
        if (j < n) {
            int32_t &k = keys[(int64_t)i * ldk + j];
            const int32_t key = k;
            T dist = Ar<T>::inf();
            int32_t hop = -1;
            if (key < kKeyInfFloor) {
                v = key >> kKeyBits;
                dist = (T)v;
                const int32_t h = key & kKeyHop;
                if (i != j && h != kKeyHop) hop = h;
            } else {
                unreachable = true;
            }
            d[(int64_t)i * ld + j] = dist;
            k = hop;
        }
        if constexpr (I32) {
            cmin = v < cmin ? v : cmin;
            const int32_t rm = wave_min(v);
            if ((threadIdx.x & 63) == 0) wmin[wave][r] = rm;
        }
    }
    if constexpr (!I32) return;
    __syncthreads();
    if ((int)threadIdx.x < rows) {
        const int t = threadIdx.x;
        int32_t m = wmin[0][t];
        m = wmin[1][t] < m ? wmin[1][t] : m;
        m = wmin[2][t] < m ? wmin[2][t] : m;
        m = wmin[3][t] < m ? wmin[3][t] : m;
        if (m < 0) atomicMin(rowmin + r0 + t, m);
    }
    if (j < n && cmin < 0) atomicMin(colmin + j, cmin);
    if (unreachable) scratch[1] = 1;
}

// Where j is not reachable from i: the value the int32 sweep over the
// complete graph reaches, FW_I32_INF + (row i's minimum) + (column j's
// minimum) -- the cheapest path i ~> u -> v ~> j through one absent edge
// u -> v splits into independent best prefix and suffix, every such (u, v)
// pair being absent.  Runs only if the unpack found such a pair.
__global__ void __launch_bounds__(256)
key_inf_kernel(int32_t *__restrict__ d, int n, int64_t ld, const int32_t *__restrict__ scratch) {
    if (scratch[0] != 0 || scratch[1] == 0) return;
    const int32_t *rowmin = scratch + 4, *colmin = scratch + 4 + n;
    for (int i = blockIdx.y; i < n; i += gridDim.y) {
        const int32_t rm = rowmin[i];
        for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
            int32_t &v = d[(int64_t)i * ld + j];
            if (v == kI32Inf) v = kI32Inf + rm + colmin[j];
        }
    }
}

// The vertices i with d_ii < 0 after a solve, in ascending order, and their
// number; one workgroup of 1024 threads walks the diagonal in chunks of 1024,
// each chunk compacted by wave ballots and a scan of the 16 wave counts.
// Either output may be NULL (the flag-only call passes list = NULL).
template <typename T>
__global__ void __launch_bounds__(1024)
negcycle_kernel(const T *__restrict__ d, int n, int64_t ld, int32_t *__restrict__ list,
                int32_t *__restrict__ count) {
    __shared__ int wave_cnt[16];
    __shared__ int total;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const bool neg = i < n && d[(int64_t)i * ld + i] < T(0);
        const uint64_t mask = __ballot(neg);
        if (lane == 0) wave_cnt[wave] = __popcll(mask);
        __syncthreads();
        int before = total;  // entries of earlier chunks and earlier waves
        for (int w = 0; w < wave; ++w) before += wave_cnt[w];
        const uint64_t below = lane ? (mask & (~0ull >> (64 - lane))) : 0ull;
        if (neg && list) list[before + __popcll(below)] = i;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w = 0; w < 16; ++w) total += wave_cnt[w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && count) *count = total;
}

// About 8K workgroups whatever n: enough to stream the matrix, and cheap to
// dispatch when a gated launch finds its gate closed.
dim3 elementwise_grid(int n) {
    int gx = (n + 255) / 256 < 64 ? (n + 255) / 256 : 64;
    gx = gx > 0 ? gx : 1;
    int gy = 8192 / gx;
    gy = n < gy ? n : gy;
    return dim3(gx, gy > 0 ? gy : 1);
}

// ---------------------------------------------------------------------------
// Dispatch: compile-time tile configurations.
//   tile  BK  TM x TN  threads   diag TM (threads)
//   128   16   8 x 8     256       4 (1024)
//    64   16   4 x 4     256       4 (256)
//    32   16   4 x 4      64       2 (256)
// ---------------------------------------------------------------------------
template <typename T, bool PRED, class A>
hipError_t diag_t(int tile, T *d, int32_t *p, int n, int64_t ld, int64_t ldp, int b,
                  hipStream_t st, int32_t *flag, const int32_t *gate) {
    switch (tile) {
    case 128:
        diag_kernel<T, 128, 4, PRED, A><<<1, 1024, 0, st>>>(d, p, n, ld, ldp, b, flag, gate);
        break;
    case 64:
        diag_kernel<T, 64, 4, PRED, A><<<1, 256, 0, st>>>(d, p, n, ld, ldp, b, flag, gate);
        break;
    case 32:
        diag_kernel<T, 32, 2, PRED, A><<<1, 256, 0, st>>>(d, p, n, ld, ldp, b, flag, gate);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


#ifndef FW_PRED128_TM
#define FW_PRED128_TM 4
#define FW_PRED128_TN 4
#define FW_PRED128_BK 32
#endif

template <typename T, bool VEC, bool PRED, class A>
hipError_t tile_t(int tile, T *d, int32_t *p, int n, int64_t ld, int64_t ldp, int b, int nb,
                  int mode, unsigned grid, hipStream_t st, int close_next, int32_t *flag,
                  const int32_t *gate) {
    switch (tile) {
    case 128:
        if constexpr (PRED) {
            // the predecessor update keeps twice the state per cell; 4 x 4
            // sub-tiles over 1024 threads keep it at 4 waves per SIMD
            constexpr int TMP = FW_PRED128_TM, TNP = FW_PRED128_TN;
            tile_kernel<T, 128, FW_PRED128_BK, TMP, TNP, VEC, PRED, A>
                <<<grid, (128 / TMP) * (128 / TNP), 0, st>>>(d, p, n, ld, ldp, b, nb, mode,
                                                             close_next, flag, gate);
        } else {
            tile_kernel<T, 128, 16, 8, 8, VEC, PRED, A><<<grid, 256, 0, st>>>(
                d, p, n, ld, ldp, b, nb, mode, 0, flag, gate);
        }
        break;
    case 64:
        tile_kernel<T, 64, 16, 4, 4, VEC, PRED, A><<<grid, 256, 0, st>>>(
            d, p, n, ld, ldp, b, nb, mode, close_next, flag, gate);
        break;
    case 32:
        tile_kernel<T, 32, 16, 4, 4, VEC, PRED, A><<<grid, 64, 0, st>>>(
            d, p, n, ld, ldp, b, nb, mode, 0, flag, gate);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The bulk of stage b goes through bulk_dma_kernel: 128-wide tiles, no
// predecessors, 16-byte aligned rows, a full k-block, and 32-bit per-lane
// copy offsets (ld below 2^25).
bool bulk_copy_path(int tile, bool vec, int n, int64_t ld, int b) {
#if FW_BULK_DMA
    return tile == 128 && vec && b < n / 128 && ld < (int64_t(1) << 25);
#else
    (void)tile, (void)vec, (void)n, (void)ld, (void)b;
    return false;
#endif
}

template <typename T, class A, bool ALLOW_PRED>
hipError_t tile_dispatch(int tile, T *d, int32_t *p, int n, int64_t ld, int64_t ldp, int b,
                         int nb, int mode, bool close_next, hipStream_t st, int32_t *flag,
                         const int32_t *gate) {
    // gates: the predecessor forms (the pair-form sweep behind a keyed one),
    // and without predecessors the register-staged tiles (the distances of
    // the fp32 canonical path)
    if (gate && !p && tile > 64) return hipErrorInvalidValue;
    const int64_t m = nb - 1;
    const int64_t grid = mode == 0 ? 2 * m : m * m;
    if (grid <= 0) return close_next ? hipErrorInvalidValue : hipSuccess;
    if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
    const bool vec = vec_ok(d, ld) && (p == nullptr || vec_ok(p, ldp));
    // closing the next diagonal: tile 64 in any form, the copy path at 128
    // without predecessors, the 128-wide predecessor kernel with them
    if (close_next &&
        (mode != 1 || b + 1 >= nb ||
         (tile != 64 &&
          (p ? (!ALLOW_PRED || tile != 128) : !bulk_copy_path(tile, vec, n, ld, b)))))
        return hipErrorInvalidValue;
    const int c = close_next ? 1 : 0;
    // the keyed 128-wide sweep's cleared column panel (in the solve's scratch)
    T *acol = nullptr;
    if constexpr (A::kChecked) acol = reinterpret_cast<T *>(flag + key_acol_offset(n));
    if constexpr (ALLOW_PRED) {
        if (p) {
            return vec ? tile_t<T, true, true, A>(tile, d, p, n, ld, ldp, b, nb, mode,
                                                  (unsigned)grid, st, c, flag, gate)
                       : tile_t<T, false, true, A>(tile, d, p, n, ld, ldp, b, nb, mode,
                                                   (unsigned)grid, st, c, flag, gate);
        }
    } else {
        if (p) return hipErrorInvalidValue;
    }
    if (tile == 64)
        return vec ? tile_t<T, true, false, A>(tile, d, p, n, ld, ldp, b, nb, mode,
                                               (unsigned)grid, st, c, flag, gate)
                   : tile_t<T, false, false, A>(tile, d, p, n, ld, ldp, b, nb, mode,
                                                (unsigned)grid, st, c, flag, gate);
#if FW_PANEL_STRIPS
    if (mode == 0 && tile == 128) {
        if (4 * grid > 0x7fffffffLL) return hipErrorInvalidValue;
        if (vec)
            panel_strip_kernel<T, true, A><<<(unsigned)(4 * grid), 256, 0, st>>>(d, n, ld, b, nb,
                                                                                flag, acol);
        else
            panel_strip_kernel<T, false, A><<<(unsigned)(4 * grid), 256, 0, st>>>(
                d, n, ld, b, nb, flag, acol);
        return hipGetLastError();
    }
#endif
    // Stage with a full k-block: full tiles through bulk_dma_kernel, the
    // tiles of a partial last block (if any) through tile_kernel mode 4.
    const int nf = n / 128;
    // the keyed copy path reads the cleared column panel the strips write
    if (mode == 1 && bulk_copy_path(tile, vec, n, ld, b) && (!A::kChecked || FW_PANEL_STRIPS)) {
        const int64_t mf = nf - 1;
        if (close_next && b + 1 >= nf) return hipErrorInvalidValue;
        if (mf > 0) {
            bulk_dma_kernel<T, A><<<(unsigned)(mf * mf), 256, 0, st>>>(
                d, n, ld, b, (int)mf, close_next ? 1 : 0, flag, acol);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (nf < nb)
            return tile_t<T, true, false, A>(tile, d, p, n, ld, ldp, b, nb, 2,
                                             (unsigned)(2 * m - 1), st, 0, flag, nullptr);
        return hipSuccess;
    }
    if (close_next) return hipErrorInvalidValue;  // every closing form is handled above
    return vec ? tile_t<T, true, false, A>(tile, d, p, n, ld, ldp, b, nb, mode, (unsigned)grid, st,
                                           0, flag, gate)
               : tile_t<T, false, false, A>(tile, d, p, n, ld, ldp, b, nb, mode, (unsigned)grid,
                                            st, 0, flag, gate);
}

template <typename T>
hipError_t tile_any(int sr, int tile, T *d, int32_t *p, int n, int64_t ld, int64_t ldp, int b,
                    int nb, int mode, bool close_next, hipStream_t st, int32_t *flag,
                    const int32_t *gate) {
    if (gate && sr != kMinPlus) return hipErrorInvalidValue;
    if (sr == kMaxMin)
        return tile_dispatch<T, ArMaxMin<T>, false>(tile, d, p, n, ld, ldp, b, nb, mode,
                                                     close_next, st, nullptr, gate);
    if (sr == kKey) {
        if constexpr (std::is_same<T, int32_t>::value) {
            if (!flag) return hipErrorInvalidValue;
            return tile_dispatch<int32_t, ArKey, false>(tile, d, p, n, ld, ldp, b, nb, mode,
                                                        close_next, st, flag, gate);
        }
        return hipErrorInvalidValue;
    }
    return tile_dispatch<T, Ar<T>, true>(tile, d, p, n, ld, ldp, b, nb, mode, close_next, st,
                                         nullptr, gate);
}

}  // namespace

hipError_t launch_diag(int dtype, int sr, int tile, void *d, int32_t *p, int n, int64_t ld,
                       int64_t ldp, int b, hipStream_t st, int32_t *flag, const int32_t *gate) {
    if (gate && (sr != kMinPlus || (!p && tile > 64))) return hipErrorInvalidValue;
    if (sr == kMaxMin) {
        if (p) return hipErrorInvalidValue;
        if (dtype == 0)
            return diag_t<float, false, ArMaxMin<float>>(tile, (float *)d, p, n, ld, ldp, b, st,
                                                         nullptr, nullptr);
        return diag_t<int32_t, false, ArMaxMin<int32_t>>(tile, (int32_t *)d, p, n, ld, ldp, b,
                                                         st, nullptr, nullptr);
    }
    if (sr == kKey) {
        if (p || dtype != 1 || !flag) return hipErrorInvalidValue;
        return diag_t<int32_t, false, ArKey>(tile, (int32_t *)d, p, n, ld, ldp, b, st, flag,
                                             nullptr);
    }
    if (dtype == 0)
        return p ? diag_t<float, true, Ar<float>>(tile, (float *)d, p, n, ld, ldp, b, st, nullptr,
                                                  gate)
                 : diag_t<float, false, Ar<float>>(tile, (float *)d, p, n, ld, ldp, b, st,
                                                   nullptr, gate);
    return p ? diag_t<int32_t, true, Ar<int32_t>>(tile, (int32_t *)d, p, n, ld, ldp, b, st,
                                                  nullptr, gate)
             : diag_t<int32_t, false, Ar<int32_t>>(tile, (int32_t *)d, p, n, ld, ldp, b, st,
                                                   nullptr, gate);
}

hipError_t launch_panels(int dtype, int sr, int tile, void *d, int32_t *p, int n, int64_t ld,
                         int64_t ldp, int b, int nb, hipStream_t st, int32_t *flag,
                         const int32_t *gate) {
    if (dtype == 0)
        return tile_any<float>(sr, tile, (float *)d, p, n, ld, ldp, b, nb, 0, false, st, flag,
                               gate);
    return tile_any<int32_t>(sr, tile, (int32_t *)d, p, n, ld, ldp, b, nb, 0, false, st, flag,
                             gate);
}

bool bulk_closes_next_diag(int sr, int tile, const void *d, const int32_t *p, int n, int64_t ld,
                           int b) {
#if FW_FUSE_DIAG
    if (tile == 64) return (!p || sr == kMinPlus) && b + 1 < (n + 63) / 64;
    if (p) return sr == kMinPlus && tile == 128 && b + 1 < (n + 127) / 128;
    if (sr == kKey && !FW_PANEL_STRIPS) return false;
    return bulk_copy_path(tile, vec_ok(d, ld), n, ld, b) && b + 1 < n / 128;
#else
    (void)sr, (void)tile, (void)d, (void)p, (void)n, (void)ld, (void)b;
    return false;
#endif
}

hipError_t launch_bulk(int dtype, int sr, int tile, void *d, int32_t *p, int n, int64_t ld,
                       int64_t ldp, int b, int nb, bool close_next, hipStream_t st, int32_t *flag,
                       const int32_t *gate) {
    if (dtype == 0)
        return tile_any<float>(sr, tile, (float *)d, p, n, ld, ldp, b, nb, 1, close_next, st,
                               flag, gate);
    return tile_any<int32_t>(sr, tile, (int32_t *)d, p, n, ld, ldp, b, nb, 1, close_next, st,
                             flag, gate);
}

hipError_t launch_pred_init(int dtype, const void *d, int32_t *p, int n, int64_t ld,
                            int64_t ldp, hipStream_t st, const int32_t *gate) {
    const dim3 g = elementwise_grid(n);
    if (dtype == 0)
        pred_init_kernel<float><<<g, 256, 0, st>>>((const float *)d, p, n, ld, ldp, gate);
    else
        pred_init_kernel<int32_t><<<g, 256, 0, st>>>((const int32_t *)d, p, n, ld, ldp, gate);
    return hipGetLastError();
}

hipError_t launch_pred_fix(int dtype, const void *d, int32_t *p, int n, int64_t ld,
                           int64_t ldp, hipStream_t st, const int32_t *gate) {
    const dim3 g = elementwise_grid(n);
    if (dtype == 0)
        pred_fix_kernel<float><<<g, 256, 0, st>>>((const float *)d, p, n, ld, ldp, gate);
    else
        pred_fix_kernel<int32_t><<<g, 256, 0, st>>>((const int32_t *)d, p, n, ld, ldp, gate);
    return hipGetLastError();
}

hipError_t launch_key_prepare(int dtype, const void *d, int32_t *keys, int n, int64_t ld,
                              int64_t ldk, int32_t *scratch, hipStream_t st) {
    const int64_t words = key_acol_offset(n);
    key_zero_kernel<<<(unsigned)((words + 255) / 256), 256, 0, st>>>(scratch, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (dtype == 0)
        key_pack_kernel<float><<<elementwise_grid(n), 256, 0, st>>>((const float *)d, keys, n, ld,
                                                                   ldk, scratch);
    else
        key_pack_kernel<int32_t><<<elementwise_grid(n), 256, 0, st>>>((const int32_t *)d, keys,
                                                                     n, ld, ldk, scratch);
    return hipGetLastError();
}

hipError_t launch_key_finish(int dtype, void *d, int32_t *keys, int n, int64_t ld, int64_t ldk,
                             int32_t *scratch, hipStream_t st) {
    key_diag_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(keys, n, ldk, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 gu((unsigned)((n + 255) / 256), (unsigned)((n + kMinRows - 1) / kMinRows));
    if (dtype == 0) {
        key_unpack_kernel<float><<<gu, 256, 0, st>>>((float *)d, keys, n, ld, ldk, scratch);
        return hipGetLastError();
    }
    key_unpack_kernel<int32_t><<<gu, 256, 0, st>>>((int32_t *)d, keys, n, ld, ldk, scratch);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    key_inf_kernel<<<elementwise_grid(n), 256, 0, st>>>((int32_t *)d, n, ld, scratch);
    return hipGetLastError();
}

hipError_t launch_canon_gate(int32_t *scratch, bool direct, hipStream_t st) {
    canon_gate_kernel<<<1, 64, 0, st>>>(scratch, direct ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_canon_restore(float *d, const int32_t *p, int n, int64_t ld, int64_t ldp,
                                const int32_t *gate, hipStream_t st) {
    canon_restore_kernel<<<elementwise_grid(n), 256, 0, st>>>(d, p, n, ld, ldp, gate);
    return hipGetLastError();
}

hipError_t launch_canon_save(const float *d, int32_t *p, int n, int64_t ld, int64_t ldp,
                             const int32_t *gate, hipStream_t st) {
    canon_save_kernel<<<elementwise_grid(n), 256, 0, st>>>(d, p, n, ld, ldp, gate);
    return hipGetLastError();
}

hipError_t launch_canon_strip(const int32_t *p, int n, int64_t ldp, int j0, int w, float *strip,
                              const int32_t *gate, hipStream_t st) {
    if (n <= 0 || w <= 0 || j0 < 0 || j0 + w > n) return hipErrorInvalidValue;
    const int gx = (w + 255) / 256, gy = n < 8192 / gx ? n : 8192 / gx;
    canon_strip_kernel<<<dim3((unsigned)gx, (unsigned)gy), 256, 0, st>>>(p, n, ldp, j0, w, strip,
                                                                         gate);
    return hipGetLastError();
}

hipError_t launch_canon_pred(const float *d, int n, int64_t ld, const float *strip, int j0, int w,
                             int32_t *p, int64_t ldp, const int32_t *gate, hipStream_t st) {
    if (n <= 0 || w <= 0 || j0 < 0 || j0 + w > n) return hipErrorInvalidValue;
    const dim3 g((unsigned)((w + kCanonTile - 1) / kCanonTile),
                 (unsigned)((n + kCanonTile - 1) / kCanonTile));
    canon_pred_kernel<<<g, 256, 0, st>>>(d, n, ld, strip, j0, w, p, ldp, gate);
    return hipGetLastError();
}

int64_t pred_fallbacks() {
    unsigned long long v = 0;
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_pred_fallbacks), sizeof(v), 0,
                            hipMemcpyDeviceToHost) != hipSuccess)
        return -1;
    return (int64_t)v;
}

hipError_t launch_negcycle(int dtype, const void *d, int n, int64_t ld, int32_t *list,
                           int32_t *count, hipStream_t st) {
    if (dtype == 0)
        negcycle_kernel<float><<<1, 1024, 0, st>>>((const float *)d, n, ld, list, count);
    else
        negcycle_kernel<int32_t><<<1, 1024, 0, st>>>((const int32_t *)d, n, ld, list, count);
    return hipGetLastError();
}

}  // namespace fw
