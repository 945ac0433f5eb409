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
// Bulk/panel kernel design (the paper's "staged load", section 4, rebuilt for
// 64-wide wavefronts rather than copied from the C1060 layout):
//   * each thread owns a TM x TN register sub-tile of C for the whole stage
//     (section 4.1: the doubly dependent tile lives in registers);
//   * A and B are staged through LDS in k-slices of depth BK, double
//     buffered, with the next slice prefetched from HBM into registers while
//     the current one is consumed (section 4.2's staged load);
//   * the A slice is stored k-major (transposed) so both operands are read
//     with 16-byte LDS loads;
//   * two k-steps are fused into one three-input minimum per cell,
//     c = min(c, a0 + b0, a1 + b1), legal because the bulk's tasks may run in
//     any order (section 3.2).
// MFMA is not used: min-plus is not a multiply-add contraction.
#include "fw_internal.h"

namespace fw {
namespace {

template <typename T> struct Ar;

template <> struct Ar<float> {
    __device__ __forceinline__ static float inf() { return __builtin_inff(); }
    __device__ __forceinline__ static float add(float a, float b) { return a + b; }
    __device__ __forceinline__ static float min2(float a, float b) {
        return __builtin_fminf(a, b);
    }
    __device__ __forceinline__ static float min3(float a, float b, float c) {
        return __builtin_fminf(__builtin_fminf(a, b), c);
    }
    __device__ __forceinline__ static bool absent(float v) { return v == __builtin_inff(); }
    __device__ __forceinline__ static bool unreachable(float v) { return v == __builtin_inff(); }
};

template <> struct Ar<int32_t> {
    __device__ __forceinline__ static int32_t inf() { return kI32Inf; }
    __device__ __forceinline__ static int32_t add(int32_t a, int32_t b) {
        return (int32_t)((uint32_t)a + (uint32_t)b);
    }
    __device__ __forceinline__ static int32_t min2(int32_t a, int32_t b) { return a < b ? a : b; }
    __device__ __forceinline__ static int32_t min3(int32_t a, int32_t b, int32_t c) {
        return min2(min2(a, b), c);
    }
    __device__ __forceinline__ static bool absent(int32_t v) { return v == kI32Inf; }
    __device__ __forceinline__ static bool unreachable(int32_t v) { return v > kI32Inf / 2; }
};

// Lexicographic minimum of (distance, last hop): the candidate replaces the
// current pair when it is strictly shorter, or equally short with a smaller
// last hop.  This keeps, for every pair, the smallest last hop over all
// shortest paths, a quantity independent of the order of the updates.
template <typename T>
__device__ __forceinline__ void lex_update(T &c, int32_t &p, T cand, int32_t pc) {
    const bool take = (cand < c) || (cand == c && pc < p);
    c = take ? cand : c;
    p = take ? pc : p;
}

template <typename T> struct Vec4 { typedef T type __attribute__((ext_vector_type(4))); };

// ---------------------------------------------------------------------------
// Phase 1: closure of the diagonal tile (b, b).
//
// One workgroup of (S/TM)^2 threads; thread (ty, tx) keeps the TM x TM cells
// rows ty*TM.., columns tx*TM.. in registers for all S steps.  Step k needs
// row k and column k as they are after step k-1; their owners publish them to
// a double-buffered LDS row/column before the step's barrier.  Row k and
// column k do not change during step k (d_kk >= 0), so one barrier per step
// suffices.  The loop over the TM steps of a register row is unrolled so that
// the owner's register index is a compile-time constant.
// ---------------------------------------------------------------------------
template <typename T, int S, int TM, bool PRED>
__global__ void __launch_bounds__((S / TM) * (S / TM))
diag_kernel(T *__restrict__ d, int32_t *__restrict__ P, int n, int64_t ld, int64_t ldp,
            int b) {
    constexpr int G = S / TM;
    __shared__ T rowb[2][S];
    __shared__ T colb[2][S];
    __shared__ int32_t rowp[PRED ? 2 : 1][PRED ? S : 1];

    const int tx = threadIdx.x % G, ty = threadIdx.x / G;
    const int base = b * S;
    T c[TM][TM];
    int32_t pc[TM][TM];
#pragma unroll
    for (int r = 0; r < TM; ++r) {
        const int gi = base + ty * TM + r;
#pragma unroll
        for (int q = 0; q < TM; ++q) {
            const int gj = base + tx * TM + q;
            const bool ok = gi < n && gj < n;
            c[r][q] = ok ? d[(int64_t)gi * ld + gj] : Ar<T>::inf();
            if constexpr (PRED) pc[r][q] = ok ? P[(int64_t)gi * ldp + gj] : kPredNone;
        }
    }

    for (int kb = 0; kb < G; ++kb) {
#pragma unroll
        for (int r = 0; r < TM; ++r) {
            const int buf = (kb * TM + r) & 1;
            if (ty == kb) {
#pragma unroll
                for (int q = 0; q < TM; ++q) {
                    rowb[buf][tx * TM + q] = c[r][q];
                    if constexpr (PRED) rowp[buf][tx * TM + q] = pc[r][q];
                }
            }
            if (tx == kb) {
#pragma unroll
                for (int q = 0; q < TM; ++q) colb[buf][ty * TM + q] = c[q][r];
            }
            __syncthreads();
            T rk[TM], ck[TM];
            int32_t pk[TM];
#pragma unroll
            for (int q = 0; q < TM; ++q) {
                rk[q] = rowb[buf][tx * TM + q];
                ck[q] = colb[buf][ty * TM + q];
                if constexpr (PRED) pk[q] = rowp[buf][tx * TM + q];
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TM; ++j) {
                    const T cand = Ar<T>::add(ck[i], rk[j]);
                    if constexpr (PRED)
                        lex_update(c[i][j], pc[i][j], cand, pk[j]);
                    else
                        c[i][j] = Ar<T>::min2(c[i][j], cand);
                }
        }
    }

#pragma unroll
    for (int r = 0; r < TM; ++r) {
        const int gi = base + ty * TM + r;
#pragma unroll
        for (int q = 0; q < TM; ++q) {
            const int gj = base + tx * TM + q;
            if (gi < n && gj < n) {
                d[(int64_t)gi * ld + gj] = c[r][q];
                if constexpr (PRED) P[(int64_t)gi * ldp + gj] = pc[r][q];
            }
        }
    }
}

// Load E consecutive elements of one matrix row starting at column `col`.
// Out-of-range elements (row >= n or column >= n) read as "infinity": the
// padded vertices behave as isolated vertices and change no real distance.
template <typename T, int E, bool VEC>
__device__ __forceinline__ void row_load(T (&v)[E], const T *__restrict__ base, int row,
                                         int col, int n, int64_t ld, bool full, T fill) {
    if (VEC && full) {
        const T *src = base + (int64_t)row * ld + col;
#pragma unroll
        for (int e = 0; e < E; e += 4) {
            const typename Vec4<T>::type x =
                *reinterpret_cast<const typename Vec4<T>::type *>(src + e);
            v[e] = x[0];
            v[e + 1] = x[1];
            v[e + 2] = x[2];
            v[e + 3] = x[3];
        }
    } else if (full) {
        const T *src = base + (int64_t)row * ld + col;
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = src[e];
    } else {
        const bool rok = row < n;
        const T *src = base + (rok ? (int64_t)row * ld : 0);
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = (rok && col + e < n) ? src[col + e] : fill;
    }
}

template <typename T, int E, bool VEC>
__device__ __forceinline__ void row_store(const T (&v)[E], T *__restrict__ base, int row,
                                          int col, int n, int64_t ld, bool full) {
    if (VEC && full) {
        T *dst = base + (int64_t)row * ld + col;
#pragma unroll
        for (int e = 0; e < E; e += 4) {
            typename Vec4<T>::type x;
            x[0] = v[e];
            x[1] = v[e + 1];
            x[2] = v[e + 2];
            x[3] = v[e + 3];
            *reinterpret_cast<typename Vec4<T>::type *>(dst + e) = x;
        }
    } else if (full) {
        T *dst = base + (int64_t)row * ld + col;
#pragma unroll
        for (int e = 0; e < E; ++e) dst[e] = v[e];
    } else if (row < n) {
        T *dst = base + (int64_t)row * ld;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (col + e < n) dst[col + e] = v[e];
    }
}

// ---------------------------------------------------------------------------
// Phases 2 and 3: register-tiled min-plus tile update (see file comment).
//   mode 0: blockIdx.x enumerates the 2(nb-1) panel tiles of stage b
//           (first the row panel (b, j != b), then the column panel);
//   mode 1: blockIdx.x enumerates the (nb-1)^2 bulk tiles (i != b, j != b).
// ---------------------------------------------------------------------------
template <typename T, int S, int BK, int TM, int TN, bool VEC, bool PRED>
__global__ void __launch_bounds__((S / TM) * (S / TN))
tile_kernel(T *__restrict__ d, int32_t *__restrict__ P, int n, int64_t ld, int64_t ldp, int b,
            int nb, int mode) {
    constexpr int NT = (S / TM) * (S / TN);
    constexpr int GX = S / TN;            // threads along a tile row
    constexpr int EA = S * BK / NT;       // A-slice elements per thread
    constexpr int TPA = BK / EA;          // threads per A-slice row
    constexpr int EB = BK * S / NT;       // B-slice elements per thread
    constexpr int TPB = S / EB;           // threads per B-slice row
    constexpr int NS = S / BK;            // k-slices per stage
    static_assert(EA * NT == S * BK && EB * NT == S * BK, "slice split");
    static_assert(!VEC || (EA % 4 == 0 && EB % 4 == 0 && TN % 4 == 0), "vector split");
    static_assert(BK % 2 == 0, "k-steps are fused in pairs");

    __shared__ T As[2][BK][S];
    __shared__ T Bs[2][BK][S];
    __shared__ int32_t Bp[PRED ? 2 : 1][PRED ? BK : 1][PRED ? S : 1];

    int bi, bj;
    const int m = nb - 1;
    if (mode == 0) {
        int idx = blockIdx.x;
        if (idx < m) {
            bi = b;
            bj = idx < b ? idx : idx + 1;
        } else {
            idx -= m;
            bi = idx < b ? idx : idx + 1;
            bj = b;
        }
    } else {
        const int q = blockIdx.x / m, r = blockIdx.x - q * m;
        bi = q < b ? q : q + 1;
        bj = r < b ? r : r + 1;
    }

    const int tid = threadIdx.x;
    const int tx = tid % GX, ty = tid / GX;
    const int row0 = bi * S, col0 = bj * S, k0 = b * S;
    const bool full = (row0 + S <= n) && (col0 + S <= n) && (k0 + S <= n);
    const T INF = Ar<T>::inf();

    // this thread's share of each slice load
    const int ia = tid / TPA, ka = (tid % TPA) * EA;
    const int kbr = tid / TPB, jb = (tid % TPB) * EB;

    T ra[EA], rb[EB];
    int32_t rp[PRED ? EB : 1];

    auto fetch = [&](int s) {
        row_load<T, EA, VEC>(ra, d, row0 + ia, k0 + s * BK + ka, n, ld, full, INF);
        row_load<T, EB, VEC>(rb, d, k0 + s * BK + kbr, col0 + jb, n, ld, full, INF);
        if constexpr (PRED)
            row_load<int32_t, EB, VEC>(rp, P, k0 + s * BK + kbr, col0 + jb, n, ldp, full,
                                       kPredNone);
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int e = 0; e < EA; ++e) As[buf][ka + e][ia] = ra[e];
#pragma unroll
        for (int e = 0; e < EB; ++e) Bs[buf][kbr][jb + e] = rb[e];
        if constexpr (PRED) {
#pragma unroll
            for (int e = 0; e < EB; ++e) Bp[buf][kbr][jb + e] = rp[e];
        }
    };

    // C first: the first slice's LDS store then waits for every load issued
    // so far, and the k loop never waits on a global load.
    T acc[TM][TN];
    int32_t accp[PRED ? TM : 1][PRED ? TN : 1];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        row_load<T, TN, VEC>(acc[i], d, row0 + ty * TM + i, col0 + tx * TN, n, ld, full, INF);
        if constexpr (PRED)
            row_load<int32_t, TN, VEC>(accp[i], P, row0 + ty * TM + i, col0 + tx * TN, n, ldp,
                                       full, kPredNone);
    }
    fetch(0);
    stash(0);
    __syncthreads();

    for (int s = 0; s < NS; ++s) {
        const int cur = s & 1;
        if (s + 1 < NS) fetch(s + 1);
        // one k-pair per iteration: unrolling further makes the compiler hoist
        // every LDS read of the slice and spill
#pragma unroll 1
        for (int kk = 0; kk < BK; kk += 2) {
            T a0[TM], a1[TM], b0[TN], b1[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                a0[i] = As[cur][kk][ty * TM + i];
                a1[i] = As[cur][kk + 1][ty * TM + i];
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                b0[j] = Bs[cur][kk][tx * TN + j];
                b1[j] = Bs[cur][kk + 1][tx * TN + j];
            }
            if constexpr (PRED) {
                int32_t p0[TN], p1[TN];
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    p0[j] = Bp[cur][kk][tx * TN + j];
                    p1[j] = Bp[cur][kk + 1][tx * TN + j];
                }
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) {
                        lex_update(acc[i][j], accp[i][j], Ar<T>::add(a0[i], b0[j]), p0[j]);
                        lex_update(acc[i][j], accp[i][j], Ar<T>::add(a1[i], b1[j]), p1[j]);
                    }
            } else {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = Ar<T>::min3(acc[i][j], Ar<T>::add(a0[i], b0[j]),
                                                Ar<T>::add(a1[i], b1[j]));
            }
        }
        if (s + 1 < NS) stash(cur ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < TM; ++i) {
        row_store<T, TN, VEC>(acc[i], d, row0 + ty * TM + i, col0 + tx * TN, n, ld, full);
        if constexpr (PRED)
            row_store<int32_t, TN, VEC>(accp[i], P, row0 + ty * TM + i, col0 + tx * TN, n, ldp,
                                        full);
    }
}

// ---------------------------------------------------------------------------
// Predecessor initialisation and final fix-up, negative-cycle scan.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
pred_init_kernel(const T *__restrict__ d, int32_t *__restrict__ P, int n, int64_t ld,
                 int64_t ldp) {
    for (int i = blockIdx.y; i < n; i += gridDim.y)
        for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
            const T w = d[(int64_t)i * ld + j];
            P[(int64_t)i * ldp + j] = (i != j && !Ar<T>::absent(w)) ? i : kPredNone;
        }
}

template <typename T>
__global__ void __launch_bounds__(256)
pred_fix_kernel(const T *__restrict__ d, int32_t *__restrict__ P, int n, int64_t ld,
                int64_t ldp) {
    for (int i = blockIdx.y; i < n; i += gridDim.y)
        for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
            const T v = d[(int64_t)i * ld + j];
            int32_t &p = P[(int64_t)i * ldp + j];
            if (i == j || p == kPredNone || Ar<T>::unreachable(v)) p = -1;
        }
}

template <typename T>
__global__ void __launch_bounds__(1024)
negcycle_kernel(const T *__restrict__ d, int n, int64_t ld, int32_t *__restrict__ flag) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    int mine = 0;
    for (int i = threadIdx.x; i < n; i += 1024) mine |= (d[(int64_t)i * ld + i] < T(0)) ? 1 : 0;
    if (mine) atomicOr(&any, 1);
    __syncthreads();
    if (threadIdx.x == 0) *flag = any;
}

dim3 elementwise_grid(int n) {
    const int gx = (n + 255) / 256 < 64 ? (n + 255) / 256 : 64;
    const int gy = n < 16384 ? n : 16384;
    return dim3(gx > 0 ? gx : 1, gy > 0 ? gy : 1);
}

// ---------------------------------------------------------------------------
// Dispatch: compile-time tile configurations.
//   tile  BK  TM x TN  threads   diag TM (threads)
//   128   16   8 x 8     256       4 (1024)
//    64   16   4 x 4     256       4 (256)
//    32   16   4 x 4      64       2 (256)
// ---------------------------------------------------------------------------
template <typename T, bool PRED>
hipError_t diag_t(int tile, T *d, int32_t *p, int n, int64_t ld, int64_t ldp, int b,
                  hipStream_t st) {
    switch (tile) {
    case 128: diag_kernel<T, 128, 4, PRED><<<1, 1024, 0, st>>>(d, p, n, ld, ldp, b); break;
    case 64: diag_kernel<T, 64, 4, PRED><<<1, 256, 0, st>>>(d, p, n, ld, ldp, b); break;
    case 32: diag_kernel<T, 32, 2, PRED><<<1, 256, 0, st>>>(d, p, n, ld, ldp, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool VEC, bool PRED>
hipError_t tile_t(int tile, T *d, int32_t *p, int n, int64_t ld, int64_t ldp, int b, int nb,
                  int mode, unsigned grid, hipStream_t st) {
    switch (tile) {
    case 128:
        tile_kernel<T, 128, 16, 8, 8, VEC, PRED><<<grid, 256, 0, st>>>(d, p, n, ld, ldp, b, nb,
                                                                      mode);
        break;
    case 64:
        tile_kernel<T, 64, 16, 4, 4, VEC, PRED><<<grid, 256, 0, st>>>(d, p, n, ld, ldp, b, nb,
                                                                     mode);
        break;
    case 32:
        tile_kernel<T, 32, 16, 4, 4, VEC, PRED><<<grid, 64, 0, st>>>(d, p, n, ld, ldp, b, nb,
                                                                    mode);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t tile_dispatch(int tile, T *d, int32_t *p, int n, int64_t ld, int64_t ldp, int b,
                         int nb, int mode, hipStream_t st) {
    const int64_t m = nb - 1;
    const int64_t grid = mode == 0 ? 2 * m : m * m;
    if (grid <= 0) return hipSuccess;
    if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
    const bool vec = vec_ok(d, ld) && (p == nullptr || vec_ok(p, ldp));
    if (p) {
        return vec ? tile_t<T, true, true>(tile, d, p, n, ld, ldp, b, nb, mode, (unsigned)grid, st)
                   : tile_t<T, false, true>(tile, d, p, n, ld, ldp, b, nb, mode, (unsigned)grid,
                                            st);
    }
    return vec ? tile_t<T, true, false>(tile, d, p, n, ld, ldp, b, nb, mode, (unsigned)grid, st)
               : tile_t<T, false, false>(tile, d, p, n, ld, ldp, b, nb, mode, (unsigned)grid, st);
}

}  // namespace

hipError_t launch_diag(int dtype, int tile, void *d, int32_t *p, int n, int64_t ld, int64_t ldp,
                       int b, hipStream_t st) {
    if (dtype == 0)
        return p ? diag_t<float, true>(tile, (float *)d, p, n, ld, ldp, b, st)
                 : diag_t<float, false>(tile, (float *)d, p, n, ld, ldp, b, st);
    return p ? diag_t<int32_t, true>(tile, (int32_t *)d, p, n, ld, ldp, b, st)
             : diag_t<int32_t, false>(tile, (int32_t *)d, p, n, ld, ldp, b, st);
}

hipError_t launch_panels(int dtype, int tile, void *d, int32_t *p, int n, int64_t ld,
                         int64_t ldp, int b, int nb, hipStream_t st) {
    if (dtype == 0) return tile_dispatch<float>(tile, (float *)d, p, n, ld, ldp, b, nb, 0, st);
    return tile_dispatch<int32_t>(tile, (int32_t *)d, p, n, ld, ldp, b, nb, 0, st);
}

hipError_t launch_bulk(int dtype, int tile, void *d, int32_t *p, int n, int64_t ld, int64_t ldp,
                       int b, int nb, hipStream_t st) {
    if (dtype == 0) return tile_dispatch<float>(tile, (float *)d, p, n, ld, ldp, b, nb, 1, st);
    return tile_dispatch<int32_t>(tile, (int32_t *)d, p, n, ld, ldp, b, nb, 1, st);
}

hipError_t launch_pred_init(int dtype, const void *d, int32_t *p, int n, int64_t ld,
                            int64_t ldp, hipStream_t st) {
    const dim3 g = elementwise_grid(n);
    if (dtype == 0)
        pred_init_kernel<float><<<g, 256, 0, st>>>((const float *)d, p, n, ld, ldp);
    else
        pred_init_kernel<int32_t><<<g, 256, 0, st>>>((const int32_t *)d, p, n, ld, ldp);
    return hipGetLastError();
}

hipError_t launch_pred_fix(int dtype, const void *d, int32_t *p, int n, int64_t ld,
                           int64_t ldp, hipStream_t st) {
    const dim3 g = elementwise_grid(n);
    if (dtype == 0)
        pred_fix_kernel<float><<<g, 256, 0, st>>>((const float *)d, p, n, ld, ldp);
    else
        pred_fix_kernel<int32_t><<<g, 256, 0, st>>>((const int32_t *)d, p, n, ld, ldp);
    return hipGetLastError();
}

hipError_t launch_negcycle(int dtype, const void *d, int n, int64_t ld, int32_t *flag,
                           hipStream_t st) {
    if (dtype == 0)
        negcycle_kernel<float><<<1, 1024, 0, st>>>((const float *)d, n, ld, flag);
    else
        negcycle_kernel<int32_t><<<1, 1024, 0, st>>>((const int32_t *)d, n, ld, flag);
    return hipGetLastError();
}

}  // namespace fw
