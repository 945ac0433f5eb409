// Workgroup-level building blocks of blocked Floyd-Warshall on gfx950.
//
// Both are executed by one whole workgroup and shared by the per-phase
// kernels (one tile per workgroup, fw_kernels.hip) and by the persistent
// batched kernel (one graph per workgroup, fw_batched.hip), so a graph gets
// the same per-cell candidate sequence -- hence the same bits -- either way.
//
//   closure_tile  -- Floyd-Warshall (section 3.1, Fig. FW-Alg) restricted to
//                    one s x s tile whose origin is on the diagonal: the
//                    paper's "independent block" (section 3.2).  When the
//                    tile covers the whole graph this IS the plain algorithm.
//   product_tile  -- C <- min(C, A (x) B) over one k-block: the paper's
//                    "doubly dependent" update (section 3.2) with A = tile
//                    (bi, b), B = tile (b, bj), C = tile (bi, bj).
//
// Padding: cells outside the n x n matrix read as "infinity" and are never
// written, i.e. the padded vertices are isolated and change no distance.
#pragma once

#include "fw_internal.h"

namespace fw {

template <typename T> struct Ar;

// fp32 minimum and maximum.  With FW_MINIMUM the IEEE 754-2019 forms
// (gfx950's v_minimum3_f32 / v_maximum3_f32): IEEE-mode v_min_f32 needs its
// operands quieted first, and wherever the compiler cannot prove a value is
// already canonical (a load, a value pinned across a barrier) it spends a
// v_max_f32 x, x, x on it; the 2019 forms need none.  The two agree except
// on NaN (excluded by the contract) and on which zero of +0 / -0 is
// returned (left open by the contract).
#ifndef FW_MINIMUM
#define FW_MINIMUM 1
#endif
__device__ __forceinline__ float fmin32(float a, float b) {
#if FW_MINIMUM
    return __builtin_elementwise_minimum(a, b);
#else
    return __builtin_fminf(a, b);
#endif
}
__device__ __forceinline__ float fmax32(float a, float b) {
#if FW_MINIMUM
    return __builtin_elementwise_maximum(a, b);
#else
    return __builtin_fmaxf(a, b);
#endif
}

// Every policy says whether its values need settle() before they are stored
// or handed to other cells as operands (only the keyed policy does).
template <> struct Ar<float> {
    static constexpr bool kChecked = false;
    __device__ __forceinline__ static float inf() { return __builtin_inff(); }
    __device__ __forceinline__ static float add(float a, float b) { return a + b; }
    __device__ __forceinline__ static float min2(float a, float b) { return fmin32(a, b); }
    __device__ __forceinline__ static float min3(float a, float b, float c) {
        return fmin32(fmin32(a, b), c);
    }
    __device__ __forceinline__ static bool absent(float v) { return v == __builtin_inff(); }
    __device__ __forceinline__ static bool unreachable(float v) { return v == __builtin_inff(); }
};

template <> struct Ar<int32_t> {
    static constexpr bool kChecked = false;
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

// The (max, min) semiring through the same code: "add" is min (a path is as
// wide as its narrowest edge) and "min" is max (keep the widest path).  The
// padding value is the max-identity, so padded vertices stay isolated.  Over
// {0, 1} this is the transitive closure.  min and max are exact, so every
// order of the updates gives the same bits.
template <typename T> struct ArMaxMin;

template <> struct ArMaxMin<float> {
    static constexpr bool kChecked = false;
    __device__ __forceinline__ static float inf() { return -__builtin_inff(); }
    __device__ __forceinline__ static float add(float a, float b) { return fmin32(a, b); }
    __device__ __forceinline__ static float min2(float a, float b) { return fmax32(a, b); }
    __device__ __forceinline__ static float min3(float a, float b, float c) {
        return fmax32(fmax32(a, b), c);
    }
};

template <> struct ArMaxMin<int32_t> {
    static constexpr bool kChecked = false;
    __device__ __forceinline__ static int32_t inf() { return (int32_t)0x80000000; }
    __device__ __forceinline__ static int32_t add(int32_t a, int32_t b) { return a < b ? a : b; }
    __device__ __forceinline__ static int32_t min2(int32_t a, int32_t b) { return a > b ? a : b; }
    __device__ __forceinline__ static int32_t min3(int32_t a, int32_t b, int32_t c) {
        return min2(min2(a, b), c);
    }
};

// Min-plus over the 32-bit (distance, last hop) keys of fw_internal.h: the
// int32 form of the lexicographic update below in one add and (for two
// k-steps) one three-input minimum, the arithmetic of the distances-only
// sweep.  "add" clears the hop field of its first operand -- always the
// (i, k) cell, whose last hop the candidate does not inherit -- and adds the
// (k, j) key.  settle() brings a value back to the key invariant before it is
// stored or published to other cells: an infinite-class value becomes exactly
// kKeyInf, and a real value outside [kKeyLow, kKeyReal) (|d| >= 2^14) is
// recorded in the KeyCheck (the solve is then redone by the 64-bit form).
//
// KeyCheck: two running minima instead of a flag, so the check costs a few
// vector instructions per value and no lane-mask state.  Values that reach
// settle() lie in (-2^29, 2^29) (real) or [kKeyInf - 2^28, kKeyInf] (infinite
// class, at or above 3 * 2^28 - 2^14), so a real value is too large exactly
// when v - kKeyReal, as unsigned, is below kKeyReal, and too small exactly
// when v < kKeyLow.
struct KeyCheck {
    uint32_t hi = 0xffffffffu;  // min over values of (uint32)(v - kKeyReal)
    int32_t lo = 0;             // min over values
    __device__ __forceinline__ bool bad() const {
        return hi < (uint32_t)kKeyReal || lo < kKeyLow;
    }
};

struct ArKey {
    static constexpr bool kChecked = true;
    __device__ __forceinline__ static int32_t inf() { return kKeyInf; }
    __device__ __forceinline__ static int32_t add(int32_t a, int32_t b) {
        return (int32_t)(((uint32_t)a & ~(uint32_t)kKeyHop) + (uint32_t)b);
    }
    // add for a first operand whose hop field is already clear
    __device__ __forceinline__ static int32_t add_cleared(int32_t a, int32_t b) {
        return (int32_t)((uint32_t)a + (uint32_t)b);
    }
    __device__ __forceinline__ static int32_t clear_hop(int32_t a) {
        return (int32_t)((uint32_t)a & ~(uint32_t)kKeyHop);
    }
    __device__ __forceinline__ static int32_t min2(int32_t a, int32_t b) { return a < b ? a : b; }
    __device__ __forceinline__ static int32_t min3(int32_t a, int32_t b, int32_t c) {
        return min2(min2(a, b), c);
    }
    __device__ __forceinline__ static int32_t settle(int32_t v, KeyCheck &c) {
        const uint32_t up = (uint32_t)v - (uint32_t)kKeyReal;
        c.hi = up < c.hi ? up : c.hi;
        c.lo = v < c.lo ? v : c.lo;
        return v >= kKeyInfFloor ? kKeyInf : v;
    }
};

template <class A, typename T>
__device__ __forceinline__ T settle(T v, KeyCheck &c) {
    if constexpr (A::kChecked)
        return A::settle(v, c);
    else
        return v;
}

// Raise the solve's flag from every lane whose check found a bad key.
template <class A>
__device__ __forceinline__ void raise_flag(int32_t *flag, const KeyCheck &c) {
    if constexpr (A::kChecked) {
        if (c.bad()) *flag = 1;
    }
}

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

// The predecessor a cell keeps after the sweep: -1 where no last hop was
// found, for an unreachable pair, and on the diagonal -- except where d_ii < 0
// (a negative cycle through i, outside the problem statement), whose last hop
// is kept so that the cycle can be walked back from the matrix.
template <typename T>
__device__ __forceinline__ int32_t final_pred(int i, int j, T v, int32_t p) {
    if (p == kPredNone) return -1;
    if (i == j) return v < T(0) ? p : -1;
    return Ar<T>::unreachable(v) ? -1 : p;
}

template <typename T> struct Vec4 { typedef T type __attribute__((ext_vector_type(4))); };

// Load E consecutive elements of one matrix row starting at column `col`;
// out-of-range elements read as `fill`.
template <typename T, int E, bool VEC>
__device__ __forceinline__ void row_load(T (&v)[E], const T *__restrict__ base, int row, int col,
                                         int n, int64_t ld, bool full, T fill) {
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
__device__ __forceinline__ void row_store(const T (&v)[E], T *__restrict__ base, int row, int col,
                                          int n, int64_t ld, bool full) {
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
// closure_tile: s dependent k-steps on the tile with origin (base, base).
//
// (S/TM)^2 threads; thread (ty, tx) keeps the TM x TM cells rows ty*TM..,
// columns tx*TM.. in registers for all S steps.  Step k needs row k and
// column k as they are after step k-1; their owners publish them to a
// double-buffered LDS row/column before the step's barrier.  Row k and column
// k do not change during step k (d_kk >= 0), so one barrier per step
// suffices.  The TM steps of one register row are unrolled so the owner's
// register index is a compile-time constant.
// ---------------------------------------------------------------------------
// (without predecessors: room for closure_tile_pairs' double-buffered rows
// and columns k and k+1)
template <typename T, int S, bool PRED>
constexpr int closure_smem_bytes() {
    return PRED ? 4 * S * (int)sizeof(T) + 2 * S * 4 : 8 * S * (int)sizeof(T);
}

// FULL: the caller guarantees a tile inside the matrix with 16-byte aligned
// rows (no predecessors); cells move as 16-byte row pieces, no bounds tests.
template <typename T, int S, int TM, bool PRED, class A = Ar<T>, bool FULL = false>
__device__ __forceinline__ void closure_tile(T *__restrict__ d, int32_t *__restrict__ P, int n,
                                             int64_t ld, int64_t ldp, int base, char *smem,
                                             int32_t *flag = nullptr) {
    static_assert(!FULL || (!PRED && TM % 4 == 0), "full-tile form: no predecessors");
    constexpr int G = S / TM;
    T(*rowb)[S] = reinterpret_cast<T(*)[S]>(smem);
    T(*colb)[S] = reinterpret_cast<T(*)[S]>(smem + 2 * S * sizeof(T));
    int32_t(*rowp)[S] = reinterpret_cast<int32_t(*)[S]>(smem + 4 * S * sizeof(T));

    const int tx = threadIdx.x % G, ty = threadIdx.x / G;
    T c[TM][TM];
    int32_t pc[TM][TM];
    KeyCheck bad;
    if constexpr (FULL) {
#pragma unroll
        for (int r = 0; r < TM; ++r)
            row_load<T, TM, true>(c[r], d, base + ty * TM + r, base + tx * TM, n, ld, true,
                                  A::inf());
    } else {
#pragma unroll
        for (int r = 0; r < TM; ++r) {
            const int gi = base + ty * TM + r;
#pragma unroll
            for (int q = 0; q < TM; ++q) {
                const int gj = base + tx * TM + q;
                const bool ok = gi < n && gj < n;
                c[r][q] = ok ? d[(int64_t)gi * ld + gj] : A::inf();
                if constexpr (PRED) pc[r][q] = ok ? P[(int64_t)gi * ldp + gj] : kPredNone;
            }
        }
    }

    // steps k >= n only involve padded (isolated) vertices and change no real
    // cell, so the loop stops at the first register row past the last real k
    const int kreal = n - base < S ? n - base : S;
    const int kb_end = (kreal + TM - 1) / TM;
    for (int kb = 0; kb < kb_end; ++kb) {
#pragma unroll
        for (int r = 0; r < TM; ++r) {
            const int buf = (kb * TM + r) & 1;
            int oty = ty, otx = tx;
            if constexpr (FULL) {
                // opaque copies (no instruction is emitted): otherwise the
                // compiler threads the owner tests, equal across the TM
                // unrolled steps, and duplicates the step code per owner
                // class, which costs far more registers than the tile
                asm volatile("" : "+v"(oty), "+v"(otx));
            }
            if (oty == kb) {
#pragma unroll
                for (int q = 0; q < TM; ++q) {
                    rowb[buf][tx * TM + q] = settle<A>(c[r][q], bad);
                    if constexpr (PRED) rowp[buf][tx * TM + q] = pc[r][q];
                }
            }
            if (otx == kb) {
#pragma unroll
                for (int q = 0; q < TM; ++q) colb[buf][ty * TM + q] = settle<A>(c[q][r], bad);
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
                    const T cand = A::add(ck[i], rk[j]);
                    if constexpr (PRED)
                        lex_update(c[i][j], pc[i][j], cand, pk[j]);
                    else
                        c[i][j] = A::min2(c[i][j], cand);
                }
            if constexpr (FULL) {
                // finish this step's updates here: left alone, the compiler
                // sinks them past later barriers and keeps every step's row
                // and column live
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TM; ++j) asm volatile("" : "+v"(c[i][j]));
            }
        }
    }

    if constexpr (A::kChecked) {
#pragma unroll
        for (int r = 0; r < TM; ++r)
#pragma unroll
            for (int q = 0; q < TM; ++q) c[r][q] = settle<A>(c[r][q], bad);
        raise_flag<A>(flag, bad);
    }
    if constexpr (FULL) {
        // addresses recomputed from opaque copies rather than kept live
        // through the k loop
        int sty = ty, stx = tx;
        asm volatile("" : "+v"(sty), "+v"(stx));
#pragma unroll
        for (int r = 0; r < TM; ++r)
            row_store<T, TM, true>(c[r], d, base + sty * TM + r, base + stx * TM, n, ld, true);
    } else {
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
    // the LDS row/column buffers may be reused by the caller right away
    __syncthreads();
}

// closure_tile two k-steps per barrier, with closure_tile's bits (no
// predecessors, no range-checked keys; TM x TM cells per thread, TM even).
// Before steps k and k+1 (k even) the owners publish rows k, k+1 and columns
// k, k+1 as they stand.  Every thread then forms row k+1 and column k+1 as
// step k leaves them -- c[k+1][j] <- c[k+1][j] + (c[k+1][k] x c[k][j]), and
// c[i][k+1] <- c[i][k+1] + (c[i][k] x c[k][k+1]) in the semiring's (+, x) --
// and applies both steps at once with one 3-input reduction:
// c[i][j] <- c[i][j] + c[i][k] x c[k][j] + c'[i][k+1] x c'[k+1][j].  These are
// the same operations on the same values as the two steps in turn, so the
// result is bit-identical for any weights.  Half the barriers of closure_tile
// for the same VALU count.  Steps past the last vertex (the padded k that
// rounds an odd count up) change no real cell: the padded rows and columns
// are absent.
template <typename T, int S, int TM, class A = Ar<T>>
__device__ __forceinline__ void closure_tile_pairs(T *__restrict__ d, int n, int64_t ld, int base,
                                                   char *smem) {
    static_assert(TM % 2 == 0, "a thread owns both rows (columns) of a step pair");
    static_assert(!A::kChecked, "range-checked keys take closure_tile");
    constexpr int G = S / TM;
    T(*rowb)[2][S] = reinterpret_cast<T(*)[2][S]>(smem);  // [parity][k, k+1][S]
    T(*colb)[2][S] = reinterpret_cast<T(*)[2][S]>(smem + 4 * S * sizeof(T));
    const int tx = threadIdx.x % G, ty = threadIdx.x / G;
    T c[TM][TM];
#pragma unroll
    for (int r = 0; r < TM; ++r) {
        const int gi = base + ty * TM + r;
#pragma unroll
        for (int q = 0; q < TM; ++q) {
            const int gj = base + tx * TM + q;
            c[r][q] = (gi < n && gj < n) ? d[(int64_t)gi * ld + gj] : A::inf();
        }
    }
    const int kreal = n - base < S ? n - base : S;
    const int kb_end = (kreal + TM - 1) / TM;
    for (int kb = 0; kb < kb_end; ++kb) {
#pragma unroll
        for (int rp = 0; rp < TM; rp += 2) {
            const int buf = ((kb * TM + rp) >> 1) & 1;
            if (ty == kb) {
#pragma unroll
                for (int q = 0; q < TM; ++q) {
                    rowb[buf][0][tx * TM + q] = c[rp][q];
                    rowb[buf][1][tx * TM + q] = c[rp + 1][q];
                }
            }
            if (tx == kb) {
#pragma unroll
                for (int q = 0; q < TM; ++q) {
                    colb[buf][0][ty * TM + q] = c[q][rp];
                    colb[buf][1][ty * TM + q] = c[q][rp + 1];
                }
            }
            __syncthreads();
            const int k = kb * TM + rp;
            const T a = colb[buf][0][k + 1];  // c[k+1][k]
            const T e = rowb[buf][0][k + 1];  // c[k][k+1]
            T r0[TM], r1[TM], c0[TM], c1[TM];
#pragma unroll
            for (int q = 0; q < TM; ++q) {
                r0[q] = rowb[buf][0][tx * TM + q];
                r1[q] = A::min2(rowb[buf][1][tx * TM + q], A::add(a, r0[q]));
                c0[q] = colb[buf][0][ty * TM + q];
                c1[q] = A::min2(colb[buf][1][ty * TM + q], A::add(c0[q], e));
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TM; ++j)
                    c[i][j] = A::min3(c[i][j], A::add(c0[i], r0[j]), A::add(c1[i], r1[j]));
        }
    }
#pragma unroll
    for (int r = 0; r < TM; ++r) {
        const int gi = base + ty * TM + r;
#pragma unroll
        for (int q = 0; q < TM; ++q) {
            const int gj = base + tx * TM + q;
            if (gi < n && gj < n) d[(int64_t)gi * ld + gj] = c[r][q];
        }
    }
}

// The diagonal closure in the form its arguments allow: two k-steps per
// barrier without predecessors or range-checked keys, else closure_tile.
#ifndef FW_CLOSURE_PAIRS
#define FW_CLOSURE_PAIRS 1
#endif
template <typename T, int S, int TM, bool PRED, class A = Ar<T>>
__device__ __forceinline__ void closure_tile_any(T *__restrict__ d, int32_t *__restrict__ P, int n,
                                                 int64_t ld, int64_t ldp, int base, char *smem,
                                                 int32_t *flag = nullptr) {
    if constexpr (FW_CLOSURE_PAIRS && !PRED && !A::kChecked && TM % 2 == 0)
        closure_tile_pairs<T, S, TM, A>(d, n, ld, base, smem);
    else
        closure_tile<T, S, TM, PRED, A>(d, P, n, ld, ldp, base, smem, flag);
}

// ---------------------------------------------------------------------------
// product_tile: register-tiled min-plus update of tile (bi, bj) over block b.
//
//   * each thread owns a TM x TN register sub-tile of C for the whole k-block
//     (section 4.1: the doubly dependent tile lives in registers);
//   * A and B are staged through LDS in k-slices of depth BK, double
//     buffered, the next slice prefetched from HBM into registers while the
//     current one is consumed (section 4.2's staged load);
//   * the A slice is stored k-major (transposed) so both operands are read
//     with 16-byte LDS loads;
//   * two k-steps are fused into one three-input minimum per cell,
//     c = min(c, a0 + b0, a1 + b1), legal because the tasks of a doubly
//     dependent tile may run in any order (section 3.2).
// ---------------------------------------------------------------------------
template <typename T, int S, int BK, bool PRED>
constexpr int product_smem_bytes() {
    return 4 * BK * S * (int)sizeof(T) + (PRED ? 2 * BK * S * 4 : 0);
}

template <typename T, int S, int BK, int TM, int TN, bool VEC, bool PRED, class A = Ar<T>>
__device__ __forceinline__ void product_tile(T *__restrict__ d, int32_t *__restrict__ P, int n,
                                             int64_t ld, int64_t ldp, int bi, int bj, int b,
                                             char *smem, int32_t *flag = nullptr) {
    constexpr int NT = (S / TM) * (S / TN);
    constexpr int GX = S / TN;       // threads along a tile row
    constexpr int EA = S * BK / NT;  // A-slice elements per thread
    constexpr int TPA = BK / EA;     // threads per A-slice row
    constexpr int EB = BK * S / NT;  // B-slice elements per thread
    constexpr int TPB = S / EB;      // threads per B-slice row
    constexpr int NS = S / BK;       // k-slices per block
    static_assert(EA * NT == S * BK && EB * NT == S * BK, "slice split");
    static_assert(TPA * EA == BK && TPB * EB == S, "slice rows");
    static_assert(!VEC || (EA % 4 == 0 && EB % 4 == 0 && TN % 4 == 0), "vector split");
    static_assert(BK % 2 == 0, "k-steps are fused in pairs");

    T(*As)[BK][S] = reinterpret_cast<T(*)[BK][S]>(smem);
    T(*Bs)[BK][S] = reinterpret_cast<T(*)[BK][S]>(smem + 2 * BK * S * sizeof(T));
    int32_t(*Bp)[BK][S] = reinterpret_cast<int32_t(*)[BK][S]>(smem + 4 * BK * S * sizeof(T));

    const int tid = threadIdx.x;
    const int tx = tid % GX, ty = tid / GX;
    const int row0 = bi * S, col0 = bj * S, k0 = b * S;
    const bool full = (row0 + S <= n) && (col0 + S <= n) && (k0 + S <= n);
    const T INF = A::inf();

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
                        lex_update(acc[i][j], accp[i][j], A::add(a0[i], b0[j]), p0[j]);
                        lex_update(acc[i][j], accp[i][j], A::add(a1[i], b1[j]), p1[j]);
                    }
            } else {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = A::min3(acc[i][j], A::add(a0[i], b0[j]),
                                                A::add(a1[i], b1[j]));
            }
        }
        if (s + 1 < NS) stash(cur ^ 1);
        __syncthreads();
    }

    if constexpr (A::kChecked) {
        KeyCheck bad;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = settle<A>(acc[i][j], bad);
        raise_flag<A>(flag, bad);
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
// bulk_tile_dma: the 128 x 128 tile update of product_tile (no predecessors)
// for a tile that lies inside the matrix with a full k-block, the k-slices
// moved from global memory straight into LDS by gfx950's global->LDS dwordx4
// loads instead of through registers.  A thread keeps only its 8 x 8 cells
// and one k-pair of operands, so four waves fit on a SIMD where the
// register-staged form fits three, and the copy costs no LDS store
// instructions.
//
// LDS layout (four separate arrays, so that the compiler's wait-count
// tracking can tell the buffer being filled from the one being read):
//   A slice: 128 rows x 16 k, row-major as in global memory; the four
//            16-byte chunks of row r are permuted, chunk c stored at
//            position c ^ ((r / 8) % 4), so that the 4 rows one wave reads
//            together fall in different banks;
//   B slice: 16 k x 128 columns, as in global memory.
// Requirements on the caller: 256 threads, 16-byte aligned rows (base
// aligned, ld % 4 == 0), tile and k-block inside the matrix.  Per cell the
// same candidates are formed, one add each, as in product_tile, hence the
// same bits.  With `close` (uniform per workgroup; the tile is (b+1, b+1))
// the tile's closure for stage b+1 follows the store.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void_t;

template <typename T>
struct Pair;
template <>
struct Pair<float> {
    using type = float2;
};
template <>
struct Pair<int32_t> {
    using type = int2;
};

// With the keyed policy the A slices come from `acol` (the stage's column
// panel with the hop fields cleared, 128 values per row, written by the
// panel launch), so the k loop adds without clearing.
template <typename T, class A = Ar<T>>
__device__ __forceinline__ void bulk_tile_dma(T *__restrict__ d, int n, int64_t ld, int bi,
                                              int bj, int b, bool close, int32_t *flag = nullptr,
                                              const T *__restrict__ acol = nullptr) {
    static_assert(sizeof(T) == 4, "32-bit values");
    constexpr int S = 128, BK = 16, TM = 8, NS = S / BK;
    static_assert(NS % 2 == 0, "slices alternate between two buffers");
    __shared__ __align__(16) T A0[S * BK];
    __shared__ __align__(16) T A1[S * BK];
    __shared__ __align__(16) T B0[BK * S];
    __shared__ __align__(16) T B1[BK * S];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tx = tid & 15, ty = tid >> 4;
    const int64_t row0 = (int64_t)bi * S, col0 = (int64_t)bj * S, k0 = (int64_t)b * S;

    // thread (tx, ty) owns rows 8*ty .. 8*ty + 7 and the two 4-column groups
    // starting at 4*tx and 64 + 4*tx: the 16 column groups a B read touches
    // are contiguous, so the read has no bank conflicts
    T acc[TM][TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        T *row = d + (row0 + ty * TM + i) * ld + col0 + tx * 4;
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

    // Copy sources: wave-uniform bases plus 32-bit per-lane offsets.  The
    // wave copies A rows 32*wave + lane/4 (and +16) and B k-rows
    // 4*wave + lane/32 (and +2) of each slice.
    const int64_t lda = A::kChecked ? (int64_t)S : ld;
    const T *a_base = A::kChecked ? acol + (row0 + wave * 32) * S
                                  : d + (row0 + wave * 32) * ld + k0;
    const T *b_base = d + (k0 + wave * 4) * ld + col0;
    const int ar = wave * 32 + (lane >> 2);
    const uint32_t a_off0 = (uint32_t)((lane >> 2) * lda) + (((lane & 3) ^ ((ar >> 3) & 3)) << 2);
    const uint32_t a_off1 =
        (uint32_t)(((lane >> 2) + 16) * lda) + (((lane & 3) ^ (((ar + 16) >> 3) & 3)) << 2);
    const uint32_t b_off0 = (uint32_t)((lane >> 5) * ld) + ((lane & 31) << 2);
    const uint32_t b_off1 = b_off0 + (uint32_t)(2 * ld);
    auto issue = [&](int s, T *Ad, T *Bd) {
        const T *as = a_base + s * BK;
        const T *bs = b_base + (int64_t)s * BK * ld;
        T *a = Ad + wave * 32 * BK;
        T *bb = Bd + wave * 4 * S;
        __builtin_amdgcn_global_load_lds(as + a_off0, (lds_void_t *)a, 16, 0, 0);
        __builtin_amdgcn_global_load_lds(as + a_off1, (lds_void_t *)(a + 16 * BK), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(bs + b_off0, (lds_void_t *)bb, 16, 0, 0);
        __builtin_amdgcn_global_load_lds(bs + b_off1, (lds_void_t *)(bb + 2 * S), 16, 0, 0);
    };
    auto compute = [&](const T *Ab, const T *Bb) {
        // one k-pair per iteration (see product_tile)
#pragma unroll 1
        for (int kk = 0; kk < BK; kk += 2) {
            const int aoff = ty * (TM * BK) + (((kk >> 2) ^ (ty & 3)) << 2) + (kk & 3);
            T a0[TM], a1[TM], b0[TM], b1[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const typename Pair<T>::type v =
                    *reinterpret_cast<const typename Pair<T>::type *>(Ab + aoff + i * BK);
                a0[i] = v.x;
                a1[i] = v.y;
            }
#pragma unroll
            for (int j = 0; j < TM; ++j) {
                const int c = (j >> 2) * 64 + tx * 4 + (j & 3);
                b0[j] = Bb[kk * S + c];
                b1[j] = Bb[(kk + 1) * S + c];
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TM; ++j) {
                    if constexpr (A::kChecked)
                        acc[i][j] = A::min3(acc[i][j], A::add_cleared(a0[i], b0[j]),
                                            A::add_cleared(a1[i], b1[j]));
                    else
                        acc[i][j] = A::min3(acc[i][j], A::add(a0[i], b0[j]), A::add(a1[i], b1[j]));
                }
        }
    };

    // vmcnt(0): this wave's copies (and its C loads) have landed; the
    // barrier after it makes every wave's copies visible and guarantees that
    // every wave is done reading the buffer the next copy overwrites
    constexpr int kWaitVm0 = 0x0F70;
    issue(0, A0, B0);
#pragma unroll 1
    for (int s = 0; s < NS; s += 2) {
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        __syncthreads();
        issue(s + 1, A1, B1);
        compute(A0, B0);
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        __syncthreads();
        if (s + 2 < NS) issue(s + 2, A0, B0);
        compute(A1, B1);
    }

    // store addresses recomputed from opaque copies of the thread ids (no
    // instruction is emitted): the load addresses would otherwise stay live
    // through the k loop, 16 VGPRs
    int stx = tx, sty = ty;
    asm volatile("" : "+v"(stx), "+v"(sty));
    if constexpr (A::kChecked) {
        KeyCheck bad;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TM; ++j) acc[i][j] = settle<A>(acc[i][j], bad);
        raise_flag<A>(flag, bad);
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        T *row = d + (row0 + sty * TM + i) * ld + col0 + stx * 4;
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
    if (close) {
        // the next stage's diagonal tile: reread by the same workgroup (the
        // barrier orders its stores before the loads) and closed in place;
        // the product's LDS buffers are free by now
        __syncthreads();
        closure_tile<T, S, TM, false, A, true>(d, nullptr, n, ld, 0, (int)row0,
                                               reinterpret_cast<char *>(A0), flag);
    }
}

// ---------------------------------------------------------------------------
// product_tile_key: product_tile with predecessors for int32 matrices, the
// (distance, last hop) pair of a cell held as one 64-bit key, distance in the
// high word and last hop (>= 0) in the low word.  Compared as signed 64-bit
// integers, keys order exactly as lex_update orders pairs (shorter first,
// then smaller last hop), so one compare and two selects replace it.  The
// candidate through k is B's key plus the A distance shifted into the high
// word -- one 64-bit shift-and-add; the low word (B's last hop) is unchanged
// because the added value's low word is zero, and the high word is the int32
// sum the unkeyed form computes.  Same candidates, same order rule, hence
// the same distances and predecessors.  B is staged in LDS as keys.
// ---------------------------------------------------------------------------
template <int S, int BK>
constexpr int product_key_smem_bytes() {
    return 2 * BK * S * 4 + 2 * BK * S * 8;
}

__device__ __forceinline__ uint64_t make_key(int32_t d, int32_t p) {
    return ((uint64_t)(uint32_t)d << 32) | (uint32_t)p;
}

template <int S, int BK, int TM, int TN, bool VEC>
__device__ __forceinline__ void product_tile_key(int32_t *__restrict__ d, int32_t *__restrict__ P,
                                                 int n, int64_t ld, int64_t ldp, int bi, int bj,
                                                 int b, char *smem) {
    using T = int32_t;
    constexpr int NT = (S / TM) * (S / TN);
    constexpr int GX = S / TN;
    constexpr int EA = S * BK / NT, TPA = BK / EA;
    constexpr int EB = BK * S / NT, TPB = S / EB;
    constexpr int NS = S / BK;
    static_assert(EA * NT == S * BK && EB * NT == S * BK, "slice split");
    static_assert(TPA * EA == BK && TPB * EB == S, "slice rows");
    static_assert(!VEC || (EA % 4 == 0 && EB % 4 == 0 && TN % 4 == 0), "vector split");
    static_assert(BK % 2 == 0, "k-steps are taken in pairs");

    T(*As)[BK][S] = reinterpret_cast<T(*)[BK][S]>(smem);
    uint64_t(*Bk)[BK][S] = reinterpret_cast<uint64_t(*)[BK][S]>(smem + 2 * BK * S * sizeof(T));

    const int tid = threadIdx.x;
    const int tx = tid % GX, ty = tid / GX;
    const int row0 = bi * S, col0 = bj * S, k0 = b * S;
    const bool full = (row0 + S <= n) && (col0 + S <= n) && (k0 + S <= n);
    const int ia = tid / TPA, ka = (tid % TPA) * EA;
    const int kbr = tid / TPB, jb = (tid % TPB) * EB;

    T ra[EA], rb[EB];
    int32_t rp[EB];
    auto fetch = [&](int s) {
        row_load<T, EA, VEC>(ra, d, row0 + ia, k0 + s * BK + ka, n, ld, full, kI32Inf);
        row_load<T, EB, VEC>(rb, d, k0 + s * BK + kbr, col0 + jb, n, ld, full, kI32Inf);
        row_load<int32_t, EB, VEC>(rp, P, k0 + s * BK + kbr, col0 + jb, n, ldp, full, kPredNone);
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int e = 0; e < EA; ++e) As[buf][ka + e][ia] = ra[e];
#pragma unroll
        for (int e = 0; e < EB; ++e) Bk[buf][kbr][jb + e] = make_key(rb[e], rp[e]);
    };

    uint64_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        T cd[TN];
        int32_t cp[TN];
        row_load<T, TN, VEC>(cd, d, row0 + ty * TM + i, col0 + tx * TN, n, ld, full, kI32Inf);
        row_load<int32_t, TN, VEC>(cp, P, row0 + ty * TM + i, col0 + tx * TN, n, ldp, full,
                                   kPredNone);
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = make_key(cd[j], cp[j]);
    }
    fetch(0);
    stash(0);
    __syncthreads();

    for (int s = 0; s < NS; ++s) {
        const int cur = s & 1;
        if (s + 1 < NS) fetch(s + 1);
#pragma unroll 1
        for (int kk = 0; kk < BK; kk += 2) {
            T a0[TM], a1[TM];
            uint64_t b0[TN], b1[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                a0[i] = As[cur][kk][ty * TM + i];
                a1[i] = As[cur][kk + 1][ty * TM + i];
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                b0[j] = Bk[cur][kk][tx * TN + j];
                b1[j] = Bk[cur][kk + 1][tx * TN + j];
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const uint64_t c0 = ((uint64_t)(uint32_t)a0[i] << 32) + b0[j];
                    const uint64_t c1 = ((uint64_t)(uint32_t)a1[i] << 32) + b1[j];
                    uint64_t v = acc[i][j];
                    v = (int64_t)c0 < (int64_t)v ? c0 : v;
                    v = (int64_t)c1 < (int64_t)v ? c1 : v;
                    acc[i][j] = v;
                }
        }
        if (s + 1 < NS) stash(cur ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < TM; ++i) {
        T cd[TN];
        int32_t cp[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            cd[j] = (int32_t)(uint32_t)(acc[i][j] >> 32);
            cp[j] = (int32_t)(uint32_t)acc[i][j];
        }
        row_store<T, TN, VEC>(cd, d, row0 + ty * TM + i, col0 + tx * TN, n, ld, full);
        row_store<int32_t, TN, VEC>(cp, P, row0 + ty * TM + i, col0 + tx * TN, n, ldp, full);
    }
}

// ---------------------------------------------------------------------------
// strip_tile: the panel update of product_tile on one strip of a panel tile,
// R rows x CW columns with the full k-block of K, so that a stage's 2(nb-1)
// panel tiles give four times as many workgroups (one 128 x 128 tile per
// workgroup leaves a CU with a single wave per SIMD).  A row-panel tile is
// cut into column strips and a column-panel tile into row strips: the panel
// operand a strip reads (its own columns of B, or its own rows of A) is then
// exactly the part it writes, and no two workgroups touch the same cell.
// Same per-cell candidates as product_tile, hence the same bits.
// ---------------------------------------------------------------------------
template <typename T, int R, int CW, int K, int BK>
constexpr int strip_smem_bytes() {
    return 2 * BK * (R + CW) * (int)sizeof(T);
}

// With the keyed policy and `acol` non-NULL (a column-panel strip of a 128-
// wide sweep), the strip also writes its cells with the hop field cleared to
// acol (row r, column c - col0 at acol[r * CW + c - col0]): the bulk's A
// operand, ready to be added.
template <typename T, int R, int CW, int K, int BK, int TM, int TN, bool VEC, class A = Ar<T>>
__device__ __forceinline__ void strip_tile(T *__restrict__ d, int n, int64_t ld, int row0,
                                           int col0, int k0, char *smem,
                                           int32_t *flag = nullptr, T *acol = nullptr) {
    constexpr int GX = CW / TN, GY = R / TM, NT = GX * GY;
    constexpr int EA = R * BK / NT, TPA = BK / EA;   // A slice: elements per thread
    constexpr int EB = BK * CW / NT, TPB = CW / EB;  // B slice
    constexpr int NS = K / BK;
    static_assert(EA * NT == R * BK && EB * NT == BK * CW, "slice split");
    static_assert(TPA * EA == BK && TPB * EB == CW, "slice rows");
    static_assert(!VEC || TN % 4 == 0, "vector split");
    // a slice share of fewer than 4 values per thread is loaded element-wise
    constexpr bool VA = VEC && EA % 4 == 0, VB = VEC && EB % 4 == 0;
    static_assert(BK % 2 == 0 && K % BK == 0, "k-steps are fused in pairs");

    T(*As)[BK][R] = reinterpret_cast<T(*)[BK][R]>(smem);
    T(*Bs)[BK][CW] = reinterpret_cast<T(*)[BK][CW]>(smem + 2 * BK * R * sizeof(T));

    const int tid = threadIdx.x;
    const int tx = tid % GX, ty = tid / GX;
    const bool full = (row0 + R <= n) && (col0 + CW <= n) && (k0 + K <= n);
    const T INF = A::inf();
    const int ia = tid / TPA, ka = (tid % TPA) * EA;
    const int kbr = tid / TPB, jb = (tid % TPB) * EB;

    T ra[EA], rb[EB];
    auto fetch = [&](int s) {
        row_load<T, EA, VA>(ra, d, row0 + ia, k0 + s * BK + ka, n, ld, full, INF);
        row_load<T, EB, VB>(rb, d, k0 + s * BK + kbr, col0 + jb, n, ld, full, INF);
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int e = 0; e < EA; ++e) As[buf][ka + e][ia] = ra[e];
#pragma unroll
        for (int e = 0; e < EB; ++e) Bs[buf][kbr][jb + e] = rb[e];
    };

    T acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
        row_load<T, TN, VEC>(acc[i], d, row0 + ty * TM + i, col0 + tx * TN, n, ld, full, INF);
    fetch(0);
    stash(0);
    __syncthreads();
    for (int s = 0; s < NS; ++s) {
        const int cur = s & 1;
        if (s + 1 < NS) fetch(s + 1);
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
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = A::min3(acc[i][j], A::add(a0[i], b0[j]), A::add(a1[i], b1[j]));
        }
        if (s + 1 < NS) stash(cur ^ 1);
        __syncthreads();
    }
    if constexpr (A::kChecked) {
        KeyCheck bad;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = settle<A>(acc[i][j], bad);
        raise_flag<A>(flag, bad);
        if (acol) {
            static_assert(TN % 4 == 0, "16-byte pieces");
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int r = row0 + ty * TM + i;
                T *dst = acol + (int64_t)r * CW + tx * TN;
                if (full) {
#pragma unroll
                    for (int j = 0; j < TN; j += 4) {
                        typename Vec4<T>::type x;
                        x[0] = A::clear_hop(acc[i][j]);
                        x[1] = A::clear_hop(acc[i][j + 1]);
                        x[2] = A::clear_hop(acc[i][j + 2]);
                        x[3] = A::clear_hop(acc[i][j + 3]);
                        *reinterpret_cast<typename Vec4<T>::type *>(dst + j) = x;
                    }
                } else if (r < n) {
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        if (col0 + tx * TN + j < n) dst[j] = A::clear_hop(acc[i][j]);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
        row_store<T, TN, VEC>(acc[i], d, row0 + ty * TM + i, col0 + tx * TN, n, ld, full);
}

// Tile coordinates of the stage-b panel tile number idx (0 <= idx < 2m,
// m = nb - 1): the row panel (b, j != b) first, then the column panel.
__device__ __forceinline__ void panel_coords(int idx, int b, int m, int &bi, int &bj) {
    if (idx < m) {
        bi = b;
        bj = idx < b ? idx : idx + 1;
    } else {
        idx -= m;
        bi = idx < b ? idx : idx + 1;
        bj = b;
    }
}

// Tile coordinates of the stage-b bulk tile number idx (0 <= idx < m^2).
__device__ __forceinline__ void bulk_coords(int idx, int b, int m, int &bi, int &bj) {
    const int q = idx / m, r = idx - q * m;
    bi = q < b ? q : q + 1;
    bj = r < b ? r : r + 1;
}

// Bulk tiles of stage b (b < nb - 1) that lie in the last block row or
// column, nb - 1 being a partial block: 2m - 1 of them (m = nb - 1).  The
// other bulk tiles are the (m - 1)^2 of bulk_coords over the first nb - 1
// blocks.
__device__ __forceinline__ void edge_coords(int idx, int b, int m, int &bi, int &bj) {
    if (idx < m) {
        bi = m;
        bj = idx < b ? idx : idx + 1;
    } else {
        idx -= m;
        bi = idx < b ? idx : idx + 1;
        bj = m;
    }
}

}  // namespace fw
