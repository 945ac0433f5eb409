// Reachability (transitive closure) on bit-packed adjacency matrices: the
// blocked schedule of section 3.2 over the boolean semiring (OR for min, AND
// for +).  Row i of the n x n matrix is ceil(n / 32) 32-bit words; bit j % 32
// of word j / 32 is the edge (or, after the solve, the path) i -> j.  A cell
// update of the bulk ("row i gains row k if i reaches k") is one
// v_and_or_b32 per 32 cells: the bit of i -> k, sign-extended to a full-word
// mask, ANDed with word w of row k and ORed into word w of row i.
//
// k-blocks are 256 bits (8 words) wide; stage b runs
//   bits_diag_kernel       the 256 x 256 diagonal block, closed by one wave
//                          (Warshall's k-ordered steps, row k broadcast from
//                          its owner lane with v_readlane);
//   bits_row_panel_kernel  rows of block b, every other 8-word column block:
//                          P <- P | D* x P (D* the closed diagonal block);
//   bits_col_panel_kernel  columns of block b, every other 256-row block:
//                          C <- C | C x D*;
//   bits_bulk_kernel       the rest: X <- X | C x P.
// As for distances, the panel and bulk steps are products with closed
// blocks, so the result is exact reachability; OR is idempotent, so nothing
// depends on the order of the updates.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fwapsp.h"
#include "fw_internal.h"

namespace fw {
namespace {

constexpr int kBW = 8;          // words per k-block
constexpr int kBK = 32 * kBW;   // bits (vertices) per k-block

// all ones where bit t of x is set, else 0 (v_bfe_i32)
__device__ __forceinline__ uint32_t bitmask(uint32_t x, int t) {
    return (uint32_t)__builtin_amdgcn_sbfe((int)x, t, 1);
}

// (m & p) | acc.  With m from v_bfe_i32 the compiler selects one
// v_and_or_b32 per 32 cells.
__device__ __forceinline__ uint32_t and_or(uint32_t m, uint32_t p, uint32_t acc) {
    return (m & p) | acc;
}

// The same, written out as the instruction for the bulk kernel's unrolled
// k loop, where the compiler otherwise merges the ORs of two k steps into a
// v_or3_b32 fed by two v_and_b32 (1.5 instructions per 32 cells instead of
// 1).  Pure vector ALU on vector registers, no memory access.
__device__ __forceinline__ uint32_t and_or_v(uint32_t m, uint32_t p, uint32_t acc) {
    uint32_t d;
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(d) : "v"(m), "v"(p), "v"(acc));
    return d;
}

// Sets bit (i, i) for every vertex: the reflexive closure.
__global__ void __launch_bounds__(256)
bits_reflexive_kernel(uint32_t *__restrict__ bits, int n, int64_t ldw) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) bits[(int64_t)i * ldw + (i >> 5)] |= 1u << (i & 31);
}

// Closure of a 256 x 256 diagonal block by a workgroup of 256 threads,
// thread t holding row t (8 words) in x.  The block is cut into eight
// 32-vertex sub-blocks K, taken in order (the blocked schedule once more,
// one level down).  For each K:
//   1. the wave holding K's 32 rows closes their word of K alone (32
//      k-ordered steps on one word, row k broadcast by v_readlane): D*;
//   2. every row i closes its own word of K through D*:
//      y' = y | OR over k in y of D*[k];
//   3. every row ORs in the old rows k (all 8 words, staged in LDS before
//      step 1) selected by y'.
// Steps 2-3 give exactly the result of the 32 Warshall steps over K: a
// vertex reached from i through K is reached by a first hop into K followed
// by a path inside K, whose last vertex's old row holds the target.  (For a
// row of K, y' is its closed row D*.)  Rows past n hold 0 and stay 0.
// lds: 32 x 8 + 32 words.  kreal is the number of the block's vertices below n.
__device__ __forceinline__ void close_block_wg(uint32_t (&x)[kBW], uint32_t *lds, int kreal) {
    const int t = threadIdx.x, wave = t >> 6;
    uint32_t(*R)[kBW] = reinterpret_cast<uint32_t(*)[kBW]>(lds);  // old rows of K
    uint32_t *Dk = lds + 32 * kBW;                                 // D*, word K of K's rows
#pragma unroll
    for (int kb = 0; kb < kBW; ++kb) {
        if (32 * kb >= kreal) break;  // uniform
        const bool in_k = (t >> 5) == kb;
        if (in_k) {
#pragma unroll
            for (int c = 0; c < kBW; ++c) R[t & 31][c] = x[c];
        }
        if (wave == (kb >> 1)) {
            // lanes of the other half compute nothing that is kept
            const int base = 32 * (kb & 1);
            const int steps = kreal - 32 * kb;
            uint32_t d = x[kb];
            if (steps >= 32) {
#pragma unroll
                for (int s = 0; s < 32; ++s) {
                    const uint32_t rk = (uint32_t)__builtin_amdgcn_readlane((int)d, base + s);
                    d = and_or(bitmask(d, s), rk, d);
                }
            } else {  // the last block's last vertices
#pragma unroll 1
                for (int s = 0; s < steps; ++s) {
                    const uint32_t rk = (uint32_t)__builtin_amdgcn_readlane((int)d, base + s);
                    d = and_or(bitmask(d, s), rk, d);
                }
            }
            if (in_k) Dk[t & 31] = d;
        }
        __syncthreads();
        const uint32_t y0 = x[kb];
        uint32_t y = y0;
#pragma unroll 8
        for (int s = 0; s < 32; ++s) y = and_or(bitmask(y0, s), Dk[s], y);
#pragma unroll 4
        for (int s = 0; s < 32; ++s) {
            const uint32_t m = bitmask(y, s);
            const uint4 ra = *reinterpret_cast<const uint4 *>(&R[s][0]);
            const uint4 rb = *reinterpret_cast<const uint4 *>(&R[s][4]);
            x[0] = and_or(m, ra.x, x[0]);
            x[1] = and_or(m, ra.y, x[1]);
            x[2] = and_or(m, ra.z, x[2]);
            x[3] = and_or(m, ra.w, x[3]);
            x[4] = and_or(m, rb.x, x[4]);
            x[5] = and_or(m, rb.y, x[5]);
            x[6] = and_or(m, rb.z, x[6]);
            x[7] = and_or(m, rb.w, x[7]);
        }
        __syncthreads();  // R and Dk are rewritten for the next K
    }
}

// Stage b's diagonal block (stage 0 only: every later diagonal block is
// closed inside the previous stage's bulk launch).  Thread t owns row k0 + t.
__global__ void __launch_bounds__(256)
bits_diag_kernel(uint32_t *__restrict__ bits, int n, int64_t ldw, int nw, int b) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[32 * kBW + 32];
    const int t = threadIdx.x;
    const int k0 = b * kBK, w0 = b * kBW;
    const int i = k0 + t;
    uint32_t x[kBW];
#pragma unroll
    for (int c = 0; c < kBW; ++c) x[c] = (i < n && w0 + c < nw) ? bits[(int64_t)i * ldw + w0 + c] : 0u;
    close_block_wg(x, lds, n - k0 < kBK ? n - k0 : kBK);
#pragma unroll
    for (int c = 0; c < kBW; ++c)
        if (i < n && w0 + c < nw) bits[(int64_t)i * ldw + w0 + c] = x[c];
}

// The panels of stage b, each workgroup on kPW of a word block's 8 words:
// the update of one word depends only on that word's column slice and on
// the masks, so the 8 words split over kBW / kPW workgroups.  That fills the
// GPU (8 (nb - 1) workgroups at kPW = 2) and shortens each workgroup's chain
// of 256 dependent k steps per word.
constexpr int kPW = 2;
constexpr int kParts = kBW / kPW;

// Row panel: rows of block b, words w0 .. w0 + kPW - 1 of word block wb != b.
// Thread t owns row k0 + t; the slice of every row of the block is staged in
// S (old values) before any is written.
__device__ __forceinline__ void row_panel(uint32_t (*S)[kPW], uint32_t *__restrict__ bits, int n,
                                          int64_t ldw, int nw, int b, int w0) {
    const int t = threadIdx.x;
    const int k0 = b * kBK;
    const int i = k0 + t;
    const bool row_ok = i < n;
    uint32_t dk[kBW], acc[kPW];
#pragma unroll
    for (int c = 0; c < kBW; ++c)  // the thread's row of the closed diagonal block (its masks)
        dk[c] = (row_ok && b * kBW + c < nw) ? bits[(int64_t)i * ldw + b * kBW + c] : 0u;
#pragma unroll
    for (int c = 0; c < kPW; ++c) {
        acc[c] = (row_ok && w0 + c < nw) ? bits[(int64_t)i * ldw + w0 + c] : 0u;
        S[t][c] = acc[c];
    }
    __syncthreads();
#pragma unroll
    for (int cw = 0; cw < kBW; ++cw) {
#pragma unroll 8
        for (int s = 0; s < 32; ++s) {
            const uint32_t m = bitmask(dk[cw], s);
            const int k = 32 * cw + s;
#pragma unroll
            for (int c = 0; c < kPW; ++c) acc[c] = and_or(m, S[k][c], acc[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < kPW; ++c)
        if (row_ok && w0 + c < nw) bits[(int64_t)i * ldw + w0 + c] = acc[c];
}

// Column panel: words w0 .. w0 + kPW - 1 (inside word block b) of the rows of
// row block rb != b.  Thread t owns row 256 rb + t; its masks are its whole
// old word block b (the product with the closed block needs no order); the
// closed diagonal block's slice is staged in S.
__device__ __forceinline__ void col_panel(uint32_t (*S)[kPW], uint32_t *__restrict__ bits, int n,
                                          int64_t ldw, int nw, int b, int rb, int w0) {
    const int t = threadIdx.x;
    const int k0 = b * kBK, wb0 = b * kBW;
    {
        const int k = k0 + t;
#pragma unroll
        for (int c = 0; c < kPW; ++c)
            S[t][c] = (k < n && w0 + c < nw) ? bits[(int64_t)k * ldw + w0 + c] : 0u;
    }
    const int i = rb * kBK + t;
    const bool row_ok = i < n;
    uint32_t y[kBW], acc[kPW];
#pragma unroll
    for (int c = 0; c < kBW; ++c) y[c] = (row_ok && wb0 + c < nw) ? bits[(int64_t)i * ldw + wb0 + c] : 0u;
#pragma unroll
    for (int c = 0; c < kPW; ++c) acc[c] = y[w0 - wb0 + c];
    __syncthreads();
#pragma unroll
    for (int cw = 0; cw < kBW; ++cw) {
#pragma unroll 8
        for (int s = 0; s < 32; ++s) {
            const uint32_t m = bitmask(y[cw], s);
            const int k = 32 * cw + s;
#pragma unroll
            for (int c = 0; c < kPW; ++c) acc[c] = and_or(m, S[k][c], acc[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < kPW; ++c)
        if (row_ok && w0 + c < nw) bits[(int64_t)i * ldw + w0 + c] = acc[c];
}

// Both panels of stage b in one launch of 2 (nb - 1) kParts workgroups: the
// first half takes the row panel's word blocks, the rest the column panel's
// row blocks, kParts workgroups per block.  The two panels write disjoint
// words and read only their own words and the closed diagonal block.
__global__ void __launch_bounds__(256)
bits_panel_kernel(uint32_t *__restrict__ bits, int n, int64_t ldw, int nw, int b, int nb) {
    __shared__ uint32_t S[kBK][kPW];
    const int x = (int)blockIdx.x / kParts, part = (int)blockIdx.x % kParts;
    if (x < nb - 1) {
        const int wb = x < b ? x : x + 1;
        row_panel(S, bits, n, ldw, nw, b, wb * kBW + kPW * part);
    } else {
        const int y = x - (nb - 1);
        col_panel(S, bits, n, ldw, nw, b, y < b ? y : y + 1, b * kBW + kPW * part);
    }
}

// Inside the bulk launch of stage b: applies stage b to diagonal block b + 1
// (X <- X | C x P over the 256 vertices of block b, as every bulk tile does)
// and closes it, so stage b + 1 needs no diagonal launch.  Block b is full
// here (it is not the last block).  The bulk tiles leave block b + 1's
// diagonal words to this workgroup.
__device__ __forceinline__ void bulk_close_next(uint32_t *L, uint32_t *__restrict__ bits, int n,
                                                int64_t ldw, int nw, int b) {
    // This workgroup's waves share their SIMDs with bulk waves, and the next
    // stage waits for its result: let them issue first whenever they are
    // ready.
    __builtin_amdgcn_s_setprio(3);
    const int t = threadIdx.x;
    const int k0 = b * kBK, k1 = k0 + kBK, w0 = b * kBW, w1 = w0 + kBW;
    const int i = k1 + t;
    const bool row_ok = i < n;
    uint32_t(*Pn)[kBW] = reinterpret_cast<uint32_t(*)[kBW]>(L);  // row panel, words of block b+1
    uint32_t y[kBW], acc[kBW];
#pragma unroll
    for (int c = 0; c < kBW; ++c) {
        Pn[t][c] = (w1 + c < nw) ? bits[(int64_t)(k0 + t) * ldw + w1 + c] : 0u;
        y[c] = row_ok ? bits[(int64_t)i * ldw + w0 + c] : 0u;
        acc[c] = (row_ok && w1 + c < nw) ? bits[(int64_t)i * ldw + w1 + c] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int cw = 0; cw < kBW; ++cw) {
#pragma unroll 4
        for (int s = 0; s < 32; ++s) {
            const uint32_t m = bitmask(y[cw], s);
            const int k = 32 * cw + s;
#pragma unroll
            for (int c = 0; c < kBW; ++c) acc[c] = and_or(m, Pn[k][c], acc[c]);
        }
    }
    __syncthreads();  // Pn is read no more; its space is reused
    close_block_wg(acc, L, n - k1 < kBK ? n - k1 : kBK);
#pragma unroll
    for (int c = 0; c < kBW; ++c)
        if (row_ok && w1 + c < nw) bits[(int64_t)i * ldw + w1 + c] = acc[c];
}

// Bulk: 64 rows x 128 words per workgroup (rows outside block b; the words
// of block b, the column panel, are not written).  Thread (tx, ty) owns rows
// 4 ty .. 4 ty + 3 and words 4 tx .. 4 tx + 3 and 64 + 4 tx .. 64 + 4 tx + 3
// of the tile (two 16-byte LDS reads per k, each contiguous across tx).  The
// rows of the row panel are staged in LDS 32 k at a time; the next 32 are
// loaded into registers while the current ones are applied.
//
// Loads are unconditional from clamped addresses: a row past n or a word
// past the last one reads some valid word instead.  Such values only reach
// accumulators that are never stored (rows past n, words past the last), or
// row-panel rows past n, whose masks are cleared (bits of vertices >= n are
// dropped from the column-panel words before use).
constexpr int kTR = 64, kTW = 128;

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
bits_bulk_kernel(uint32_t *__restrict__ bits, int n, int64_t ldw, int nw, int b, int nrt, int nwt,
                 int close_next) {
    __shared__ __attribute__((aligned(16))) uint32_t P[32][kTW];
    if (close_next && blockIdx.x == 0) {  // first, so it starts at once
        bulk_close_next(&P[0][0], bits, n, ldw, nw, b);
        return;
    }
    const int tile = (int)blockIdx.x - close_next;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int k0 = b * kBK, wk0 = b * kBW;
    // row tiles of block b (rows k0 .. k0 + 255) are skipped
    const int skip0 = k0 / kTR, nskip = (nrt - skip0) < 4 ? (nrt - skip0) : 4;
    const int ty_tile = tile / nwt;
    const int rt = ty_tile < skip0 ? ty_tile : ty_tile + nskip;
    const int row0 = rt * kTR, col0 = (tile - ty_tile * nwt) * kTW;
    // block b + 1's diagonal words, written by the closing workgroup
    const int k1 = k0 + kBK, wk1 = wk0 + kBW;
    auto word_of = [&](int j) { return col0 + (j < 4 ? 4 * tx + j : 64 + 4 * tx + j - 4); };
    auto clampi = [](int v, int hi) { return v < hi ? v : hi; };

    // this thread's rows, clamped
    const uint32_t *rowp[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) rowp[r] = bits + (int64_t)clampi(row0 + 4 * ty + r, n - 1) * ldw;
    // The accumulators start at 0, the identity of OR; the tile's own words
    // are loaded during the last slice and ORed in at the end, so the launch
    // does not start with every workgroup waiting on HBM at once.
    uint32_t acc[4][8];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[r][j] = 0u;

    // row-panel staging: thread loads word (tid & 127) of rows 2 e + (tid >> 7);
    // the row is the same across a wave, so its address is scalar work
    const int wl = tid & (kTW - 1);
    const int kl = __builtin_amdgcn_readfirstlane(tid >> 7);
    const int wcl = clampi(col0 + wl, nw - 1);
    const int klast = n - 1 - k0;  // last valid row of the block, relative
    uint32_t pf[16], yn[4];
    auto fetch = [&](int cw) {
#pragma unroll
        for (int e = 0; e < 16; ++e)
            pf[e] = bits[(int64_t)(k0 + clampi(32 * cw + 2 * e + kl, klast)) * ldw + wcl];
        const int wy = clampi(wk0 + cw, nw - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) yn[r] = rowp[r][wy];
    };
    auto slice = [&](int cw) {
        __syncthreads();  // every wave is done with the previous slice
#pragma unroll
        for (int e = 0; e < 16; ++e) P[2 * e + kl][wl] = pf[e];
        // bits 32 cw .. 32 cw + 31 of block b in the thread's rows (the
        // column panel, final since the panel launch), vertices >= n dropped
        const int valid = n - (k0 + 32 * cw);
        const uint32_t vmask = valid >= 32 ? ~0u : valid <= 0 ? 0u : (1u << valid) - 1u;
        uint32_t yw[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) yw[r] = yn[r] & vmask;
        __syncthreads();
        if (cw + 1 < kBW) fetch(cw + 1);
        // the LDS words of step s + 1 are read before step s is applied (the
        // compiler keeps the written order around the and_or statements)
        uint4 pa = *reinterpret_cast<const uint4 *>(&P[0][4 * tx]);
        uint4 pb = *reinterpret_cast<const uint4 *>(&P[0][64 + 4 * tx]);
#pragma unroll
        for (int s = 0; s < 32; ++s) {
            uint4 na = pa, nb = pb;
            if (s + 1 < 32) {
                na = *reinterpret_cast<const uint4 *>(&P[s + 1][4 * tx]);
                nb = *reinterpret_cast<const uint4 *>(&P[s + 1][64 + 4 * tx]);
            }
            const uint32_t p[8] = {pa.x, pa.y, pa.z, pa.w, pb.x, pb.y, pb.z, pb.w};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t m = bitmask(yw[r], s);
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[r][j] = and_or_v(m, p[j], acc[r][j]);
            }
            pa = na;
            pb = nb;
        }
    };
    fetch(0);
    for (int cw = 0; cw < kBW - 1; ++cw) slice(cw);
    uint32_t x[4][8];  // the tile's own words, in flight during the last slice
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < 8; ++j) x[r][j] = rowp[r][clampi(word_of(j), nw - 1)];
    slice(kBW - 1);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[r][j] |= x[r][j];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = row0 + 4 * ty + r;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int w = word_of(j);
            const bool diag1 = close_next && i >= k1 && i < k1 + kBK && w >= wk1 && w < wk1 + kBW;
            if (i < n && w < nw && (w < wk0 || w >= wk0 + kBW) && !diag1)
                bits[(int64_t)i * ldw + w] = acc[r][j];
        }
    }
}

// Pack / unpack between an int32 0/1 matrix and the bit layout, one wave per
// 512 columns of a row (8 coalesced 256-byte accesses per wave); waves stride
// over the groups, so the grid stays bounded for any n.  Pack: each lane
// reads one int per 64-column chunk and the wave's ballot is the chunk's two
// words (lanes 0 and 1 store them).  Unpack: each lane writes one int per
// chunk from the word holding its bit.
constexpr int kPackCols = 512;
constexpr int64_t kPackMaxBlocks = 1 << 20;

// the first group of the calling wave (wave-uniform: scalar arithmetic)
__device__ __forceinline__ int64_t first_group() {
    return (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__global__ void __launch_bounds__(256)
bits_pack_kernel(const int32_t *__restrict__ adj, int n, int64_t ld, uint32_t *__restrict__ bits,
                 int64_t ldw, int nw) {
    const int lane = threadIdx.x & 63;
    const int ng = (n + kPackCols - 1) / kPackCols;
    const int64_t groups = (int64_t)n * ng, stride = (int64_t)gridDim.x * 4;
    for (int64_t grp = first_group(); grp < groups; grp += stride) {
        const int i = (int)(grp / ng), g = (int)(grp - (int64_t)(grp / ng) * ng);
        const int32_t *row = adj + (int64_t)i * ld;
        bool e[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = kPackCols * g + 64 * q + lane;
            e[q] = j < n && row[j] != 0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint64_t m = __ballot(e[q]);
            const int w = 16 * g + 2 * q + lane;
            if (lane < 2 && w < nw) bits[(int64_t)i * ldw + w] = (uint32_t)(m >> (32 * lane));
        }
    }
}

__global__ void __launch_bounds__(256)
bits_unpack_kernel(const uint32_t *__restrict__ bits, int n, int64_t ldw, int32_t *__restrict__ adj,
                   int64_t ld) {
    const int lane = threadIdx.x & 63;
    const int ng = (n + kPackCols - 1) / kPackCols;
    const int64_t groups = (int64_t)n * ng, stride = (int64_t)gridDim.x * 4;
    for (int64_t grp = first_group(); grp < groups; grp += stride) {
        const int i = (int)(grp / ng), g = (int)(grp - (int64_t)(grp / ng) * ng);
        const uint32_t *brow = bits + (int64_t)i * ldw;
        int32_t *row = adj + (int64_t)i * ld;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = kPackCols * g + 64 * q + lane;
            if (j < n) row[j] = (int32_t)((brow[j >> 5] >> (j & 31)) & 1u);
        }
    }
}

// One stage's launches, each timed as its own phase kind when profiling is on.
struct BitsStage {
    uint32_t *bits;
    int n, nw, b, nb, nrt, nwt, close_next;
    int64_t ldw;
    hipStream_t st;
};

hipError_t run_bits_diag(void *c) {
    const auto *a = static_cast<const BitsStage *>(c);
    bits_diag_kernel<<<1, 256, 0, a->st>>>(a->bits, a->n, a->ldw, a->nw, a->b);
    return hipGetLastError();
}

hipError_t run_bits_panels(void *c) {
    const auto *a = static_cast<const BitsStage *>(c);
    bits_panel_kernel<<<(unsigned)(2 * (a->nb - 1) * kParts), 256, 0, a->st>>>(a->bits, a->n, a->ldw,
                                                                             a->nw, a->b, a->nb);
    return hipGetLastError();
}

hipError_t run_bits_bulk(void *c) {
    const auto *a = static_cast<const BitsStage *>(c);
    const int skip0 = a->b * kBK / kTR;
    const int nskip = (a->nrt - skip0) < 4 ? (a->nrt - skip0) : 4;
    const int64_t groups = (int64_t)a->nwt * (a->nrt - nskip) + a->close_next;
    bits_bulk_kernel<<<(unsigned)groups, 256, 0, a->st>>>(a->bits, a->n, a->ldw, a->nw, a->b, a->nrt,
                                                         a->nwt, a->close_next);
    return hipGetLastError();
}

int status_of(hipError_t e) {
    if (e == hipSuccess) return FW_OK;
    if (e == hipErrorOutOfMemory) return FW_ERR_NOMEM;
    return FW_ERR_HIP;
}

int64_t words_of(int64_t n) { return (n + 31) / 32; }

constexpr int64_t kMaxBitsN = 1LL << 21;

// workgroups of the pack / unpack launches: four 512-column groups (one per
// wave) each, at most kPackMaxBlocks (the waves then loop)
int64_t pack_blocks(int64_t n) {
    const int64_t g = (n * ((n + kPackCols - 1) / kPackCols) + 3) / 4;
    return g < kPackMaxBlocks ? g : kPackMaxBlocks;
}

// ceil(a / b) blocks of a 1-D launch over `count` items, or -1 if too many
int64_t blocks_for(int64_t count) {
    const int64_t g = (count + 255) / 256;
    return g > 0x7fffffffLL ? -1 : g;
}

}  // namespace
}  // namespace fw

using namespace fw;

extern "C" {

int fw_transitive_closure_bits(uint32_t *bits, int64_t n, int64_t ldw, int reflexive,
                               void *stream) {
    if (n < 0 || (n > 0 && !bits) || ldw < words_of(n)) return FW_ERR_INVALID;
    // past 2^21 vertices (a 512 GiB matrix) the bulk grid would overflow
    if (n > kMaxBitsN || ldw > (1LL << 40) / (n > 0 ? n : 1)) return FW_ERR_UNSUPPORTED;
    if (n == 0) return FW_OK;
    hipStream_t st = (hipStream_t)stream;
    const int nn = (int)n, nw = (int)words_of(n);
    if (reflexive) {
        bits_reflexive_kernel<<<(unsigned)blocks_for(n), 256, 0, st>>>(bits, nn, ldw);
        if (hipGetLastError() != hipSuccess) return FW_ERR_HIP;
    }
    const int nb = (nn + kBK - 1) / kBK;          // k-blocks = row blocks = word blocks
    const int nrt = (nn + kTR - 1) / kTR;         // bulk row tiles
    const int nwt = (nw + kTW - 1) / kTW;         // bulk word tiles
    for (int b = 0; b < nb; ++b) {
        // cell updates of each phase (for the profile counters): kb vertices
        // in block b, the rest of the matrix outside it
        const double kb = (double)(nn - b * kBK < kBK ? nn - b * kBK : kBK), rest = (double)nn - kb;
        BitsStage a{bits, nn, nw, b, nb, nrt, nwt, b + 1 < nb ? 1 : 0, ldw, st};
        hipError_t e = hipSuccess;
        // later diagonal blocks are closed by the previous bulk launch
        if (b == 0) e = timed_launch(kBitsDiag, kb * kb * kb, st, run_bits_diag, &a);
        if (e == hipSuccess && nb > 1) {
            e = timed_launch(kBitsPanel, 2.0 * rest * kb * kb, st, run_bits_panels, &a);
            // the bulk launch also closes block b + 1 (kn vertices)
            const double kn = a.close_next ? (double)(nn - (b + 1) * kBK < kBK ? nn - (b + 1) * kBK : kBK) : 0.0;
            if (e == hipSuccess)
                e = timed_launch(kBitsBulk, rest * rest * kb + kn * kn * kn, st, run_bits_bulk, &a);
        }
        if (e != hipSuccess) return status_of(e);
    }
    return FW_OK;
}

int fw_pack_bits(const int32_t *adj, int64_t n, int64_t ld, uint32_t *bits, int64_t ldw,
                 void *stream) {
    if (n < 0 || (n > 0 && (!adj || !bits)) || ld < n || ldw < words_of(n))
        return FW_ERR_INVALID;
    if (n == 0) return FW_OK;
    if (n > kMaxBitsN) return FW_ERR_UNSUPPORTED;
    const int64_t g = pack_blocks(n);
    bits_pack_kernel<<<(unsigned)g, 256, 0, (hipStream_t)stream>>>(adj, (int)n, ld, bits, ldw,
                                                                    (int)words_of(n));
    return status_of(hipGetLastError());
}

int fw_unpack_bits(const uint32_t *bits, int64_t n, int64_t ldw, int32_t *adj, int64_t ld,
                   void *stream) {
    if (n < 0 || (n > 0 && (!adj || !bits)) || ld < n || ldw < words_of(n))
        return FW_ERR_INVALID;
    if (n == 0) return FW_OK;
    if (n > kMaxBitsN) return FW_ERR_UNSUPPORTED;
    const int64_t g = pack_blocks(n);
    bits_unpack_kernel<<<(unsigned)g, 256, 0, (hipStream_t)stream>>>(bits, (int)n, ldw, adj, ld);
    return status_of(hipGetLastError());
}

}  // extern "C"
