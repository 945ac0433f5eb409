// Internal declarations shared by the host driver and the kernel files of
// libfwapsp.  Not part of the public ABI (see include/fwapsp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fw {

constexpr int32_t kI32Inf = 1073741823;   // "no edge" for int32
constexpr int32_t kPredNone = 0x7fffffff; // in-sweep "no last hop yet"

// 32-bit keys of the int32 sweep with predecessors.  A cell's (distance d,
// last hop p) pair is held as key = d * 2^kKeyBits + p with 0 <= p <=
// kKeyHop, so that keys order exactly as the pairs do lexicographically; the
// candidate through k is (key_ik with its hop field cleared) + key_kj, the
// int32 sum of the distances with kj's last hop.  The hop value kKeyHop means
// "no last hop" (it orders after every vertex), so graphs have at most
// kKeyMaxN vertices.  Real (finite) distances must keep |d| < 2^14, i.e.
// keys in [kKeyLow, kKeyReal); every key at or above kKeyInfFloor is
// infinite and is stored as kKeyInf.  Within those bounds no sum overflows and a finite key
// never meets an infinite one: finite sums lie in (-2^29, 2^29), sums with an
// infinite operand in [kKeyInf - 2^28, 2 kKeyInf] with 2 kKeyInf < 2^31.
constexpr int kKeyBits = 14;
constexpr int32_t kKeyHop = (1 << kKeyBits) - 1;
constexpr int32_t kKeyInf = (1 << 30) - (1 << kKeyBits);
constexpr int32_t kKeyReal = 1 << 28;
constexpr int32_t kKeyLow = -kKeyReal + (1 << kKeyBits);
constexpr int32_t kKeyInfFloor = 1 << 29;
constexpr int kKeyMaxN = kKeyHop;
// Scratch of one keyed solve, int32 words: [0] the fallback flag (set when an
// entry is not a key, a real key left its range or a diagonal went
// negative), [1] set when some pair is unreachable, [2] set when a diagonal
// went negative, [3] the gate of the fp32 canonical path (see
// launch_canon_gate), then the row minima and the column minima of the finite
// distances (n each); from the 64-word (256-byte) boundary after them, the
// current stage's column panel with the hop fields cleared (n rows of 128),
// the A operand of the 128-wide keyed bulk.  fp32 solves add, after that,
// one strip of the original weights (n rows of canon_strip_cols(n)) for the
// canonical path.
constexpr int64_t key_acol_offset(int64_t n) { return (4 + 2 * n + 63) / 64 * 64; }
constexpr int64_t key_scratch_words(int64_t n) { return key_acol_offset(n) + 128 * n; }
constexpr int kCanonStripMax = 1024;
constexpr int canon_strip_cols(int64_t n) {
    return (int)((n + 63) / 64 * 64 < kCanonStripMax ? (n + 63) / 64 * 64 : kCanonStripMax);
}
// dtype: 0 fp32, 1 int32
constexpr int64_t key_scratch_words_for(int dtype, int64_t n) {
    return key_scratch_words(n) + (dtype == 0 ? n * canon_strip_cols(n) : 0);
}
// Scratch of an fp32 canonical path with no keyed sweep before it (graphs
// beyond the keys' vertices): the four flag words as above (64 words), then
// the strip.
constexpr int64_t canon_scratch_words(int64_t n) { return 64 + n * canon_strip_cols(n); }

enum PhaseKind {
    kDiag = 0,
    kPanel = 1,
    kBulk = 2,      // the bulk (+ the next diagonal tile where the kernel closes it)
    kPredFix = 3,
    kBatched = 4,
    kBitsDiag = 5,  // bit-packed reachability: stage 0's diagonal block
    kBitsPanel = 6, // bit-packed reachability: both panels
    kBitsBulk = 7,  // bit-packed reachability: the bulk (+ next diagonal block)
    kPredFallback = 8, // the 64-bit predecessor sweep behind a keyed one (gated)
    kNumKinds = 9
};

// Phase timing for launches made outside the host driver: calls
// launch(ctx), bracketed by HIP events on st while profiling is enabled.
hipError_t timed_launch(int kind, double updates, hipStream_t st, hipError_t (*launch)(void *),
                        void *ctx);

// What the sweep runs over: closed semirings, and kKey, min-plus over the
// 32-bit (distance, last hop) keys above (int32 only, no predecessor matrix:
// the keys are the matrix).
enum Semiring { kMinPlus = 0, kMaxMin = 1, kKey = 2 };

// One stage-phase launch of the blocked schedule.  `d`/`p` are the matrix
// and the (optional) predecessor matrix; `b` is the k-block index, `nb` the
// number of tile rows.  `flag` (kKey only, device int32): set to 1 when a
// real key leaves its range.  `gate` (device int32 or NULL): when non-NULL
// the launch does nothing unless *gate != 0 at the time it runs; min-plus
// only, and without predecessors only at tiles 64 and 32 (the 128-wide
// copy path takes no gate).  Returns hipSuccess or the launch error.
hipError_t launch_diag(int dtype, int sr, int tile, void *d, int32_t *p, int n, int64_t ld,
                       int64_t ldp, int b, hipStream_t st, int32_t *flag = nullptr,
                       const int32_t *gate = nullptr);
hipError_t launch_panels(int dtype, int sr, int tile, void *d, int32_t *p, int n, int64_t ld,
                         int64_t ldp, int b, int nb, hipStream_t st, int32_t *flag = nullptr,
                         const int32_t *gate = nullptr);
// With close_next the launch also closes the next stage's diagonal tile
// (b+1, b+1), which replaces launch_diag(b + 1); allowed exactly when
// bulk_closes_next_diag(sr, tile, d, p, n, ld, b) holds.
hipError_t launch_bulk(int dtype, int sr, int tile, void *d, int32_t *p, int n, int64_t ld,
                       int64_t ldp, int b, int nb, bool close_next, hipStream_t st,
                       int32_t *flag = nullptr, const int32_t *gate = nullptr);
bool bulk_closes_next_diag(int sr, int tile, const void *d, const int32_t *p, int n, int64_t ld,
                           int b);
hipError_t launch_pred_init(int dtype, const void *d, int32_t *p, int n, int64_t ld,
                            int64_t ldp, hipStream_t st, const int32_t *gate = nullptr);
// With a gate, a fix-up that runs also counts one fallback (pred_fallbacks).
hipError_t launch_pred_fix(int dtype, const void *d, int32_t *p, int n, int64_t ld,
                           int64_t ldp, hipStream_t st, const int32_t *gate = nullptr);
// The keyed predecessor solve around the sweep (d int32 or fp32; scratch as
// key_scratch_words): key_prepare zeroes the scratch and writes the keys of
// d into `keys`; key_finish takes the row and column minima, raises the flag
// on a negative diagonal, and -- unless the flag is set -- writes the
// distances into d and the predecessors into `keys`, in place.
hipError_t launch_key_prepare(int dtype, const void *d, int32_t *keys, int n, int64_t ld,
                              int64_t ldk, int32_t *scratch, hipStream_t st);
hipError_t launch_key_finish(int dtype, void *d, int32_t *keys, int n, int64_t ld, int64_t ldk,
                             int32_t *scratch, hipStream_t st);
// The fp32 canonical path, for a keyed solve whose input was not keys (an
// entry not an integer of the key range, or a real key out of range) and
// whose diagonals stayed non-negative: the distances by the distances-only
// sweep, then p_ij = the smallest q != j with (q == i ? 0 : d_iq) + w_qj ==
// d_ij in fp32 arithmetic (-1 for i == j, for unreachable pairs and when no q
// matches), the oracle's definition of the canonical last hop, over the
// original weights.  The predecessor matrix holds the weights meanwhile.
//   canon_gate:  scratch[3] = (direct || scratch[0]) && !scratch[2] (the gate
//                of the rest; direct: no keyed sweep before, scratch[2] the
//                negative-diagonal count of the distances).
//   canon_save:  P = the bits of d (the weights); gated, counts one fallback.
//   canon_strip: strip = columns [j0, j0 + w) of those weights (n x w, ld w).
//   canon_pred:  columns [j0, j0 + w) of P from the final d and the strip.
//   canon_restore: d = the weights saved in P (before the compare form that
//                a negative diagonal takes instead).
// With a gate a launch does nothing unless *gate != 0.
hipError_t launch_canon_gate(int32_t *scratch, bool direct, hipStream_t st);
hipError_t launch_canon_restore(float *d, const int32_t *p, int n, int64_t ld, int64_t ldp,
                                const int32_t *gate, hipStream_t st);
hipError_t launch_canon_save(const float *d, int32_t *p, int n, int64_t ld, int64_t ldp,
                             const int32_t *gate, hipStream_t st);
hipError_t launch_canon_strip(const int32_t *p, int n, int64_t ldp, int j0, int w, float *strip,
                              const int32_t *gate, hipStream_t st);
hipError_t launch_canon_pred(const float *d, int n, int64_t ld, const float *strip, int j0, int w,
                             int32_t *p, int64_t ldp, const int32_t *gate, hipStream_t st);
// Number of gated predecessor fallbacks (64-bit or compare-form sweeps, and
// fp32 canonical paths) that ran on the current device (synchronises the
// device).
int64_t pred_fallbacks();
// Vertices with d_ii < 0, ascending, into list (NULL: not written) and their
// number into *count (device memory).
hipError_t launch_negcycle(int dtype, const void *d, int n, int64_t ld, int32_t *list,
                           int32_t *count, hipStream_t st);

// Descriptor of one graph of a persistent batched launch.
struct BatchItem {
    void *d;
    int32_t *p;
    int64_t ld, ldp;
    int32_t n, tile;
    int32_t vec, pad;
};

// Head of a batched descriptor table (the items follow it).
struct BatchHeader {
    int32_t next;   // work counter, 0 at launch
    int32_t count;  // number of items
    int32_t pad[14];
};

// Persistent batched kernel (fw_batched.hip) and host helpers (fw_api.cpp)
// shared by the batch plans and the server.
// big: some item has a 128-wide tile (selects the kernel form that has the
// 128-wide path; the other one runs more workgroups per CU).  Callers compute
// it from the items with batch_needs_big: the form without the 128-wide path
// cannot solve a 128-wide item.
hipError_t launch_batched_raw(int dtype, bool pred, BatchHeader *hdr, const BatchItem *items,
                              int grid, hipStream_t st, bool big);
bool batch_needs_big(const BatchItem *items, int64_t count);
int batched_resident_grid(int dtype, bool pred);
void fill_batch_item(BatchItem &it, void *d, int dtype, int64_t n, int64_t ld, int32_t *p,
                     int64_t ldp);
// Buffers a caller owns for enqueue_batch_buffered: the descriptor table
// (header + items) and the stage-batched work table, each as pinned host
// memory and a device copy, with their capacities in bytes.  The host
// buffers must stay untouched until the stream has run the copies.
struct BatchBuffers {
    void *host_table, *dev_table;
    size_t table_bytes;
    void *host_work, *dev_work;
    size_t work_bytes;
};
// One batch (no predecessors) through the batch-plan schedule -- stage-
// batched launches, then the persistent kernel for the smallest graphs --
// with the tables staged through `buf` and copied on `st`.
// FW_ERR_UNSUPPORTED when the tables exceed the buffers (nothing enqueued).
int enqueue_batch_buffered(void *const *d, const int64_t *n, const int64_t *ld, int64_t count,
                           int dtype, const BatchBuffers &buf, hipStream_t st);
// Upper bound on the work-table entries one graph adds to a batch.
int64_t batch_work_entries(int dtype, int64_t n, bool pred);
// The plan table's tile for (dtype, n), from the table of solves with
// predecessors when `pred`.
int plan_tile_for(int dtype, int64_t n, bool pred);
// One solve with the given tile, eager launches (pred may be NULL).
int solve_with_tile(void *d, int dtype, int n, int64_t ld, int32_t *pred, int64_t ldp, int tile,
                    hipStream_t st);
int validate_matrix(const void *d, int dtype, int64_t n, int64_t ld, const int32_t *pred,
                    int64_t ldp);
int solve_single(void *d, int dtype, int64_t n, int64_t ld, int32_t *pred, int64_t ldp,
                 hipStream_t st);

// True when the vectorised (16-byte) load/store path may be used for a
// matrix: 16-byte aligned base and a leading dimension divisible by 4.
inline bool vec_ok(const void *ptr, int64_t ld) {
    return ((uintptr_t)ptr % 16 == 0) && (ld % 4 == 0);
}

}  // namespace fw
