// Internal declarations shared by the host driver and the kernel files of
// libfwapsp.  Not part of the public ABI (see include/fwapsp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fw {

constexpr int32_t kI32Inf = 1073741823;   // "no edge" for int32
constexpr int32_t kPredNone = 0x7fffffff; // in-sweep "no last hop yet"

enum PhaseKind {
    kDiag = 0,
    kPanel = 1,
    kBulk = 2,      // the bulk (+ the next diagonal tile where the kernel closes it)
    kPredFix = 3,
    kBatched = 4,
    kBitsDiag = 5,  // bit-packed reachability: stage 0's diagonal block
    kBitsPanel = 6, // bit-packed reachability: both panels
    kBitsBulk = 7,  // bit-packed reachability: the bulk (+ next diagonal block)
    kNumKinds = 8
};

// Phase timing for launches made outside the host driver: calls
// launch(ctx), bracketed by HIP events on st while profiling is enabled.
hipError_t timed_launch(int kind, double updates, hipStream_t st, hipError_t (*launch)(void *),
                        void *ctx);

// Closed semirings the sweep runs over.
enum Semiring { kMinPlus = 0, kMaxMin = 1 };

// One stage-phase launch of the blocked schedule.  `d`/`p` are the matrix
// and the (optional) predecessor matrix; `b` is the k-block index, `nb` the
// number of tile rows.  Returns hipSuccess or the launch error.
hipError_t launch_diag(int dtype, int sr, int tile, void *d, int32_t *p, int n, int64_t ld,
                       int64_t ldp, int b, hipStream_t st);
hipError_t launch_panels(int dtype, int sr, int tile, void *d, int32_t *p, int n, int64_t ld,
                         int64_t ldp, int b, int nb, hipStream_t st);
// With close_next the launch also closes the next stage's diagonal tile
// (b+1, b+1), which replaces launch_diag(b + 1); allowed exactly when
// bulk_closes_next_diag(sr, tile, d, p, n, ld, b) holds.
hipError_t launch_bulk(int dtype, int sr, int tile, void *d, int32_t *p, int n, int64_t ld,
                       int64_t ldp, int b, int nb, bool close_next, hipStream_t st);
bool bulk_closes_next_diag(int sr, int tile, const void *d, const int32_t *p, int n, int64_t ld,
                           int b);
hipError_t launch_pred_init(int dtype, const void *d, int32_t *p, int n, int64_t ld,
                            int64_t ldp, hipStream_t st);
hipError_t launch_pred_fix(int dtype, const void *d, int32_t *p, int n, int64_t ld,
                           int64_t ldp, hipStream_t st);
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
