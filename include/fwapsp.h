/*
 * fwapsp.h -- C ABI of the MI355X (gfx950) blocked Floyd-Warshall APSP library
 * (libfwapsp.so).
 *
 * Paper: B. Lund, J. W. Smith, "A Multi-Stage CUDA Kernel for Floyd-Warshall"
 * (arXiv 1001.4108).  The operation is the problem of section 3.1: given a
 * weighted directed graph as a dense matrix W with w_ii = 0 and "infinity" on
 * absent edges and no negative cycle, overwrite W with the shortest-path
 * lengths d_ij (Fig. FW-Alg).  The library computes it by the blocked
 * schedule of section 3.2 / Fig. BFW-Alg (per k-block: the diagonal tile, the
 * row and column panels, then all remaining tiles).
 *
 * Common conventions
 *   - Matrices are row-major: entry (i, j) lives at d[i * ld + j], 0 <= i, j < n,
 *     ld >= n.  Columns n .. ld-1 of every row are never read or written.
 *   - Every matrix and output pointer is DEVICE memory owned by the caller; the
 *     library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     compute calls are stream-ordered and asynchronous: they return after
 *     enqueueing work; results are valid once the stream has been
 *     synchronised.  Faults of enqueued kernels surface from later HIP calls,
 *     as with any stream API.
 *   - Argument errors are detected before anything is enqueued and return
 *     FW_ERR_INVALID with no side effect.  HIP launch/allocation failures
 *     return FW_ERR_HIP / FW_ERR_NOMEM.
 *   - fp32: "infinity" is IEEE +INF.  Inputs must not contain NaN or -INF.
 *     Where both signs of zero meet, either zero may be returned.
 *   - int32: "infinity" is FW_I32_INF and sums are plain 32-bit adds (no
 *     saturation): the library solves APSP on the complete graph whose missing
 *     edges weigh FW_I32_INF.  Precondition: every simple-path weight sum of
 *     the real edges lies in (-2^29, 2^29) and every entry lies in
 *     [-2^29, FW_I32_INF]; then no add overflows, reachable distances are
 *     exact and unreachable pairs end at values above FW_I32_INF / 2.
 *   - Exactness: blocked Floyd-Warshall evaluates path sums in a different
 *     association than the plain triple loop.  Results are bit-identical to the
 *     triple loop whenever the arithmetic is exact (int32 under the
 *     precondition; fp32 with integer-valued weights whose true distances are
 *     below 2^24).  Otherwise fp32 results are valid shortest-path values that
 *     may differ from the triple loop's in the last bits.
 *   - Negative cycles violate the problem statement (section 3.1); the
 *     distances are then unspecified.  fw_negative_cycle detects them.
 */
#ifndef FWAPSP_H
#define FWAPSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FW_I32_INF 1073741823 /* INT32_MAX / 2: "no edge" for int32 matrices */

typedef enum { FW_F32 = 0, FW_I32 = 1 } fw_dtype;

typedef enum {
    FW_OK = 0,
    FW_ERR_INVALID = 1,     /* bad argument; nothing was enqueued            */
    FW_ERR_HIP = 2,         /* a HIP call failed                             */
    FW_ERR_NOMEM = 3,       /* device or host allocation failed              */
    FW_ERR_UNSUPPORTED = 4, /* valid request the library cannot serve         */
    FW_ERR_BUSY = 5,        /* server: admission refused (budget or queue)   */
    FW_ERR_NOT_FOUND = 6    /* server: unknown request id                    */
} fw_status;

/* Human-readable name of a status code (static string, never NULL). */
const char *fw_status_string(int status);

/* Library version string (static). */
const char *fw_version(void);

/*
 * fw_apsp -- all-pairs shortest paths in place, fp32 (section 3.1, solved by
 * the blocked schedule of section 3.2).
 *   d      device, n x n fp32 matrix with leading dimension ld (in elements);
 *          on entry the edge weights (0 diagonal, +INF absent), on completion
 *          the shortest-path lengths.
 *   n      number of vertices, 0 <= n < 2^31.  n = 0 or 1 returns FW_OK and
 *          enqueues nothing.
 *   ld     leading dimension, ld >= n.
 * Errors: FW_ERR_INVALID for d == NULL with n > 0, n < 0, ld < n, or n*ld
 * overflowing int64.
 */
int fw_apsp(float *d, int64_t n, int64_t ld, void *stream);

/* fw_apsp for int32 weights (FW_I32_INF = absent edge); same contract. */
int fw_apsp_i32(int32_t *d, int64_t n, int64_t ld, void *stream);

/*
 * fw_apsp_pred -- distances plus the optional predecessor matrix.
 *   d, n, ld   as fw_apsp; `dtype` (fw_dtype) says whether d is fp32 or int32.
 *   pred       device int32 n x n matrix (leading dimension ld_pred >= n), or
 *              NULL for distances only.  It need not be initialised.  On
 *              completion pred[i*ld_pred+j] is -1 when i == j or j is not
 *              reachable from i (fp32: d_ij == +INF; int32: d_ij > FW_I32_INF/2),
 *              and otherwise the canonical predecessor: the smallest vertex p
 *              that is the last hop of some shortest i -> j path.  (The paper
 *              computes distances only; this reading is unique, so it is the
 *              same for every tile size and batch composition.)  It is computed
 *              during the sweep by a lexicographic minimum over (distance, last
 *              hop) -- fp32 inputs that are not keys (below): after it, from
 *              the final distances -- and requires, besides the distance
 *              preconditions, that the graph has no zero-weight cycle.  Outside the problem statement
 *              (a negative cycle), pred[i*ld_pred+i] keeps the last hop of the
 *              closed walk that made d_ii negative (see
 *              fw_negative_cycle_find); the other entries are then as
 *              computed.
 * With pred and 2 <= n <= 16383 the (distance, last hop) pairs are first
 * swept as 32-bit integer keys (distance * 2^14 + last hop) held in `pred`,
 * at the cost of the int32 distances-only sweep; this takes 16 + 8n + 512n
 * bytes (rounded to 256), and for fp32 another 4 n min(n rounded up to 64,
 * 1024) bytes, of stream-ordered device memory (hipMallocAsync on `stream`,
 * freed on it).  When an entry of d is not an integer with |w| < 2^14
 * (fp32: also a fraction), some distance met during that sweep has
 * |d| >= 2^14, or a diagonal entry ends negative, a second form already
 * queued behind it (each launch gated on a device flag) solves again from
 * the untouched d: int32, the pair form with 64-bit keys; fp32, the
 * canonical path -- the distances by the distances-only sweep, then every
 * last hop from the definition above (the smallest q != j with
 * (q == i ? 0 : d_iq) + w_qj == d_ij in fp32, over the original weights,
 * held in `pred` meanwhile) -- or, after a negative diagonal, the compare
 * form, whose pred leads a walk to the cycle.  Within the precondition the
 * results are the same in every case and the choice is invisible except in
 * time (fw_pred_fallbacks counts the second forms).
 * fp32 with pred and n > 16383 (beyond the keys) takes the canonical path
 * directly: the weights saved in `pred`, the distances-only sweep, then
 * every last hop from the definition; after a negative diagonal instead the
 * compare form from the saved weights (counted by fw_pred_fallbacks).  This
 * takes 256 + 4 n min(n rounded up to 64, 1024) bytes of stream-ordered
 * device memory; where it cannot be had, the compare form runs alone.
 * Errors: as fw_apsp, plus FW_ERR_INVALID for a bad dtype or, with pred
 * non-NULL, ld_pred < n or n*ld_pred overflowing int64.
 */
int fw_apsp_pred(void *d, int dtype, int64_t n, int64_t ld, int32_t *pred,
                 int64_t ld_pred, void *stream);

/*
 * fw_apsp_plan -- fw_apsp_pred with an explicit tile size (the k-block depth
 * s of section 3.2) instead of the library's choice.  tile must be one of
 * fw_plan_tiles(); results are identical for every tile (the exactness rule
 * above).  Used to test every plan and by the autotuner.
 */
int fw_apsp_plan(void *d, int dtype, int64_t n, int64_t ld, int32_t *pred,
                 int64_t ld_pred, int tile, void *stream);

/*
 * fw_apsp_semiring -- the same in-place blocked sweep over another closed
 * semiring (section 3.2's schedule is valid for any of them).
 *   FW_SR_MINPLUS  shortest paths, exactly fw_apsp / fw_apsp_i32;
 *   FW_SR_MAXMIN   widest (bottleneck) paths: d_ij becomes the largest, over
 *                  all i -> j paths, of the smallest edge weight on the path,
 *                  i.e. the update is d_ij <- max(d_ij, min(d_ik, d_kj)).
 *                  Absent edges must hold the max-identity (-INF for fp32,
 *                  INT32_MIN for int32; for non-negative weights 0 works);
 *                  the diagonal is kept unless a cycle through i is wider
 *                  (use +INF / INT32_MAX for "a vertex reaches itself").  Over
 *                  int32 weights in {0, 1} with 1 on the diagonal this is the
 *                  transitive closure.  min and max are exact, so results are
 *                  bit-identical to the triple loop for every input (no
 *                  precondition, no negative-cycle issue).
 * d, n, ld, stream as fw_apsp; dtype is fw_dtype.  Errors: FW_ERR_INVALID for
 * a bad semiring or the argument errors of fw_apsp.
 */
#define FW_SR_MINPLUS 0
#define FW_SR_MAXMIN 1
int fw_apsp_semiring(void *d, int dtype, int semiring, int64_t n, int64_t ld, void *stream);

/*
 * fw_transitive_closure_bits -- reachability on a bit-packed adjacency matrix:
 * the blocked schedule (section 3.2) over the boolean semiring, in place.
 * Row i is ceil(n / 32) 32-bit words; bit j % 32 of word j / 32 is the edge
 * i -> j on input and "j is reachable from i" on output.
 *   bits       device, n rows of ldw words (ldw >= ceil(n / 32)); bits of
 *              columns >= n must be 0 (they stay 0); words past ceil(n / 32)
 *              are neither read nor written.
 *   reflexive  non-zero: every vertex reaches itself (the diagonal is set
 *              first); zero: paths of one edge or more only (i reaches i iff
 *              i lies on a cycle).
 * Stream-ordered.  Errors: FW_ERR_INVALID for bits == NULL with n > 0, n < 0
 * or ldw too small; FW_ERR_UNSUPPORTED for n > 2^21 (a 512 GiB matrix).
 */
int fw_transitive_closure_bits(uint32_t *bits, int64_t n, int64_t ldw, int reflexive,
                               void *stream);

/*
 * fw_pack_bits / fw_unpack_bits -- convert between an n x n int32 matrix (ld
 * >= n; non-zero = edge) and the bit layout above (ldw >= ceil(n / 32); the
 * pack writes words 0 .. ceil(n / 32) - 1 of each row, column bits >= n as 0;
 * the unpack writes 0 / 1).  Stream-ordered; the same errors as
 * fw_transitive_closure_bits.
 */
int fw_pack_bits(const int32_t *adj, int64_t n, int64_t ld, uint32_t *bits, int64_t ldw,
                 void *stream);
int fw_unpack_bits(const uint32_t *bits, int64_t n, int64_t ldw, int32_t *adj, int64_t ld,
                   void *stream);

/*
 * Tile sizes fw_apsp_plan accepts: writes up to `cap` of them to `tiles`
 * (host memory) and returns how many exist.
 */
int fw_plan_tiles(int *tiles, int cap);

/*
 * Plan keys.  The plan table has one part per key: a fw_dtype, or'd with
 * FW_PLAN_PRED for the solves that also compute predecessors (fw_apsp_pred
 * with a non-NULL pred, batched graphs with a predecessor matrix), whose
 * kernels favour other tiles.  The fw_plan_tile / fw_plan_set / fw_autotune
 * calls take a key where they take a dtype.
 */
#define FW_PLAN_PRED 2

/*
 * Tile size the library picks for (key, n), from its tuned plan table.
 * Returns the tile, or 0 for n <= 1, or -1 for a bad key / n < 0.
 */
int fw_plan_tile(int key, int64_t n);

/*
 * fw_plan_set -- replace the plan table entry for a size bucket: solves of
 * plan key `key` (dtype [| FW_PLAN_PRED]) with n_lo <= n <= n_hi use `tile`.
 * Used by the autotuner to install measured choices.  Returns FW_OK or
 * FW_ERR_INVALID.
 */
int fw_plan_set(int key, int64_t n_lo, int64_t n_hi, int tile);

/* Restore the built-in plan table. */
void fw_plan_reset(void);

/*
 * fw_apsp_ladder -- the same solve by one rung of an ablation ladder that
 * mirrors the columns of the paper's Table 1 with gfx950 kernels (for
 * measuring what each design step buys; every rung gives the same bits):
 *   0  one launch per k, one thread per cell (section 3.1's direct form);
 *   1  blocked (section 3.2), 32 x 32 tiles held in LDS, one cell per thread,
 *      k-ordered diagonal and panel phases;
 *   2  blocked, 64 x 64 tiles, 4 x 4 register sub-tiles, two k-steps fused,
 *      the whole operand tiles in LDS (64 KB per workgroup);
 *   3  as 2 with the operands staged in 16-deep LDS slices (the tile-64 path
 *      of fw_apsp_plan);
 *   4  tile 128: direct global->LDS slice copies, 8 x 8 register sub-tiles,
 *      strip panels, the next diagonal tile closed in the bulk launch (the
 *      path the plan table picks for large solves; rung 3 is its pick for
 *      mid sizes).
 * d, dtype, n, ld, stream as fw_apsp_pred without predecessors.  Errors:
 * FW_ERR_INVALID for a bad rung or the argument errors of fw_apsp,
 * FW_ERR_UNSUPPORTED for n > 65536.
 */
int fw_apsp_ladder(void *d, int dtype, int64_t n, int64_t ld, int rung, void *stream);

/*
 * fw_autotune -- the plan table's autotuner (dtype: a plan key; with
 * FW_PLAN_PRED the timed solves compute predecessors).  For each size bucket
 * [lo[k], hi[k]] (2 <= lo <= hi <= 65536) it times every tile of
 * fw_plan_tiles() and installs the fastest with fw_plan_set.  objective 0
 * times one single-graph solve of the bucket's geometric-middle size,
 * objective 1 one eager launch of a batch plan of `batch` graphs whose sizes
 * spread log-uniformly over the bucket (graph g at quantile (g + 1/2) / batch;
 * persistent or stage-batched, as batch plans run those sizes; plans read the
 * same table).  While a candidate is timed it is installed for its bucket, so
 * concurrent solves may see it.  Each (bucket, tile) is run reps + 1
 * times, the first as a warm-up, and scored by the median.  Writes the chosen
 * tile of bucket k to tile_out[k] and, if ms_out is non-NULL, the median ms of
 * tile t to ms_out[k * ntiles + t].  Synchronous; allocates and frees its own
 * zero-filled scratch matrices (the sweep's run time does not depend on the
 * data).  Errors: FW_ERR_INVALID for bad arguments, FW_ERR_NOMEM/FW_ERR_HIP.
 */
int fw_autotune(int dtype, const int64_t *lo, const int64_t *hi, int nbuckets, int objective,
                int batch, int reps, int *tile_out, double *ms_out);

/*
 * fw_autotune_batch -- tunes the plan table for one batch as a whole (dtype:
 * a plan key, as for fw_autotune).  n[0..count) are the batch's graph sizes
 * (0 <= n[g] <= fw_batched_max_n, 1 <= count <= 2^20); buckets [lo[k], hi[k]]
 * as for fw_autotune (a bucket may lie inside a wider one installed before:
 * the most recent entry covering a size wins).  The tiles of different
 * buckets interact inside one batch plan (each tile size is its own chain of
 * stage launches, and the chains share the GPU), so the objective is a
 * launch of a batch plan over zero matrices of exactly these sizes, in `mode`
 * as for fw_batch_plan_launch (0: eager kernel launches, 1: a replay of the
 * plan's captured graph; the two can favour different tiles):
 * starting from the table's current tile at each bucket's geometric middle,
 * `passes` rounds of coordinate descent, in which every bucket that holds
 * some of the graphs times every tile of fw_plan_tiles() (reps + 1 launches,
 * the first a warm-up, scored by the median) with the other buckets fixed,
 * and installs the fastest with fw_plan_set.  Writes the chosen tiles to
 * tile_out[k] and, if ms_out is non-NULL, the last pass's median ms of tile t
 * for bucket k to ms_out[k * ntiles + t] (0 for buckets skipped).
 * Synchronous; allocates and frees its own scratch matrices.  Errors:
 * FW_ERR_INVALID for bad arguments, FW_ERR_UNSUPPORTED for a size above
 * fw_batched_max_n, FW_ERR_NOMEM/FW_ERR_HIP.
 */
int fw_autotune_batch(int dtype, const int64_t *n, int64_t count, const int64_t *lo,
                      const int64_t *hi, int nbuckets, int mode, int reps, int passes,
                      int *tile_out, double *ms_out);

/*
 * fw_apsp_batched -- many independent graphs in one call.  Graphs of 33
 * vertices and more are stage-batched: for each tile size (from the plan
 * table: a graph with a predecessor matrix reads the FW_PLAN_PRED part),
 * stage b of the blocked schedule (section 3.2) is at most three launches
 * shared by all such graphs that have a stage b -- their diagonal tiles,
 * their panel tiles, their bulk tiles (the bulk launch also closes each
 * graph's next diagonal tile where the tile size allows).  Smaller graphs go
 * through one persistent launch whose workgroups take graphs from a device
 * work counter, largest first, and solve each alone.
 *   d        HOST array of `count` device pointers, one n[g] x n[g] matrix
 *            each (leading dimension ld[g] >= n[g]); graphs must not alias.
 *   n, ld    HOST arrays of `count` sizes and leading dimensions.
 *   dtype    fw_dtype of every matrix.
 *   pred     NULL, or a HOST array of `count` device pointers (entries may be
 *            NULL) to int32 predecessor matrices with leading dimensions
 *            ld_pred[g] (ld_pred may be NULL only if pred is NULL).
 *   count    number of graphs (0 = no-op).
 * A graph's result is bit-identical to fw_apsp_pred on the same graph alone.
 * Errors: FW_ERR_INVALID if any graph's arguments are invalid (nothing is
 * enqueued), FW_ERR_UNSUPPORTED if a graph exceeds fw_batched_max_n().
 * The call uploads the descriptor table and the stage-batched work table
 * (graph, tile) synchronously on a private stream, then enqueues the launches
 * on `stream`; it may be called again at once.
 */
int fw_apsp_batched(void *const *d, const int64_t *n, const int64_t *ld,
                    int64_t count, int dtype, int32_t *const *pred,
                    const int64_t *ld_pred, void *stream);

/*
 * fw_apsp_batched_noalloc -- fw_apsp_batched for callers that cannot
 * allocate (code under stream capture of their own, tight serving loops,
 * harnesses that forbid allocation): the same arguments, plan and kernels,
 * bit-identical results, but the descriptor table and the stage-batched work
 * table go to a static device array of FW_BATCHED_NOALLOC_MAX_BYTES (16 MiB)
 * that the library holds on each GPU it runs on until the process ends;
 * nothing is allocated on the device and no HIP event or stream is created.
 * The tables (64 bytes + 48 bytes per graph, then 8 bytes per tile-phase
 * entry of the stage-batched graphs: about 1.8 MB for 4096 graphs of 16-512
 * vertices) are copied there on `stream`, which the call then synchronises
 * (the host tables are freed on return); the kernels are enqueued after
 * that.  Every call on a GPU shares that GPU's array and overwrites the
 * previous call's tables: calls on one GPU must not overlap in time (two
 * streams running them at once race on the array).  Errors: those of
 * fw_apsp_batched, and FW_ERR_UNSUPPORTED when the tables exceed the array
 * (nothing is enqueued).
 */
#define FW_BATCHED_NOALLOC_MAX_BYTES (16 << 20)
int fw_apsp_batched_noalloc(void *const *d, const int64_t *n, const int64_t *ld,
                            int64_t count, int dtype, int32_t *const *pred,
                            const int64_t *ld_pred, void *stream);

/* Size of the static array of fw_apsp_batched_noalloc, in bytes. */
int64_t fw_batched_noalloc_max_bytes(void);

/* Largest n fw_apsp_batched accepts for a dtype (with or without pred). */
int64_t fw_batched_max_n(int dtype, int with_pred);

/*
 * Reusable batch plans.  fw_batch_plan_create validates the graphs exactly as
 * fw_apsp_batched does and builds the descriptor table (pinned host memory
 * plus a device copy) and the stage-batched work table (device), both
 * uploaded at creation and owned by the plan; the matrices must stay allocated for the
 * plan's lifetime and are re-solved in place on every launch.  The tiles are
 * read from the plan table at creation.  fw_batch_plan_launch enqueues on
 * `stream`, by `mode`:
 *   0  the stage-batched launches, the reset of the device work counter (a
 *      kernel) and the persistent kernel, as plain stream operations;
 *   1  the same operations captured once into a hipGraph, replayed by every
 *      later launch (one graph launch per batch);
 *   2  no persistent kernel: every graph through the single-graph stage
 *      loop of fw_apsp_pred (the per-graph launch baseline).
 * All modes give bit-identical results.  Launches of one plan must not
 * overlap in time (they share the work counter).  fw_batch_plan_destroy synchronises
 * the device and frees the plan.  fw_batch_plan_grid returns the persistent
 * grid size (workgroups), or -1 for a NULL plan.
 */
typedef struct fw_batch_plan_s *fw_batch_plan;
int fw_batch_plan_create(void *const *d, const int64_t *n, const int64_t *ld, int64_t count,
                         int dtype, int32_t *const *pred, const int64_t *ld_pred,
                         fw_batch_plan *out);
int fw_batch_plan_launch(fw_batch_plan plan, int mode, void *stream);
int fw_batch_plan_destroy(fw_batch_plan plan);
int64_t fw_batch_plan_grid(fw_batch_plan plan);

/*
 * Serving loop (continuous batching).  Requests are admitted in arrival order
 * while their device footprint (n x round_up(n, 4) x 4 bytes) fits
 * `budget_bytes`; each admitted payload is copied into a resident slot.
 * Whenever one of `streams` worker streams is free, every admitted request
 * with n <= small_n (up to max_batch of them) goes into one persistent
 * batched launch, or the oldest admitted larger request runs the single-graph
 * stage loop alone; groups on different streams overlap on the device.
 * Finished requests return their memory and wake the dispatcher, so waiting
 * requests are admitted as soon as memory and streams free up.  A request's
 * result is bit-identical to fw_apsp / fw_apsp_i32 on the same matrix alone.
 * The server runs its own host threads (one dispatcher, one completion thread
 * per stream); every stream keeps the default priority.
 */
typedef struct {
    int dtype;            /* fw_dtype of every request                        */
    int streams;          /* worker streams, 1 .. 16                          */
    int64_t budget_bytes; /* device memory for resident request matrices      */
    int64_t small_n;      /* n <= small_n: batched path                       */
    int max_batch;        /* most requests per batched launch                 */
    int64_t queue_cap;    /* most requests waiting for admission              */
} fw_server_config;

typedef struct {
    int64_t id, n;
    int status;           /* FW_OK, or the error that ended the request       */
    int group_size;       /* requests in the launch group it ran in           */
    int64_t t_submit_ns;  /* host steady-clock timestamps                     */
    int64_t t_admit_ns;
    int64_t t_done_ns;    /* completion observed (after any copy-back)        */
} fw_completion;

typedef struct {
    int64_t submitted, admitted, completed, failed, rejected, deferrals;
    int64_t batched_groups, single_groups, max_group;
    int64_t waiting, bytes_in_use, peak_bytes, budget_bytes;
} fw_server_stats;

typedef struct fw_server_s *fw_server;

/* Allocates the budget arena, worker streams and threads on the current
 * device.  FW_ERR_INVALID for a bad config, FW_ERR_NOMEM if allocation fails. */
int fw_server_create(const fw_server_config *cfg, fw_server *out);

/*
 * Submit one request (thread-safe, non-blocking).  `src` (host or device, n x n
 * with leading dimension ld_src >= n) must stay valid until the request's
 * completion is reported.  If dst_host is non-NULL the result is copied there
 * (leading dimension ld_dst) before completion.  keep != 0 keeps the result
 * resident until fw_server_release (fetch it with fw_server_fetch); otherwise
 * its memory returns to the budget at completion.  Writes the request id.
 * Errors: FW_ERR_INVALID for bad arguments, FW_ERR_UNSUPPORTED when the
 * footprint exceeds the whole budget, FW_ERR_BUSY when queue_cap requests are
 * already waiting.
 */
int fw_server_submit(fw_server s, const void *src, int64_t n, int64_t ld_src, void *dst_host,
                     int64_t ld_dst, int keep, int64_t *id_out);

/* Up to `cap` completion records (host array), waiting up to timeout_us for
 * the first; returns how many were written (negative status on bad args). */
int fw_server_poll(fw_server s, fw_completion *out, int cap, int64_t timeout_us);

/* Copy a finished kept result to `dst` (host or device, ld_dst >= n),
 * stream-ordered on `stream`.  FW_ERR_NOT_FOUND for an unknown id,
 * FW_ERR_INVALID if the request is not finished or was not kept. */
int fw_server_fetch(fw_server s, int64_t id, void *dst, int64_t ld_dst, void *stream);

/* Return a finished kept request's memory to the budget. */
int fw_server_release(fw_server s, int64_t id);

/* Wait until every submitted request has completed (timeout_us < 0: no limit);
 * FW_ERR_BUSY on timeout. */
int fw_server_drain(fw_server s, int64_t timeout_us);

int fw_server_get_stats(fw_server s, fw_server_stats *out);

/* Cancel requests not yet admitted (status FW_ERR_BUSY), finish the running
 * ones, join the threads and free everything. */
int fw_server_destroy(fw_server s);

/*
 * fw_negative_cycle -- after a solve, write to *flag_dev (device int32) the
 * number of vertices i with d_ii < 0 (a negative cycle through i: the case
 * the problem statement of section 3.1 excludes), 0 when there is none.
 * Stream-ordered.  Errors: the argument errors of fw_apsp_pred, or
 * FW_ERR_INVALID for flag_dev == NULL.
 */
int fw_negative_cycle(const void *d, int dtype, int64_t n, int64_t ld,
                      int32_t *flag_dev, void *stream);

/*
 * fw_negative_cycle_vertices -- the vertices i with d_ii < 0 after a solve,
 * in ascending order, written to list_dev[0 .. c-1] (device int32, capacity
 * n), and c written to *count_dev (device int32).  One workgroup scans the
 * diagonal.  Stream-ordered.  Errors: the argument errors of fw_apsp_pred, or
 * FW_ERR_INVALID for count_dev == NULL or list_dev == NULL with n > 0.
 */
int fw_negative_cycle_vertices(const void *d, int dtype, int64_t n, int64_t ld,
                               int32_t *list_dev, int32_t *count_dev, void *stream);

/*
 * fw_negative_cycle_find -- one negative cycle reachable from vertex v, for
 * v with d_vv < 0 (from fw_negative_cycle_vertices: a negative closed walk
 * runs through v, so one is reachable).  Host call; every pointer is HOST
 * memory.
 *   w_host     the ORIGINAL weights (n x n, leading dimension ld, fw_dtype
 *              `dtype`), the matrix before the solve overwrote it.
 *   pred_host  NULL, or the predecessor matrix of the same solve
 *              (fw_apsp_pred; ld_pred >= n).  When d_vv < 0 the solve keeps
 *              P_vv, the last hop of the closed walk that made d_vv negative,
 *              and the walk back along row v (v <- P_vv <- P_v,P_vv <- ...)
 *              runs into a cycle of edges.  That cycle is returned if its
 *              weight over w_host is negative (*from_pred = 1).
 *   otherwise  (no pred, or the walk's cycle is not negative) Bellman-Ford
 *              from v over w_host, in-place relaxation, stopping at the
 *              first pass after which the parent graph holds a cycle (which
 *              then has negative weight); O(n^2) per pass, at most n + 1
 *              passes.
 * Writes the cycle c_0, ..., c_{m-1} (edges c_t -> c_{t+1} and c_{m-1} ->
 * c_0, weights summed exactly in double) to `cycle` (capacity cap) and
 * returns m; returns 0 if no negative cycle is reachable from v, and -1 for
 * invalid arguments or insufficient capacity.  from_pred may be NULL.
 */
int64_t fw_negative_cycle_find(const void *w_host, int dtype, int64_t n, int64_t ld,
                               const int32_t *pred_host, int64_t ld_pred, int64_t v,
                               int64_t *cycle, int64_t cap, int *from_pred);

/*
 * fw_path -- reconstruct one shortest path from a predecessor matrix that was
 * copied to HOST memory.  Writes the vertices i = v_0, v_1, ..., v_m = j to
 * `path` (host, capacity `cap`) and returns m + 1, or 0 when j is unreachable
 * from i, or -1 for invalid arguments / a predecessor chain that does not
 * lead back to i within n steps / insufficient capacity.
 */
int64_t fw_path(const int32_t *pred_host, int64_t n, int64_t ld_pred, int64_t i,
                int64_t j, int64_t *path, int64_t cap);

/*
 * Solve plans: the stage loop of section 3.2 for one matrix, captured once
 * into a hipGraph and replayed by one graph launch per solve.
 *   fw_solve_plan_create  validates (d, dtype, n, ld, pred, ld_pred) as
 *                         fw_apsp_pred does and fixes the tile: `tile` (one
 *                         of fw_plan_tiles()) or 0 for the plan table's
 *                         choice at creation.  Nothing is enqueued; the
 *                         matrices must stay allocated for the plan's
 *                         lifetime and are re-solved in place on every
 *                         launch.  A plan with predecessors allocates the
 *                         keyed sweep's scratch here (FW_ERR_NOMEM if it
 *                         cannot); its launches then allocate nothing.
 *   fw_solve_plan_launch  mode 0: the solve as eager launches on `stream`
 *                         (fw_apsp_plan); mode 1: on the first call the
 *                         launches are captured into a hipGraph on a stream
 *                         the plan owns (kept, with the graph, until the plan
 *                         is destroyed; no event is recorded during the
 *                         capture, so phase timing does not see graph
 *                         launches), and every call launches that graph on
 *                         `stream`.  Both modes give bit-identical results.
 *                         Launches of one plan must not overlap in time.
 *   fw_solve_plan_tile    the plan's tile (-1 for NULL).
 *   fw_solve_plan_destroy synchronises the plan's device and frees it.
 * Errors: FW_ERR_INVALID for bad arguments (NULL plan, bad mode or tile),
 * FW_ERR_HIP / FW_ERR_NOMEM when capture or instantiation fails.
 */
typedef struct fw_solve_plan_s *fw_solve_plan;
int fw_solve_plan_create(void *d, int dtype, int64_t n, int64_t ld, int32_t *pred,
                         int64_t ld_pred, int tile, fw_solve_plan *out);
int fw_solve_plan_launch(fw_solve_plan plan, int mode, void *stream);
int fw_solve_plan_tile(fw_solve_plan plan);
int fw_solve_plan_destroy(fw_solve_plan plan);

/*
 * Phase timing.  While enabled, every eager phase launch of the calls above
 * is bracketed by HIP events on its stream (graph launches of solve plans and
 * batch plans are not).  fw_profile_read synchronises those events and
 * writes, per phase kind, the summed kernel time in ms and the launch count
 * (kinds: 0 = diagonal tile, 1 = panels, 2 = bulk tiles (with the next
 * diagonal tile where the bulk launch closes it), 3 = predecessor
 * init/fix-up (and the key packing and unpacking of int32 solves with
 * predecessors), 4 = batched persistent kernel; fw_transitive_closure_bits:
 * 5 = stage 0's diagonal block, 6 = panels, 7 = bulk with the next diagonal
 * block; 8 = the gated 64-bit predecessor sweep behind a keyed one, every
 * launch whether it ran or found its gate closed); it returns the number of
 * kinds written and clears the accumulators.
 */
int fw_profile_enable(int on);
int fw_profile_read(double *ms, int64_t *launches, int cap);

/* Work counters of the last fw_profile_read window: algorithmic cell updates
 * per kind (the n^3 tasks of section 1 split by phase). */
int fw_profile_updates(double *updates, int cap);

/*
 * fw_pred_fallbacks -- how many solves with predecessors on the current
 * device have run their second form (pair-form sweep, or fp32 canonical
 * path) because the 32-bit keyed one gave up (see fw_apsp_pred), since the
 * library was loaded.  Synchronises the device; -1 when the count cannot be
 * read.
 */
int64_t fw_pred_fallbacks(void);

#ifdef __cplusplus
}
#endif

#endif /* FWAPSP_H */
