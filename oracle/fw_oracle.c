/*
 * Plain CPU oracle for all-pairs shortest paths.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the package's smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header, table or
 * helper with the HIP library.
 *
 * Paper: B. Lund, J. W. Smith, "A Multi-Stage CUDA Kernel for Floyd-Warshall"
 * (arXiv 1001.4108).  Every routine below names the passage it follows.
 *
 * Conventions (the paper's problem statement, section 3.1):
 *   - a dense n x n row-major matrix with leading dimension ld >= n;
 *   - w_ii = 0, w_ij = "infinity" when (v_i, v_j) is not an edge;
 *   - fp32: infinity is IEEE +INF;
 *   - int32: infinity is the sentinel M = 1073741823 (= INT32_MAX / 2) and
 *     additions are plain 32-bit two's-complement adds (no saturation), i.e.
 *     the oracle solves APSP on the complete graph whose missing edges weigh M.
 *   - min(a, b) := (b < a) ? b : a  (ties keep the current value).
 *
 * Readings where the paper is silent (zero sign, the int32 sentinel, the
 * predecessor definition, reachability under the sentinel) are stated at each
 * routine.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_I32_INF 1073741823

static int oracle_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads <= 0) return omp_get_max_threads();
    return nthreads;
#else
    (void)nthreads;
    return 1;
#endif
}

/* Number of threads an OpenMP region of this library would use. */
int oracle_max_threads(void) { return oracle_threads(0); }

/*
 * Floyd-Warshall, section 3.1, Fig. FW-Alg:
 *     for k: for i: for j: w_ij <- min(w_ij, w_ik + w_kj)
 * performed in place on w for k in [k_begin, k_end) (the full algorithm is
 * k_begin = 0, k_end = n; a prefix of the k loop is what the CPU timing leg
 * runs on large matrices).
 *
 * Order of the i and j loops.  The figure writes them as "for all", and when
 * w_kk >= 0 they are order-free: row k and column k cannot change during
 * iteration k (w_kj <- min(w_kj, w_kk + w_kj) and w_ik <- min(w_ik, w_ik + w_kk)
 * keep the old value), so every (i, j) of iteration k reads the same w_ik and
 * w_kj as the serial i-then-j loop does, and the rows can be run in parallel.
 * When w_kk < 0 (a negative cycle, excluded by the problem statement) the
 * iteration runs as the literal serial double loop instead, re-reading w_ik
 * and w_kj at every task, so the routine equals the serial triple loop for
 * every input.
 */
void oracle_fw_f32(float *w, int64_t n, int64_t ld, int64_t k_begin,
                   int64_t k_end, int nthreads) {
    int nt = oracle_threads(nthreads);
    for (int64_t k = k_begin; k < k_end; ++k) {
        const float *wk = w + k * ld;
        if (!(wk[k] >= 0.0f)) {
            for (int64_t i = 0; i < n; ++i)
                for (int64_t j = 0; j < n; ++j) {
                    float s = w[i * ld + k] + w[k * ld + j];
                    if (s < w[i * ld + j]) w[i * ld + j] = s;
                }
            continue;
        }
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t i = 0; i < n; ++i) {
            if (i == k) continue; /* row k is unchanged in iteration k */
            float *restrict wi = w + i * ld;
            const float *restrict wkr = wk;
            const float wik = wi[k];
            for (int64_t j = 0; j < n; ++j) {
                float s = wik + wkr[j];
                wi[j] = (s < wi[j]) ? s : wi[j];
            }
        }
    }
}

/* Two's-complement 32-bit add, defined for every input (the device adds wrap
 * the same way; the int32 precondition keeps real sums far from the wrap). */
static inline int32_t add_wrap_i32(int32_t a, int32_t b) {
    return (int32_t)((uint32_t)a + (uint32_t)b);
}

/* Fig. FW-Alg with int32 weights; same loop structure and argument as
 * oracle_fw_f32. */
void oracle_fw_i32(int32_t *w, int64_t n, int64_t ld, int64_t k_begin,
                   int64_t k_end, int nthreads) {
    int nt = oracle_threads(nthreads);
    for (int64_t k = k_begin; k < k_end; ++k) {
        const int32_t *wk = w + k * ld;
        if (wk[k] < 0) {
            for (int64_t i = 0; i < n; ++i)
                for (int64_t j = 0; j < n; ++j) {
                    int32_t s = add_wrap_i32(w[i * ld + k], w[k * ld + j]);
                    if (s < w[i * ld + j]) w[i * ld + j] = s;
                }
            continue;
        }
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t i = 0; i < n; ++i) {
            if (i == k) continue;
            int32_t *restrict wi = w + i * ld;
            const int32_t *restrict wkr = wk;
            const int32_t wik = wi[k];
            for (int64_t j = 0; j < n; ++j) {
                int32_t s = add_wrap_i32(wik, wkr[j]);
                wi[j] = (s < wi[j]) ? s : wi[j];
            }
        }
    }
}

/* dtype codes of this file: 0 = fp32, 1 = int32. */
static inline int is_edge(const void *W, int dtype, int64_t ld, int64_t p,
                          int64_t j) {
    if (p == j) return 0; /* the diagonal is not an edge */
    if (dtype == 0) {
        float v = ((const float *)W)[p * ld + j];
        return !(isinf(v) && v > 0.0f);
    }
    return ((const int32_t *)W)[p * ld + j] != ORACLE_I32_INF;
}

static inline double weight_f64(const void *W, int dtype, int64_t ld, int64_t p,
                                int64_t j) {
    if (dtype == 0) return (double)((const float *)W)[p * ld + j];
    return (double)((const int32_t *)W)[p * ld + j];
}

/*
 * Reachability from src over the edges of W (the edge set E of section 3.1:
 * every off-diagonal entry that is not infinity).  Breadth-first search on the
 * dense matrix; reach[j] = 1 iff a path of edges leads from src to j
 * (reach[src] = 1).
 */
void oracle_reach_row(const void *W, int dtype, int64_t n, int64_t ld,
                      int64_t src, uint8_t *reach) {
    int64_t *queue = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    memset(reach, 0, (size_t)n);
    int64_t head = 0, tail = 0;
    reach[src] = 1;
    queue[tail++] = src;
    while (head < tail) {
        int64_t u = queue[head++];
        for (int64_t v = 0; v < n; ++v)
            if (!reach[v] && is_edge(W, dtype, ld, u, v)) {
                reach[v] = 1;
                queue[tail++] = v;
            }
    }
    free(queue);
}

/*
 * Canonical predecessor matrix (the paper computes distances only; this is
 * the reading the library adopts for its optional predecessor output).
 *
 * For each listed source row i = rows[r] (r = 0 .. nrows-1), given the final
 * distance row D[r*ldd + *] of i and the ORIGINAL weights W:
 *   P[r][i] = -1;
 *   P[r][j] = -1 when j is not reachable from i over the edges of W;
 *   otherwise P[r][j] = min { p : p != j, (p, j) is an edge of W,
 *                                 p reachable from i,
 *                                 d(i, p) + W[p][j] == D[i][j] },
 * the smallest last hop over all shortest i -> j paths, where d(i, p) is the
 * weight of the best i -> p prefix: D[i][p] for p != i, and 0 for p = i (the
 * empty path -- a path from i does not pass through the diagonal entry, which
 * holds the best cycle through i, or a non-zero w_ii).  The sum is taken in
 * the matrix's own precision (fp32 round-to-nearest, or exact int64 for
 * int32), and -1 is written if no p qualifies (which cannot happen for exact
 * shortest-path distances).
 *
 * Search order: for each (i, j) the candidates p are tested in increasing
 * order and the first that qualifies is the minimum of the set above.  The
 * weights are read through a transposed copy (column j of W as one
 * contiguous row, its diagonal entry marked absent, since p != j), in chunks
 * of 64 candidates whose tests are independent of each other.  Reachability
 * from i is a breadth-first search over the edges, with the adjacency rows
 * and the visited set held as 64-bit masks.
 */
static void adjacency_masks(const void *W, int dtype, int64_t ldw, int64_t n,
                            uint64_t *adj, int64_t nw) {
    for (int64_t u = 0; u < n; ++u) {
        uint64_t *row = adj + u * nw;
        memset(row, 0, (size_t)nw * sizeof(uint64_t));
        for (int64_t v = 0; v < n; ++v)
            if (is_edge(W, dtype, ldw, u, v)) row[v >> 6] |= 1ull << (v & 63);
    }
}

/* reach[j] = 1 iff j is reachable from src over the edges (reach[src] = 1). */
static void reach_masks(const uint64_t *adj, int64_t nw, int64_t n, int64_t src,
                        uint64_t *seen, int64_t *queue, uint8_t *reach) {
    memset(seen, 0, (size_t)nw * sizeof(uint64_t));
    int64_t head = 0, tail = 0;
    seen[src >> 6] |= 1ull << (src & 63);
    queue[tail++] = src;
    while (head < tail) {
        const uint64_t *row = adj + queue[head++] * nw;
        for (int64_t w = 0; w < nw; ++w) {
            uint64_t fresh = row[w] & ~seen[w];
            seen[w] |= fresh;
            while (fresh) {
                const int b = __builtin_ctzll(fresh);
                fresh &= fresh - 1;
                queue[tail++] = w * 64 + b;
            }
        }
    }
    for (int64_t v = 0; v < n; ++v) reach[v] = (uint8_t)((seen[v >> 6] >> (v & 63)) & 1);
}

/* First p in [0, n) with ok[p] and dr[p] + wt[p] == target (fp32 sum), or -1. */
static int64_t first_hit_f32(const float *dr, const float *wt, const uint8_t *ok, int64_t n,
                             float target) {
    for (int64_t p0 = 0; p0 < n; p0 += 64) {
        const int64_t cnt = n - p0 < 64 ? n - p0 : 64;
        uint8_t hit[64];
        for (int64_t q = 0; q < cnt; ++q) {
            const float w = wt[p0 + q];
            const float sum = dr[p0 + q] + w;
            hit[q] = (uint8_t)(ok[p0 + q] & (w != INFINITY) & (sum == target));
        }
        for (int64_t q = 0; q < cnt; ++q)
            if (hit[q]) return p0 + q;
    }
    return -1;
}

/* As first_hit_f32 for int32 weights, the sum exact in int64. */
static int64_t first_hit_i32(const int32_t *dr, const int32_t *wt, const uint8_t *ok, int64_t n,
                             int64_t target) {
    for (int64_t p0 = 0; p0 < n; p0 += 64) {
        const int64_t cnt = n - p0 < 64 ? n - p0 : 64;
        uint8_t hit[64];
        for (int64_t q = 0; q < cnt; ++q) {
            const int32_t w = wt[p0 + q];
            const int64_t sum = (int64_t)dr[p0 + q] + (int64_t)w;
            hit[q] = (uint8_t)(ok[p0 + q] & (w != ORACLE_I32_INF) & (sum == target));
        }
        for (int64_t q = 0; q < cnt; ++q)
            if (hit[q]) return p0 + q;
    }
    return -1;
}

void oracle_canonical_pred_rows(const void *D, int64_t ldd, const void *W,
                                int64_t ldw, int dtype, int64_t n,
                                const int64_t *rows, int64_t nrows, int32_t *P,
                                int64_t ldp, int nthreads) {
    int nt = oracle_threads(nthreads);
    const int64_t nw = (n + 63) / 64;
    const size_t nn = (size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1);
    uint64_t *adj = (uint64_t *)malloc((size_t)(n > 0 ? n : 1) * (size_t)(nw > 0 ? nw : 1) *
                                       sizeof(uint64_t));
    adjacency_masks(W, dtype, ldw, n, adj, nw);
    /* wt[j * n + p] = W[p][j]; the diagonal marked absent (p != j) */
    void *wt = malloc(nn * 4);
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t q = 0; q < n; ++q) {
            if (dtype == 0)
                ((float *)wt)[j * n + q] =
                    q == j ? INFINITY : ((const float *)W)[q * ldw + j];
            else
                ((int32_t *)wt)[j * n + q] =
                    q == j ? ORACLE_I32_INF : ((const int32_t *)W)[q * ldw + j];
        }
#pragma omp parallel num_threads(nt)
    {
        uint8_t *reach = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
        void *drow = malloc((size_t)(n > 0 ? n : 1) * 4);  /* d(i, .) of the row */
        uint64_t *seen = (uint64_t *)malloc((size_t)(nw > 0 ? nw : 1) * sizeof(uint64_t));
        int64_t *queue = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < nrows; ++r) {
            const int64_t i = rows[r];
            reach_masks(adj, nw, n, i, seen, queue, reach);
            memcpy(drow, (const char *)D + (size_t)(r * ldd) * 4, (size_t)n * 4);
            if (dtype == 0)
                ((float *)drow)[i] = 0.0f;
            else
                ((int32_t *)drow)[i] = 0;
            int32_t *Pr = P + r * ldp;
            for (int64_t j = 0; j < n; ++j) {
                int64_t p = -1;
                if (j != i && reach[j]) {
                    if (dtype == 0) {
                        const float *Dr = (const float *)D + r * ldd;
                        p = first_hit_f32((const float *)drow, (const float *)wt + j * n, reach,
                                          n, Dr[j]);
                    } else {
                        const int32_t *Dr = (const int32_t *)D + r * ldd;
                        p = first_hit_i32((const int32_t *)drow, (const int32_t *)wt + j * n,
                                          reach, n, (int64_t)Dr[j]);
                    }
                }
                Pr[j] = (int32_t)p;
            }
        }
        free(drow);
        free(queue);
        free(seen);
        free(reach);
    }
    free(wt);
    free(adj);
}

/*
 * Single-source shortest paths by Dijkstra's algorithm (textbook dense
 * O(n^2) form, no heap), used to check large solves row by row.  Weights must
 * be non-negative; distances are accumulated in float64, which is exact for
 * integer weights whose path sums stay below 2^53.  out[s*ldo + v] is the
 * distance from srcs[s] to v, +inf when v is unreachable.
 * Returns 0, or -1 if a negative edge weight was found (nothing is computed).
 */
int oracle_dijkstra_rows(const void *W, int dtype, int64_t n, int64_t ld,
                         const int64_t *srcs, int64_t nsrc, double *out,
                         int64_t ldo, int nthreads) {
    for (int64_t p = 0; p < n; ++p)
        for (int64_t j = 0; j < n; ++j)
            if (is_edge(W, dtype, ld, p, j) && weight_f64(W, dtype, ld, p, j) < 0.0)
                return -1;
    int nt = oracle_threads(nthreads);
#pragma omp parallel num_threads(nt)
    {
        uint8_t *done = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < nsrc; ++s) {
            double *dist = out + s * ldo;
            for (int64_t v = 0; v < n; ++v) dist[v] = INFINITY;
            memset(done, 0, (size_t)n);
            dist[srcs[s]] = 0.0;
            for (int64_t it = 0; it < n; ++it) {
                int64_t u = -1;
                double best = INFINITY;
                for (int64_t v = 0; v < n; ++v)
                    if (!done[v] && dist[v] < best) {
                        best = dist[v];
                        u = v;
                    }
                if (u < 0) break;
                done[u] = 1;
                for (int64_t v = 0; v < n; ++v) {
                    if (done[v] || !is_edge(W, dtype, ld, u, v)) continue;
                    double nd = best + weight_f64(W, dtype, ld, u, v);
                    if (nd < dist[v]) dist[v] = nd;
                }
            }
        }
        free(done);
    }
    return 0;
}

/*
 * Widest (bottleneck) paths: the Floyd-Warshall loop of Fig. FW-Alg over the
 * (max, min) semiring, the same k-ordered triple loop with
 *     w_ij <- max(w_ij, min(w_ik, w_kj)),
 * i.e. d_ij = the largest, over all i -> j paths, of the smallest edge weight
 * on the path.  Absent edges carry the max-identity (-INF for fp32,
 * INT32_MIN for int32).  Over weights in {0, 1} this is the transitive
 * closure.  min and max are exact, and row k / column k cannot change in
 * iteration k (min(w_kk, w_kj) <= w_kj), so rows may run in parallel for any
 * input.  max(a, b) := (b > a) ? b : a.
 */
void oracle_fw_maxmin_f32(float *w, int64_t n, int64_t ld, int nthreads) {
    int nt = oracle_threads(nthreads);
    for (int64_t k = 0; k < n; ++k) {
        const float *wk = w + k * ld;
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t i = 0; i < n; ++i) {
            if (i == k) continue;
            float *restrict wi = w + i * ld;
            const float *restrict wkr = wk;
            const float wik = wi[k];
            for (int64_t j = 0; j < n; ++j) {
                float s = (wkr[j] < wik) ? wkr[j] : wik;
                wi[j] = (s > wi[j]) ? s : wi[j];
            }
        }
    }
}

void oracle_fw_maxmin_i32(int32_t *w, int64_t n, int64_t ld, int nthreads) {
    int nt = oracle_threads(nthreads);
    for (int64_t k = 0; k < n; ++k) {
        const int32_t *wk = w + k * ld;
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t i = 0; i < n; ++i) {
            if (i == k) continue;
            int32_t *restrict wi = w + i * ld;
            const int32_t *restrict wkr = wk;
            const int32_t wik = wi[k];
            for (int64_t j = 0; j < n; ++j) {
                int32_t s = (wkr[j] < wik) ? wkr[j] : wik;
                wi[j] = (s > wi[j]) ? s : wi[j];
            }
        }
    }
}

/*
 * Single-source widest paths by the bottleneck variant of Dijkstra's
 * algorithm (dense O(n^2) form): width[src] = +inf, every other vertex starts
 * at -inf; repeatedly finalise the unvisited vertex of largest width u and
 * relax width[v] <- max(width[v], min(width[u], w_uv)) over the edges of W
 * (entries other than -INF; the diagonal is skipped).  Used to check rows of
 * large (max, min) solves.  out[s*ldo + v] = width from srcs[s] to v.
 */
void oracle_widest_rows_f32(const float *W, int64_t n, int64_t ld, const int64_t *srcs,
                            int64_t nsrc, double *out, int64_t ldo, int nthreads) {
    int nt = oracle_threads(nthreads);
#pragma omp parallel num_threads(nt)
    {
        uint8_t *done = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < nsrc; ++s) {
            double *wd = out + s * ldo;
            for (int64_t v = 0; v < n; ++v) wd[v] = -INFINITY;
            memset(done, 0, (size_t)n);
            wd[srcs[s]] = INFINITY;
            for (int64_t it = 0; it < n; ++it) {
                int64_t u = -1;
                double best = -INFINITY;
                for (int64_t v = 0; v < n; ++v)
                    if (!done[v] && (u < 0 || wd[v] > best)) {
                        best = wd[v];
                        u = v;
                    }
                if (u < 0 || best == -INFINITY) break;
                done[u] = 1;
                for (int64_t v = 0; v < n; ++v) {
                    if (done[v] || v == u) continue;
                    const float e = W[u * ld + v];
                    if (isinf(e) && e < 0.0f) continue;
                    const double c = best < (double)e ? best : (double)e;
                    if (c > wd[v]) wd[v] = c;
                }
            }
        }
        free(done);
    }
}
