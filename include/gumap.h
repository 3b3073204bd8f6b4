/*
 * gumap -- BFS-based graph-theoretic kNN construction of the GUMAP family
 * (arXiv 2509.19703) on one AMD MI355X (gfx950).
 *
 * What it computes (paper sections):
 *   - all-source BFS hop distances of an undirected unweighted graph
 *     (Sec. 3.1, Alg. 1 step C0, "AllPairsShortestPath");
 *   - the kNN graph of those distances (Alg. 1 step C1), each row the k
 *     nearest OTHER vertices ordered by (hop, vertex id);
 *   - the truncated partial BFS that stops once k other vertices are
 *     reached (Sec. 3.3.1, Alg. 4 "PartialBFS"), whose rows are identical
 *     to those of the full construction under the (hop, id) order;
 *   - the UMAP fuzzy-membership weights of a kNN row (Sec. 2.1):
 *     w_j = exp(-(d_j - rho) / sigma), rho = hop of the nearest neighbour,
 *     sigma solving sum_j w_j = log2(k).
 *
 * Conventions shared by every call
 *   - Graphs are CSR with int32 row_ptr[n+1] and col_idx[nnz], both in
 *     device memory.  The graph is read as the undirected edge set
 *     {u, col_idx[e]}: repeated entries and self-loops are ignored and rows
 *     may be in any order unless the caller sets GUMAP_CSR_SORTED.  The
 *     caller guarantees a well-formed, symmetric CSR unless it sets
 *     GUMAP_VALIDATE, in which case a malformed one returns GUMAP_EGRAPH.
 *   - Output rows are k entries wide, row-major, sorted by (hop, id)
 *     ascending; a row with fewer than k reachable other vertices is
 *     padded with id -1, hop 255 and weight 0.
 *   - Hops are uint8; 255 means unreachable (the paper's "infinite"
 *     distance for disconnected pairs, Sec. 3.2).
 *   - Pointers to arrays are device pointers owned by the caller; the
 *     library owns its scratch memory (cached per device, grow-only).
 *   - Calls are host-synchronous: they return after `stream` has finished
 *     the work (0 selects the null stream).  Calls from several host
 *     threads are serialised.
 *   - Every call returns a status code; on failure gumap_last_error() holds
 *     a message for the calling thread.
 */
#ifndef GUMAP_H
#define GUMAP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define GUMAP_OK 0
#define GUMAP_PENDING 1      /* served job still running (gumap_poll only) */
#define GUMAP_EINVAL (-1)    /* bad argument: null pointer, n < 0, k outside [1, 254], bad source id */
#define GUMAP_EGRAPH (-2)    /* GUMAP_VALIDATE: malformed or asymmetric CSR */
#define GUMAP_ERANGE (-3)    /* hop_matrix requested and a finite hop exceeds 254 */
#define GUMAP_ENOMEM (-4)    /* device or host allocation failed */
#define GUMAP_EDEVICE (-5)   /* HIP runtime error */
#define GUMAP_E2BIG (-6)     /* served job larger than the server's memory budget, or input too large
                                for gumap_knn_partial_noalloc's fixed scratch */
#define GUMAP_ENOTFOUND (-7) /* unknown or released ticket */

/* Graph flags. */
#define GUMAP_CSR_SORTED 1u  /* caller asserts: rows sorted ascending, no repeats, no self-loops */
#define GUMAP_VALIDATE 2u    /* check the CSR on the device; malformed -> GUMAP_EGRAPH */

#define GUMAP_MAX_K 254

typedef struct gumap_graph {
    int32_t n;              /* vertices, >= 0 */
    int32_t nnz;            /* col_idx entries, >= 0 */
    const int32_t *row_ptr; /* device, n + 1 entries; row_ptr[0] = 0, row_ptr[n] = nnz */
    const int32_t *col_idx; /* device, nnz entries in [0, n) */
    uint32_t flags;         /* GUMAP_CSR_SORTED | GUMAP_VALIDATE */
} gumap_graph;

/*
 * CSR ingest.  The input of every method step is an undirected unweighted
 * graph G = (V, E) (Sec. 3.1, Alg. 1 input); this writes the canonical CSR
 * of its edge set: rows sorted ascending, repeated entries and self-loops
 * removed.  The other calls do this themselves unless GUMAP_CSR_SORTED is
 * set; calling it once lets a caller pass the result with that flag.
 *   out_row_ptr device int32[n + 1]; out_col_idx device int32[g->nnz]
 *   (capacity); *out_nnz (host) receives the kept entry count.  The
 *   outputs must not overlap the input arrays.
 * Errors: GUMAP_EINVAL, GUMAP_EGRAPH (with GUMAP_VALIDATE), GUMAP_ENOMEM,
 *         GUMAP_EDEVICE.
 */
int gumap_csr_canonicalize(const gumap_graph *g, int32_t *out_row_ptr, int32_t *out_col_idx,
                           int32_t *out_nnz, hipStream_t stream);

/*
 * GUMAP steps C0 + C1 (Sec. 3.1, Alg. 1): BFS hop distances from each source
 * and the (hop, id)-ordered k nearest other vertices of each source.
 *   sources    device int32[n_sources] vertex ids, or NULL for all n vertices
 *              in order (n_sources is then ignored).  Repeats are allowed.
 *   nbr_ids    device int32[rows * k], rows = n_sources (or n)
 *   nbr_hops   device uint8[rows * k]
 *   hop_matrix device uint8[rows * n] or NULL; row r receives the hop from
 *              source r to every vertex (0 at the source, 255 unreachable).
 * Errors: GUMAP_EINVAL (arguments, a source id outside [0, n)),
 *         GUMAP_EGRAPH, GUMAP_ERANGE (only with hop_matrix), GUMAP_ENOMEM,
 *         GUMAP_EDEVICE.  On error the outputs are unspecified.
 */
int gumap_knn_build(const gumap_graph *g, int32_t k, const int32_t *sources, int32_t n_sources,
                    int32_t *nbr_ids, uint8_t *nbr_hops, uint8_t *hop_matrix, hipStream_t stream);

/*
 * Autotuning of gumap_knn_build (the same outputs; only the speed of the
 * search depends on these settings).  gumap_knn_build_tune runs the call
 * on the caller's graph, sources and outputs once per candidate setting --
 * one warm-up, then the fastest of three timed calls -- by a coordinate
 * descent from the defaults over: the one-workgroup-per-group form for
 * small graphs; the source-bitset width (64 x {1, 2, 4, 8} sources per
 * group); (vertex, word) items per thread of the level kernel {1, 2, 4, 8};
 * level 1 as a top-down scatter from the sources or a range scan; the
 * degree above which a vertex is searched by a whole wave {default rule,
 * 32, 128, 512}; hops kept as frontiers {0, 15}; levels 2.. that may run
 * top-down {0, 2}.  The pick is written to *out and recorded for the shape
 * of the call (floor(log2) of n, of the mean degree nnz / n, of the number
 * of sources and of k, and whether hop_matrix is given); later
 * gumap_knn_build calls of that shape (and gumap_stress calls, k = 1 with
 * hop rows) use it.  A setting given in the environment (GUMAP_FUSED,
 * GUMAP_FORCE_WORDS, GUMAP_LEVEL_VERTS, GUMAP_FIRST_LEVEL,
 * GUMAP_HEAVY_DEGREE, GUMAP_HIST_LEVELS, GUMAP_PUSH_LEVELS) overrides the
 * recorded one.  If GUMAP_AUTOTUNE_CACHE names a file, the recorded picks
 * are read from it on first use and the file is rewritten (JSON) after each
 * tuning.  Arguments and errors as gumap_knn_build; GUMAP_EINVAL also for
 * out == NULL or an unwritable cache file.
 */
typedef struct gumap_build_tuning {
    int32_t fused;        /* 1: every level of a group in one workgroup (words = 1) */
    int32_t words;        /* 64-bit source words per vertex per group */
    int32_t level_verts;  /* (vertex, word) items per thread of the level kernel */
    int32_t first_level;  /* 1: fill + top-down scatter from the sources; 0: range scan */
    int32_t heavy_degree; /* whole-wave search above this degree; 0: max(64, 8 x mean degree) */
    int32_t hist_levels;  /* hops kept as frontiers instead of bit-plane updates */
    int32_t push_levels;  /* levels after the sources that may run top-down */
    int32_t candidates;   /* settings timed */
    float best_ms;        /* one call with the pick */
    float default_ms;     /* one call with the defaults */
} gumap_build_tuning;
int gumap_knn_build_tune(const gumap_graph *g, int32_t k, const int32_t *sources, int32_t n_sources,
                         int32_t *nbr_ids, uint8_t *nbr_hops, uint8_t *hop_matrix, hipStream_t stream,
                         gumap_build_tuning *out);
/* The recorded pick for calls of this shape (hop_matrix != 0: hop rows
 * wanted); host only.  Returns 1 and fills *out if there is one, 0 if not,
 * GUMAP_EINVAL for out == NULL, a negative size or k < 1. */
int gumap_build_tuning_lookup(int32_t n, int64_t nnz, int64_t n_sources, int32_t k, int hop_matrix,
                              gumap_build_tuning *out);
/* Replace the recorded picks by those of a cache file / write them to one;
 * host only.  GUMAP_EINVAL if the file cannot be read or written or is not a
 * cache written by this library (the picks are then unchanged). */
int gumap_autotune_cache_load(const char *path);
int gumap_autotune_cache_save(const char *path);
/* Forget every recorded pick (and do not read GUMAP_AUTOTUNE_CACHE again). */
void gumap_autotune_clear(void);

/*
 * Aggregated stress of a drawing (Sec. 4.1.3 quality metrics): the sum over
 * ordered pairs (s, v), s in `sources` (every vertex when sources is NULL;
 * a source listed twice counts twice) and v != s reachable from s, of
 * ((d(s,v) - |X_s - X_v|) / d(s,v))^2, with d the hop distance of the graph
 * and |.| the Euclidean distance of the drawing, computed in FP64, plus the
 * number of such pairs.  The metric is *sum / *pairs (the paper's 1/(n^2-n)
 * normalisation on a connected graph).  Runs the all-source BFS of
 * gumap_knn_build and folds the terms into its hop-row pass; no hop rows are
 * written.
 *   xy       device float[2 * n]: x and y of vertex v at xy[2v], xy[2v + 1]
 *   sources  device int32[n_sources] or NULL
 *   sum      host double (out);  pairs  host int64 (out)
 * Errors: GUMAP_EINVAL (NULL pointer, bad source id), GUMAP_EGRAPH (with
 * GUMAP_VALIDATE), GUMAP_ERANGE (a finite hop distance above 254),
 * GUMAP_ENOMEM, GUMAP_EDEVICE.
 */
int gumap_stress(const gumap_graph *g, const float *xy, const int32_t *sources, int32_t n_sources,
                 double *sum, int64_t *pairs, hipStream_t stream);

/*
 * Neighbourhood preservation of a drawing (Sec. 4.1.3 quality metrics), per
 * vertex: the Jaccard index |N_G & N_D| / |N_G | N_D| of the graph ball
 * N_G(v, r) (vertices u != v within r hops) and N_D(v, r), the |N_G(v, r)|
 * vertices u != v nearest to v in the drawing, ranked by squared Euclidean
 * distance (FP64, dx*dx + dy*dy without fused multiply-add) and then by id.
 * The paper's metric is the sum of the scores (r = 2).
 *   xy        device float[2 * n] (x, y of each vertex)
 *   r         1 or 2
 *   vertices  device int32[n_vertices] or NULL (every vertex, n_vertices ignored)
 *   score     device double[rows]: the score of each listed vertex, NaN when
 *             its ball is empty
 *   ball      device int32[rows] or NULL: |N_G(v, r)|
 * Each vertex costs a few passes over all n vertices of the drawing; n is
 * limited to about 1.2 million (the ball is a bit set in LDS).
 * Errors: GUMAP_EINVAL (NULL pointer, r, vertex id, n too large),
 * GUMAP_EGRAPH (with GUMAP_VALIDATE), GUMAP_ENOMEM, GUMAP_EDEVICE.
 */
int gumap_neighborhood(const gumap_graph *g, const float *xy, int32_t r, const int32_t *vertices,
                       int32_t n_vertices, double *score, int32_t *ball, hipStream_t stream);

/*
 * SL-/SSSL-GUMAP steps C0 + C1 (Sec. 3.3.1, Alg. 4 PartialBFS): for every
 * vertex v, a BFS that stops at the level completing k other vertices; the
 * row holds all earlier levels and the smallest ids of that last level.
 * Rows are identical to gumap_knn_build's for sources = all vertices.
 *   nbr_ids  device int32[n * k];  nbr_hops device uint8[n * k]
 * Errors: GUMAP_EINVAL, GUMAP_EGRAPH, GUMAP_ENOMEM, GUMAP_EDEVICE.
 */
int gumap_knn_partial(const gumap_graph *g, int32_t k, int32_t *nbr_ids, uint8_t *nbr_hops,
                      hipStream_t stream);

/*
 * gumap_knn_partial_noalloc: gumap_knn_partial for callers that cannot
 * allocate device or host memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, results
 * and kernels as gumap_knn_partial; it calls no hipMalloc, hipFree or other
 * allocating routine.  The canonical CSR and the canonicalisation's work
 * arrays live in one fixed device array of GUMAP_NOALLOC_SCRATCH_BYTES that
 * each device the library runs on holds until the process ends; its address
 * on a device is looked up on the first call there.
 * Differences from gumap_knn_partial:
 *   - GUMAP_VALIDATE is rejected (GUMAP_EINVAL): validation reads its result
 *     back through pinned host memory that the library allocates;
 *   - without GUMAP_CSR_SORTED the graph must fit the fixed scratch:
 *     256-byte-rounded 4 (n + 1) + 4 nnz bytes for the canonical CSR plus the
 *     canonicalisation's work arrays (about 12 n + 4 nnz bytes more); a larger
 *     one returns GUMAP_E2BIG (with GUMAP_CSR_SORTED no scratch is used and
 *     any size is accepted);
 *   - every call on a device shares that device's array, so calls that
 *     overlap on one device (from several processes' streams, or a captured
 *     graph replayed while a call runs) race; calls from threads of one
 *     process are serialised like every other call.
 * Errors: GUMAP_EINVAL, GUMAP_E2BIG, GUMAP_EDEVICE.
 */
#define GUMAP_NOALLOC_SCRATCH_BYTES (64u << 20)
int gumap_knn_partial_noalloc(const gumap_graph *g, int32_t k, int32_t *nbr_ids, uint8_t *nbr_hops,
                              hipStream_t stream);

/*
 * UMAP fuzzy membership of kNN rows (Sec. 2.1): per row with K valid
 * entries (hop != 255) sorted ascending, rho = the first hop and sigma
 * solves sum_j exp(-(h_j - rho)/sigma) = log2(k), k the row width.
 * Rows without a root take the limits: K = 0 -> rho = sigma = 0, weights 0;
 * #{h_j = rho} >= log2 k -> sigma = 0, weight 1 at h_j = rho and 0 beyond;
 * K <= log2 k -> sigma = +inf, weights 1.  The root is found in double
 * precision; weights, rho and sigma are written as float.
 *   nbr_hops device uint8[rows * k] (as written by the kNN calls)
 *   weights  device float[rows * k];  rho, sigma device float[rows] or NULL
 * Errors: GUMAP_EINVAL, GUMAP_EDEVICE.
 */
int gumap_membership(int32_t rows, int32_t k, const uint8_t *nbr_hops, float *weights, float *rho,
                     float *sigma, hipStream_t stream);

/*
 * Layout step C2 (Sec. 2.1 cost C; Sec. 3.3, Alg. 3 and Alg. 5 GradSample).
 *
 * gumap_fuzzy_union: the symmetric graph of UMAP's fuzzy union of a
 * directed kNN membership graph.  With A[i][j] the weight of j in row i
 * (0 when absent), U[i][j] = A[i][j] + A[j][i] - A[i][j] * A[j][i],
 * evaluated in FP64 as (a + b) - a * b and rounded to float; entries with
 * U = 0 are dropped.
 *   rows, k   the kNN has rows x k cells (rows = number of vertices)
 *   ids       device int32[rows * k]: neighbour ids; a negative id marks an
 *             empty slot (gumap_knn_partial pads with -1)
 *   weights   device float[rows * k] (gumap_membership's output)
 *   row_ptr   device int32[rows + 1] (out);  col device int32[cap],
 *   val       device float[cap] (out): columns ascending within a row
 *   cap       capacity of col / val; 2 * rows * k always suffices
 *   nnz       host int64 (out): stored entries
 * Errors: GUMAP_EINVAL (NULL pointer, rows < 0, k outside [1, 254],
 * 2 * rows * k >= 2^31, an id at or above rows, or equal to its row),
 * GUMAP_ERANGE (more than cap entries: *nnz holds the count needed),
 * GUMAP_ENOMEM, GUMAP_EDEVICE.
 */
int gumap_fuzzy_union(int32_t rows, int32_t k, const int32_t *ids, const float *weights, int32_t *row_ptr,
                      int32_t *col, float *val, int64_t cap, int64_t *nnz, hipStream_t stream);

/*
 * gumap_edge_shuffle: the edge array E_k of Alg. 5 in shuffled order.  E_k
 * lists every stored entry (i, j, w) of a symmetric CSR (so each undirected
 * edge once per direction); entry e (CSR order) gets the key
 * SplitMix64(seed, e + 1) (the (e + 1)-th output of the generator seeded
 * with `seed`) and the array is ordered by (key, e).
 *   n, row_ptr, col, val   device CSR (gumap_fuzzy_union's output)
 *   m                      number of entries, must equal row_ptr[n]
 *   head, tail             device int32[m] (out): the entry's row and column
 *   w                      device float[m] (out): its weight
 * Errors: GUMAP_EINVAL (NULL pointer, n < 0, m != row_ptr[n], m >= 2^31),
 * GUMAP_ENOMEM, GUMAP_EDEVICE.
 */
int gumap_edge_shuffle(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *val, int64_t m,
                       uint64_t seed, int32_t *head, int32_t *tail, float *w, hipStream_t stream);

/*
 * Spectral sparsification front end of SS-GUMAP / SSSL-GUMAP (Sec. 3.2,
 * Alg. 2 and Alg. 6): rank the edges by effective resistance, keep a maximum
 * spanning tree (forest) of the resistances and then the edges of highest
 * resistance until about n log n edges.  The edges of a graph are its
 * entries (u, v) with u < v, numbered in CSR order of the canonical CSR.
 *
 * gumap_effective_resistance: R_e of every edge of the (unweighted,
 * symmetric) graph, estimated by random projection (Spielman and
 * Srivastava): with q sign vectors s_k over the edges (s_k(e) = -1 when bit
 * 63 of SplitMix64(seed, k m + e + 1) is set, else +1), x_k solves
 * L x_k = B^T s_k (L = D - W, B the edge-vertex incidence) by conjugate
 * gradients preconditioned with the degrees, from x = 0, each until
 * |r| <= tol |b| or max_iters iterations; R_e = (1/q) sum_k (x_k(u) - x_k(v))^2.
 * The estimate is unbiased with relative spread about sqrt(2 / q).  FP64.
 *   q           sign vectors, 1 .. 1024 (n q < 2^31)
 *   resistance  device double[g->nnz / 2] (out), indexed by edge
 *   edges       host int64 or NULL (out): number of edges m
 *   iterations  host int32 or NULL (out): CG iterations run (the slowest column)
 * Errors: GUMAP_EINVAL (NULL pointer, q, tol <= 0, max_iters < 1),
 * GUMAP_EGRAPH (malformed under GUMAP_VALIDATE; not symmetric or with
 * self-loops after canonicalisation), GUMAP_ENOMEM, GUMAP_EDEVICE.
 */
int gumap_effective_resistance(const gumap_graph *g, int32_t q, uint64_t seed, double tol, int32_t max_iters,
                               double *resistance, int64_t *edges, int32_t *iterations, hipStream_t stream);

/*
 * gumap_sparsify_select: the sparsified graph G' for given edge weights
 * (the resistances): the maximum spanning forest in the order (resistance
 * descending, edge index ascending), which makes it unique, then the
 * further edges first in that order until `target` edges (target <= 0:
 * ceil(n ln n); at most m; the forest is kept whole if it alone exceeds
 * the target).
 *   resistance   device double[m], non-negative (gumap_effective_resistance's output)
 *   out_row_ptr  device int32[n + 1], out_col_idx device int32[g->nnz] (out):
 *                the symmetric CSR of G', columns ascending
 *   out_nnz      host int32 (out): entries of G' (twice its edges)
 * Errors: as gumap_effective_resistance (NULL pointer, graph).
 */
int gumap_sparsify_select(const gumap_graph *g, const double *resistance, int64_t target, int32_t *out_row_ptr,
                          int32_t *out_col_idx, int32_t *out_nnz, hipStream_t stream);

/* Parameters of gumap_spectral_layout (zero fields take the defaults). */
typedef struct {
    int32_t max_steps;  /* Lanczos steps at most (default 600, never more than n - 1) */
    int32_t pad;
    double tol;         /* residual |A x - mu x| of each eigenvector (default 1e-5) */
    uint64_t seed;      /* SplitMix64 seed of the starting vector */
} gumap_spectral_params;

/*
 * gumap_spectral_layout: the spectral initial drawing of the layout step
 * (the paper starts its layout from a spectral layout, Sec. 3.2, as UMAP
 * does): the eigenvectors of the 2nd and 3rd smallest eigenvalues of the
 * normalised Laplacian L = I - D^-1/2 W D^-1/2 of the symmetric weighted
 * graph W (D: weighted degrees), each of unit norm with the sign that makes
 * positive its first entry of magnitude above half its largest, the two
 * scaled together so that the largest coordinate magnitude is 10.  Computed
 * by Lanczos iteration with full reorthogonalisation in FP64 on the
 * complement of the known eigenvector D^1/2 1, until both residuals are at
 * most tol; the result approximates the exact eigenvectors to about
 * tol / (eigenvalue gap).
 *   n, row_ptr, col, val   device symmetric CSR with non-negative float weights
 *                          (gumap_fuzzy_union's output), connected
 *   params                 host, may be NULL (defaults)
 *   xy                     device float[2 n] (out): x, y of vertex v at xy[2v], xy[2v + 1]
 *   eigenvalues            host double[2] or NULL (out): the two eigenvalues of L
 *   steps                  host int32 or NULL (out): Lanczos steps taken
 * Scratch: (min(max_steps, n - 1) + 6) * n doubles of device memory.
 * Errors: GUMAP_EINVAL (NULL pointer, n < 3, a weight negative or not
 * finite), GUMAP_EGRAPH (a vertex of zero degree, or a disconnected graph:
 * second eigenvalue below 1e-10), GUMAP_ERANGE (no convergence within
 * max_steps), GUMAP_ENOMEM, GUMAP_EDEVICE.
 */
int gumap_spectral_layout(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *val,
                          const gumap_spectral_params *params, float *xy, double *eigenvalues, int32_t *steps,
                          hipStream_t stream);

/* Parameters of gumap_grad_sample. */
typedef struct {
    double alpha;      /* low-dimensional similarity 1 / (1 + alpha d^(2 beta)) */
    double beta;
    double gamma;      /* weight of the repulsive (negative-sample) moves */
    double alpha0;     /* learning rate of iteration 0; iteration it uses alpha0 (1 - it / t) */
    double samp;       /* window = floor(m^samp) when window is 0 (the paper uses 0.9) */
    int64_t window;    /* edges per iteration s, 1 <= s <= m; 0 = from samp */
    int32_t neg;       /* negative samples per edge (>= 0) */
    int32_t t;         /* iterations of the whole run (>= 1) */
    uint64_t seed;     /* seed of the negative samples */
    int32_t parts;     /* synchronous parts per window (>= 0; 0 = GUMAP_LAYOUT_DEFAULT_PARTS) */
    int32_t pad;
} gumap_layout_params;

/* Default number of synchronous parts of a GradSample window. */
#define GUMAP_LAYOUT_DEFAULT_PARTS 4

/*
 * gumap_grad_sample: iterations [it_begin, it_end) of a t-iteration
 * GradSample run on a 2-D drawing.  Iteration it processes the entries at
 * positions (it * s + l) mod m, l = 0..s-1, of the shuffled edge array
 * (consecutive windows slide without gaps or overlap) at learning rate
 * lr = alpha0 (1 - it / t).  For entry (a, b, h), with D = X_a - X_b,
 * d2 = |D|^2 and T = d2^beta:
 *   attraction   g = clip(c D, -4, 4), c = -2 alpha beta T / (d2 (1 + alpha T))
 *                (0 when d2 = 0); X_a += lr h g, X_b -= lr h g;
 *   repulsion    for q < neg: v = SplitMix64(seed, (it s + l) neg + q + 1) mod n,
 *                skipped when v = a; with E = X_a - X_v, e2 = |E|^2:
 *                g = clip(c E, -4, 4), c = 2 gamma beta / ((0.001 + e2)(1 + alpha e2^beta)),
 *                or g = (4, 4) when e2 = 0; X_a += lr h g.
 * Alg. 5 (Sec. 3.3.2) takes the window's entries one after the other, each
 * reading the coordinates as moved by the entries before it.  Here the window
 * is cut into P = min(parts, s) consecutive parts (entries l in
 * [c s / P, (c + 1) s / P), c = 0..P-1) that are applied one after the
 * other; within a part the entries are applied at once: each entry starts
 * from the positions at the start of its part and takes its own steps in
 * Alg. 5's order on its private copy of its vertices (attraction on a and b,
 * then each negative sample from the moved X_a, reading the moved X_b when
 * v = b), and the part's moves are added afterwards.  Where no two entries
 * of a part share a vertex (negative samples included) this is exactly the
 * serial order; otherwise it is a synchronous approximation of it, closer
 * the more parts.  Positions are kept in fixed point (round(X * 2^32) in
 * int64) during the call and every move is rounded to that grid, so results
 * do not depend on thread scheduling; xy is read at the start and written at
 * the end.  FP64 arithmetic throughout.  Splitting a run into several calls
 * over consecutive iteration ranges gives the same drawing as one call, up
 * to the rounding of xy to float between calls.
 *   n               vertices;  xy device float[2 n] (in/out): x, y of vertex v
 *                   at xy[2v], xy[2v + 1], each of magnitude below 2^20
 *   m, head, tail, w  the shuffled edge array (gumap_edge_shuffle's output)
 *   p               parameters (host)
 * Errors: GUMAP_EINVAL (NULL pointer, n < 0, m < 0, m >= 2^30, m > 0 with n = 0,
 * window outside [1, m], neg < 0, t < 1, parts < 0, iteration range outside [0, t],
 * an endpoint outside [0, n), a coordinate out of range), GUMAP_ENOMEM,
 * GUMAP_EDEVICE.
 */
int gumap_grad_sample(int32_t n, float *xy, int64_t m, const int32_t *head, const int32_t *tail, const float *w,
                      const gumap_layout_params *p, int32_t it_begin, int32_t it_end, hipStream_t stream);

/*
 * Many graphs at once (partial BFS + membership fused, one persistent
 * launch over all vertices of all graphs).
 * Packing: graph i has n_i = vtx_offset[i+1] - vtx_offset[i] vertices and
 * its own local CSR: row_ptr[vtx_offset[i] + i .. vtx_offset[i+1] + i]
 * (n_i + 1 entries, starting at 0) and col_idx[edge_offset[i] ..
 * edge_offset[i+1]) holding local ids in [0, n_i).  Output row of vertex v of
 * graph i is vtx_offset[i] + v; ids in it are local to graph i.
 */
typedef struct gumap_batch {
    int32_t n_graphs;
    int64_t total_vertices;     /* vtx_offset[n_graphs] (host copy) */
    int64_t total_nnz;          /* edge_offset[n_graphs] (host copy) */
    const int64_t *vtx_offset;  /* device, n_graphs + 1 */
    const int64_t *edge_offset; /* device, n_graphs + 1 */
    const int32_t *row_ptr;     /* device, total_vertices + n_graphs */
    const int32_t *col_idx;     /* device, total_nnz */
    uint32_t flags;             /* GUMAP_CSR_SORTED | GUMAP_VALIDATE */
} gumap_batch;

/*
 * Rows of every graph of the batch: nbr_ids/nbr_hops as gumap_knn_partial,
 * weights/rho/sigma as gumap_membership (weights, rho, sigma may be NULL to
 * skip membership).  All outputs are device arrays indexed by packed row.
 * Errors: GUMAP_EINVAL, GUMAP_EGRAPH, GUMAP_ENOMEM, GUMAP_EDEVICE.
 */
int gumap_knn_partial_batch(const gumap_batch *b, int32_t k, int32_t *nbr_ids, uint8_t *nbr_hops,
                            float *weights, float *rho, float *sigma, hipStream_t stream);

/*
 * Captured form of gumap_knn_partial_batch for repeated calls on the same
 * packed batch and output buffers: the launch sequence is recorded once into
 * a HIP graph and replayed.  The batch arrays and outputs must stay valid and
 * unchanged in size until gumap_batch_plan_destroy.  The batch must be
 * canonical (GUMAP_CSR_SORTED).  Replays give the same results as the plain
 * call.
 * Before capture the launch is autotuned on this batch: every candidate
 * (lanes per source in {16, 32, 64} where k + 1 fits, or one wave per source;
 * rows per work grab in {16, 32, 64}; half or all of the resident-workgroup
 * grid) is timed (one warm-up and two timed launches, writing the outputs),
 * and the fastest is recorded.  Every candidate computes the same rows.
 * Setting the environment variable GUMAP_PLAN_TUNE=0 skips the tuning.
 */
typedef struct gumap_batch_plan gumap_batch_plan;
int gumap_batch_plan_create(const gumap_batch *b, int32_t k, int32_t *nbr_ids, uint8_t *nbr_hops,
                            float *weights, float *rho, float *sigma, hipStream_t stream,
                            gumap_batch_plan **plan);
int gumap_batch_plan_launch(gumap_batch_plan *plan, hipStream_t stream); /* host-synchronous */
void gumap_batch_plan_destroy(gumap_batch_plan *plan);

/* What the autotuner of gumap_batch_plan_create picked (all zero when it did
 * not run).  Errors: GUMAP_EINVAL for a NULL argument. */
typedef struct gumap_batch_tuning {
    int32_t lanes;      /* lanes per source: 16, 32, 64; -1 one wave per source; 0 default */
    int32_t chunk;      /* rows per work grab */
    int32_t blocks;     /* persistent workgroups */
    int32_t candidates; /* configurations timed */
    float best_ms;      /* one launch with the pick */
    float default_ms;   /* one launch with the defaults of gumap_knn_partial_batch */
} gumap_batch_tuning;
int gumap_batch_plan_tuning(const gumap_batch_plan *plan, gumap_batch_tuning *out);

/* ----------------------------------------------------------- serving --- */

/*
 * A request loop that takes layout-preparation jobs (one host CSR graph +
 * k) as they arrive, keeps their CSR and results resident in device memory
 * while they run, admits them first-come-first-served under a byte budget,
 * and runs the admitted jobs' rows together (continuous batching: jobs that
 * arrive while others run join the next device iteration).  Each job's
 * result is the same as gumap_knn_partial + gumap_membership on its graph.
 */
typedef struct gumap_server gumap_server;

typedef struct gumap_job {
    int32_t n, nnz;
    const int32_t *row_ptr;  /* HOST, n + 1; copied before gumap_submit returns */
    const int32_t *col_idx;  /* HOST, nnz */
    int32_t k;               /* 1..254 */
    int32_t want_weights;    /* nonzero: also weights, rho, sigma */
    uint32_t flags;          /* GUMAP_CSR_SORTED | GUMAP_VALIDATE */
} gumap_job;

typedef struct gumap_result {
    int32_t status;          /* GUMAP_OK or the job's error */
    int32_t n, k;
    const int32_t *nbr_ids;  /* HOST, n * k; owned by the server until gumap_release */
    const uint8_t *nbr_hops; /* HOST, n * k */
    const float *weights;    /* HOST, n * k, or NULL */
    const float *rho;        /* HOST, n, or NULL */
    const float *sigma;      /* HOST, n, or NULL */
    uint64_t t_submit_ns, t_admit_ns, t_start_ns, t_done_ns; /* steady clock */
} gumap_result;

typedef struct gumap_server_stats {
    uint64_t submitted, completed, failed, iterations;
    uint64_t queued, running;          /* jobs now waiting / admitted */
    uint64_t resident_bytes, peak_resident_bytes, budget_bytes;
} gumap_server_stats;

/* Server flag: run the scheduler without a device (results are zeros); for
 * testing admission and ordering logic on machines without a GPU.  In this
 * mode the environment variable GUMAP_SERVE_NODEV_FAIL_ITER=N makes the
 * executor report iteration N as failed, as a device error would: every job
 * with rows in it ends with GUMAP_EDEVICE and the others are unaffected. */
#define GUMAP_SERVER_NO_DEVICE 1u

/* hbm_budget_bytes: device bytes the resident jobs may hold together;
 * max_slots: jobs admitted at once (0 = no limit).  Job inputs and results
 * are staged in a pinned host pool (GUMAP_SERVE_HOST_POOL_MB, default 16384,
 * touched once at creation).  A submission that finds the pool full waits up
 * to 200 ms while inputs of earlier jobs are still in it (each leaves once
 * uploaded), then uses pageable host memory; results that find it full use
 * pageable memory.  t_submit_ns is taken when gumap_submit is entered, so
 * latencies include the copy of the CSR. */
gumap_server *gumap_server_create(size_t hbm_budget_bytes, int32_t max_slots, uint32_t flags,
                                  int *status);
/* Copies the job and returns a ticket.  GUMAP_E2BIG if it can never fit. */
int gumap_submit(gumap_server *s, const gumap_job *job, uint64_t *ticket);
/* GUMAP_PENDING while the job runs, else fills *out and returns its status. */
int gumap_poll(gumap_server *s, uint64_t ticket, gumap_result *out);
/* Blocks until the job ends (or timeout_ms elapses: GUMAP_PENDING; < 0 = forever). */
int gumap_wait(gumap_server *s, uint64_t ticket, int64_t timeout_ms, gumap_result *out);
/* Frees a finished job's host results.  GUMAP_ENOTFOUND if unknown/released,
 * GUMAP_PENDING if still running. */
int gumap_release(gumap_server *s, uint64_t ticket);
int gumap_server_get_stats(gumap_server *s, gumap_server_stats *out);
/* Stops the scheduler; jobs still queued or running end with GUMAP_EDEVICE
 * status semantics are not observable afterwards (the server is gone). */
void gumap_server_destroy(gumap_server *s);

/* Message of the calling thread's last failure ("" if none). */
const char *gumap_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GUMAP_H */
