/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU statement of what the GPU library
 * computes.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it.  It shares no code, header, table or helper with the GPU
 * path, and the GPU path never calls it.
 *
 * Contents (paper: arXiv 2509.19703, "Fast UMAP-based graph drawing"):
 *   oracle_bfs_dist      one-source queue BFS hop distances
 *                        (Sec. 3.1, Alg. 1, step C0: shortest paths of G)
 *   oracle_knn_build     all-source hops + k nearest by (hop, id)
 *                        (Sec. 3.1, Alg. 1, steps C0 and C1)
 *   oracle_knn_partial   truncated BFS that stops at the level completing k
 *                        other vertices (Sec. 3.3.1, Alg. 4 PartialBFS)
 *   oracle_membership    UMAP fuzzy membership rho, sigma and weights in FP64
 *                        (Sec. 2.1, high-dimensional similarity h_ij)
 *   oracle_stress        aggregated stress of a drawing against hop
 *                        distances (Sec. 4.1.3, quality metrics)
 *   oracle_neighborhood  neighbourhood preservation of a drawing, per vertex
 *                        (Sec. 4.1.3, quality metrics)
 *   oracle_splitmix64    the SplitMix64 generator (published definition)
 *   oracle_fuzzy_union   symmetric fuzzy union of the kNN membership weights
 *                        (UMAP's graph symmetrisation before step C2)
 *   oracle_edge_shuffle  shuffled edge array E_k (Alg. 5, first step)
 *   oracle_grad_sample   sliding-window gradient iterations of the layout in
 *                        the paper's serial order (Alg. 5 GradSample,
 *                        Sec. 3.3.2; cost C of Sec. 2.1)
 *   oracle_grad_sample_window  the same iterations with each window applied
 *                        synchronously in fixed point (the device's form; a
 *                        check of the kernels' arithmetic, not of the paper)
 *
 * Readings where the paper is silent or garbled (each is listed with its
 * justification in the design notes):
 *   - true hop distances: the source is at hop 0, its neighbours at hop 1;
 *   - a kNN row lists k OTHER vertices (the source itself is excluded);
 *   - ties at equal hop are broken by ascending vertex id (the paper breaks
 *     them at random, which is not reproducible);
 *   - a level is a set (a vertex enters a level once);
 *   - unreachable vertices (the paper's "infinite" distance, Sec. 3.2) are
 *     never neighbours; missing slots are padded with id -1 and hop 255;
 *   - hop values are uint8, 255 meaning unreachable; a finite hop above 254
 *     cannot be stored in a hop matrix (status -3);
 *   - h_ij = exp(-(d_ij - rho_i) / sigma_i) (the printed sign is a typo) with
 *     sigma_i solving sum_j h_ij = log2(k) over the row's valid entries, k the
 *     requested neighbourhood size; rows with no root take the limits
 *     described at oracle_membership;
 *   - stress sums over ordered pairs of distinct vertices that are connected
 *     (the paper evaluates on connected graphs, where these are all n^2 - n
 *     pairs), the graph distance being the hop count, the drawing distance
 *     the Euclidean one in FP64 of float coordinates; the sum and the number
 *     of pairs are returned, stress = sum / pairs;
 *   - neighbourhood preservation: N_G(v, r) holds the vertices u != v at hop
 *     distance 1..r; N_D(v, r) the |N_G(v, r)| vertices u != v nearest to v in
 *     the drawing, ordered by squared Euclidean distance (FP64, computed as
 *     dx*dx + dy*dy without fused multiply-add) and then by id; a vertex's
 *     score is |N_G & N_D| / |N_G | N_D|, undefined (NaN) when N_G is empty;
 *     the metric sums the defined scores;
 *   - layout step: the readings are stated at each function below (fuzzy
 *     union as in UMAP, E_k holding both directions of each edge, windows
 *     of s consecutive positions, entries moved one after the other, UMAP's
 *     attractive and negative-sample moves scaled by the edge weight,
 *     learning rate alpha0 (1 - it / t)).
 *
 * Threads: rows are independent; `nthreads` worker threads take rows from a
 * shared counter.  This parallelism does not change any result.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ERANGE (-3)
#define ORACLE_ENOMEM (-4)

/* ------------------------------------------------------------------------
 * One-source BFS (FIFO queue).  dist[v] = number of edges on a shortest
 * path from s to v, or -1 if v is not reachable.  Repeated entries and
 * self-loops in the adjacency are harmless: a vertex is labelled only the
 * first time it is seen.
 * ---------------------------------------------------------------------- */
int oracle_bfs_dist(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                    int32_t s, int32_t *dist)
{
    if (n < 0 || s < 0 || s >= n) return ORACLE_EINVAL;
    int32_t *queue = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!queue) return ORACLE_ENOMEM;
    for (int32_t v = 0; v < n; ++v) dist[v] = -1;
    int32_t head = 0, tail = 0;
    dist[s] = 0;
    queue[tail++] = s;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t w = col_idx[e];
            if (dist[w] < 0) {
                dist[w] = dist[u] + 1;
                queue[tail++] = w;
            }
        }
    }
    free(queue);
    return ORACLE_OK;
}

/* --------------------------------------------------------- thread pool -- */

typedef struct {
    int64_t next;          /* next row to take */
    int64_t count;         /* rows in total */
    pthread_mutex_t lock;
    int status;            /* first non-OK status seen */
    void *job;
    int (*row_fn)(void *job, int64_t row, void *scratch);
    size_t scratch_bytes;
} pool_t;

static void *pool_worker(void *arg)
{
    pool_t *p = (pool_t *)arg;
    void *scratch = p->scratch_bytes ? calloc(1, p->scratch_bytes) : NULL;
    if (p->scratch_bytes && !scratch) {
        pthread_mutex_lock(&p->lock);
        if (p->status == ORACLE_OK) p->status = ORACLE_ENOMEM;
        pthread_mutex_unlock(&p->lock);
        return NULL;
    }
    for (;;) {
        pthread_mutex_lock(&p->lock);
        int64_t row = p->next++;
        pthread_mutex_unlock(&p->lock);
        if (row >= p->count) break;
        int st = p->row_fn(p->job, row, scratch);
        if (st != ORACLE_OK) {
            pthread_mutex_lock(&p->lock);
            if (p->status == ORACLE_OK) p->status = st;
            pthread_mutex_unlock(&p->lock);
        }
    }
    free(scratch);
    return NULL;
}

static int run_rows(int64_t count, int nthreads, void *job,
                    int (*row_fn)(void *, int64_t, void *), size_t scratch_bytes)
{
    pool_t p;
    p.next = 0;
    p.count = count;
    pthread_mutex_init(&p.lock, NULL);
    p.status = ORACLE_OK;
    p.job = job;
    p.row_fn = row_fn;
    p.scratch_bytes = scratch_bytes;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int t = 1; t < nthreads; ++t)
        if (pthread_create(&th[started], NULL, pool_worker, &p) == 0) ++started;
    pool_worker(&p);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&p.lock);
    return p.status;
}

/* ------------------------------------------------------------ kNN build --
 * Alg. 1 C0 then C1 for each requested source s:
 *   1. dist = BFS hop distances from s;
 *   2. the pairs (dist[v], v) with v != s and v reachable, sorted
 *      lexicographically; the first min(k, count) of them form the row;
 *   3. remaining slots are padded with (id -1, hop 255).
 * If hop_matrix is not NULL, row r of it (n bytes) receives dist from
 * sources[r] with 255 for unreachable; a finite distance above 254 makes the
 * call fail with ORACLE_ERANGE.
 * ---------------------------------------------------------------------- */

typedef struct { int32_t hop, id; } pair_t;

static int cmp_pair(const void *a, const void *b)
{
    const pair_t *x = (const pair_t *)a, *y = (const pair_t *)b;
    if (x->hop != y->hop) return (x->hop > y->hop) - (x->hop < y->hop);
    return (x->id > y->id) - (x->id < y->id);
}

typedef struct {
    int32_t n;
    const int32_t *row_ptr, *col_idx;
    int32_t k;
    const int32_t *sources;
    int32_t *ids;
    uint8_t *hops;
    uint8_t *hop_matrix;
} build_job;

static int build_row(void *jp, int64_t r, void *scratch)
{
    build_job *j = (build_job *)jp;
    int32_t n = j->n;
    int32_t s = j->sources ? j->sources[r] : (int32_t)r;
    int32_t *dist = (int32_t *)scratch;
    pair_t *pairs = (pair_t *)(dist + n);
    int st = oracle_bfs_dist(n, j->row_ptr, j->col_idx, s, dist);
    if (st != ORACLE_OK) return st;
    int32_t cnt = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (v == s || dist[v] < 0) continue;
        pairs[cnt].hop = dist[v];
        pairs[cnt].id = v;
        ++cnt;
    }
    qsort(pairs, (size_t)cnt, sizeof(pair_t), cmp_pair);
    int32_t *ids = j->ids + r * (int64_t)j->k;
    uint8_t *hops = j->hops + r * (int64_t)j->k;
    for (int32_t i = 0; i < j->k; ++i) {
        if (i < cnt) {
            ids[i] = pairs[i].id;
            hops[i] = (uint8_t)(pairs[i].hop > 254 ? 255 : pairs[i].hop);
        } else {
            ids[i] = -1;
            hops[i] = 255;
        }
    }
    if (j->hop_matrix) {
        uint8_t *row = j->hop_matrix + r * (int64_t)n;
        for (int32_t v = 0; v < n; ++v) {
            if (dist[v] < 0) row[v] = 255;
            else if (dist[v] > 254) return ORACLE_ERANGE;
            else row[v] = (uint8_t)dist[v];
        }
    }
    return ORACLE_OK;
}

int oracle_knn_build(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t k,
                     const int32_t *sources, int32_t n_sources, int32_t *ids, uint8_t *hops,
                     uint8_t *hop_matrix, int nthreads)
{
    if (n < 0 || k < 1 || !ids || !hops) return ORACLE_EINVAL;
    int64_t rows = sources ? n_sources : n;
    if (rows < 0) return ORACLE_EINVAL;
    if (sources)
        for (int64_t r = 0; r < rows; ++r)
            if (sources[r] < 0 || sources[r] >= n) return ORACLE_EINVAL;
    build_job j = {n, row_ptr, col_idx, k, sources, ids, hops, hop_matrix};
    size_t scratch = (size_t)(n > 0 ? n : 1) * (sizeof(int32_t) + sizeof(pair_t));
    return run_rows(rows, nthreads, &j, build_row, scratch);
}

/* ---------------------------------------------------------- PartialBFS --
 * Alg. 4, per source v: BFS one level at a time.  Level h+1 is the set of
 * vertices adjacent to level h that no earlier level contains.  Let c be the
 * number of other vertices already taken.  If c + |level| >= k, the level is
 * sorted by id and its first k - c members are taken, and the search stops;
 * otherwise the whole level is taken (in id order) and the search goes on.
 * The search also stops when a level comes out empty (the component of v has
 * fewer than k + 1 vertices); the row is then padded.
 * Each row is therefore sorted by (hop, id), hops 1..h.
 * ---------------------------------------------------------------------- */

typedef struct {
    int32_t n;
    const int32_t *row_ptr, *col_idx;
    int32_t k;
    const int32_t *sources;
    int32_t *ids;
    uint8_t *hops;
} partial_job;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int partial_row(void *jp, int64_t r, void *scratch)
{
    partial_job *j = (partial_job *)jp;
    int32_t n = j->n, k = j->k;
    int32_t v = j->sources ? j->sources[r] : (int32_t)r;
    int32_t *seen = (int32_t *)scratch;   /* n entries: 0 = not seen, else level + 1 */
    int32_t *cur = seen + n;              /* current level   */
    int32_t *nxt = cur + n;               /* next level      */
    int32_t *touched = nxt + n;           /* vertices marked, cleared again at the end */
    int32_t ntouched = 0;
    int32_t *ids = j->ids + r * (int64_t)k;
    uint8_t *hops = j->hops + r * (int64_t)k;

    seen[v] = 1;
    touched[ntouched++] = v;
    int32_t ncur = 1, taken = 0, h = 0;
    cur[0] = v;
    while (taken < k && ncur > 0) {
        ++h;
        int32_t nnext = 0;
        for (int32_t i = 0; i < ncur; ++i) {
            int32_t u = cur[i];
            for (int32_t e = j->row_ptr[u]; e < j->row_ptr[u + 1]; ++e) {
                int32_t w = j->col_idx[e];
                if (seen[w] == 0) {
                    seen[w] = h + 1;
                    touched[ntouched++] = w;
                    nxt[nnext++] = w;
                }
            }
        }
        qsort(nxt, (size_t)nnext, sizeof(int32_t), cmp_i32);
        int32_t take = nnext < k - taken ? nnext : k - taken;
        for (int32_t i = 0; i < take; ++i) {
            ids[taken + i] = nxt[i];
            hops[taken + i] = (uint8_t)(h > 254 ? 255 : h);
        }
        taken += take;
        memcpy(cur, nxt, (size_t)nnext * sizeof(int32_t));
        ncur = nnext;
    }
    for (int32_t i = taken; i < k; ++i) {
        ids[i] = -1;
        hops[i] = 255;
    }
    for (int32_t i = 0; i < ntouched; ++i) seen[touched[i]] = 0;
    return ORACLE_OK;
}

int oracle_knn_partial(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t k,
                       const int32_t *sources, int32_t n_sources, int32_t *ids, uint8_t *hops,
                       int nthreads)
{
    if (n < 0 || k < 1 || !ids || !hops) return ORACLE_EINVAL;
    int64_t rows = sources ? n_sources : n;
    if (rows < 0) return ORACLE_EINVAL;
    if (sources)
        for (int64_t r = 0; r < rows; ++r)
            if (sources[r] < 0 || sources[r] >= n) return ORACLE_EINVAL;
    partial_job j = {n, row_ptr, col_idx, k, sources, ids, hops};
    size_t scratch = (size_t)(n > 0 ? n : 1) * 4 * sizeof(int32_t);
    return run_rows(rows, nthreads, &j, partial_row, scratch);
}

/* ---------------------------------------------------------- membership --
 * Sec. 2.1: h_j = exp(-(d_j - rho) / sigma) over the row's K valid entries
 * (hop != 255), rho = the hop of the nearest neighbour (the row's first
 * entry), sigma chosen so that f(sigma) = sum_j exp(-(d_j - rho)/sigma)
 * equals T = log2(k).  f rises from c0 = #{j : d_j = rho} (sigma -> 0+) to K
 * (sigma -> infinity), so:
 *   K = 0          rho = 0, sigma = 0, every weight 0;
 *   c0 >= T        no root; sigma -> 0+ limit: sigma = 0, weight 1 where
 *                  d_j = rho and 0 elsewhere;
 *   K <= T         no root (or a root at infinity): sigma = +inf, weights 1;
 *   otherwise      bisection on sigma in double precision: bracket [0, hi]
 *                  with hi doubled from 1 until f(hi) >= T, then halve the
 *                  bracket (f(mid) < T moves lo up, else hi down) until mid
 *                  equals an end point or 2000 steps; sigma = hi.
 * Padding slots get weight 0.  rho and sigma are returned as float, the
 * weights as float(exp(-(d_j - rho)/sigma)) computed in double.
 * ---------------------------------------------------------------------- */

typedef struct {
    int32_t k;
    const uint8_t *hops;
    float *weights, *rho, *sigma;
} memb_job;

static double memb_f(const uint8_t *h, int32_t K, double rho, double sigma)
{
    double s = 0.0;
    for (int32_t j = 0; j < K; ++j) s += exp(-((double)h[j] - rho) / sigma);
    return s;
}

static int memb_row(void *jp, int64_t r, void *scratch)
{
    (void)scratch;
    memb_job *j = (memb_job *)jp;
    int32_t k = j->k;
    const uint8_t *h = j->hops + r * (int64_t)k;
    float *w = j->weights + r * (int64_t)k;
    int32_t K = 0;
    while (K < k && h[K] != 255) ++K;
    double rho = 0.0, sigma = 0.0;
    if (K == 0) {
        for (int32_t i = 0; i < k; ++i) w[i] = 0.0f;
    } else {
        rho = (double)h[0];
        double T = log2((double)k);
        int32_t c0 = 0;
        for (int32_t i = 0; i < K; ++i) c0 += (h[i] == h[0]);
        if ((double)c0 >= T) {
            sigma = 0.0;
            for (int32_t i = 0; i < K; ++i) w[i] = (h[i] == h[0]) ? 1.0f : 0.0f;
        } else if ((double)K <= T) {
            sigma = INFINITY;
            for (int32_t i = 0; i < K; ++i) w[i] = 1.0f;
        } else {
            double lo = 0.0, hi = 1.0;
            while (memb_f(h, K, rho, hi) < T) hi *= 2.0;
            for (int it = 0; it < 2000; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid == lo || mid == hi) break;
                if (memb_f(h, K, rho, mid) < T) lo = mid;
                else hi = mid;
            }
            sigma = hi;
            for (int32_t i = 0; i < K; ++i) w[i] = (float)exp(-((double)h[i] - rho) / sigma);
        }
        for (int32_t i = K; i < k; ++i) w[i] = 0.0f;
    }
    if (j->rho) j->rho[r] = (float)rho;
    if (j->sigma) j->sigma[r] = (float)sigma;
    return ORACLE_OK;
}

int oracle_membership(int64_t rows, int32_t k, const uint8_t *hops, float *weights,
                      float *rho, float *sigma, int nthreads)
{
    if (rows < 0 || k < 1 || !hops || !weights) return ORACLE_EINVAL;
    memb_job j = {k, hops, weights, rho, sigma};
    return run_rows(rows, nthreads, &j, memb_row, 0);
}

/* ------------------------------------------------------------------------
 * Aggregated stress (Sec. 4.1.3): for each listed source s and every vertex
 * v != s reachable from s, ((d(s,v) - |X_s - X_v|) / d(s,v))^2, with d the
 * BFS hop distance and |.| the Euclidean distance of the drawing (xy holds
 * x, y per vertex as float; the arithmetic is FP64).  Per-source sums and
 * pair counts go to row_sum[r] / row_pairs[r]; the caller adds them up.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t n;
    const int32_t *row_ptr, *col_idx, *src;
    const float *xy;
    double *row_sum;
    int64_t *row_pairs;
} stress_job_t;

static int stress_row(void *jp, int64_t r, void *scratch)
{
    stress_job_t *j = (stress_job_t *)jp;
    int32_t *dist = (int32_t *)scratch;
    const int32_t s = j->src ? j->src[r] : (int32_t)r;
    int st = oracle_bfs_dist(j->n, j->row_ptr, j->col_idx, s, dist);
    if (st != ORACLE_OK) return st;
    double sum = 0.0;
    int64_t pairs = 0;
    const double xs = (double)j->xy[2 * (size_t)s], ys = (double)j->xy[2 * (size_t)s + 1];
    for (int32_t v = 0; v < j->n; ++v) {
        if (v == s || dist[v] < 0) continue;
        const double dx = xs - (double)j->xy[2 * (size_t)v];
        const double dy = ys - (double)j->xy[2 * (size_t)v + 1];
        const double e = sqrt(dx * dx + dy * dy);
        const double d = (double)dist[v];
        const double t = (d - e) / d;
        sum += t * t;
        ++pairs;
    }
    j->row_sum[r] = sum;
    j->row_pairs[r] = pairs;
    return ORACLE_OK;
}

int oracle_stress(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const float *xy,
                  const int32_t *sources, int64_t rows, double *row_sum, int64_t *row_pairs, int nthreads)
{
    if (n < 0 || rows < 0) return ORACLE_EINVAL;
    for (int64_t r = 0; sources && r < rows; ++r)
        if (sources[r] < 0 || sources[r] >= n) return ORACLE_EINVAL;
    stress_job_t j = {n, row_ptr, col_idx, sources, xy, row_sum, row_pairs};
    return run_rows(rows, nthreads, &j, stress_row, (size_t)(n > 0 ? n : 1) * sizeof(int32_t));
}

/* ------------------------------------------------------------------------
 * Neighbourhood preservation (Sec. 4.1.3): per vertex v, the Jaccard index of
 * its graph ball N_G(v, r) (hops 1..r) and the same number of nearest
 * vertices in the drawing, ranked by (squared distance, id).  score[v] is
 * NaN when the ball is empty; ball[v] receives |N_G(v, r)|.
 * ---------------------------------------------------------------------- */
typedef struct {
    double d2;
    int32_t id;
} np_key_t;

static int cmp_np_key(const void *a, const void *b)
{
    const np_key_t *x = (const np_key_t *)a, *y = (const np_key_t *)b;
    if (x->d2 < y->d2) return -1;
    if (x->d2 > y->d2) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

typedef struct {
    int32_t n, r;
    const int32_t *row_ptr, *col_idx;
    const float *xy;
    const int32_t *verts;
    double *score;
    int32_t *ball;
} np_job_t;

static int np_row(void *jp, int64_t row, void *scratch)
{
    np_job_t *j = (np_job_t *)jp;
    const int32_t n = j->n, v = j->verts ? j->verts[row] : (int32_t)row;
    int32_t *dist = (int32_t *)scratch;
    np_key_t *keys = (np_key_t *)(dist + n);
    char *in_ball = (char *)(keys + n);
    int st = oracle_bfs_dist(n, j->row_ptr, j->col_idx, v, dist);
    if (st != ORACLE_OK) return st;
    int32_t K = 0;
    for (int32_t u = 0; u < n; ++u) {
        in_ball[u] = (u != v && dist[u] >= 1 && dist[u] <= j->r);
        K += in_ball[u];
    }
    j->ball[row] = K;
    if (K == 0) {
        j->score[row] = NAN;
        return ORACLE_OK;
    }
    const double xv = (double)j->xy[2 * (size_t)v], yv = (double)j->xy[2 * (size_t)v + 1];
    int32_t m = 0;
    for (int32_t u = 0; u < n; ++u) {
        if (u == v) continue;
        const double dx = (double)j->xy[2 * (size_t)u] - xv;
        const double dy = (double)j->xy[2 * (size_t)u + 1] - yv;
        const double sx = dx * dx, sy = dy * dy;
        keys[m].d2 = sx + sy;
        keys[m].id = u;
        ++m;
    }
    qsort(keys, (size_t)m, sizeof(np_key_t), cmp_np_key);
    int32_t common = 0;
    for (int32_t i = 0; i < K; ++i) common += in_ball[keys[i].id];
    j->score[row] = (double)common / (double)(2 * K - common);
    return ORACLE_OK;
}

int oracle_neighborhood(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const float *xy, int32_t r,
                        const int32_t *verts, int64_t rows, double *score, int32_t *ball, int nthreads)
{
    if (n < 0 || r < 1 || rows < 0) return ORACLE_EINVAL;
    for (int64_t i = 0; verts && i < rows; ++i)
        if (verts[i] < 0 || verts[i] >= n) return ORACLE_EINVAL;
    np_job_t j = {n, r, row_ptr, col_idx, xy, verts, score, ball};
    const size_t nn = (size_t)(n > 0 ? n : 1);
    return run_rows(verts ? rows : n, nthreads, &j, np_row, nn * (sizeof(int32_t) + sizeof(np_key_t) + 1));
}

/* ========================================================================
 * Layout step C2 of SL-GUMAP (Sec. 2.1 cost C, Sec. 3.3 Alg. 3 and Alg. 5
 * GradSample), after the kNN graph and its membership weights.
 * ====================================================================== */

/* ------------------------------------------------------------------------
 * SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): the i-th output (i >= 1) of the stream seeded
 * with `seed` mixes seed + i * 0x9E3779B97F4A7C15 by two xor-shift-multiply
 * rounds and a final xor-shift.
 * ---------------------------------------------------------------------- */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------
 * Fuzzy union of the directed kNN membership graph (UMAP's symmetrisation,
 * which the paper inherits from its UMAP implementation, Sec. 4.1.1): with
 * A[i][j] = weight of j in row i (0 when j is not in row i), the symmetric
 * graph has U[i][j] = A[i][j] + A[j][i] - A[i][j] * A[j][i] for every pair
 * where this is positive.  Evaluated in FP64 as (a + b) - a * b without
 * fused multiply-add and rounded to float.
 * Output: CSR with n = rows, columns ascending in each row; `cap` entries
 * of capacity (2 * rows * k always suffices); *nnz receives the count.
 * ---------------------------------------------------------------------- */
typedef struct { int32_t r, c; } rc_t;

static int cmp_rc(const void *a, const void *b)
{
    const rc_t *x = (const rc_t *)a, *y = (const rc_t *)b;
    if (x->r != y->r) return (x->r > y->r) - (x->r < y->r);
    return (x->c > y->c) - (x->c < y->c);
}

static double knn_weight(int32_t k, const int32_t *ids, const float *w, int32_t i, int32_t j)
{
    for (int32_t q = 0; q < k; ++q)
        if (ids[(size_t)i * k + q] == j) return (double)w[(size_t)i * k + q];
    return 0.0;
}

int oracle_fuzzy_union(int32_t rows, int32_t k, const int32_t *ids, const float *w, int32_t *row_ptr,
                       int32_t *col, float *val, int64_t cap, int64_t *nnz)
{
    if (rows < 0 || k < 1 || !row_ptr || !nnz) return ORACLE_EINVAL;
    const size_t cells = (size_t)rows * (size_t)k;
    rc_t *cand = (rc_t *)malloc((2 * cells + 1) * sizeof(rc_t));
    if (!cand) return ORACLE_ENOMEM;
    size_t m = 0;
    for (int32_t i = 0; i < rows; ++i)
        for (int32_t q = 0; q < k; ++q) {
            const int32_t j = ids[(size_t)i * k + q];
            if (j < 0) continue;
            if (j >= rows || j == i) { free(cand); return ORACLE_EINVAL; }
            cand[m].r = i; cand[m].c = j; ++m;
            cand[m].r = j; cand[m].c = i; ++m;
        }
    qsort(cand, m, sizeof(rc_t), cmp_rc);
    int64_t out = 0;
    for (int32_t i = 0; i <= rows; ++i) row_ptr[i] = 0;
    for (size_t e = 0; e < m; ++e) {
        if (e > 0 && cand[e].r == cand[e - 1].r && cand[e].c == cand[e - 1].c) continue;
        const double a = knn_weight(k, ids, w, cand[e].r, cand[e].c);
        const double b = knn_weight(k, ids, w, cand[e].c, cand[e].r);
        const double s = a + b;
        const double p = a * b;
        const double u = s - p;
        if (!(u > 0.0)) continue;
        if (out >= cap) { free(cand); return ORACLE_ERANGE; }
        col[out] = cand[e].c;
        val[out] = (float)u;
        ++out;
        ++row_ptr[cand[e].r + 1];
    }
    for (int32_t i = 0; i < rows; ++i) row_ptr[i + 1] += row_ptr[i];
    *nnz = out;
    free(cand);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * Shuffle of the edge array E_k (Alg. 5, first step): E_k lists every
 * stored entry (i, j, U[i][j]) of the symmetric graph, so each undirected
 * edge appears once per direction, as in the positive-sample arrays of
 * UMAP's optimiser.  Entry e (CSR order) gets the key
 * splitmix64(seed, e + 1); the shuffled order sorts by (key, e).
 * ---------------------------------------------------------------------- */
typedef struct { uint64_t key; int64_t e; } shuf_t;

static int cmp_shuf(const void *a, const void *b)
{
    const shuf_t *x = (const shuf_t *)a, *y = (const shuf_t *)b;
    if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
    return (x->e > y->e) - (x->e < y->e);
}

int oracle_edge_shuffle(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *val, uint64_t seed,
                        int32_t *head, int32_t *tail, float *w)
{
    if (n < 0 || !row_ptr) return ORACLE_EINVAL;
    const int64_t m = row_ptr[n];
    shuf_t *ks = (shuf_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(shuf_t));
    int32_t *row_of = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!ks || !row_of) { free(ks); free(row_of); return ORACLE_ENOMEM; }
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) row_of[e] = i;
    for (int64_t e = 0; e < m; ++e) {
        ks[e].key = oracle_splitmix64(seed, (uint64_t)e + 1);
        ks[e].e = e;
    }
    qsort(ks, (size_t)m, sizeof(shuf_t), cmp_shuf);
    for (int64_t p = 0; p < m; ++p) {
        head[p] = row_of[ks[p].e];
        tail[p] = col[ks[p].e];
        w[p] = val[ks[p].e];
    }
    free(ks);
    free(row_of);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * GradSample (Alg. 5, Sec. 3.3.2) on a 2-D drawing, in the paper's serial
 * order: the entries of a window are taken one after the other, and each
 * reads the CURRENT coordinates of its vertices (as moved by every earlier
 * entry) and moves them before the next entry is read.  Coordinates are
 * plain FP64 for the whole call (read from float, written back as float).
 *
 * s = window (edges per iteration, 1 <= s <= m).  Iteration it in
 * [it_begin, it_end) of a run of t iterations:
 *   lr = alpha0 * (1 - it / t)      (UMAP's linear learning-rate decay)
 *   the window holds the array positions (it * s + l) mod m, l = 0..s-1,
 *   i.e. consecutive windows slide over the shuffled array without gaps.
 * For the window entry (a, b, h) at position l, in this order:
 *   attraction (gradient of h * log(1 + alpha_ab * d^(2 beta)), the
 *   attractive part of the cross-entropy C of Sec. 2.1 with
 *   w = 1 / (1 + alpha_ab * d^(2 beta))), from the current X_a, X_b:
 *     D = X_a - X_b, d2 = Dx*Dx + Dy*Dy, T = d2^beta,
 *     c = -2 alpha_ab beta T / (d2 (1 + alpha_ab T)) if d2 > 0 else 0,
 *     g = clip(c * D, -4, 4) per coordinate,
 *     X_a += lr * h * g,  X_b -= lr * h * g;
 *   then the negative samples of UMAP's optimiser, one after the other: the
 *   q-th is vertex v = splitmix64(seed, ((it * s + l) * neg + q) + 1) mod n;
 *   v == a is skipped; from the current X_a and X_v, E = X_a - X_v,
 *   e2 = |E|^2, T = e2^beta:
 *     c = 2 gamma beta / ((0.001 + e2) (1 + alpha_ab T)),
 *     g = clip(c * E, -4, 4) if e2 > 0, else 4 in each coordinate,
 *     X_a += lr * h * g.
 * The FP64 expressions are evaluated in the order written, without fused
 * multiply-add.  visits (optional) counts how often each array position was
 * processed.
 * ---------------------------------------------------------------------- */
static double clip4(double v)
{
    return v > 4.0 ? 4.0 : (v < -4.0 ? -4.0 : v);
}

int oracle_grad_sample(int32_t n, int64_t m, const int32_t *head, const int32_t *tail, const float *w, float *xy,
                       double alpha_ab, double beta, double gamma, double alpha0, int64_t s, int32_t neg,
                       int32_t t, uint64_t seed, int32_t it_begin, int32_t it_end, int32_t *visits)
{
    if (n < 0 || m < 0 || neg < 0 || t < 1 || it_begin < 0 || it_end > t || it_begin > it_end) return ORACLE_EINVAL;
    if (m == 0 || n == 0 || it_begin == it_end) return ORACLE_OK;
    if (s < 1 || s > m) return ORACLE_EINVAL;
    for (int64_t e = 0; e < m; ++e)
        if (head[e] < 0 || head[e] >= n || tail[e] < 0 || tail[e] >= n) return ORACLE_EINVAL;
    double *X = (double *)malloc((size_t)n * 2 * sizeof(double));
    if (!X) return ORACLE_ENOMEM;
    for (size_t i = 0; i < (size_t)n * 2; ++i) X[i] = (double)xy[i];
    for (int32_t it = it_begin; it < it_end; ++it) {
        const double lr = alpha0 * (1.0 - (double)it / (double)t);
        const int64_t j0 = (int64_t)(((__int128)it * s) % m);
        for (int64_t l = 0; l < s; ++l) {
            const int64_t p = (j0 + l) % m;
            if (visits) ++visits[p];
            const size_t a = (size_t)head[p], b = (size_t)tail[p];
            const double lh = lr * (double)w[p];
            const double dx = X[2 * a] - X[2 * b], dy = X[2 * a + 1] - X[2 * b + 1];
            const double sx = dx * dx, sy = dy * dy;
            const double d2 = sx + sy;
            if (d2 > 0.0) {
                const double T = pow(d2, beta);
                const double num = -2.0 * alpha_ab * beta * T;
                const double den = d2 * (1.0 + alpha_ab * T);
                const double c = num / den;
                const double mx = lh * clip4(c * dx), my = lh * clip4(c * dy);
                X[2 * a] += mx;
                X[2 * a + 1] += my;
                X[2 * b] -= mx;
                X[2 * b + 1] -= my;
            }
            for (int32_t q = 0; q < neg; ++q) {
                const uint64_t idx = ((uint64_t)it * (uint64_t)s + (uint64_t)l) * (uint64_t)neg + (uint64_t)q;
                const size_t v = (size_t)(oracle_splitmix64(seed, idx + 1) % (uint64_t)n);
                if (v == a) continue;
                const double ex = X[2 * a] - X[2 * v], ey = X[2 * a + 1] - X[2 * v + 1];
                const double tx = ex * ex, ty = ey * ey;
                const double e2 = tx + ty;
                double gx = 4.0, gy = 4.0;
                if (e2 > 0.0) {
                    const double T = pow(e2, beta);
                    const double num = 2.0 * gamma * beta;
                    const double den = (0.001 + e2) * (1.0 + alpha_ab * T);
                    const double c = num / den;
                    gx = clip4(c * ex);
                    gy = clip4(c * ey);
                }
                X[2 * a] += lh * gx;
                X[2 * a + 1] += lh * gy;
            }
        }
    }
    for (size_t i = 0; i < (size_t)n * 2; ++i) xy[i] = (float)X[i];
    free(X);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * GradSample with synchronous parts in fixed point: the form the device
 * runs (many entries of a window at once).  A window is cut into
 * P = min(parts, s) consecutive parts, entries l in [c s / P, (c + 1) s / P),
 * applied one after the other.  Every entry of a part starts from the
 * positions at the start of its part and applies its own steps in Alg. 5's
 * order to a private copy of its vertices (attraction moves X_a and X_b, then
 * each negative sample reads the entry's moved X_a, and X_b as moved when the
 * sample is b); the part's moves are added to the positions after the part.  Positions are held as P = round(X * 2^32) (int64 per coordinate,
 * round half to even) and every single move is rounded to that grid, so the
 * sum of a window's moves does not depend on their order.  Schedule, learning
 * rate, attraction and repulsion are those of oracle_grad_sample; where no
 * two entries of a part share a vertex (negative samples included) the two
 * agree up to the grid rounding (at most 2^-33 per move).
 * ---------------------------------------------------------------------- */
int oracle_grad_sample_window(int32_t n, int64_t m, const int32_t *head, const int32_t *tail, const float *w,
                              float *xy, double alpha_ab, double beta, double gamma, double alpha0, int64_t s,
                              int32_t neg, int32_t t, uint64_t seed, int32_t it_begin, int32_t it_end,
                              int32_t *visits, int32_t parts)
{
    if (n < 0 || m < 0 || neg < 0 || t < 1 || it_begin < 0 || it_end > t || it_begin > it_end || parts < 1)
        return ORACLE_EINVAL;
    if (m == 0 || n == 0 || it_begin == it_end) return ORACLE_OK;
    if (s < 1 || s > m) return ORACLE_EINVAL;
    const double scale = 4294967296.0, inv = 1.0 / 4294967296.0;
    for (int64_t e = 0; e < m; ++e)
        if (head[e] < 0 || head[e] >= n || tail[e] < 0 || tail[e] >= n) return ORACLE_EINVAL;
    int64_t *P = (int64_t *)malloc((size_t)n * 2 * sizeof(int64_t));
    int64_t *acc = (int64_t *)calloc((size_t)n * 2, sizeof(int64_t));
    if (!P || !acc) { free(P); free(acc); return ORACLE_ENOMEM; }
    for (size_t i = 0; i < (size_t)n * 2; ++i) P[i] = llrint((double)xy[i] * scale);
    const int64_t np = parts < s ? parts : s;
    for (int32_t it = it_begin; it < it_end; ++it) {
        const double lr = alpha0 * (1.0 - (double)it / (double)t);
        const int64_t j0 = (int64_t)(((__int128)it * s) % m);
        for (int64_t c = 0; c < np; ++c) {
          for (int64_t l = s * c / np; l < s * (c + 1) / np; ++l) {
            const int64_t p = (j0 + l) % m;
            if (visits) ++visits[p];
            const size_t a = (size_t)head[p], b = (size_t)tail[p];
            const double lh = lr * (double)w[p];
            /* the entry's private copies of its two vertices */
            int64_t pax = P[2 * a], pay = P[2 * a + 1], pbx = P[2 * b], pby = P[2 * b + 1];
            const double dx = (double)pax * inv - (double)pbx * inv, dy = (double)pay * inv - (double)pby * inv;
            const double sx = dx * dx, sy = dy * dy;
            const double d2 = sx + sy;
            if (d2 > 0.0) {
                const double T = pow(d2, beta);
                const double num = -2.0 * alpha_ab * beta * T;
                const double den = d2 * (1.0 + alpha_ab * T);
                const double c = num / den;
                const int64_t qx = llrint(lh * clip4(c * dx) * scale);
                const int64_t qy = llrint(lh * clip4(c * dy) * scale);
                pax += qx; pay += qy;
                pbx -= qx; pby -= qy;
            }
            for (int32_t q = 0; q < neg; ++q) {
                const uint64_t idx = ((uint64_t)it * (uint64_t)s + (uint64_t)l) * (uint64_t)neg + (uint64_t)q;
                const size_t v = (size_t)(oracle_splitmix64(seed, idx + 1) % (uint64_t)n);
                if (v == a) continue;
                const int64_t pvx = v == b ? pbx : P[2 * v], pvy = v == b ? pby : P[2 * v + 1];
                const double ex = (double)pax * inv - (double)pvx * inv, ey = (double)pay * inv - (double)pvy * inv;
                const double tx = ex * ex, ty = ey * ey;
                const double e2 = tx + ty;
                double gx = 4.0, gy = 4.0;
                if (e2 > 0.0) {
                    const double T = pow(e2, beta);
                    const double num = 2.0 * gamma * beta;
                    const double den = (0.001 + e2) * (1.0 + alpha_ab * T);
                    const double c = num / den;
                    gx = clip4(c * ex);
                    gy = clip4(c * ey);
                }
                pax += llrint(lh * gx * scale);
                pay += llrint(lh * gy * scale);
            }
            acc[2 * a] += pax - P[2 * a];
            acc[2 * a + 1] += pay - P[2 * a + 1];
            if (b != a) {
                acc[2 * b] += pbx - P[2 * b];
                acc[2 * b + 1] += pby - P[2 * b + 1];
            }
          }
          for (size_t i = 0; i < (size_t)n * 2; ++i) {
              P[i] += acc[i];
              acc[i] = 0;
          }
        }
    }
    for (size_t i = 0; i < (size_t)n * 2; ++i) xy[i] = (float)((double)P[i] * inv);
    free(P);
    free(acc);
    return ORACLE_OK;
}
