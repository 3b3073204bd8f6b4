/*
 * Drives the C oracle and the C graph generators under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_sanitizers_cpu.py with gcc,
 * host code only).  Every function is called on seeded graphs of each
 * generator, on dirty rows (repeats, self-loops), and on the degenerate
 * inputs the library accepts (n = 0, isolated vertices, k above n, windows
 * of one entry); results are checked only for internal consistency, since
 * the pinned tests check the values.  Exit status 0 means every call
 * returned and the sanitizers reported nothing.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t gg_ba(int32_t n, int32_t m_attach, uint64_t seed, int32_t **edges);
int64_t gg_er(int32_t n, double p, uint64_t seed, int32_t **edges);
int64_t gg_sbm(int32_t n, int32_t blocks, double p_in, double p_out, uint64_t seed, int32_t **edges);
int64_t gg_rgg(int32_t n, double radius, uint64_t seed, int32_t **edges);
int64_t gg_csr(int32_t n, int64_t m, const int32_t *edges, int32_t *row_ptr, int32_t *col_idx);
uint64_t gg_mix_seed(uint64_t base, uint64_t index);
double gg_uniform(uint64_t seed, int64_t count, double *out);
void gg_free(void *p);

int oracle_bfs_dist(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t s, int32_t *dist);
int oracle_knn_build(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t k, const int32_t *sources,
                     int32_t n_sources, int32_t *ids, uint8_t *hops, uint8_t *hop_matrix, int nthreads);
int oracle_knn_partial(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t k, const int32_t *sources,
                       int32_t n_sources, int32_t *ids, uint8_t *hops, int nthreads);
int oracle_membership(int64_t rows, int32_t k, const uint8_t *hops, float *weights, float *rho, float *sigma,
                      int nthreads);
int oracle_stress(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const float *xy, const int32_t *sources,
                  int64_t rows, double *row_sum, int64_t *row_pairs, int nthreads);
int oracle_neighborhood(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const float *xy, int32_t r,
                        const int32_t *verts, int64_t rows, double *score, int32_t *ball, int nthreads);
uint64_t oracle_splitmix64(uint64_t seed, uint64_t i);
int oracle_fuzzy_union(int32_t rows, int32_t k, const int32_t *ids, const float *w, int32_t *row_ptr, int32_t *col,
                       float *val, int64_t cap, int64_t *nnz);
int oracle_edge_shuffle(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *val, uint64_t seed,
                        int32_t *head, int32_t *tail, float *w);
int oracle_grad_sample(int32_t n, int64_t m, const int32_t *head, const int32_t *tail, const float *w, float *xy,
                       double alpha_ab, double beta, double gamma, double alpha0, int64_t s, int32_t neg, int32_t t,
                       uint64_t seed, int32_t it_begin, int32_t it_end, int32_t *visits);
int oracle_grad_sample_window(int32_t n, int64_t m, const int32_t *head, const int32_t *tail, const float *w,
                              float *xy, double alpha_ab, double beta, double gamma, double alpha0, int64_t s,
                              int32_t neg, int32_t t, uint64_t seed, int32_t it_begin, int32_t it_end,
                              int32_t *visits, int32_t parts);

static int failures = 0;

#define CHECK(cond, what)                                        \
    do {                                                         \
        if (!(cond)) {                                           \
            fprintf(stderr, "check failed: %s (%s)\n", what, #cond); \
            ++failures;                                          \
        }                                                        \
    } while (0)

typedef struct {
    int32_t n;
    int64_t nnz;
    int32_t *rp, *col;
} csr_t;

static csr_t make_csr(int32_t n, int64_t m, int32_t *edges)
{
    csr_t g;
    g.n = n;
    g.rp = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    g.col = (int32_t *)malloc((size_t)(2 * m > 0 ? 2 * m : 1) * sizeof(int32_t));
    g.nnz = gg_csr(n, m, edges, g.rp, g.col);
    gg_free(edges);
    return g;
}

/* the same edge set with every row reversed, each row's first entry
 * repeated and a self-loop appended */
static csr_t make_dirty(const csr_t *g)
{
    csr_t d;
    d.n = g->n;
    d.rp = (int32_t *)calloc((size_t)g->n + 1, sizeof(int32_t));
    d.col = (int32_t *)malloc((size_t)(g->nnz + 2 * (int64_t)g->n + 1) * sizeof(int32_t));
    int64_t o = 0;
    for (int32_t v = 0; v < g->n; ++v) {
        d.rp[v] = (int32_t)o;
        for (int32_t e = g->rp[v + 1] - 1; e >= g->rp[v]; --e) d.col[o++] = g->col[e];
        if (g->rp[v + 1] > g->rp[v]) d.col[o++] = g->col[g->rp[v]];
        d.col[o++] = v;
    }
    d.rp[g->n] = (int32_t)o;
    d.nnz = o;
    return d;
}

static void free_csr(csr_t *g)
{
    free(g->rp);
    free(g->col);
}

static void exercise(const csr_t *g, int32_t k, const char *name)
{
    const int32_t n = g->n;
    const int32_t srcs = n < 40 ? n : 40;
    int32_t *src = (int32_t *)malloc((size_t)(srcs > 0 ? srcs : 1) * sizeof(int32_t));
    for (int32_t i = 0; i < srcs; ++i) src[i] = (int32_t)(((int64_t)i * 7919) % (n > 0 ? n : 1));
    int32_t *ids = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * (size_t)k * sizeof(int32_t));
    uint8_t *hops = (uint8_t *)malloc((size_t)(n > 0 ? n : 1) * (size_t)k);
    int32_t *pids = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * (size_t)k * sizeof(int32_t));
    uint8_t *phops = (uint8_t *)malloc((size_t)(n > 0 ? n : 1) * (size_t)k);
    uint8_t *hm = (uint8_t *)malloc((size_t)(srcs > 0 ? srcs : 1) * (size_t)(n > 0 ? n : 1));
    int st = oracle_knn_build(n, g->rp, g->col, k, src, srcs, ids, hops, hm, 3);
    CHECK(st == 0 || st == -3, name);
    st = oracle_knn_partial(n, g->rp, g->col, k, src, srcs, pids, phops, 2);
    CHECK(st == 0, name);
    if (st == 0) CHECK(memcmp(phops, hops, (size_t)srcs * (size_t)k) == 0 || n > 255, name);
    st = oracle_knn_partial(n, g->rp, g->col, k, NULL, 0, ids, hops, 4);
    CHECK(st == 0, name);
    if (n > 0) {
        int32_t *dist = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        CHECK(oracle_bfs_dist(n, g->rp, g->col, n - 1, dist) == 0, name);
        free(dist);
    }
    float *w = (float *)malloc((size_t)(n > 0 ? n : 1) * (size_t)k * sizeof(float));
    float *rho = (float *)malloc((size_t)(n > 0 ? n : 1) * sizeof(float));
    float *sig = (float *)malloc((size_t)(n > 0 ? n : 1) * sizeof(float));
    CHECK(oracle_membership(n, k, hops, w, rho, sig, 3) == 0, name);
    float *xy = (float *)malloc((size_t)(n > 0 ? n : 1) * 2 * sizeof(float));
    double *u = (double *)malloc((size_t)(n > 0 ? n : 1) * 2 * sizeof(double));
    gg_uniform(gg_mix_seed(7, (uint64_t)n), 2 * (int64_t)n, u);
    for (int64_t i = 0; i < 2 * (int64_t)n; ++i) xy[i] = (float)(u[i] * 20.0 - 10.0);
    double *rs = (double *)malloc((size_t)(srcs > 0 ? srcs : 1) * sizeof(double));
    int64_t *rpairs = (int64_t *)malloc((size_t)(srcs > 0 ? srcs : 1) * sizeof(int64_t));
    CHECK(oracle_stress(n, g->rp, g->col, xy, src, srcs, rs, rpairs, 2) == 0, name);
    double *score = (double *)malloc((size_t)(srcs > 0 ? srcs : 1) * sizeof(double));
    int32_t *ball = (int32_t *)malloc((size_t)(srcs > 0 ? srcs : 1) * sizeof(int32_t));
    CHECK(oracle_neighborhood(n, g->rp, g->col, xy, 2, src, srcs, score, ball, 2) == 0, name);
    /* layout step on the partial kNN */
    const int64_t cap = 2 * (int64_t)n * k + 1;
    int32_t *urp = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t *ucol = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    float *uval = (float *)malloc((size_t)cap * sizeof(float));
    int64_t unnz = 0;
    CHECK(oracle_fuzzy_union(n, k, ids, w, urp, ucol, uval, cap, &unnz) == 0, name);
    if (unnz > 0) {
        int32_t *head = (int32_t *)malloc((size_t)unnz * sizeof(int32_t));
        int32_t *tail = (int32_t *)malloc((size_t)unnz * sizeof(int32_t));
        float *ew = (float *)malloc((size_t)unnz * sizeof(float));
        int32_t *vis = (int32_t *)calloc((size_t)unnz, sizeof(int32_t));
        CHECK(oracle_edge_shuffle(n, urp, ucol, uval, 99, head, tail, ew) == 0, name);
        const int64_t s = unnz > 3 ? unnz / 3 : 1;
        CHECK(oracle_grad_sample(n, unnz, head, tail, ew, xy, 1.577, 0.895, 1.0, 1.0, s, 3, 6, 5, 0, 6, vis) == 0,
              name);
        CHECK(oracle_grad_sample_window(n, unnz, head, tail, ew, xy, 1.577, 0.895, 1.0, 1.0, s, 3, 6, 5, 1, 4, vis,
                                        4) == 0, name);
        CHECK(oracle_grad_sample(n, unnz, head, tail, ew, xy, 1.577, 0.895, 1.0, 1.0, 1, 0, 2, 5, 1, 2, NULL) == 0,
              name);
        free(head);
        free(tail);
        free(ew);
        free(vis);
    }
    free(urp);
    free(ucol);
    free(uval);
    free(score);
    free(ball);
    free(rs);
    free(rpairs);
    free(u);
    free(xy);
    free(w);
    free(rho);
    free(sig);
    free(hm);
    free(src);
    free(ids);
    free(hops);
    free(pids);
    free(phops);
}

int main(void)
{
    int32_t *e = NULL;
    int64_t m;
    csr_t gs[6];
    const char *names[6] = {"ba", "er", "sbm", "rgg", "edgeless", "empty"};
    m = gg_ba(700, 3, gg_mix_seed(1, 1), &e);
    gs[0] = make_csr(700, m, e);
    m = gg_er(300, 0.05, gg_mix_seed(1, 2), &e);
    gs[1] = make_csr(300, m, e);
    m = gg_sbm(640, 8, 0.2, 0.01, gg_mix_seed(1, 3), &e);
    gs[2] = make_csr(640, m, e);
    m = gg_rgg(500, 0.08, gg_mix_seed(1, 4), &e);
    gs[3] = make_csr(500, m, e);
    m = gg_er(20, 0.0, gg_mix_seed(1, 5), &e);
    gs[4] = make_csr(20, m, e);
    m = gg_er(0, 0.5, gg_mix_seed(1, 6), &e);
    gs[5] = make_csr(0, m, e);
    const int32_t ks[3] = {1, 15, 40};
    for (int i = 0; i < 6; ++i) {
        for (int q = 0; q < 3; ++q) exercise(&gs[i], ks[q], names[i]);
        csr_t d = make_dirty(&gs[i]);
        exercise(&d, 15, names[i]);
        free_csr(&d);
    }
    CHECK(oracle_splitmix64(1234567, 1) == oracle_splitmix64(1234567, 1), "splitmix64");
    for (int i = 0; i < 6; ++i) free_csr(&gs[i]);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("sanitized oracle and generators: ok\n");
    return 0;
}
