/*
 * Seeded synthetic graph generators (input side only).
 *
 * These produce undirected, unweighted graphs shaped like the workloads the
 * paper evaluates on (its dataset table: scale-free, mesh-like and locally
 * dense graphs), plus the dense random graph its complexity discussion flags
 * as the costly case.  They hold none of the kNN method's arithmetic: no
 * traversal, no distance, no selection.  Both the CPU oracle's tests and the
 * GPU path's tests read the CSR arrays that come out of here.
 *
 * Random numbers: xoshiro256** seeded through splitmix64 (both published
 * generators by Blackman and Vigna).  Every generator takes a 64-bit seed and
 * is deterministic for a given seed.
 *
 * Memory: generators that produce a random number of edges allocate the edge
 * list themselves and hand it back; the caller releases it with gg_free().
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- RNG --- */

static uint64_t splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static void rng_seed(rng_t *r, uint64_t seed)
{
    uint64_t sm = seed;
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64_next(&sm);
}

static uint64_t rng_next(rng_t *r)
{
    uint64_t *s = r->s;
    const uint64_t result = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}

/* uniform double in [0, 1) with 53 random bits */
static double rng_unif(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* uniform integer in [0, bound) without modulo bias (rejection) */
static uint64_t rng_below(rng_t *r, uint64_t bound)
{
    uint64_t threshold = (0 - bound) % bound;
    for (;;) {
        uint64_t x = rng_next(r);
        if (x >= threshold) return x % bound;
    }
}

/* Derive the seed of item `index` of a family seeded with `base`. */
uint64_t gg_mix_seed(uint64_t base, uint64_t index)
{
    uint64_t s = base ^ (0xD1B54A32D192ED03ULL * (index + 1));
    return splitmix64_next(&s);
}

double gg_uniform(uint64_t seed, int64_t count, double *out)
{
    rng_t r;
    rng_seed(&r, seed);
    for (int64_t i = 0; i < count; ++i) out[i] = rng_unif(&r);
    return count > 0 ? out[0] : 0.0;
}

void gg_free(void *p) { free(p); }

/* ------------------------------------------------------- edge buffers --- */

typedef struct {
    int32_t *e;    /* pairs (u, v) */
    int64_t m;     /* pairs stored */
    int64_t cap;   /* pairs allocated */
    int failed;
} edgebuf;

static void eb_push(edgebuf *b, int32_t u, int32_t v)
{
    if (b->failed) return;
    if (b->m == b->cap) {
        int64_t nc = b->cap ? b->cap * 2 : 1024;
        int32_t *ne = (int32_t *)realloc(b->e, (size_t)nc * 2 * sizeof(int32_t));
        if (!ne) { b->failed = 1; return; }
        b->e = ne;
        b->cap = nc;
    }
    b->e[2 * b->m] = u;
    b->e[2 * b->m + 1] = v;
    b->m++;
}

static int64_t eb_finish(edgebuf *b, int32_t **out)
{
    if (b->failed) { free(b->e); *out = NULL; return -1; }
    *out = b->e;
    return b->m;
}

/* ------------------------------------------------------------ models ---- */

/*
 * Barabasi-Albert preferential attachment.  Starts from a clique on
 * m_attach + 1 vertices; every later vertex attaches to m_attach distinct
 * earlier vertices drawn with probability proportional to their degree
 * (uniform draw from the list of edge endpoints, redrawn on repeats).
 */
int64_t gg_ba(int32_t n, int32_t m_attach, uint64_t seed, int32_t **edges)
{
    *edges = NULL;
    if (n <= 0 || m_attach < 1) return 0;
    int32_t m0 = m_attach + 1;
    if (m0 > n) m0 = n;
    int64_t total = (int64_t)m0 * (m0 - 1) / 2 + (int64_t)(n - m0) * m_attach;
    int32_t *e = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * 2 * sizeof(int32_t));
    int32_t *ends = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * 2 * sizeof(int32_t));
    int32_t *chosen = (int32_t *)malloc((size_t)m_attach * sizeof(int32_t));
    if (!e || !ends || !chosen) { free(e); free(ends); free(chosen); return -1; }
    rng_t r;
    rng_seed(&r, seed);
    int64_t m = 0, ne = 0;
    for (int32_t u = 0; u < m0; ++u)
        for (int32_t v = u + 1; v < m0; ++v) {
            e[2 * m] = u; e[2 * m + 1] = v; ++m;
            ends[ne++] = u; ends[ne++] = v;
        }
    for (int32_t v = m0; v < n; ++v) {
        int32_t got = 0;
        while (got < m_attach) {
            int32_t t = ends[rng_below(&r, (uint64_t)ne)];
            int dup = 0;
            for (int32_t i = 0; i < got; ++i) dup |= (chosen[i] == t);
            if (!dup) chosen[got++] = t;
        }
        for (int32_t i = 0; i < m_attach; ++i) {
            e[2 * m] = chosen[i]; e[2 * m + 1] = v; ++m;
            ends[ne++] = chosen[i]; ends[ne++] = v;
        }
    }
    free(ends);
    free(chosen);
    *edges = e;
    return m;
}

/*
 * Walk the pairs of a rectangular or triangular block in a fixed order and
 * keep each with probability p, jumping over runs of rejected pairs with a
 * geometric draw (Batagelj and Brandes, 2005).
 *   triangular: pairs (a0+i, a0+j) with 0 <= j < i < na
 *   rectangular: pairs (a0+i, b0+j) with 0 <= i < na, 0 <= j < nb
 */
static void skip_sample(edgebuf *b, rng_t *r, double p, int32_t a0, int32_t na,
                        int32_t b0, int32_t nb, int triangular)
{
    if (p <= 0.0 || na <= 0 || (!triangular && nb <= 0)) return;
    if (p >= 1.0) {
        for (int32_t i = 0; i < na; ++i) {
            int32_t lim = triangular ? i : nb;
            for (int32_t j = 0; j < lim; ++j)
                eb_push(b, triangular ? a0 + j : a0 + i, triangular ? a0 + i : b0 + j);
        }
        return;
    }
    double lq = log(1.0 - p);
    int64_t total = triangular ? (int64_t)na * (na - 1) / 2 : (int64_t)na * nb;
    int64_t pos = -1;
    for (;;) {
        double u = rng_unif(r);
        int64_t skip = (int64_t)floor(log(1.0 - u) / lq);
        pos += 1 + skip;
        if (pos >= total || pos < 0) break;
        int32_t i, j;
        if (triangular) {
            /* row i holds pairs i*(i-1)/2 .. i*(i+1)/2 - 1 */
            double di = floor((1.0 + sqrt(1.0 + 8.0 * (double)pos)) / 2.0);
            int64_t ii = (int64_t)di;
            while (ii * (ii - 1) / 2 > pos) --ii;
            while ((ii + 1) * ii / 2 <= pos) ++ii;
            i = (int32_t)ii;
            j = (int32_t)(pos - ii * (ii - 1) / 2);
            eb_push(b, a0 + j, a0 + i);
        } else {
            i = (int32_t)(pos / nb);
            j = (int32_t)(pos % nb);
            eb_push(b, a0 + i, b0 + j);
        }
    }
}

/* Erdos-Renyi G(n, p). */
int64_t gg_er(int32_t n, double p, uint64_t seed, int32_t **edges)
{
    edgebuf b = {0};
    rng_t r;
    rng_seed(&r, seed);
    skip_sample(&b, &r, p, 0, n, 0, 0, 1);
    return eb_finish(&b, edges);
}

/*
 * Stochastic block model: `blocks` near-equal consecutive id blocks, edge
 * probability p_in inside a block and p_out across blocks.
 */
int64_t gg_sbm(int32_t n, int32_t blocks, double p_in, double p_out, uint64_t seed, int32_t **edges)
{
    edgebuf b = {0};
    rng_t r;
    rng_seed(&r, seed);
    if (blocks < 1) blocks = 1;
    for (int32_t a = 0; a < blocks; ++a) {
        int32_t a0 = (int32_t)((int64_t)n * a / blocks), a1 = (int32_t)((int64_t)n * (a + 1) / blocks);
        skip_sample(&b, &r, p_in, a0, a1 - a0, 0, 0, 1);
        for (int32_t c = a + 1; c < blocks; ++c) {
            int32_t c0 = (int32_t)((int64_t)n * c / blocks), c1 = (int32_t)((int64_t)n * (c + 1) / blocks);
            skip_sample(&b, &r, p_out, a0, a1 - a0, c0, c1 - c0, 0);
        }
    }
    return eb_finish(&b, edges);
}

/*
 * 2-D random geometric graph: n points uniform in the unit square, an edge
 * between every pair at Euclidean distance <= radius.  Cell lists of side
 * >= radius keep it near-linear.
 */
int64_t gg_rgg(int32_t n, double radius, uint64_t seed, int32_t **edges)
{
    edgebuf b = {0};
    *edges = NULL;
    if (n <= 0) return 0;
    rng_t r;
    rng_seed(&r, seed);
    double *x = (double *)malloc((size_t)n * sizeof(double));
    double *y = (double *)malloc((size_t)n * sizeof(double));
    int32_t nc = radius > 0 ? (int32_t)floor(1.0 / radius) : 1;
    if (nc < 1) nc = 1;
    if (nc > 4096) nc = 4096;
    int32_t *head = (int32_t *)malloc((size_t)nc * nc * sizeof(int32_t));
    int32_t *nxt = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!x || !y || !head || !nxt) { free(x); free(y); free(head); free(nxt); return -1; }
    for (int32_t i = 0; i < n; ++i) { x[i] = rng_unif(&r); y[i] = rng_unif(&r); }
    for (int64_t c = 0; c < (int64_t)nc * nc; ++c) head[c] = -1;
    /* insert in decreasing id so every cell list runs in increasing id */
    for (int32_t i = n - 1; i >= 0; --i) {
        int32_t cx = (int32_t)(x[i] * nc), cy = (int32_t)(y[i] * nc);
        if (cx >= nc) cx = nc - 1;
        if (cy >= nc) cy = nc - 1;
        nxt[i] = head[cy * nc + cx];
        head[cy * nc + cx] = i;
    }
    double r2 = radius * radius;
    for (int32_t i = 0; i < n; ++i) {
        int32_t cx = (int32_t)(x[i] * nc), cy = (int32_t)(y[i] * nc);
        if (cx >= nc) cx = nc - 1;
        if (cy >= nc) cy = nc - 1;
        for (int32_t dy = -1; dy <= 1; ++dy)
            for (int32_t dx = -1; dx <= 1; ++dx) {
                int32_t ax = cx + dx, ay = cy + dy;
                if (ax < 0 || ay < 0 || ax >= nc || ay >= nc) continue;
                for (int32_t j = head[ay * nc + ax]; j >= 0; j = nxt[j]) {
                    if (j <= i) continue;
                    double ddx = x[i] - x[j], ddy = y[i] - y[j];
                    if (ddx * ddx + ddy * ddy <= r2) eb_push(&b, i, j);
                }
            }
    }
    free(x); free(y); free(head); free(nxt);
    return eb_finish(&b, edges);
}

/* ------------------------------------------------------------- CSR ------ */

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Undirected edge list -> canonical CSR: both directions stored, self-loops
 * dropped, every row sorted ascending with duplicates removed.
 * row_ptr has n+1 entries; col_idx must hold 2*m entries.  Returns nnz.
 */
int64_t gg_csr(int32_t n, int64_t m, const int32_t *edges, int32_t *row_ptr, int32_t *col_idx)
{
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *pos = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!deg || !pos) { free(deg); free(pos); return -1; }
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u == v || u < 0 || v < 0 || u >= n || v >= n) continue;
        deg[u]++; deg[v]++;
    }
    pos[0] = 0;
    for (int32_t v = 0; v < n; ++v) pos[v + 1] = pos[v] + deg[v];
    int64_t *fill = deg; /* reuse */
    for (int32_t v = 0; v < n; ++v) fill[v] = pos[v];
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u == v || u < 0 || v < 0 || u >= n || v >= n) continue;
        col_idx[fill[u]++] = v;
        col_idx[fill[v]++] = u;
    }
    int64_t out = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t a = pos[v], b = pos[v + 1];
        qsort(col_idx + a, (size_t)(b - a), sizeof(int32_t), cmp_i32);
        row_ptr[v] = (int32_t)out;
        for (int64_t i = a; i < b; ++i)
            if (i == a || col_idx[i] != col_idx[i - 1]) col_idx[out++] = col_idx[i];
    }
    row_ptr[n] = (int32_t)out;
    free(deg);
    free(pos);
    return out;
}
