// Spectral sparsification front end of SS-GUMAP and SSSL-GUMAP (Sec. 3.2,
// Alg. 2 and Alg. 6): effective resistances of the edges, then a maximum
// spanning forest with the resistances as weights and further edges in
// decreasing resistance until n ln n edges.
//
// Resistances are estimated by random projection (Spielman and Srivastava):
// with q sign vectors s_k over the edges, x_k solves L x_k = B^T s_k and
// R_e = (1/q) sum_k (x_k(u) - x_k(v))^2.  The q systems are solved together
// by conjugate gradients preconditioned with the degrees, the iterates held
// row-major (q values per vertex, so a vertex's row of the product is one
// coalesced segment); each column stops on its own residual test, as a
// separate solve would.  The right-hand sides are gathered per (vertex,
// column) from the signs of the vertex's edges, so no atomics are needed;
// every reduction runs in a fixed order, so a run is reproducible.
//
// The spanning forest is Boruvka's: each component takes its best edge in
// the order (resistance descending, edge index ascending), a total order,
// so the forest is unique (found per vertex by a wave over its row, then one
// atomic per vertex); components are hooked along the chosen edges and the
// labels compressed, until no component gains an edge.  The remaining
// edges are ranked by a stable radix sort on the resistance bits.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.h"

namespace gm {
namespace {

constexpr int kSsBlock = 256;
constexpr int kSsTile = 128;    // vertices per partial sum (a thread per tile and column)

__device__ __forceinline__ uint64_t ss_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int ss_grid(int64_t work)
{
    int64_t b = (work + kSsBlock - 1) / kSsBlock;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    return (int)b;
}

// ------------------------------------------------------------- edge ids --
// upper[u] = entries of row u with a larger column (the edges (u, v), u < v)
__global__ void ss_upper_count_kernel(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                      int32_t *__restrict__ upper)
{
    for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        // rows are sorted: the upper entries are a suffix, found by binary search
        int32_t lo = rp[u], hi = rp[u + 1];
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (col[mid] <= u) lo = mid + 1;
            else hi = mid;
        }
        upper[u] = rp[u + 1] - lo;
    }
}

// eid[j] for every entry j = (u, w): the index of edge (min, max) in CSR
// order of the upper entries; eu / ev list the edges.  A wave per row, the
// lanes striding over its entries (each lower entry searches row w for u).
__global__ void __launch_bounds__(kSsBlock)
ss_edge_ids_kernel(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                   const int32_t *__restrict__ eoff, int32_t *__restrict__ eid, int32_t *__restrict__ eu,
                   int32_t *__restrict__ ev)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t uu = wave; uu < n; uu += waves) {
        const int32_t u = (int32_t)uu;
        const int32_t e1 = rp[u + 1];
        const int32_t first_up = e1 - (eoff[u + 1] - eoff[u]);
        for (int32_t j = rp[u] + lane; j < e1; j += 64) {
            const int32_t w = col[j];
            if (w == u) {   // a self-loop is not an edge
                eid[j] = -1;
                continue;
            }
            if (j >= first_up) {
                const int32_t e = eoff[u] + (j - first_up);
                eid[j] = e;
                eu[e] = u;
                ev[e] = w;
            } else {
                // position of u in row w (sorted), among w's upper entries
                int32_t lo = rp[w], hi = rp[w + 1];
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (col[mid] < u) lo = mid + 1;
                    else hi = mid;
                }
                const int32_t wfirst = rp[w + 1] - (eoff[w + 1] - eoff[w]);
                // an entry without its mirror (asymmetric input) is not an edge
                eid[j] = (lo < rp[w + 1] && col[lo] == u && lo >= wfirst) ? eoff[w] + (lo - wfirst) : -1;
            }
        }
    }
}

// --------------------------------------------------------- projections --
// B[v][k] = sum over v's edges e of +s_k(e) (v the smaller end) or -s_k(e)
__global__ void __launch_bounds__(kSsBlock)
ss_rhs_kernel(int32_t n, int32_t q, int64_t m, uint64_t seed, const int32_t *__restrict__ rp,
              const int32_t *__restrict__ col, const int32_t *__restrict__ eid, double *__restrict__ B)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)n * q;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(t / q);
        const int32_t k = (int32_t)(t % q);
        double acc = 0.0;
        for (int32_t j = rp[v]; j < rp[v + 1]; ++j) {
            if (eid[j] < 0) continue;
            const uint64_t r = ss_splitmix64(seed, (uint64_t)k * (uint64_t)m + (uint64_t)eid[j] + 1);
            const double s = (r >> 63) ? -1.0 : 1.0;
            acc += col[j] > v ? s : -s;
        }
        B[t] = acc;
    }
}

// Y = L P (rows of q values), and per (tile, column) partial sums of P . Y
__global__ void __launch_bounds__(kSsBlock)
ss_lap_kernel(int32_t n, int32_t q, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
              const double *__restrict__ P, double *__restrict__ Y, const int *__restrict__ active)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)n * q;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(t / q);
        const int32_t k = (int32_t)(t % q);
        if (!active[k]) continue;
        const int32_t b = rp[v], e = rp[v + 1];
        double s = 0.0;
        for (int32_t j = b; j < e; ++j) s += P[(int64_t)col[j] * q + k];
        Y[t] = (double)(e - b) * P[t] - s;
    }
}

// part[(tile * q + k) * 3 + f] for the products f: 0 = a.b, 1 = c.d, 2 = c.c
// (the vertices of the tile, column k); a thread takes one column of a tile.
__global__ void __launch_bounds__(kSsBlock)
ss_dots_kernel(int32_t n, int32_t q, const double *__restrict__ A, const double *__restrict__ Bv,
               const double *__restrict__ C, const double *__restrict__ D, double *__restrict__ part, int tiles)
{
    const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= (int64_t)tiles * q) return;
    const int t = (int)(item / q), k = (int)(item % q);
    const int32_t v0 = t * kSsTile, v1 = min(n, v0 + kSsTile);
    double ab = 0.0, cd = 0.0, cc = 0.0;
    for (int32_t v = v0; v < v1; ++v) {
        const int64_t i = (int64_t)v * q + k;
        if (A) ab += A[i] * Bv[i];
        if (C) {
            cd += C[i] * D[i];
            cc += C[i] * C[i];
        }
    }
    part[item * 3] = ab;
    part[item * 3 + 1] = cd;
    part[item * 3 + 2] = cc;
}

// Column sums of the partials into sums[k * 3 + f]: a block per column, the
// threads striding over the tiles, then a tree (a fixed order throughout).
__global__ void __launch_bounds__(kSsBlock)
ss_reduce_kernel(int32_t q, int tiles, const double *__restrict__ part, double *__restrict__ sums)
{
    __shared__ double sh[3][kSsBlock];
    const int k = blockIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < tiles; t += blockDim.x)
        for (int f = 0; f < 3; ++f) acc[f] += part[((int64_t)t * q + k) * 3 + f];
    for (int f = 0; f < 3; ++f) sh[f][threadIdx.x] = acc[f];
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int f = 0; f < 3; ++f) sh[f][threadIdx.x] += sh[f][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int f = 0; f < 3; ++f) sums[k * 3 + f] = sh[f][0];
}

// CG state per column k: st[k * 8 + .] = {rz, |b|, alpha, iterations}.
// After L p: alpha = rz / (p . Ap).
__global__ void ss_alpha_kernel(int32_t q, const double *__restrict__ sums, double *__restrict__ st,
                                const int *__restrict__ active)
{
    for (int k = threadIdx.x; k < q; k += blockDim.x)
        if (active[k]) st[k * 8 + 2] = st[k * 8 + 0] / sums[k * 3 + 0];
}

// x += alpha p, r -= alpha Ap, z = r / deg
__global__ void __launch_bounds__(kSsBlock)
ss_update_kernel(int32_t n, int32_t q, const int32_t *__restrict__ rp, const double *__restrict__ st,
                 const int *__restrict__ active, double *__restrict__ X, double *__restrict__ R,
                 double *__restrict__ Z, const double *__restrict__ P, const double *__restrict__ AP)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)n * q;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(t / q);
        const int32_t k = (int32_t)(t % q);
        if (!active[k]) continue;
        const double a = st[k * 8 + 2];
        X[t] += a * P[t];
        R[t] -= a * AP[t];
        const int32_t d = rp[v + 1] - rp[v];
        Z[t] = d > 0 ? R[t] / (double)d : 0.0;
    }
}

// After the update: rz_new = r . z, |r| = sqrt(r . r); beta = rz_new / rz;
// a column whose |r| <= tol |b| (or which reached max_iters) stops.
__global__ void ss_beta_kernel(int32_t q, const double *__restrict__ sums, double *__restrict__ st,
                               int *__restrict__ active, double tol, int max_iters, int *__restrict__ n_active)
{
    for (int k = threadIdx.x; k < q; k += blockDim.x) {
        if (!active[k]) continue;
        const double rz_new = sums[k * 3 + 1], rr = sums[k * 3 + 2];
        st[k * 8 + 4] = rz_new / st[k * 8 + 0];   // beta
        st[k * 8 + 0] = rz_new;
        st[k * 8 + 3] += 1.0;
        if (!(sqrt(rr) > tol * st[k * 8 + 1]) || st[k * 8 + 3] >= (double)max_iters) active[k] = 2;
    }
}

// p = z + beta p for the columns still running; columns that just stopped
// (active = 2) become inactive.
__global__ void __launch_bounds__(kSsBlock)
ss_direction_kernel(int32_t n, int32_t q, const double *__restrict__ st, const int *__restrict__ active,
                    const double *__restrict__ Z, double *__restrict__ P)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)n * q;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = (int32_t)(t % q);
        if (active[k] != 1) continue;
        P[t] = Z[t] + st[k * 8 + 4] * P[t];
    }
}

__global__ void ss_settle_kernel(int32_t q, int *__restrict__ active, int *__restrict__ n_active)
{
    if (blockIdx.x != 0) return;
    for (int k = threadIdx.x; k < q; k += blockDim.x) {
        if (active[k] == 2) active[k] = 0;
        if (active[k] == 1) atomicAdd(n_active, 1);
    }
}

// Initial state: x = 0, r = b, z = r / deg, p = z
__global__ void __launch_bounds__(kSsBlock)
ss_init_kernel(int32_t n, int32_t q, const int32_t *__restrict__ rp, const double *__restrict__ B,
               double *__restrict__ X, double *__restrict__ R, double *__restrict__ Z, double *__restrict__ P)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)n * q;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(t / q);
        const int32_t d = rp[v + 1] - rp[v];
        X[t] = 0.0;
        R[t] = B[t];
        Z[t] = d > 0 ? B[t] / (double)d : 0.0;
        P[t] = Z[t];
    }
}

// st from the first dot products: rz = r . z, |b| = sqrt(b . b); a column
// with b = 0 (or already small) is inactive from the start.
__global__ void ss_start_kernel(int32_t q, const double *__restrict__ sums, double *__restrict__ st,
                                int *__restrict__ active, double tol)
{
    for (int k = threadIdx.x; k < q; k += blockDim.x) {
        st[k * 8 + 0] = sums[k * 3 + 1];
        st[k * 8 + 1] = sqrt(sums[k * 3 + 2]);
        st[k * 8 + 3] = 0.0;
        active[k] = sqrt(sums[k * 3 + 2]) > tol * st[k * 8 + 1] ? 1 : 0;
    }
}

// R_e = (1/q) sum_k (x_k(u) - x_k(v))^2
__global__ void __launch_bounds__(kSsBlock)
ss_resistance_kernel(int64_t m, int32_t q, const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
                     const double *__restrict__ X, double *__restrict__ Rout)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const double *a = X + (int64_t)eu[e] * q, *b = X + (int64_t)ev[e] * q;
        double s = 0.0;
        for (int k = 0; k < q; ++k) {
            const double d = a[k] - b[k];
            s += d * d;
        }
        Rout[e] = s / (double)q;
    }
}

// ------------------------------------------------------- spanning forest --
__global__ void ss_forest_init_kernel(int32_t n, int64_t m, int32_t *__restrict__ comp, uint8_t *__restrict__ keep)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n > m ? n : m);
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < n) comp[i] = (int32_t)i;
        if (i < m) keep[i] = 0;
    }
}

__global__ void ss_best_clear_kernel(int32_t n, unsigned long long *__restrict__ bestR, int32_t *__restrict__ bestE)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        bestR[i] = 0ull;
        bestE[i] = INT32_MAX;
    }
}

// Non-negative doubles order as their bit patterns; +1 keeps 0 above "none".
__device__ __forceinline__ unsigned long long r_key(double r) { return (unsigned long long)__double_as_longlong(r) + 1ull; }

// Each vertex's best edge to another component, a wave per vertex (the
// order: larger key first, then the smaller edge index); then one atomic
// per vertex on its component instead of one per edge end, since late
// rounds have few components and millions of edges between them.
__global__ void __launch_bounds__(kSsBlock)
ss_vertex_best_kernel(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                      const int32_t *__restrict__ eid, const int32_t *__restrict__ comp, const double *__restrict__ R,
                      unsigned long long *__restrict__ vkey, int32_t *__restrict__ ve,
                      unsigned long long *__restrict__ bestR)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t v = wave; v < n; v += waves) {
        const int32_t c = comp[v];
        unsigned long long key = 0ull;
        int32_t e = INT32_MAX;
        for (int32_t j = rp[v] + lane; j < rp[v + 1]; j += 64) {
            const int32_t x = eid[j];
            if (x < 0 || comp[col[j]] == c) continue;
            const unsigned long long k = r_key(R[x]);
            if (k > key || (k == key && x < e)) {
                key = k;
                e = x;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long k2 = __shfl_xor(key, o, 64);
            const int32_t e2 = __shfl_xor(e, o, 64);
            if (k2 > key || (k2 == key && e2 < e)) {
                key = k2;
                e = e2;
            }
        }
        if (lane == 0) {
            vkey[v] = key;
            ve[v] = e;
            if (key) atomicMax(&bestR[c], key);
        }
    }
}

__global__ void __launch_bounds__(kSsBlock)
ss_vertex_best_e_kernel(int32_t n, const int32_t *__restrict__ comp, const unsigned long long *__restrict__ vkey,
                        const int32_t *__restrict__ ve, const unsigned long long *__restrict__ bestR,
                        int32_t *__restrict__ bestE)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int32_t c = comp[v];
        if (vkey[v] && vkey[v] == bestR[c]) atomicMin(&bestE[c], ve[v]);
    }
}

// Each root c with a best edge e hooks onto the other end's component; when
// both ends chose the same edge the smaller root stays a root.  The edge is
// kept; added counts the edges of this round.
__global__ void ss_hook_kernel(int32_t n, const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
                               const int32_t *__restrict__ comp, const int32_t *__restrict__ bestE,
                               int32_t *__restrict__ parent, uint8_t *__restrict__ keep, int *__restrict__ added)
{
    for (int32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        if (comp[c] != c) continue;   // not a root
        const int32_t e = bestE[c];
        if (e == INT32_MAX) {
            parent[c] = c;
            continue;
        }
        const int32_t a = comp[eu[e]], b = comp[ev[e]];
        const int32_t other = a == c ? b : a;
        if (bestE[other] == e && c < other) {
            parent[c] = c;
        } else {
            parent[c] = other;
        }
        if (!(bestE[other] == e && c > other)) {   // count a mutual edge once
            keep[e] = 1;
            atomicAdd(added, 1);
        }
    }
}

// comp[v] = the root reached from comp[v] along parent (roots point to themselves)
__global__ void ss_compress_kernel(int32_t n, const int32_t *__restrict__ parent, int32_t *__restrict__ comp)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        int32_t r = comp[v];
        while (parent[r] != r) r = parent[r];
        comp[v] = r;
    }
}

// Roots keep parent[c] = c for the next round; others copy their new root.
__global__ void ss_parent_reset_kernel(int32_t n, const int32_t *__restrict__ comp, int32_t *__restrict__ parent)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) parent[v] = comp[v];
}

// ----------------------------------------------------------- top edges --
__global__ void __launch_bounds__(kSsBlock)
ss_rank_keys_kernel(int64_t m, const double *__restrict__ R, unsigned long long *__restrict__ keys,
                    int32_t *__restrict__ idx)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        keys[e] = ~(unsigned long long)__double_as_longlong(R[e]);   // ascending key = descending resistance
        idx[e] = (int32_t)e;
    }
}

// flags[i] = 1 if the i-th ranked edge is not in the forest
__global__ void __launch_bounds__(kSsBlock)
ss_rest_flags_kernel(int64_t m, const int32_t *__restrict__ order, const uint8_t *__restrict__ keep,
                     int32_t *__restrict__ flags)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        flags[i] = keep[order[i]] ? 0 : 1;
}

__global__ void __launch_bounds__(kSsBlock)
ss_take_kernel(int64_t m, const int32_t *__restrict__ order, const int32_t *__restrict__ flags,
               const int32_t *__restrict__ pos, int64_t need, uint8_t *__restrict__ keep)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        if (flags[i] && pos[i] < need) keep[order[i]] = 1;
}

// ----------------------------------------------------------- output CSR --
// A wave per row: kept entries counted, then written in row order (the
// lanes' ballot of kept entries gives each its place).
__global__ void __launch_bounds__(kSsBlock)
ss_out_count_kernel(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ eid,
                    const uint8_t *__restrict__ keep, int32_t *__restrict__ cnt)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t u = wave; u < n; u += waves) {
        int32_t c = 0;
        for (int32_t j = rp[u] + lane; j < rp[u + 1]; j += 64) c += eid[j] >= 0 ? keep[eid[j]] : 0;
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (lane == 0) cnt[u] = c;
    }
}

__global__ void __launch_bounds__(kSsBlock)
ss_out_fill_kernel(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                   const int32_t *__restrict__ eid, const uint8_t *__restrict__ keep,
                   const int32_t *__restrict__ out_rp, int32_t *__restrict__ out_col)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t u = wave; u < n; u += waves) {
        int32_t o = out_rp[u];
        const int32_t e1 = rp[u + 1];
        for (int32_t j0 = rp[u]; j0 < e1; j0 += 64) {
            const int32_t j = j0 + lane;
            const bool k = j < e1 && eid[j] >= 0 && keep[eid[j]];
            const uint64_t mask = __ballot(k);
            if (k) out_col[o + __popcll(mask & ((1ull << lane) - 1ull))] = col[j];
            o += __popcll(mask);
        }
    }
}

}  // namespace

// ---------------------------------------------------------- launchers --
int sparsify_tiles(int32_t n) { return (n + kSsTile - 1) / kSsTile; }

hipError_t launch_edge_ids(const SparsifyArgs &a, void *scan_tmp, hipStream_t s)
{
    hipLaunchKernelGGL(ss_upper_count_kernel, dim3(ss_grid(a.n)), dim3(kSsBlock), 0, s, a.n, a.row_ptr, a.col, a.upper);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_exclusive_scan(a.upper, a.eoff, a.n, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ss_edge_ids_kernel, dim3(ss_grid((int64_t)a.n * 64)), dim3(kSsBlock), 0, s, a.n, a.row_ptr,
                       a.col, a.eoff, a.eid, a.eu, a.ev);
    return hipGetLastError();
}

hipError_t launch_resistance_setup(const SparsifyArgs &a, int32_t q, uint64_t seed, double tol, hipStream_t s)
{
    const int64_t nq = (int64_t)a.n * q;
    const int tiles = sparsify_tiles(a.n);
    hipLaunchKernelGGL(ss_rhs_kernel, dim3(ss_grid(nq)), dim3(kSsBlock), 0, s, a.n, q, a.m, seed, a.row_ptr, a.col,
                       a.eid, a.B);
    hipLaunchKernelGGL(ss_init_kernel, dim3(ss_grid(nq)), dim3(kSsBlock), 0, s, a.n, q, a.row_ptr, a.B, a.X, a.Rv,
                       a.Z, a.P);
    // r . z and b . b (r = b at the start)
    hipLaunchKernelGGL(ss_dots_kernel, dim3(ss_grid((int64_t)tiles * q)), dim3(kSsBlock), 0, s, a.n, q,
                       (const double *)nullptr, (const double *)nullptr, a.Rv, a.Z, a.part, tiles);
    hipLaunchKernelGGL(ss_reduce_kernel, dim3(q), dim3(kSsBlock), 0, s, q, tiles, a.part, a.sums);
    hipLaunchKernelGGL(ss_start_kernel, dim3(1), dim3(64), 0, s, q, a.sums, a.st, a.active, tol);
    return hipGetLastError();
}

hipError_t launch_cg_iteration(const SparsifyArgs &a, int32_t q, double tol, int max_iters, hipStream_t s)
{
    const int64_t nq = (int64_t)a.n * q;
    const int tiles = sparsify_tiles(a.n);
    hipLaunchKernelGGL(ss_lap_kernel, dim3(ss_grid(nq)), dim3(kSsBlock), 0, s, a.n, q, a.row_ptr, a.col, a.P, a.AP,
                       a.active);
    hipLaunchKernelGGL(ss_dots_kernel, dim3(ss_grid((int64_t)tiles * q)), dim3(kSsBlock), 0, s, a.n, q, a.P, a.AP,
                       (const double *)nullptr, (const double *)nullptr, a.part, tiles);
    hipLaunchKernelGGL(ss_reduce_kernel, dim3(q), dim3(kSsBlock), 0, s, q, tiles, a.part, a.sums);
    hipLaunchKernelGGL(ss_alpha_kernel, dim3(1), dim3(64), 0, s, q, a.sums, a.st, a.active);
    hipLaunchKernelGGL(ss_update_kernel, dim3(ss_grid(nq)), dim3(kSsBlock), 0, s, a.n, q, a.row_ptr, a.st, a.active,
                       a.X, a.Rv, a.Z, a.P, a.AP);
    hipLaunchKernelGGL(ss_dots_kernel, dim3(ss_grid((int64_t)tiles * q)), dim3(kSsBlock), 0, s, a.n, q,
                       (const double *)nullptr, (const double *)nullptr, a.Rv, a.Z, a.part, tiles);
    hipLaunchKernelGGL(ss_reduce_kernel, dim3(q), dim3(kSsBlock), 0, s, q, tiles, a.part, a.sums);
    hipLaunchKernelGGL(ss_beta_kernel, dim3(1), dim3(64), 0, s, q, a.sums, a.st, a.active, tol, max_iters,
                       a.n_active);
    hipLaunchKernelGGL(ss_direction_kernel, dim3(ss_grid(nq)), dim3(kSsBlock), 0, s, a.n, q, a.st, a.active, a.Z,
                       a.P);
    hipError_t e = hipMemsetAsync(a.n_active, 0, sizeof(int), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ss_settle_kernel, dim3(1), dim3(64), 0, s, q, a.active, a.n_active);
    return hipGetLastError();
}

hipError_t launch_resistance_out(const SparsifyArgs &a, int32_t q, double *R, hipStream_t s)
{
    hipLaunchKernelGGL(ss_resistance_kernel, dim3(ss_grid(a.m)), dim3(kSsBlock), 0, s, a.m, q, a.eu, a.ev, a.X, R);
    return hipGetLastError();
}

hipError_t launch_forest_init(const SparsifyArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(ss_forest_init_kernel, dim3(ss_grid(a.n > a.m ? a.n : a.m)), dim3(kSsBlock), 0, s, a.n, a.m,
                       a.comp, a.keep);
    hipLaunchKernelGGL(ss_parent_reset_kernel, dim3(ss_grid(a.n)), dim3(kSsBlock), 0, s, a.n, a.comp, a.parent);
    return hipGetLastError();
}

hipError_t launch_forest_round(const SparsifyArgs &a, const double *R, int *added, hipStream_t s)
{
    hipLaunchKernelGGL(ss_best_clear_kernel, dim3(ss_grid(a.n)), dim3(kSsBlock), 0, s, a.n, a.bestR, a.bestE);
    hipLaunchKernelGGL(ss_vertex_best_kernel, dim3(ss_grid((int64_t)a.n * 64)), dim3(kSsBlock), 0, s, a.n,
                       a.row_ptr, a.col, a.eid, a.comp, R, a.vkey, a.ve, a.bestR);
    hipLaunchKernelGGL(ss_vertex_best_e_kernel, dim3(ss_grid(a.n)), dim3(kSsBlock), 0, s, a.n, a.comp, a.vkey, a.ve,
                       a.bestR, a.bestE);
    hipLaunchKernelGGL(ss_hook_kernel, dim3(ss_grid(a.n)), dim3(kSsBlock), 0, s, a.n, a.eu, a.ev, a.comp, a.bestE,
                       a.parent, a.keep, added);
    hipLaunchKernelGGL(ss_compress_kernel, dim3(ss_grid(a.n)), dim3(kSsBlock), 0, s, a.n, a.parent, a.comp);
    hipLaunchKernelGGL(ss_parent_reset_kernel, dim3(ss_grid(a.n)), dim3(kSsBlock), 0, s, a.n, a.comp, a.parent);
    return hipGetLastError();
}

size_t rank_scratch_bytes(int64_t m, size_t *sort_tmp)
{
    size_t tmp = (radix_sort_scratch_bytes(m) + 255) & ~(size_t)255;
    *sort_tmp = tmp;
    const size_t t = (size_t)(m > 0 ? m : 1);
    return tmp + 2 * t * sizeof(unsigned long long) + 4 * t * sizeof(int32_t) + exclusive_scan_scratch_bytes(m) + 4096;
}

hipError_t launch_take_top(const SparsifyArgs &a, const double *R, int64_t need, void *scratch, hipStream_t s)
{
    if (need <= 0 || a.m == 0) return hipSuccess;
    size_t tmp = 0;
    (void)rank_scratch_bytes(a.m, &tmp);
    const size_t t = (size_t)a.m;
    char *p = (char *)scratch;
    unsigned long long *k0 = (unsigned long long *)(p + tmp), *k1 = k0 + t;
    int32_t *o0 = (int32_t *)(k1 + t), *o1 = o0 + t, *flags = o1 + t, *pos = flags + t;
    void *scan_tmp = (void *)(((uintptr_t)(pos + t + 1) + 255) & ~(uintptr_t)255);
    hipLaunchKernelGGL(ss_rank_keys_kernel, dim3(ss_grid(a.m)), dim3(kSsBlock), 0, s, a.m, R, k0, o0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    bool alt = false;   // stable: ties keep index order
    e = radix_sort_pairs<unsigned long long>(k0, k1, (uint32_t *)o0, (uint32_t *)o1, a.m, 0, 64, p, s, &alt);
    if (e != hipSuccess) return e;
    const int32_t *order = alt ? o1 : o0;
    hipLaunchKernelGGL(ss_rest_flags_kernel, dim3(ss_grid(a.m)), dim3(kSsBlock), 0, s, a.m, order, a.keep, flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = launch_exclusive_scan(flags, pos, a.m, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ss_take_kernel, dim3(ss_grid(a.m)), dim3(kSsBlock), 0, s, a.m, order, flags, pos, need,
                       a.keep);
    return hipGetLastError();
}

hipError_t launch_sparsified_csr(const SparsifyArgs &a, int32_t *out_rp, int32_t *out_col, void *scan_tmp,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(ss_out_count_kernel, dim3(ss_grid((int64_t)a.n * 64)), dim3(kSsBlock), 0, s, a.n, a.row_ptr,
                       a.eid, a.keep, a.upper);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_exclusive_scan(a.upper, out_rp, a.n, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ss_out_fill_kernel, dim3(ss_grid((int64_t)a.n * 64)), dim3(kSsBlock), 0, s, a.n, a.row_ptr,
                       a.col, a.eid, a.keep, (const int32_t *)out_rp, out_col);
    return hipGetLastError();
}

}  // namespace gm
