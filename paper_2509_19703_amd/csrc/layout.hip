// Layout step C2 of SL-GUMAP on the kNN graph (Sec. 2.1 cost C, Sec. 3.3
// Alg. 3 and Alg. 5 GradSample): the fuzzy union that makes the membership
// graph symmetric, the keyed shuffle of its edge array E_k and the
// sliding-window gradient iterations.
//
// Union and shuffle are sorts (the stable radix sort of radix_sort.hip):
// every directed kNN cell emits at most two (row, col) keys with their union
// weight, one radix sort orders them and a segment pass writes the CSR; the
// shuffle sorts the entries by a SplitMix64 key of their position.  GradSample first sorts the 2m
// incidences (each array entry at its head and at its tail) by vertex.  A
// window is then two launches: a thread per window entry computes the
// entry's moves from the positions at the start of the window (its own steps
// in Alg. 5's order: attraction, then the negative samples from the moved
// head) and stores them at the entry's array position; a thread per vertex (a wave for a
// vertex with many incidences) adds up the stored moves of its incidences
// that lie in the window and writes its next position once.  Positions are
// fixed point (int64, 2^-32 units) and moves are summed as integers, so the
// result does not depend on the order of the sum, and no atomics are needed
// (device-wide 64-bit atomics on one address serialise, and a high-degree
// vertex receives thousands of moves per window).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.h"

namespace gm {
namespace {

constexpr int kLayoutBlock = 256;
constexpr double kFix = 4294967296.0;         // 2^32
constexpr double kFixInv = 1.0 / 4294967296.0;

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double clip4(double v) { return v > 4.0 ? 4.0 : (v < -4.0 ? -4.0 : v); }

// ------------------------------------------------------------ fuzzy union --
// Cell e = i * k + q of the kNN (j = ids[e], a = weights[e]).  With b the
// weight of i in row j (0 if absent), u = (a + b) - a * b; the cell emits
// (i, j, u) when u > 0 and, when i is absent from row j, also (j, i, u).
// Unused key slots hold the sentinel rows << 32, which sorts after every
// real key.
__global__ void __launch_bounds__(kLayoutBlock)
union_emit_kernel(int32_t rows, int32_t k, const int32_t *__restrict__ ids, const float *__restrict__ w,
                  uint64_t *__restrict__ keys, float *__restrict__ vals, int *__restrict__ err)
{
#pragma clang fp contract(off)
    const int64_t cells = (int64_t)rows * k;
    const uint64_t sent = (uint64_t)rows << 32;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cells;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = (int32_t)(e / k);
        const int32_t j = ids[e];
        uint64_t k0 = sent, k1 = sent;
        float u0 = 0.0f;
        if (j >= 0) {
            if (j >= rows || j == i) {
                atomicOr(err, 1);
            } else {
                const double a = (double)w[e];
                // find i in row j, eight independent loads per round
                const int32_t *rj = ids + (int64_t)j * k;
                int32_t at = -1;
                for (int32_t q0 = 0; q0 < k && at < 0; q0 += 8) {
                    int32_t c[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) c[u] = q0 + u < k ? rj[q0 + u] : -1;
#pragma unroll
                    for (int u = 7; u >= 0; --u)
                        if (c[u] == i) at = q0 + u;
                }
                const bool found = at >= 0;
                const double b = found ? (double)w[(int64_t)j * k + at] : 0.0;
                const double s = a + b;
                const double p = a * b;
                const double u = s - p;
                if (u > 0.0) {
                    u0 = (float)u;
                    k0 = ((uint64_t)i << 32) | (uint32_t)j;
                    if (!found) k1 = ((uint64_t)j << 32) | (uint32_t)i;
                }
            }
        }
        keys[2 * e] = k0;
        keys[2 * e + 1] = k1;
        vals[2 * e] = u0;
        vals[2 * e + 1] = u0;
    }
}

// Sorted keys -> CSR.  Position e holds a real entry iff its row is below
// `rows`; the last real position publishes the count.  Each entry writes the
// row pointers of the rows between its predecessor's row and its own.
__global__ void __launch_bounds__(kLayoutBlock)
union_rows_kernel(int32_t rows, int64_t total, const uint64_t *__restrict__ keys, const float *__restrict__ vals,
                  int32_t *__restrict__ row_ptr, int32_t *__restrict__ col, float *__restrict__ val, int64_t cap,
                  int64_t *__restrict__ nnz)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[e];
        const int32_t r = (int32_t)(key >> 32);
        if (r >= rows) continue;
        if (e < cap) {
            col[e] = (int32_t)(uint32_t)key;
            val[e] = vals[e];
        }
        const int32_t prev = e == 0 ? -1 : (int32_t)(keys[e - 1] >> 32);
        for (int32_t x = prev + 1; x <= r; ++x) row_ptr[x] = (int32_t)e;
        const bool last = e + 1 == total || (int32_t)(keys[e + 1] >> 32) >= rows;
        if (last) {
            for (int32_t x = r + 1; x <= rows; ++x) row_ptr[x] = (int32_t)(e + 1);
            *nnz = e + 1;
        }
    }
}

// ----------------------------------------------------------- edge shuffle --
__global__ void __launch_bounds__(kLayoutBlock)
shuffle_keys_kernel(int64_t m, uint64_t seed, uint64_t *__restrict__ keys, int32_t *__restrict__ pos)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        keys[e] = splitmix64(seed, (uint64_t)e + 1);
        pos[e] = (int32_t)e;
    }
}

// Entry e's row: the last i with row_ptr[i] <= e (binary search).
__global__ void __launch_bounds__(kLayoutBlock)
shuffle_gather_kernel(int32_t n, int64_t m, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                      const float *__restrict__ val, const int32_t *__restrict__ order, int32_t *__restrict__ head,
                      int32_t *__restrict__ tail, float *__restrict__ w)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = order[p];
        int32_t lo = 0, hi = n;        // row_ptr[lo] <= e < row_ptr[hi]
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (row_ptr[mid] <= e) lo = mid;
            else hi = mid;
        }
        head[p] = lo;
        tail[p] = col[e];
        w[p] = val[e];
    }
}

// ------------------------------------------------------------- GradSample --
__global__ void __launch_bounds__(kLayoutBlock)
edge_check_kernel(int32_t n, int64_t m, const int32_t *__restrict__ head, const int32_t *__restrict__ tail,
                  int *__restrict__ err)
{
    int bad = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = head[e], b = tail[e];
        bad |= (a < 0 || a >= n || b < 0 || b >= n) ? 1 : 0;
    }
    if (bad) atomicOr(err, 1);
}

__global__ void __launch_bounds__(kLayoutBlock)
fix_init_kernel(int32_t n, const float *__restrict__ xy, long long *__restrict__ p0, long long *__restrict__ p1,
                int *__restrict__ err)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * (int64_t)n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double x = (double)xy[i];
        if (!(fabs(x) < kLayoutCoordLimit)) {
            atomicOr(err, 2);
            p0[i] = 0;
        } else {
            p0[i] = llrint(x * kFix);
        }
        p1[i] = 0;
    }
}

__global__ void __launch_bounds__(kLayoutBlock)
fix_out_kernel(int32_t n, const long long *__restrict__ p, float *__restrict__ xy)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * (int64_t)n;
         i += (int64_t)gridDim.x * blockDim.x)
        xy[i] = (float)((double)p[i] * kFixInv);
}

// ------------------------------------------------- incidence lists --
// Every array position p contributes two incidences: at head[p] (role 0)
// and at tail[p] (role 1).  Sorted by vertex, code[i] = p << 1 | role and
// off[v] .. off[v + 1] delimit vertex v's codes.
__global__ void __launch_bounds__(kLayoutBlock)
incidence_keys_kernel(int64_t m, const int32_t *__restrict__ head, const int32_t *__restrict__ tail,
                      uint32_t *__restrict__ keys, uint32_t *__restrict__ codes)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = i >> 1;
        keys[i] = (uint32_t)((i & 1) ? tail[p] : head[p]);
        codes[i] = (uint32_t)i;
    }
}

__global__ void __launch_bounds__(kLayoutBlock)
incidence_rows_kernel(int32_t n, int64_t total, const uint32_t *__restrict__ keys, int32_t *__restrict__ off)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)keys[i];
        const int32_t prev = i == 0 ? -1 : (int32_t)keys[i - 1];
        for (int32_t x = prev + 1; x <= v; ++x) off[x] = (int32_t)i;
        if (i + 1 == total)
            for (int32_t x = v + 1; x <= n; ++x) off[x] = (int32_t)total;
    }
}

__global__ void __launch_bounds__(kLayoutBlock)
incidence_heavy_kernel(int32_t n, const int32_t *__restrict__ off, int32_t *__restrict__ heavy,
                       int32_t *__restrict__ n_heavy)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (off[v + 1] - off[v] > kLayoutHeavyInc) heavy[atomicAdd(n_heavy, 1)] = v;
}

// ---------------------------------------------------------- one window --
__device__ __forceinline__ void attract(const LayoutArgs &g, double lh, double dx, double dy, long long &qx,
                                        long long &qy)
{
#pragma clang fp contract(off)
    const double sx = dx * dx, sy = dy * dy;
    const double d2 = sx + sy;
    qx = 0;
    qy = 0;
    if (d2 > 0.0) {
        const double T = pow(d2, g.beta);
        const double num = g.att_num * T;
        const double den = d2 * (1.0 + g.alpha * T);
        const double c = num / den;
        qx = llrint(lh * clip4(c * dx) * kFix);
        qy = llrint(lh * clip4(c * dy) * kFix);
    }
}

__device__ __forceinline__ void repel(const LayoutArgs &g, double lh, double ex, double ey, long long &hx,
                                      long long &hy)
{
#pragma clang fp contract(off)
    const double tx = ex * ex, ty = ey * ey;
    const double e2 = tx + ty;
    double gx = 4.0, gy = 4.0;
    if (e2 > 0.0) {
        const double T = pow(e2, g.beta);
        const double den = (0.001 + e2) * (1.0 + g.alpha * T);
        const double c = g.rep_num / den;
        gx = clip4(c * ex);
        gy = clip4(c * ey);
    }
    hx += llrint(lh * gx * kFix);
    hy += llrint(lh * gy * kFix);
}

__device__ __forceinline__ double fix_to_f64(long long v) { return (double)v * kFixInv; }

// Phase 1, a thread per window entry (a, b, h) at position p: the entry's
// steps in Alg. 5's order on its own copy of its vertices, starting from the
// positions at the start of the window -- the attraction moves a and b, then
// each negative sample reads a as moved so far (and b as moved when the
// sample is b).  Every move is rounded to the fixed-point grid.  Stored at
// mv[p] = {head x, head y, att x, att y}: the head's total move and the
// attraction (the tail receives -att).  The positions of up to kNegBatch
// negative samples are loaded before any of them is used.
constexpr int kNegBatch = 8;

__global__ void __launch_bounds__(kLayoutBlock)
grad_moves_kernel(LayoutArgs g, int64_t j0, int64_t l0, int64_t l1, int32_t it, double lr,
                  const longlong2 *__restrict__ R, longlong2 *__restrict__ mv)
{
#pragma clang fp contract(off)
    for (int64_t l = l0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < l1; l += (int64_t)gridDim.x * blockDim.x) {
        int64_t p = j0 + l;
        if (p >= g.m) p -= g.m;
        const int32_t a = g.head[p], b = g.tail[p];
        const double lh = lr * (double)g.w[p];
        const longlong2 ra = R[a], rb = R[b];
        long long qx, qy;
        attract(g, lh, fix_to_f64(ra.x) - fix_to_f64(rb.x), fix_to_f64(ra.y) - fix_to_f64(rb.y), qx, qy);
        long long hx = qx, hy = qy;
        const longlong2 pb = make_longlong2(rb.x - qx, rb.y - qy);
        const uint64_t base = ((uint64_t)it * (uint64_t)g.s + (uint64_t)l) * (uint64_t)g.neg;
        for (int32_t q0 = 0; q0 < g.neg; q0 += kNegBatch) {
            int32_t vq[kNegBatch];
            longlong2 rq[kNegBatch];
#pragma unroll
            for (int u = 0; u < kNegBatch; ++u)
                vq[u] = q0 + u < g.neg ? (int32_t)(splitmix64(g.seed, base + (uint64_t)(q0 + u) + 1) % (uint64_t)g.n)
                                       : a;
#pragma unroll
            for (int u = 0; u < kNegBatch; ++u) rq[u] = (vq[u] != a && vq[u] != b) ? R[vq[u]] : pb;
#pragma unroll
            for (int u = 0; u < kNegBatch; ++u)
                if (vq[u] != a)
                    repel(g, lh, fix_to_f64(ra.x + hx) - fix_to_f64(rq[u].x), fix_to_f64(ra.y + hy) - fix_to_f64(rq[u].y),
                          hx, hy);
        }
        mv[2 * p] = make_longlong2(hx, hy);
        mv[2 * p + 1] = make_longlong2(qx, qy);
    }
}

// Adds the stored moves of the incidences codes[i], i in [i0, i1) stepping by
// `step`, that lie in the window (kGatherLoads codes in flight per round).
constexpr int kGatherLoads = 4;

__device__ __forceinline__ void gather_range(const LayoutArgs &g, int64_t j0, int64_t len,
                                             const longlong2 *__restrict__ mv, int32_t i0, int32_t i1, int32_t step,
                                             long long &ax, long long &ay)
{
    for (int32_t i = i0; i < i1; i += kGatherLoads * step) {
        uint32_t c[kGatherLoads];
#pragma unroll
        for (int u = 0; u < kGatherLoads; ++u) c[u] = i + u * step < i1 ? g.code[i + u * step] : 0xFFFFFFFFu;
        longlong2 t[kGatherLoads];
        bool in[kGatherLoads];
#pragma unroll
        for (int u = 0; u < kGatherLoads; ++u) {
            int64_t l = (int64_t)(c[u] >> 1) - j0;
            if (l < 0) l += g.m;
            in[u] = c[u] != 0xFFFFFFFFu && l < len;
            t[u] = in[u] ? mv[2 * (int64_t)(c[u] >> 1) + (c[u] & 1)] : make_longlong2(0, 0);
        }
#pragma unroll
        for (int u = 0; u < kGatherLoads; ++u) {
            if (c[u] & 1) {
                ax -= t[u].x;
                ay -= t[u].y;
            } else {
                ax += t[u].x;
                ay += t[u].y;
            }
        }
    }
}

// Phase 2: N[v] = R[v] + the moves of v's incidences at array positions
// j0 .. j0 + len - 1 (mod m).  Blocks
// [0, heavy_blocks) take the heavy vertices (more than kLayoutHeavyInc
// incidences), one block each when heavy_blocks equals their count; the
// other blocks give kGatherTeam lanes to each remaining vertex.
constexpr int kGatherTeam = 8;

__global__ void __launch_bounds__(kLayoutBlock)
grad_gather_kernel(LayoutArgs g, int64_t j0, int64_t len, const longlong2 *__restrict__ mv,
                   const longlong2 *__restrict__ R, longlong2 *__restrict__ N)
{
    if ((int)blockIdx.x < g.heavy_blocks) {
        __shared__ long long part[2][kLayoutBlock / 64];
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        const int32_t cnt = *g.n_heavy;
        for (int32_t h = blockIdx.x; h < cnt; h += g.heavy_blocks) {
            const int32_t v = g.heavy[h];
            long long ax = 0, ay = 0;
            gather_range(g, j0, len, mv, g.off[v] + (int32_t)threadIdx.x, g.off[v + 1], kLayoutBlock, ax, ay);
            for (int o = 32; o > 0; o >>= 1) {
                ax += __shfl_xor(ax, o);
                ay += __shfl_xor(ay, o);
            }
            if (lane == 0) {
                part[0][wid] = ax;
                part[1][wid] = ay;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                long long sx = 0, sy = 0;
                for (int w = 0; w < kLayoutBlock / 64; ++w) {
                    sx += part[0][w];
                    sy += part[1][w];
                }
                const longlong2 r = R[v];
                N[v] = make_longlong2(r.x + sx, r.y + sy);
            }
            __syncthreads();
        }
        return;
    }
    const int32_t v = ((blockIdx.x - g.heavy_blocks) * kLayoutBlock + threadIdx.x) / kGatherTeam;
    const int32_t t = threadIdx.x % kGatherTeam;
    const bool valid = v < g.n;
    const int32_t b = valid ? g.off[v] : 0, e = valid ? g.off[v + 1] : 0;
    const bool mine = valid && e - b <= kLayoutHeavyInc;
    long long ax = 0, ay = 0;
    if (mine) gather_range(g, j0, len, mv, b + t, e, kGatherTeam, ax, ay);
    for (int o = kGatherTeam / 2; o > 0; o >>= 1) {
        ax += __shfl_xor(ax, o);
        ay += __shfl_xor(ay, o);
    }
    if (mine && t == 0) {
        const longlong2 r = R[v];
        N[v] = make_longlong2(r.x + ax, r.y + ay);
    }
}

int grid_for(int64_t work)
{
    int64_t b = (work + kLayoutBlock - 1) / kLayoutBlock;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (int)b;
}

}  // namespace

// ------------------------------------------------------------ launchers --
// Key bits of the union sort: 32 column bits below the row bits (rows
// itself, the sentinel row, must fit).
int union_key_bits(int32_t rows)
{
    int bits = 0;
    while (bits < 31 && ((int64_t)1 << bits) <= (int64_t)rows) ++bits;
    return 32 + bits;
}

size_t union_scratch_bytes(int32_t rows, int32_t k, size_t *sort_tmp)
{
    const int64_t total = 2 * (int64_t)rows * k;
    size_t tmp = (radix_sort_scratch_bytes(total) + 255) & ~(size_t)255;
    *sort_tmp = tmp;
    const size_t t = (size_t)(total > 0 ? total : 1);
    return tmp + 2 * t * sizeof(uint64_t) + 2 * t * sizeof(float) + 1024;
}

hipError_t launch_fuzzy_union(int32_t rows, int32_t k, const int32_t *ids, const float *w, int32_t *row_ptr,
                              int32_t *col, float *val, int64_t cap, int64_t *nnz, int *err, void *scratch,
                              hipStream_t s)
{
    const int64_t total = 2 * (int64_t)rows * k;
    size_t tmp = 0;
    (void)union_scratch_bytes(rows, k, &tmp);
    const size_t t = (size_t)(total > 0 ? total : 1);
    char *p = (char *)scratch;
    uint64_t *k0 = (uint64_t *)(p + tmp);
    uint64_t *k1 = k0 + t;
    float *v0 = (float *)(k1 + t);
    float *v1 = v0 + t;
    hipLaunchKernelGGL(union_emit_kernel, dim3(grid_for(total / 2)), dim3(kLayoutBlock), 0, s, rows, k, ids, w, k0,
                       v0, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    bool alt = false;
    e = radix_sort_pairs<uint64_t>(k0, k1, (uint32_t *)v0, (uint32_t *)v1, total, 0, union_key_bits(rows), p, s, &alt);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(union_rows_kernel, dim3(grid_for(total)), dim3(kLayoutBlock), 0, s, rows, total,
                       (const uint64_t *)(alt ? k1 : k0), (const float *)(alt ? v1 : v0), row_ptr, col, val, cap, nnz);
    return hipGetLastError();
}

size_t shuffle_scratch_bytes(int64_t m, size_t *sort_tmp)
{
    size_t tmp = (radix_sort_scratch_bytes(m) + 255) & ~(size_t)255;
    *sort_tmp = tmp;
    const size_t t = (size_t)(m > 0 ? m : 1);
    return tmp + 2 * t * sizeof(uint64_t) + 2 * t * sizeof(int32_t) + 1024;
}

hipError_t launch_edge_shuffle(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *val,
                               uint64_t seed, int32_t *head, int32_t *tail, float *w, void *scratch, hipStream_t s)
{
    size_t tmp = 0;
    (void)shuffle_scratch_bytes(m, &tmp);
    const size_t t = (size_t)(m > 0 ? m : 1);
    char *p = (char *)scratch;
    uint64_t *k0 = (uint64_t *)(p + tmp);
    uint64_t *k1 = k0 + t;
    int32_t *o0 = (int32_t *)(k1 + t);
    int32_t *o1 = o0 + t;
    hipLaunchKernelGGL(shuffle_keys_kernel, dim3(grid_for(m)), dim3(kLayoutBlock), 0, s, m, seed, k0, o0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    bool alt = false;
    e = radix_sort_pairs<uint64_t>(k0, k1, (uint32_t *)o0, (uint32_t *)o1, m, 0, 64, p, s, &alt);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(shuffle_gather_kernel, dim3(grid_for(m)), dim3(kLayoutBlock), 0, s, n, m, row_ptr, col, val,
                       (const int32_t *)(alt ? o1 : o0), head, tail, w);
    return hipGetLastError();
}

hipError_t launch_edge_check(int32_t n, int64_t m, const int32_t *head, const int32_t *tail, int *err, hipStream_t s)
{
    hipLaunchKernelGGL(edge_check_kernel, dim3(grid_for(m)), dim3(kLayoutBlock), 0, s, n, m, head, tail, err);
    return hipGetLastError();
}

hipError_t launch_layout_init(int32_t n, const float *xy, long long *p0, long long *p1, int *err, hipStream_t s)
{
    hipLaunchKernelGGL(fix_init_kernel, dim3(grid_for(2 * (int64_t)n)), dim3(kLayoutBlock), 0, s, n, xy, p0, p1, err);
    return hipGetLastError();
}

hipError_t launch_layout_out(int32_t n, const long long *p, float *xy, hipStream_t s)
{
    hipLaunchKernelGGL(fix_out_kernel, dim3(grid_for(2 * (int64_t)n)), dim3(kLayoutBlock), 0, s, n, p, xy);
    return hipGetLastError();
}

size_t incidence_scratch_bytes(int32_t n, int64_t m, size_t *sort_tmp)
{
    (void)n;
    size_t tmp = (radix_sort_scratch_bytes(2 * m) + 255) & ~(size_t)255;
    *sort_tmp = tmp;
    const size_t t = (size_t)(2 * m);
    return tmp + 3 * t * sizeof(uint32_t) + 1024;
}

hipError_t launch_layout_incidence(LayoutArgs &g, void *scratch, int32_t *off, uint32_t *code, int32_t *heavy,
                                   int32_t *n_heavy, hipStream_t s)
{
    size_t tmp = 0;
    (void)incidence_scratch_bytes(g.n, g.m, &tmp);
    const int64_t total = 2 * g.m;
    char *p = (char *)scratch;
    uint32_t *k0 = (uint32_t *)(p + tmp), *k1 = k0 + total, *c0 = k1 + total;
    hipLaunchKernelGGL(incidence_keys_kernel, dim3(grid_for(total)), dim3(kLayoutBlock), 0, s, g.m, g.head, g.tail,
                       k0, c0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < (int64_t)g.n) ++bits;
    bool alt = false;   // the sorted codes may end in either buffer
    e = radix_sort_pairs<uint32_t>(k0, k1, c0, code, total, 0, bits, p, s, &alt);
    if (e != hipSuccess) return e;
    if (!alt) {
        e = hipMemcpyAsync(code, c0, (size_t)total * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(incidence_rows_kernel, dim3(grid_for(total)), dim3(kLayoutBlock), 0, s, g.n, total,
                       (const uint32_t *)(alt ? k1 : k0), off);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = hipMemsetAsync(n_heavy, 0, sizeof(int32_t), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(incidence_heavy_kernel, dim3(grid_for(g.n)), dim3(kLayoutBlock), 0, s, g.n, off, heavy,
                       n_heavy);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    g.off = off;
    g.code = code;
    g.heavy = heavy;
    g.n_heavy = n_heavy;
    g.heavy_blocks = 0;   // set by the caller to the heavy count (one block each)
    return hipSuccess;
}

hipError_t launch_grad_window(const LayoutArgs &g, int32_t it, int64_t l0, int64_t l1, double lr, const long long *R,
                              long long *N, void *moves, hipStream_t s)
{
    const int64_t j0 = (int64_t)(((unsigned __int128)(uint64_t)it * (uint64_t)g.s) % (uint64_t)g.m);
    longlong2 *mv = (longlong2 *)moves;
    hipLaunchKernelGGL(grad_moves_kernel, dim3(grid_for(l1 - l0)), dim3(kLayoutBlock), 0, s, g, j0, l0, l1, it, lr,
                       (const longlong2 *)R, mv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t jp = j0 + l0;
    if (jp >= g.m) jp -= g.m;
    const int64_t light_threads = (int64_t)g.n * kGatherTeam;
    const int blocks = g.heavy_blocks + (int)((light_threads + kLayoutBlock - 1) / kLayoutBlock);
    hipLaunchKernelGGL(grad_gather_kernel, dim3(blocks), dim3(kLayoutBlock), 0, s, g, jp, l1 - l0,
                       (const longlong2 *)mv, (const longlong2 *)R, (longlong2 *)N);
    return hipGetLastError();
}

}  // namespace gm
