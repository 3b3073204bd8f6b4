// Layout step C2 of SL-GUMAP on the kNN graph (Sec. 2.1 cost C, Sec. 3.3
// Alg. 3 and Alg. 5 GradSample): the fuzzy union that makes the membership
// graph symmetric, the keyed shuffle of its edge array E_k and the
// sliding-window gradient iterations.
//
// Union and shuffle are sorts: every directed kNN cell emits at most two
// (row, col) keys with their union weight, one radix sort orders them and a
// segment pass writes the CSR; the shuffle sorts the entries by a
// SplitMix64 key of their position.  A GradSample window is one launch: a
// thread per window entry computes the attractive move and its negative
// samples from the positions at the start of the window and adds the
// rounded moves to the next positions with 64-bit integer atomics (fixed
// point, 2^-32 units), so the window's result does not depend on the order
// in which the moves land.  Positions rotate through three buffers: the one
// read, the one accumulated into, and the one cleared for the next window.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
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
                double b = 0.0;
                bool found = false;
                const int32_t *rj = ids + (int64_t)j * k;
                for (int32_t q = 0; q < k; ++q)
                    if (rj[q] == i) {
                        b = (double)w[(int64_t)j * k + q];
                        found = true;
                        break;
                    }
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

// One window: entries at array positions (j0 + l) mod m, l in [0, s).
// R: positions at the start of the window (read only); N: next positions,
// all zero on entry, receiving R and every move; Z: cleared for the window
// after this one.
__global__ void __launch_bounds__(kLayoutBlock)
grad_window_kernel(LayoutArgs g, int64_t j0, int32_t it, double lr, const long long *__restrict__ R,
                   unsigned long long *__restrict__ N, long long *__restrict__ Z)
{
#pragma clang fp contract(off)
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t v = tid; v < g.n; v += stride) {
        atomicAdd(N + 2 * v, (unsigned long long)R[2 * v]);
        atomicAdd(N + 2 * v + 1, (unsigned long long)R[2 * v + 1]);
        Z[2 * v] = 0;
        Z[2 * v + 1] = 0;
    }
    for (int64_t l = tid; l < g.s; l += stride) {
        int64_t p = j0 + l;
        if (p >= g.m) p -= g.m;
        const int32_t a = g.head[p], b = g.tail[p];
        const double lh = lr * (double)g.w[p];
        const double ax = (double)R[2 * (int64_t)a] * kFixInv, ay = (double)R[2 * (int64_t)a + 1] * kFixInv;
        const double bx = (double)R[2 * (int64_t)b] * kFixInv, by = (double)R[2 * (int64_t)b + 1] * kFixInv;
        const double dx = ax - bx, dy = ay - by;
        const double sx = dx * dx, sy = dy * dy;
        const double d2 = sx + sy;
        long long qax = 0, qay = 0;
        if (d2 > 0.0) {
            const double T = pow(d2, g.beta);
            const double num = g.att_num * T;
            const double den = d2 * (1.0 + g.alpha * T);
            const double c = num / den;
            const long long qx = llrint(lh * clip4(c * dx) * kFix);
            const long long qy = llrint(lh * clip4(c * dy) * kFix);
            qax = qx;
            qay = qy;
            atomicAdd(N + 2 * (int64_t)b, (unsigned long long)(-qx));
            atomicAdd(N + 2 * (int64_t)b + 1, (unsigned long long)(-qy));
        }
        const uint64_t base = ((uint64_t)it * (uint64_t)g.s + (uint64_t)l) * (uint64_t)g.neg;
        for (int32_t q = 0; q < g.neg; ++q) {
            const int32_t v = (int32_t)(splitmix64(g.seed, base + (uint64_t)q + 1) % (uint64_t)g.n);
            if (v == a) continue;
            const double vx = (double)R[2 * (int64_t)v] * kFixInv, vy = (double)R[2 * (int64_t)v + 1] * kFixInv;
            const double ex = ax - vx, ey = ay - vy;
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
            qax += llrint(lh * gx * kFix);
            qay += llrint(lh * gy * kFix);
        }
        if (qax) atomicAdd(N + 2 * (int64_t)a, (unsigned long long)qax);
        if (qay) atomicAdd(N + 2 * (int64_t)a + 1, (unsigned long long)qay);
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
    size_t tmp = 0;
    hipcub::DoubleBuffer<uint64_t> kb(nullptr, nullptr);
    hipcub::DoubleBuffer<float> vb(nullptr, nullptr);
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, kb, vb, (int)total, 0, union_key_bits(rows),
                                             (hipStream_t)0);
    tmp = (tmp + 255) & ~(size_t)255;
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
    hipcub::DoubleBuffer<uint64_t> kb(k0, k1);
    hipcub::DoubleBuffer<float> vb(v0, v1);
    e = hipcub::DeviceRadixSort::SortPairs(p, tmp, kb, vb, (int)total, 0, union_key_bits(rows), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(union_rows_kernel, dim3(grid_for(total)), dim3(kLayoutBlock), 0, s, rows, total,
                       (const uint64_t *)kb.Current(), (const float *)vb.Current(), row_ptr, col, val, cap, nnz);
    return hipGetLastError();
}

size_t shuffle_scratch_bytes(int64_t m, size_t *sort_tmp)
{
    size_t tmp = 0;
    hipcub::DoubleBuffer<uint64_t> kb(nullptr, nullptr);
    hipcub::DoubleBuffer<int32_t> vb(nullptr, nullptr);
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, kb, vb, (int)m, 0, 64, (hipStream_t)0);
    tmp = (tmp + 255) & ~(size_t)255;
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
    hipcub::DoubleBuffer<uint64_t> kb(k0, k1);
    hipcub::DoubleBuffer<int32_t> ob(o0, o1);
    e = hipcub::DeviceRadixSort::SortPairs(p, tmp, kb, ob, (int)m, 0, 64, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(shuffle_gather_kernel, dim3(grid_for(m)), dim3(kLayoutBlock), 0, s, n, m, row_ptr, col, val,
                       (const int32_t *)ob.Current(), head, tail, w);
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

hipError_t launch_grad_window(const LayoutArgs &g, int32_t it, double lr, const long long *R, long long *N,
                              long long *Z, hipStream_t s)
{
    const int64_t j0 = (int64_t)(((unsigned __int128)(uint64_t)it * (uint64_t)g.s) % (uint64_t)g.m);
    const int64_t work = g.s > g.n ? g.s : g.n;
    hipLaunchKernelGGL(grad_window_kernel, dim3(grid_for(work)), dim3(kLayoutBlock), 0, s, g, j0, it, lr, R,
                       (unsigned long long *)N, Z);
    return hipGetLastError();
}

}  // namespace gm
