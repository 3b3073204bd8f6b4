// Spectral initial drawing of the layout step (the drawing starts from a
// spectral layout, Sec. 3.2, as UMAP starts its optimisation): the
// eigenvectors of the 2nd and 3rd smallest eigenvalues of the normalised
// Laplacian L = I - D^-1/2 W D^-1/2 of the symmetric weighted graph W.
//
// They are the eigenvectors of the two largest eigenvalues of
// A = D^-1/2 W D^-1/2 on the complement of its top eigenvector D^1/2 1
// (eigenvalue 1), found by Lanczos iteration in FP64: the Krylov basis Q is
// kept whole (column-major, one column per step) behind the deflated
// columns, and every new vector is orthogonalised against all of it once
// after the three-term recurrence has removed the two large components
// (one classical Gram-Schmidt pass then meets only rounding error), which
// keeps Q orthonormal to rounding and removes the deflated directions.  Two runs: the first, with
// column 0 = D^1/2 1 normalised, converges the top eigenpair; the second
// also deflates that eigenvector (column 1) and converges the next, so that
// a repeated eigenvalue (a cycle's, a complete graph's) still yields two
// orthogonal eigenvectors, which one Krylov sequence cannot.  Only the top
// eigenpair of the small tridiagonal matrix of the recurrence is needed; the
// host finds it by bisection on Sturm counts and inverse iteration, in O(m).
// Partial sums are reduced in a fixed order, so a run is reproducible.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cmath>
#include <stdint.h>

#include <vector>

#include "kernels.h"

namespace gm {
namespace {

constexpr int kSpBlock = 256;
constexpr int kSpTile = 2048;   // rows per partial sum

__device__ __forceinline__ uint64_t sp_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)blockDim.x / 64; ++i) t += sh[i];
    __syncthreads();
    return t;   // valid in thread 0
}

// sinv[v] = 1 / sqrt(d_v), u[v] = sqrt(d_v), d_v = sum of row v's weights;
// err bit 1: a vertex of zero degree; bit 2: a weight negative or not finite.
__global__ void __launch_bounds__(kSpBlock)
sp_degree_kernel(int32_t n, const int32_t *__restrict__ rp, const float *__restrict__ val, double *__restrict__ sinv,
                 double *__restrict__ u, int *__restrict__ err)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        double d = 0.0;
        int bad = 0;
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            const float x = val[e];
            if (!(x >= 0.0f) || isinf(x)) bad = 2;
            d += (double)x;
        }
        if (!(d > 0.0)) bad |= 1;
        if (bad) atomicOr(err, bad);
        sinv[v] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
        u[v] = d > 0.0 ? sqrt(d) : 0.0;
    }
}

// Rows with more than kSpHeavyRow entries (listed once per call).
constexpr int kSpHeavyRow = 128;
constexpr int kSpTeam = 8;

__global__ void __launch_bounds__(kSpBlock)
sp_heavy_kernel(int32_t n, const int32_t *__restrict__ rp, int32_t *__restrict__ heavy, int32_t *__restrict__ count)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (rp[v + 1] - rp[v] > kSpHeavyRow) heavy[atomicAdd(count, 1)] = v;
}

// y = A x (minus bprev[0] * xprev when xprev is not NULL: the first term of
// the three-term recurrence): blocks [0, heavy_blocks) take one heavy row
// each (block-wide sum), the others kSpTeam lanes per remaining row.
__global__ void __launch_bounds__(kSpBlock)
sp_spmv_kernel(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
               const float *__restrict__ val, const double *__restrict__ sinv, const double *__restrict__ x,
               double *__restrict__ y, const int32_t *__restrict__ heavy, int heavy_blocks,
               const double *__restrict__ xprev, const double *__restrict__ bprev)
{
    const double fprev = xprev ? bprev[0] : 0.0;
    if ((int)blockIdx.x < heavy_blocks) {
        __shared__ double sh[kSpBlock / 64];
        const int32_t v = heavy[blockIdx.x];
        double acc = 0.0;
        for (int32_t e = rp[v] + threadIdx.x; e < rp[v + 1]; e += blockDim.x) {
            const int32_t c = col[e];
            acc += (double)val[e] * (sinv[c] * x[c]);
        }
        const double t = block_sum(acc, sh);
        if (threadIdx.x == 0) y[v] = xprev ? sinv[v] * t - fprev * xprev[v] : sinv[v] * t;
        return;
    }
    const int32_t v = (int32_t)((((int64_t)blockIdx.x - heavy_blocks) * kSpBlock + threadIdx.x) / kSpTeam);
    const int lane_t = threadIdx.x % kSpTeam;
    const bool valid = v < n;
    const int32_t b = valid ? rp[v] : 0, e1 = valid ? rp[v + 1] : 0;
    const bool mine = valid && e1 - b <= kSpHeavyRow;
    double acc = 0.0;
    if (mine)
        for (int32_t e = b + lane_t; e < e1; e += kSpTeam) {
            const int32_t c = col[e];
            acc += (double)val[e] * (sinv[c] * x[c]);
        }
    for (int o = kSpTeam / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (mine && lane_t == 0) y[v] = xprev ? sinv[v] * acc - fprev * xprev[v] : sinv[v] * acc;
}

// part[c * tiles + t] = sum over the rows of tile t of Q[:, c] * w, for
// columns c0 .. c0 + kSpCols of block (t, cb) (c < ncols): w is read once
// per column block
constexpr int kSpCols = 8;

__global__ void __launch_bounds__(kSpBlock)
sp_gemvt_kernel(int32_t n, const double *__restrict__ Q, size_t ld, int ncols, const double *__restrict__ w,
                double *__restrict__ part, int tiles)
{
    __shared__ double sh[kSpCols][kSpBlock / 64];
    const int t = blockIdx.x, c0 = blockIdx.y * kSpCols;
    const int32_t r0 = t * kSpTile, r1 = min(n, r0 + kSpTile);
    double acc[kSpCols];
#pragma unroll
    for (int u = 0; u < kSpCols; ++u) acc[u] = 0.0;
    for (int32_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        const double wi = w[i];
#pragma unroll
        for (int u = 0; u < kSpCols; ++u)
            if (c0 + u < ncols) acc[u] += Q[(size_t)(c0 + u) * ld + i] * wi;
    }
#pragma unroll
    for (int u = 0; u < kSpCols; ++u) {
        double v = acc[u];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) sh[u][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < kSpCols && c0 + (int)threadIdx.x < ncols) {
        double v = 0.0;
        for (int q = 0; q < kSpBlock / 64; ++q) v += sh[threadIdx.x][q];
        part[(size_t)(c0 + threadIdx.x) * tiles + t] = v;
    }
}

// One-column projection finished and applied: s = the sum of the tiles'
// partials of column 0 (each block sums them in the same order), h[0] =
// hacc[0] = s, and w -= s * q.
__global__ void __launch_bounds__(kSpBlock)
sp_axpy_reduce_kernel(int32_t n, const double *__restrict__ q, const double *__restrict__ part, int tiles,
                      double *__restrict__ h, double *__restrict__ hacc, double *__restrict__ w)
{
    __shared__ double sv;
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int t = 0; t < tiles; ++t) acc += part[t];
        sv = acc;
        if (blockIdx.x == 0) {
            h[0] = acc;
            hacc[0] = acc;
        }
    }
    __syncthreads();
    const double f = sv;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) w[i] -= f * q[i];
}

// h[c] = sum of the tiles' partials; hacc[c] = h[c] (first pass) or += h[c]
// (second pass, which also stores *alpha_out = hacc[jcol])
__global__ void __launch_bounds__(kSpBlock)
sp_reduce_kernel(const double *__restrict__ part, int tiles, int ncols, double *__restrict__ h,
                 double *__restrict__ hacc, int second, int jcol, double *__restrict__ alpha_out)
{
    for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
        double s = 0.0;
        for (int t = 0; t < tiles; ++t) s += part[(size_t)c * tiles + t];
        h[c] = s;
        const double a = second ? hacc[c] + s : s;
        hacc[c] = a;
        if (second && c == jcol) *alpha_out = a;
    }
}

// The full pass of a Lanczos step: h[c] = sum of the partials for every
// column; *alpha_out = the local alpha (h[0] on entry, from the projection
// on q[j] alone) + the correction h[jcol].
__global__ void __launch_bounds__(kSpBlock)
sp_reduce_full_kernel(const double *__restrict__ part, int tiles, int ncols, double *__restrict__ h, int jcol,
                      double *__restrict__ alpha_out)
{
    const double local = h[0];   // the local alpha, read before h is overwritten
    __syncthreads();
    for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
        double s = 0.0;
        for (int t = 0; t < tiles; ++t) s += part[(size_t)c * tiles + t];
        h[c] = s;
        if (c == jcol) *alpha_out = local + s;
    }
}

// w -= Q[:, 0..ncols) h
__global__ void __launch_bounds__(kSpBlock)
sp_gemv_sub_kernel(int32_t n, const double *__restrict__ Q, size_t ld, int ncols, const double *__restrict__ h,
                   double *__restrict__ w)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double acc = 0.0;
#pragma unroll 8
        for (int c = 0; c < ncols; ++c) acc += Q[(size_t)c * ld + i] * h[c];
        w[i] -= acc;
    }
}

__global__ void __launch_bounds__(kSpBlock)
sp_sumsq_kernel(int32_t n, const double *__restrict__ w, double *__restrict__ part)
{
    __shared__ double sh[kSpBlock / 64];
    const int32_t r0 = blockIdx.x * kSpTile, r1 = min(n, r0 + kSpTile);
    double acc = 0.0;
    for (int32_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) acc += w[i] * w[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[0] = sqrt(sum of the partials); below `tiny` it counts as zero (the
// Krylov space is exhausted) and the next vector is zero.
__global__ void sp_norm_kernel(const double *__restrict__ part, int tiles, double tiny, double *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int t = 0; t < tiles; ++t) s += part[t];
    const double r = sqrt(s);
    out[0] = r > tiny ? r : 0.0;
}

// The norm and the scaling in one launch: every block sums the tiles'
// squared partials in the same order, r = sqrt(sum) (zero below `tiny`),
// block 0 stores it to *out, and q = w / r (zero when r is zero).
__global__ void __launch_bounds__(kSpBlock)
sp_norm_scale_kernel(int32_t n, const double *w, const double *__restrict__ part, int tiles, double tiny,
                     double *__restrict__ out, double *q)   // w may equal q
{
    __shared__ double rv;
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int t = 0; t < tiles; ++t) acc += part[t];
        const double r0 = sqrt(acc);
        rv = r0 > tiny ? r0 : 0.0;
        if (blockIdx.x == 0) out[0] = rv;
    }
    __syncthreads();
    const double r = rv;
    const double f = r > 0.0 ? 1.0 / r : 0.0;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) q[i] = w[i] * f;
}

__global__ void __launch_bounds__(kSpBlock)
sp_scale_kernel(int32_t n, const double *w, const double *__restrict__ nrm, double *q)   // w may equal q
{
    const double r = nrm[0];
    const double f = r > 0.0 ? 1.0 / r : 0.0;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) q[i] = w[i] * f;
}

__global__ void __launch_bounds__(kSpBlock)
sp_start_kernel(int32_t n, uint64_t seed, double *__restrict__ q)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        q[i] = (double)(sp_splitmix64(seed, (uint64_t)i + 1) >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// x[i] = sum_c Q[i][c0 + c] s[c], c < m (a Ritz vector)
__global__ void __launch_bounds__(kSpBlock)
sp_ritz_kernel(int32_t n, const double *__restrict__ Q, size_t ld, int c0, int m, const double *__restrict__ s,
               double *__restrict__ x)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double a = 0.0;
        for (int c = 0; c < m; ++c) a += Q[(size_t)(c0 + c) * ld + i] * s[c];
        x[i] = a;
    }
}

// Per tile and column: sum of squares and largest magnitude.
__global__ void __launch_bounds__(kSpBlock)
sp_stats_kernel(int32_t n, const double *__restrict__ X, double *__restrict__ part, int tiles)
{
    __shared__ double sh[kSpBlock / 64];
    __shared__ double mx[kSpBlock];
    const int k = blockIdx.y;
    const double *x = X + (size_t)k * n;
    const int32_t r0 = blockIdx.x * kSpTile, r1 = min(n, r0 + kSpTile);
    double ss = 0.0, m = 0.0;
    for (int32_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        ss += x[i] * x[i];
        m = fmax(m, fabs(x[i]));
    }
    const double s = block_sum(ss, sh);
    mx[threadIdx.x] = m;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[((size_t)k * tiles + blockIdx.x) * 2] = s;
        part[((size_t)k * tiles + blockIdx.x) * 2 + 1] = mx[0];
    }
}

// stat[k] = {norm, largest magnitude} of column k
__global__ void sp_stats_reduce_kernel(const double *__restrict__ part, int tiles, double *__restrict__ stat)
{
    const int k = threadIdx.x;
    if (k >= 2 || blockIdx.x != 0) return;
    double s = 0.0, m = 0.0;
    for (int t = 0; t < tiles; ++t) {
        s += part[((size_t)k * tiles + t) * 2];
        m = fmax(m, part[((size_t)k * tiles + t) * 2 + 1]);
    }
    stat[2 * k] = sqrt(s);
    stat[2 * k + 1] = m;
}

// first[k] = the smallest index whose magnitude exceeds half the largest
__global__ void __launch_bounds__(kSpBlock)
sp_first_kernel(int32_t n, const double *__restrict__ X, const double *__restrict__ stat, int *__restrict__ first)
{
    const int k = blockIdx.y;
    const double *x = X + (size_t)k * n;
    const double thr = 0.5 * stat[2 * k + 1];
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (fabs(x[i]) > thr) atomicMin(&first[k], i);
}

// xy[2 i + k] = sign_k x_k[i] / norm_k * 10 / max_k(largest_k / norm_k)
__global__ void __launch_bounds__(kSpBlock)
sp_finish_kernel(int32_t n, const double *__restrict__ X, const double *__restrict__ stat,
                 const int *__restrict__ first, float *__restrict__ xy)
{
    if (!(stat[0] > 0.0) || !(stat[2] > 0.0)) {   // no Ritz vector (cannot happen after convergence)
        for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < 2 * n; i += gridDim.x * blockDim.x) xy[i] = 0.0f;
        return;
    }
    const double m0 = stat[1] / stat[0], m1 = stat[3] / stat[2];
    const double scale = 10.0 / fmax(m0, m1);
    const int32_t p0 = first[0] < n ? first[0] : 0, p1 = first[1] < n ? first[1] : 0;
    const double f0 = (X[p0] < 0.0 ? -scale : scale) / stat[0];
    const double f1 = (X[(size_t)n + p1] < 0.0 ? -scale : scale) / stat[2];
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        xy[2 * (size_t)i] = (float)(X[i] * f0);
        xy[2 * (size_t)i + 1] = (float)(X[(size_t)n + i] * f1);
    }
}

int sp_grid(int64_t work)
{
    int64_t b = (work + kSpBlock - 1) / kSpBlock;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    return (int)b;
}

}  // namespace

int spectral_tiles(int32_t n) { return (n + kSpTile - 1) / kSpTile; }

hipError_t launch_spectral_setup(const SpectralArgs &a, int *err, int32_t *heavy_count, hipStream_t s)
{
    const int tiles = spectral_tiles(a.n);
    hipLaunchKernelGGL(sp_heavy_kernel, dim3(sp_grid(a.n)), dim3(kSpBlock), 0, s, a.n, a.row_ptr, a.heavy,
                       heavy_count);
    hipLaunchKernelGGL(sp_degree_kernel, dim3(sp_grid(a.n)), dim3(kSpBlock), 0, s, a.n, a.row_ptr, a.val, a.sinv,
                       a.Q, err);
    // column 0: D^1/2 1 normalised
    hipLaunchKernelGGL(sp_sumsq_kernel, dim3(tiles), dim3(kSpBlock), 0, s, a.n, a.Q, a.part);
    hipLaunchKernelGGL(sp_norm_kernel, dim3(1), dim3(64), 0, s, a.part, tiles, 0.0, a.scal);
    hipLaunchKernelGGL(sp_scale_kernel, dim3(sp_grid(a.n)), dim3(kSpBlock), 0, s, a.n, a.Q, a.scal, a.Q);
    return hipGetLastError();
}

// Column c0 (the first Lanczos vector): a seeded vector orthogonalised twice
// against columns 0 .. c0 - 1 and normalised.
hipError_t launch_lanczos_start(const SpectralArgs &a, int c0, uint64_t seed, hipStream_t s)
{
    const int tiles = spectral_tiles(a.n);
    hipLaunchKernelGGL(sp_start_kernel, dim3(sp_grid(a.n)), dim3(kSpBlock), 0, s, a.n, seed, a.w);
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(sp_gemvt_kernel, dim3(tiles, (c0 + kSpCols - 1) / kSpCols), dim3(kSpBlock), 0, s, a.n, a.Q,
                           a.ld, c0, a.w, a.part, tiles);
        hipLaunchKernelGGL(sp_reduce_kernel, dim3(1), dim3(kSpBlock), 0, s, a.part, tiles, c0, a.h, a.hacc, 0, -1,
                           (double *)nullptr);
        hipLaunchKernelGGL(sp_gemv_sub_kernel, dim3(sp_grid(a.n)), dim3(kSpBlock), 0, s, a.n, a.Q, a.ld, c0, a.h,
                           a.w);
    }
    hipLaunchKernelGGL(sp_sumsq_kernel, dim3(tiles), dim3(kSpBlock), 0, s, a.n, a.w, a.part);
    hipLaunchKernelGGL(sp_norm_kernel, dim3(1), dim3(64), 0, s, a.part, tiles, 0.0, a.scal);
    hipLaunchKernelGGL(sp_scale_kernel, dim3(sp_grid(a.n)), dim3(kSpBlock), 0, s, a.n, a.w, a.scal,
                       a.Q + (size_t)c0 * a.ld);
    return hipGetLastError();
}

hipError_t launch_lanczos_step(const SpectralArgs &a, int c0, int j, hipStream_t s)
{
    const int tiles = spectral_tiles(a.n);
    const int cj = c0 + j - 1;   // column of Lanczos vector j
    const double *qj = a.Q + (size_t)cj * a.ld;
    const int light_blocks = (int)(((int64_t)a.n * kSpTeam + kSpBlock - 1) / kSpBlock);
    // the three-term recurrence first: w = A q[j] - beta[j-1] q[j-1] (in the
    // sparse product), then w -= alpha q[j] with alpha = q[j] . w; what
    // remains along the basis is rounding error, which one full projection
    // pass removes
    hipLaunchKernelGGL(sp_spmv_kernel, dim3(a.heavy_rows + light_blocks), dim3(kSpBlock), 0, s, a.n, a.row_ptr, a.col,
                       a.val, a.sinv, qj, a.w, a.heavy, a.heavy_rows, j > 1 ? qj - a.ld : (const double *)nullptr,
                       a.beta + j - 1);
    hipLaunchKernelGGL(sp_gemvt_kernel, dim3(tiles, 1), dim3(kSpBlock), 0, s, a.n, qj, a.ld, 1, a.w, a.part, tiles);
    hipLaunchKernelGGL(sp_axpy_reduce_kernel, dim3(sp_grid(a.n)), dim3(kSpBlock), 0, s, a.n, qj, a.part, tiles, a.h,
                       a.hacc, a.w);
    hipLaunchKernelGGL(sp_gemvt_kernel, dim3(tiles, (cj + 1 + kSpCols - 1) / kSpCols), dim3(kSpBlock), 0, s, a.n, a.Q,
                       a.ld, cj + 1, a.w, a.part, tiles);
    hipLaunchKernelGGL(sp_reduce_full_kernel, dim3(1), dim3(kSpBlock), 0, s, a.part, tiles, cj + 1, a.h, cj,
                       a.alpha + j);
    hipLaunchKernelGGL(sp_gemv_sub_kernel, dim3(sp_grid(a.n)), dim3(kSpBlock), 0, s, a.n, a.Q, a.ld, cj + 1, a.h, a.w);
    hipLaunchKernelGGL(sp_sumsq_kernel, dim3(tiles), dim3(kSpBlock), 0, s, a.n, a.w, a.part);
    hipLaunchKernelGGL(sp_norm_scale_kernel, dim3(sp_grid(a.n)), dim3(kSpBlock), 0, s, a.n, a.w, a.part, tiles, a.tiny,
                       a.beta + j, a.Q + (size_t)(cj + 1) * a.ld);
    return hipGetLastError();
}

hipError_t launch_ritz_vector(const SpectralArgs &a, int c0, int m, const double *svec, int k, hipStream_t s)
{
    hipLaunchKernelGGL(sp_ritz_kernel, dim3(sp_grid(a.n)), dim3(kSpBlock), 0, s, a.n, a.Q, a.ld, c0, m, svec,
                       a.X + (size_t)k * a.n);
    return hipGetLastError();
}

// Column `col` = X[:, k] normalised (for the deflation of the second run).
hipError_t launch_ritz_deflate(const SpectralArgs &a, int k, int col, hipStream_t s)
{
    const int tiles = spectral_tiles(a.n);
    const double *x = a.X + (size_t)k * a.n;
    hipLaunchKernelGGL(sp_sumsq_kernel, dim3(tiles), dim3(kSpBlock), 0, s, a.n, x, a.part);
    hipLaunchKernelGGL(sp_norm_kernel, dim3(1), dim3(64), 0, s, a.part, tiles, 0.0, a.scal);
    hipLaunchKernelGGL(sp_scale_kernel, dim3(sp_grid(a.n)), dim3(kSpBlock), 0, s, a.n, x, a.scal,
                       a.Q + (size_t)col * a.ld);
    return hipGetLastError();
}

hipError_t launch_spectral_finish(const SpectralArgs &a, int *first, float *xy, hipStream_t s)
{
    const int tiles = spectral_tiles(a.n);
    hipLaunchKernelGGL(sp_stats_kernel, dim3(tiles, 2), dim3(kSpBlock), 0, s, a.n, a.X, a.part, tiles);
    hipLaunchKernelGGL(sp_stats_reduce_kernel, dim3(1), dim3(64), 0, s, a.part, tiles, a.scal);
    hipLaunchKernelGGL(sp_first_kernel, dim3(sp_grid(a.n), 2), dim3(kSpBlock), 0, s, a.n, a.X, a.scal, first);
    hipLaunchKernelGGL(sp_finish_kernel, dim3(sp_grid(a.n)), dim3(kSpBlock), 0, s, a.n, a.X, a.scal, first, xy);
    return hipGetLastError();
}

// ------------------------------------------------------------ host side --
// Largest eigenvalue theta of the symmetric tridiagonal matrix T with
// diagonal a[0..m) and off-diagonal b[0..m-1), and its unit eigenvector z:
// theta by bisection on Sturm counts (the number of negative pivots of
// T - x I counts the eigenvalues below x), z by inverse iteration (three
// solves of (T - theta I) x = y with partial pivoting).  O(m) work per
// bisection step and per solve.
bool tridiag_top(int m, const double *a, const double *b, double *theta, double *z)
{
    if (m < 1) return false;
    if (m == 1) {
        *theta = a[0];
        z[0] = 1.0;
        return true;
    }
    const double eps = 2.220446049250313e-16;
    double lo = a[0], hi = a[0], bmax2 = 0.0;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < m ? fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
        if (i + 1 < m) bmax2 = std::max(bmax2, b[i] * b[i]);
    }
    const double pivmin = 2.2250738585072014e-308 * std::max(1.0, bmax2);
    auto below = [&](double x) {   // eigenvalues < x
        int cnt = 0;
        double q = a[0] - x;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++cnt;
        for (int i = 1; i < m; ++i) {
            q = (a[i] - x) - b[i - 1] * b[i - 1] / q;
            if (fabs(q) < pivmin) q = -pivmin;
            if (q < 0.0) ++cnt;
        }
        return cnt;
    };
    // below(x) == m exactly when x is above the largest eigenvalue
    for (int it = 0; it < 256; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi || hi - lo <= 2.0 * eps * std::max(fabs(lo), fabs(hi))) break;
        if (below(mid) == m) hi = mid;
        else lo = mid;
    }
    const double t = 0.5 * (lo + hi);
    *theta = t;
    // LU of T - t I with partial pivoting: d (diagonal), du, du2 (first and
    // second superdiagonals of U), l (multipliers), sw (row i swapped with i + 1)
    double anorm = 0.0;
    for (int i = 0; i < m; ++i) anorm = std::max(anorm, fabs(a[i] - t) + (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < m ? fabs(b[i]) : 0.0));
    const double tiny = std::max(eps * anorm, pivmin);
    std::vector<double> d(m), du(m, 0.0), du2(m, 0.0), l(m, 0.0), y(m);
    std::vector<char> sw(m, 0);
    for (int i = 0; i < m; ++i) d[i] = a[i] - t;
    for (int i = 0; i + 1 < m; ++i) du[i] = b[i];
    for (int i = 0; i + 1 < m; ++i) {
        const double sub = b[i];   // row i + 1, column i
        if (fabs(d[i]) >= fabs(sub)) {
            if (d[i] == 0.0) d[i] = tiny;
            const double f = sub / d[i];
            l[i] = f;
            d[i + 1] -= f * du[i];
        } else {
            // rows i and i + 1 exchanged, then column i eliminated from the new row i + 1
            const double f = d[i] / sub;
            const double di1 = d[i + 1], dui = du[i], dui1 = i + 2 < m ? du[i + 1] : 0.0;
            d[i] = sub;
            du[i] = di1;
            du2[i] = dui1;
            d[i + 1] = dui - f * di1;
            if (i + 2 < m) du[i + 1] = -f * dui1;
            l[i] = f;
            sw[i] = 1;
        }
    }
    for (int i = 0; i < m; ++i)
        if (fabs(d[i]) < tiny) d[i] = d[i] < 0.0 ? -tiny : tiny;
    // start vector with components of both signs' weights spread over the rows
    for (int i = 0; i < m; ++i) z[i] = 1.0 + 0.25 * (double)(i % 7);
    for (int pass = 0; pass < 3; ++pass) {
        for (int i = 0; i < m; ++i) y[i] = z[i];
        for (int i = 0; i + 1 < m; ++i) {
            if (sw[i]) std::swap(y[i], y[i + 1]);
            y[i + 1] -= l[i] * y[i];
        }
        for (int i = m - 1; i >= 0; --i) {
            double v = y[i];
            if (i + 1 < m) v -= du[i] * z[i + 1];
            if (i + 2 < m) v -= du2[i] * z[i + 2];
            z[i] = v / d[i];
        }
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += z[i] * z[i];
        nrm = sqrt(nrm);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) return false;
        for (int i = 0; i < m; ++i) z[i] /= nrm;
    }
    return true;
}

}  // namespace gm
