// Neighbourhood preservation of a drawing (Sec. 4.1.3 quality metrics).
//
// One workgroup per listed vertex v:
//   1. the graph ball N_G(v, r), r in {1, 2}: an n-bit set in LDS, marked by
//      the adjacency of v and (r = 2) of each neighbour, one wave per
//      neighbour row; K = |N_G(v, r)|;
//   2. the K-th nearest other vertex in the drawing under the order
//      (squared distance, id): a radix select over the 96-bit key
//      (bits of the FP64 squared distance, then the id).  A first pass finds
//      the smallest and largest distance so the bits all keys share are
//      skipped; then 11-bit digits, one pass over all vertices each, until
//      the K-th key is the only one left in its bucket;
//   3. |N_G & N_D| = the ball members whose key is at most the K-th key.
// The score is |N_G & N_D| / (2K - |N_G & N_D|) in FP64, NaN for an empty
// ball.  Squared distances are dx*dx + dy*dy in FP64 with no fused
// multiply-add, so every comparison matches a plain sequential evaluation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device.h"
#include "kernels.h"

namespace gm {

namespace {

constexpr int kNpBlock = 256;
constexpr int kNpWaves = kNpBlock / GM_WAVE;
constexpr int kDigitBits = 11;
constexpr int kBins = 1 << kDigitBits;

__device__ __forceinline__ double sq_dist(float2 a, float2 b)
{
#pragma clang fp contract(off)
    const double dx = (double)a.x - (double)b.x;
    const double dy = (double)a.y - (double)b.y;
    const double sx = dx * dx;
    const double sy = dy * dy;
    return sx + sy;
}

__device__ __forceinline__ unsigned long long key_hi(float2 p, float2 q)
{
    return (unsigned long long)__double_as_longlong(sq_dist(p, q));   // >= +0: bits order like the values
}

// Block-wide sum of an int (all threads call; result in every thread).
__device__ __forceinline__ int block_sum(int x, int *red)
{
    x = wave_sum(x);
    const int wid = threadIdx.x / GM_WAVE;
    __syncthreads();
    if (lane() == 0) red[wid] = x;
    __syncthreads();
    int t = 0;
#pragma unroll
    for (int i = 0; i < kNpWaves; ++i) t += red[i];
    return t;
}

__global__ void __launch_bounds__(kNpBlock)
neighborhood_kernel(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                    const float2 *__restrict__ xy, int r, const int32_t *__restrict__ verts, int32_t n_verts,
                    double *__restrict__ score, int32_t *__restrict__ ball, unsigned long long *evals)
{
    unsigned long long my_evals = 0;   // squared distances evaluated (thread 0's count of the block's passes)
    extern __shared__ unsigned int bm[];   // n-bit ball
    __shared__ unsigned int hist[kBins];
    __shared__ int red[kNpWaves];
    __shared__ unsigned long long red64[2 * kNpWaves];
    __shared__ unsigned long long sel_hi;
    __shared__ unsigned int sel_lo;
    __shared__ int sel_need, sel_count, sel_bucket;
    const int words = (n + 31) >> 5;
    const int l = lane(), wid = threadIdx.x / GM_WAVE;
    for (int32_t i = blockIdx.x; i < n_verts; i += gridDim.x) {
        const int32_t v = verts ? verts[i] : i;
        // 1. ball
        for (int w = threadIdx.x; w < words; w += kNpBlock) bm[w] = 0u;
        __syncthreads();
        const int32_t e0 = rp[v], e1 = rp[v + 1];
        for (int32_t e = e0 + threadIdx.x; e < e1; e += kNpBlock) {
            const int32_t u = col[e];
            atomicOr(&bm[u >> 5], 1u << (u & 31));
        }
        if (r >= 2) {
            for (int32_t e = e0 + wid; e < e1; e += kNpWaves) {
                const int32_t u = col[e];
                for (int32_t f = rp[u] + l; f < rp[u + 1]; f += GM_WAVE) {
                    const int32_t x = col[f];
                    atomicOr(&bm[x >> 5], 1u << (x & 31));
                }
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) bm[v >> 5] &= ~(1u << (v & 31));
        __syncthreads();
        int kc = 0;
        for (int w = threadIdx.x; w < words; w += kNpBlock) kc += __popc(bm[w]);
        const int K = block_sum(kc, red);
        if (K == 0 || K == n - 1) {
            // empty ball: undefined; everything within r hops: the drawing's
            // K nearest are all the other vertices
            if (threadIdx.x == 0) {
                score[i] = K == 0 ? __longlong_as_double(0x7ff8000000000000ll) : 1.0;
                if (ball) ball[i] = K;
            }
            __syncthreads();
            continue;
        }
        const float2 pv = xy[v];
        // 2a. smallest and largest key: skip the bits they share
        unsigned long long mn = ~0ull, mx = 0ull;
        for (int32_t u = threadIdx.x; u < n; u += kNpBlock) {
            if (u == v) continue;
            const unsigned long long k = key_hi(xy[u], pv);
            mn = k < mn ? k : mn;
            mx = k > mx ? k : mx;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long a = __shfl_xor(mn, o, GM_WAVE), b = __shfl_xor(mx, o, GM_WAVE);
            mn = a < mn ? a : mn;
            mx = b > mx ? b : mx;
        }
        if (l == 0) {
            red64[wid] = mn;
            red64[kNpWaves + wid] = mx;
        }
        if (threadIdx.x == 0) sel_need = K;
        __syncthreads();
        mn = red64[0];
        mx = red64[kNpWaves];
#pragma unroll
        for (int q = 1; q < kNpWaves; ++q) {
            mn = red64[q] < mn ? red64[q] : mn;
            mx = red64[kNpWaves + q] > mx ? red64[kNpWaves + q] : mx;
        }
        // 2b. radix passes over the 96-bit key (hi = distance bits, lo = id)
        const int shared_bits = (mn == mx) ? 64 : __clzll(mn ^ mx);
        unsigned long long pfx_hi = mn & (shared_bits == 64 ? ~0ull : ~(~0ull >> shared_bits));
        unsigned long long mask_hi = shared_bits == 64 ? ~0ull : ~(~0ull >> shared_bits);
        unsigned int pfx_lo = 0u, mask_lo = 0u;
        int bit = 96 - shared_bits;   // bits of the key still free (hi bits first)
        bool unique = false;
        while (bit > 0 && !unique) {
            const int width = bit < kDigitBits ? bit : kDigitBits;
            const int low = bit - width;   // lowest key bit of this digit, counted over 96
            for (int b = threadIdx.x; b < kBins; b += kNpBlock) hist[b] = 0u;
            __syncthreads();
            for (int32_t u = threadIdx.x; u < n; u += kNpBlock) {
                if (u == v) continue;
                const unsigned long long kh = key_hi(xy[u], pv);
                const unsigned int kl = (unsigned int)u;
                if ((kh & mask_hi) != pfx_hi || (kl & mask_lo) != pfx_lo) continue;
                // digit: key bits [low, low + width) of (kh << 32 | kl)
                unsigned int d;
                if (low >= 32) d = (unsigned int)(kh >> (low - 32));
                else if (low + width <= 32) d = kl >> low;
                else d = (unsigned int)((kh << (32 - low)) | (kl >> low));
                atomicAdd(&hist[d & ((1u << width) - 1u)], 1u);
            }
            __syncthreads();
            if (wid == 0) {
                // bucket holding the need-th key: 32 bins per lane, then a wave scan
                constexpr int per = kBins / GM_WAVE;
                int sub = 0;
                for (int b = 0; b < per; ++b) sub += (int)hist[l * per + b];
                const int incl = wave_incl_scan(sub);
                const int need = sel_need;
                const unsigned long long hit = __ballot(incl >= need);
                const int owner = __ffsll((long long)hit) - 1;
                if (l == owner) {
                    int acc = incl - sub;
                    int b = l * per;
                    while (acc + (int)hist[b] < need) acc += (int)hist[b++];
                    sel_bucket = b;
                    sel_need = need - acc;
                    sel_count = (int)hist[b];
                }
            }
            __syncthreads();
            const unsigned long long dig = (unsigned long long)sel_bucket;
            const unsigned long long dm = (width == 64 ? ~0ull : ((1ull << width) - 1ull));
            if (low >= 32) {
                pfx_hi |= dig << (low - 32);
                mask_hi |= dm << (low - 32);
            } else if (low + width <= 32) {
                pfx_lo |= (unsigned int)(dig << low);
                mask_lo |= (unsigned int)(dm << low);
            } else {
                pfx_hi |= dig >> (32 - low);
                mask_hi |= dm >> (32 - low);
                pfx_lo |= (unsigned int)(dig << low);
                mask_lo |= (unsigned int)(dm << low);
            }
            bit = low;
            unique = sel_count == 1;
            __syncthreads();
        }
        // 2c. the K-th key itself (the one key with the chosen prefix)
        if (bit > 0) {
            for (int32_t u = threadIdx.x; u < n; u += kNpBlock) {
                if (u == v) continue;
                const unsigned long long kh = key_hi(xy[u], pv);
                if ((kh & mask_hi) == pfx_hi && ((unsigned int)u & mask_lo) == pfx_lo) {
                    sel_hi = kh;
                    sel_lo = (unsigned int)u;
                }
            }
        } else if (threadIdx.x == 0) {
            sel_hi = pfx_hi;
            sel_lo = pfx_lo;
        }
        __syncthreads();
        const unsigned long long th = sel_hi;
        const unsigned int tl = sel_lo;
        // 3. ball members within the K nearest
        int common = 0;
        for (int w = threadIdx.x; w < words; w += kNpBlock) {
            unsigned int bits = bm[w];
            while (bits) {
                const int b = __ffs((int)bits) - 1;
                bits &= bits - 1u;
                const int32_t u = (w << 5) + b;
                const unsigned long long kh = key_hi(xy[u], pv);
                common += (kh < th || (kh == th && (unsigned int)u <= tl)) ? 1 : 0;
            }
        }
        const int I = block_sum(common, red);
        if (threadIdx.x == 0) {
            // min/max pass, the radix passes, the final lookup, the ball
            const int passes = 1 + ((96 - shared_bits) - bit + kDigitBits - 1) / kDigitBits + (bit > 0 ? 1 : 0);
            my_evals += (unsigned long long)passes * (unsigned long long)(n - 1) + (unsigned long long)K;
            score[i] = (double)I / (double)(2 * K - I);
            if (ball) ball[i] = K;
        }
        __syncthreads();
    }
    if (evals && threadIdx.x == 0 && my_evals) atomicAdd(evals, my_evals);
}

}  // namespace

size_t neighborhood_lds_bytes(int32_t n) { return (size_t)((n + 31) / 32) * sizeof(unsigned int); }

hipError_t launch_neighborhood(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *xy, int r,
                               const int32_t *verts, int32_t n_verts, double *score, int32_t *ball,
                               unsigned long long *evals, hipStream_t s)
{
    if (n_verts <= 0) return hipSuccess;
    const size_t lds = neighborhood_lds_bytes(n);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
    static size_t lds_set[64] = {};   // the LDS limit is an attribute of the kernel on each device
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (lds > 48 * 1024 && lds > lds_set[dev]) {
        hipError_t e = hipFuncSetAttribute((const void *)neighborhood_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set[dev] = lds;
    }
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        cus = 256;
    }
    const int blocks = (int)std::min<int64_t>(n_verts, (int64_t)cus * 8);
    hipLaunchKernelGGL(neighborhood_kernel, dim3(blocks), dim3(kNpBlock), lds, s, n, row_ptr, col,
                       (const float2 *)xy, r, verts, n_verts, score, ball, evals);
    return hipGetLastError();
}

}  // namespace gm
