// All-source BFS hop distances (GUMAP step C0, Sec. 3.1, Alg. 1) as a
// multi-source bit-parallel BFS.
//
// Sources are ranked in ascending id order ("slots") and packed into groups of
// W = 64 * words slots.  For each group every vertex owns `words` uint64 of
// each state array, laid out [group][vertex][word]:
//   front[L & 1]   bits of the sources that reached the vertex at hop L - 1
//   visited        bits of the sources that reached it at any earlier hop
//   planes[b]      bit b of the hop at which each source reached it
// One launch per level.  Level L first commits the previous level's frontier
// into `visited` and the bit-planes (the commit is lazy so one launch per
// level suffices), then finds the level-L bits bottom-up: a vertex ORs the
// frontier words of its neighbours, stopping as soon as every source that has
// not reached it yet is covered.  Level 1 needs no frontier read: a vertex
// scans the part of its sorted adjacency that falls in the id range of each
// 64-source word and sets the bits of the sources it finds.
// After the last level a transpose kernel turns the vertex-major bit-planes
// into source-major uint8 hop rows, 64 x 64 bits per wave through shuffle
// butterflies, and counts how many vertices each source reached at hops
// 1..16 (used by the kNN selection to find its last level without a
// separate pass).
#include "device.h"
#include "kernels.h"

namespace gm {

namespace {

constexpr int kLevelBlock = 256;
constexpr int kHopTilesPerWave = 16;
constexpr int kHopWaves = 4;
constexpr int kCountLevels = 16;

__device__ __forceinline__ uint64_t word_valid_mask(int32_t n_slots, int32_t local_slot0)
{
    int32_t c = n_slots - local_slot0;
    if (c <= 0) return 0ull;
    if (c >= 64) return ~0ull;
    return (1ull << c) - 1ull;
}

__global__ void msbfs_init_kernel(MsbfsArgs a)
{
    // one thread per slot of the round: set the source's own bit (hop 0)
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_slots) return;
    const int W = 64 * a.words;
    int32_t g = i / W, r = i % W, w = r >> 6, bit = r & 63;
    int32_t u = a.usrc[a.slot0 + i];
    size_t idx = ((size_t)g * a.n + u) * a.words + w;
    atomicOr((unsigned long long *)&a.front[1][idx], 1ull << bit);
}

__global__ void __launch_bounds__(kLevelBlock)
msbfs_level_kernel(MsbfsArgs a, int level, int commit_only)
{
    const int32_t g = blockIdx.y;
    if (level >= 2 && a.stats[(size_t)(level - 1) * a.stats_groups + g] == 0ull) return;
    const int lw = __ffs(a.words) - 1;                        // log2(words)
    const int64_t idx = (int64_t)blockIdx.x * kLevelBlock + threadIdx.x;
    const int64_t items = (int64_t)a.n << lw;
    uint64_t nw = 0;
    if (idx < items) {
        const int32_t v = (int32_t)(idx >> lw);
        const int32_t w = (int32_t)(idx & (a.words - 1));
        const size_t gbase = (size_t)g * a.n * a.words + w;  // + vertex * words
        const size_t me = gbase + ((size_t)v << lw);
        const uint64_t *__restrict__ fr = a.front[level & 1];
        uint64_t f = fr[me];
        uint64_t vis = a.visited[me];
        if (f) {
            vis |= f;
            a.visited[me] = vis;
            const int hop = level - 1;
            for (int b = 0; b < 8; ++b)
                if ((hop >> b) & 1) a.planes[(size_t)b * a.plane_stride + me] |= f;
        }
        if (!commit_only) {
            const int32_t ls0 = g * 64 * a.words + 64 * w;    // local slot of bit 0
            const uint64_t unv = ~vis & word_valid_mask(a.n_slots, ls0);
            if (unv) {
                const int32_t e0 = a.row_ptr[v], e1 = a.row_ptr[v + 1];
                uint64_t acc = 0;
                if (level == 1) {
                    const int32_t gs0 = a.slot0 + ls0;
                    const int32_t gl = min(gs0 + 63, a.slot0 + a.n_slots - 1);
                    const int32_t lo = a.usrc[gs0], hi = a.usrc[gl];
                    for (int32_t e = lower_bound(a.col, e0, e1, lo); e < e1; ++e) {
                        const int32_t u = a.col[e];
                        if (u > hi) break;
                        const int32_t s = a.slot_of[u];
                        if (s >= 0) acc |= 1ull << (s - gs0);
                    }
                } else {
                    for (int32_t e = e0; e < e1; ++e) {
                        const int32_t u = a.col[e];
                        acc |= fr[gbase + ((size_t)u << lw)];
                        if ((acc & unv) == unv) break;
                    }
                }
                nw = acc & unv;
            }
            a.front[(level + 1) & 1][me] = nw;
        }
    }
    if (!commit_only) {
        unsigned long long c = wave_sum_u64((unsigned long long)__popcll(nw));
        if (lane() == 0 && c) atomicAdd(&a.stats[(size_t)level * a.stats_groups + g], c);
    }
}

// Transpose of a 64 x 64 bit matrix held one row per lane: afterwards lane j
// holds column j (bit i = old bit j of lane i).
__device__ __forceinline__ uint64_t transpose64(uint64_t x)
{
    const int l = lane();
    const uint64_t M[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                           0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int s = 32 >> k;
        const uint64_t y = __shfl_xor(x, s, GM_WAVE);
        if ((l & s) == 0) x = (x & M[k]) | ((y & M[k]) << s);
        else x = (x & ~M[k]) | ((y & ~M[k]) >> s);
    }
    return x;
}

// 8 bits -> 8 bytes holding 0 or 1, bit i in byte i.
__device__ __forceinline__ uint64_t spread8(uint64_t bits8)
{
    uint64_t t = (bits8 & 0xFFull) * 0x0101010101010101ull;
    t &= 0x8040201008040201ull;
    t = ((t + 0x7F7F7F7F7F7F7F7Full) & 0x8080808080808080ull) >> 7;
    return t;
}

// Block: kHopWaves waves on one (group, word); each wave walks vertex tiles of
// 64.  Lane j ends with the hop bytes of slot (group, word, j) for the tile.
__global__ void __launch_bounds__(kHopWaves * GM_WAVE)
msbfs_hops_kernel(MsbfsArgs a, int planes_used, uint8_t *__restrict__ hop_out,
                  const int64_t *__restrict__ slot_row, int64_t row_stride,
                  unsigned int *__restrict__ lvl_cnt)
{
    __shared__ unsigned int red[kHopWaves][kCountLevels][GM_WAVE];
    const int wid = threadIdx.x / GM_WAVE, l = lane();
    const int32_t gw = blockIdx.y;                 // group * words + word
    const int32_t g = gw / a.words, w = gw % a.words;
    const int lw = __ffs(a.words) - 1;
    const int32_t local_slot = g * 64 * a.words + 64 * w + l;
    const bool slot_ok = local_slot < a.n_slots;
    const int64_t row = slot_ok ? slot_row[local_slot] : 0;
    const int32_t ntiles = (a.n + 63) / 64;
    const size_t gbase = (size_t)g * a.n * a.words + w;
    unsigned int cnt[kCountLevels];
#pragma unroll
    for (int h = 0; h < kCountLevels; ++h) cnt[h] = 0;

    const int32_t t0 = blockIdx.x * (kHopWaves * kHopTilesPerWave);
    for (int it = 0; it < kHopTilesPerWave; ++it) {
        const int32_t tile = t0 + it * kHopWaves + wid;
        if (tile >= ntiles) break;
        const int32_t v0 = tile * 64;
        const int32_t v = v0 + l;
        const size_t me = gbase + ((size_t)v << lw);
        uint64_t vis = v < a.n ? a.visited[me] : 0ull;
        uint64_t pl[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) pl[b] = (b < planes_used && v < a.n) ? a.planes[(size_t)b * a.plane_stride + me] : 0ull;
        vis = transpose64(vis);
#pragma unroll
        for (int b = 0; b < 8; ++b)
            if (b < planes_used) pl[b] = transpose64(pl[b]);
        // counts of vertices at hops 1..16 (planes 5.. must be clear)
        uint64_t high = 0;
#pragma unroll
        for (int b = 5; b < 8; ++b) high |= pl[b];
        const uint64_t low_ok = vis & ~high;
#pragma unroll
        for (int h = 1; h <= kCountLevels; ++h) {
            uint64_t m = low_ok;
#pragma unroll
            for (int b = 0; b < 5; ++b) m &= ((h >> b) & 1) ? pl[b] : ~pl[b];
            cnt[h - 1] += __popcll(m);
        }
        if (slot_ok) {
            uint8_t *dst = hop_out + row * row_stride + v0;
            const int valid = min(64, a.n - v0);
            uint64_t outw[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                uint64_t by = spread8(~vis >> (8 * c)) * 0xFFull;
#pragma unroll
                for (int b = 0; b < 8; ++b) by |= spread8(pl[b] >> (8 * c)) << b;
                outw[c] = by;
            }
            if (valid == 64 && (((uintptr_t)dst) & 15) == 0) {
                uint4 *d4 = (uint4 *)dst;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    uint4 q;
                    q.x = (uint32_t)outw[2 * c];
                    q.y = (uint32_t)(outw[2 * c] >> 32);
                    q.z = (uint32_t)outw[2 * c + 1];
                    q.w = (uint32_t)(outw[2 * c + 1] >> 32);
                    d4[c] = q;
                }
            } else {
                for (int i = 0; i < valid; ++i) dst[i] = (uint8_t)(outw[i >> 3] >> (8 * (i & 7)));
            }
        }
    }
    if (lvl_cnt) {
#pragma unroll
        for (int h = 0; h < kCountLevels; ++h) red[wid][h][l] = cnt[h];
        __syncthreads();
        if (wid == 0 && slot_ok) {
            for (int h = 0; h < kCountLevels; ++h) {
                unsigned int s = 0;
                for (int q = 0; q < kHopWaves; ++q) s += red[q][h][l];
                if (s) atomicAdd(&lvl_cnt[(size_t)local_slot * kCountLevels + h], s);
            }
        }
    }
}

}  // namespace

hipError_t launch_msbfs_init(const MsbfsArgs &a, hipStream_t s)
{
    if (a.n_slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(msbfs_init_kernel, dim3((a.n_slots + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_msbfs_level(const MsbfsArgs &a, int level, bool commit_only, hipStream_t s)
{
    const int64_t items = (int64_t)a.n * a.words;
    dim3 grid((unsigned)((items + kLevelBlock - 1) / kLevelBlock), (unsigned)a.groups);
    hipLaunchKernelGGL(msbfs_level_kernel, grid, dim3(kLevelBlock), 0, s, a, level, commit_only ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_msbfs_hops_counted(const MsbfsArgs &a, int planes_used, uint8_t *hop_out,
                                     const int64_t *slot_row, int64_t row_stride,
                                     unsigned int *lvl_cnt, hipStream_t s)
{
    const int32_t ntiles = (a.n + 63) / 64;
    const int32_t per_block = kHopWaves * kHopTilesPerWave;
    dim3 grid((unsigned)((ntiles + per_block - 1) / per_block), (unsigned)(a.groups * a.words));
    hipLaunchKernelGGL(msbfs_hops_kernel, grid, dim3(kHopWaves * GM_WAVE), 0, s, a, planes_used,
                       hop_out, slot_row, row_stride, lvl_cnt);
    return hipGetLastError();
}

hipError_t launch_msbfs_hops(const MsbfsArgs &a, int planes_used, uint8_t *hop_out,
                             const int64_t *slot_row, int64_t row_stride, hipStream_t s)
{
    return launch_msbfs_hops_counted(a, planes_used, hop_out, slot_row, row_stride, nullptr, s);
}

}  // namespace gm
