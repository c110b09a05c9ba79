// primitives.h -- device-wide building blocks on gfx950 (64-lane wavefronts):
//   * exclusive / inclusive prefix scan of u32 / u64 arrays (reduce-then-scan, LDS staged)
//   * stable LSD radix sort of multi-word bitstring keys with a u32 payload, 8-bit digits,
//     digit ranks from wavefront ballots ("match" of equal digits) and LDS counters.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccmc {

constexpr int kThreads = 256;           // 4 wavefronts of 64
constexpr int kWaves = kThreads / 64;
constexpr int kScanItems = 8;           // items per thread in scans
constexpr int kScanTile = kThreads * kScanItems;
constexpr int kSortItems = 8;           // rounds of 256 keys per radix tile
constexpr int kSortTile = kThreads * kSortItems;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x >> 6); }

// number of set bits of m below this lane
__device__ __forceinline__ int lanes_below(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename V>
__device__ __forceinline__ V wave_inclusive_scan(V v)
{
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const V t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total in *total.
template <typename V>
__device__ __forceinline__ V block_exclusive_scan(V v, V *total)
{
    __shared__ V wave_tot[kWaves];
    const V inc = wave_inclusive_scan(v);
    if (lane_id() == 63) wave_tot[wave_id()] = inc;
    __syncthreads();
    V before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        if (w < wave_id()) before += wave_tot[w];
        all += wave_tot[w];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

template <typename V>
__device__ __forceinline__ V block_reduce_sum(V v)
{
    __shared__ V wave_tot[kWaves];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane_id() == 0) wave_tot[wave_id()] = v;
    __syncthreads();
    V all = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) all += wave_tot[w];
    __syncthreads();
    return all;
}

// -------------------------------------------------------------------------- scan
// Scans read their input through a source functor: a plain array, or a transform of
// another array (the selection weights are formed while being scanned).
template <typename V>
struct ArraySrc {
    const V *p;
    __device__ __forceinline__ V operator()(uint64_t i) const { return p[i]; }
};

template <typename V, typename Src>
__global__ void __launch_bounds__(kThreads) k_scan_reduce(Src in, uint64_t n, V *__restrict__ part)
{
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    V s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const uint64_t g = base + (uint64_t)i * kThreads + threadIdx.x;
        if (g < n) s += in(g);
    }
    s = block_reduce_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Scan of one tile, staged through LDS so that global loads and stores stay coalesced
// while each thread scans kScanItems consecutive values.
template <typename V, typename Src>
__global__ void __launch_bounds__(kThreads) k_scan_tile(Src in, V *__restrict__ out, uint64_t n,
                                                        const V *__restrict__ tile_offset, int inclusive)
{
    __shared__ V buf[kScanTile];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const uint64_t g = base + (uint64_t)i * kThreads + threadIdx.x;
        buf[i * kThreads + threadIdx.x] = (g < n) ? in(g) : V(0);
    }
    __syncthreads();
    V loc[kScanItems];
    V sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        loc[i] = buf[threadIdx.x * kScanItems + i];
        sum += loc[i];
    }
    V total;
    V run = block_exclusive_scan(sum, &total) + (tile_offset ? tile_offset[blockIdx.x] : V(0));
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const V x = loc[i];
        buf[threadIdx.x * kScanItems + i] = inclusive ? run + x : run;
        run += x;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const uint64_t g = base + (uint64_t)i * kThreads + threadIdx.x;
        if (g < n) out[g] = buf[i * kThreads + threadIdx.x];
    }
}

// One block scans up to a few tiles in sequence, carrying the running total: one launch
// instead of three for the small scans of a step (radix histograms, flags of short lists).
template <typename V, typename Src>
__global__ void __launch_bounds__(kThreads) k_scan_small(Src in, V *__restrict__ out, uint64_t n, int inclusive)
{
    __shared__ V buf[kScanTile];
    V carry = 0;
    for (uint64_t base = 0; base < n; base += kScanTile) {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint64_t g = base + (uint64_t)i * kThreads + threadIdx.x;
            buf[i * kThreads + threadIdx.x] = (g < n) ? in(g) : V(0);
        }
        __syncthreads();
        V loc[kScanItems];
        V sum = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            loc[i] = buf[threadIdx.x * kScanItems + i];
            sum += loc[i];
        }
        V total;
        V run = block_exclusive_scan(sum, &total) + carry;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const V x = loc[i];
            buf[threadIdx.x * kScanItems + i] = inclusive ? run + x : run;
            run += x;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint64_t g = base + (uint64_t)i * kThreads + threadIdx.x;
            if (g < n) out[g] = buf[i * kThreads + threadIdx.x];
        }
        carry += total;
        __syncthreads();
    }
}

// ----------------------------------------------------------------- radix sort
// Keys are W words in SoA layout (word w of item i at key[w * stride + i]).  One pass sorts
// by the 8-bit digit at bit `shift` of word `word`, stably.

// Digits of equal value among the active lanes of this wave.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active)
{
    uint64_t peers = active;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint64_t m = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? m : ~m;
    }
    return peers;
}

// The live item count is read from device memory (*n_live); the grid covers a capacity and
// tiles beyond the count contribute empty histograms.
template <int W>
__global__ void __launch_bounds__(kThreads) k_radix_hist(const uint64_t *__restrict__ key, uint64_t stride,
                                                         const uint64_t *__restrict__ n_live, int word, int shift,
                                                         uint32_t *__restrict__ hist, uint32_t n_tiles)
{
    const uint64_t n = *n_live;
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    const uint64_t *kw = key + (uint64_t)word * stride;
    for (int r = 0; r < kSortItems; ++r) {
        const uint64_t g = base + (uint64_t)r * kThreads + threadIdx.x;
        const bool valid = g < n;
        const uint32_t d = valid ? (uint32_t)((kw[g] >> shift) & 0xFFu) : 0u;
        const uint64_t active = __ballot(valid);
        if (valid) {
            const uint64_t peers = match_digit(d, active);
            if (lanes_below(peers) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
        }
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: rank of an item = global digit offset of this tile + items of the same
// digit in earlier rounds + in earlier waves of this round + in lower lanes of this wave.
template <int W>
__global__ void __launch_bounds__(kThreads) k_radix_scatter(const uint64_t *__restrict__ key_in, const uint32_t *__restrict__ idx_in,
                                                            uint64_t *__restrict__ key_out, uint32_t *__restrict__ idx_out,
                                                            uint64_t stride, const uint64_t *__restrict__ n_live, int word,
                                                            int shift, const uint32_t *__restrict__ offsets, uint32_t n_tiles)
{
    const uint64_t n = *n_live;
    if ((uint64_t)blockIdx.x * kSortTile >= n) return;  // empty tile (uniform per block)
    __shared__ uint32_t run[256];
    __shared__ uint32_t wave_cnt[kWaves][256];
    run[threadIdx.x] = offsets[(uint64_t)threadIdx.x * n_tiles + blockIdx.x];
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    const uint64_t *kw = key_in + (uint64_t)word * stride;
    for (int r = 0; r < kSortItems; ++r) {
#pragma unroll
        for (int w = 0; w < kWaves; ++w) wave_cnt[w][threadIdx.x] = 0;
        __syncthreads();
        const uint64_t g = base + (uint64_t)r * kThreads + threadIdx.x;
        const bool valid = g < n;
        const uint32_t d = valid ? (uint32_t)((kw[g] >> shift) & 0xFFu) : 0u;
        const uint64_t active = __ballot(valid);
        uint64_t peers = 0;
        int rank = 0;
        if (valid) {
            peers = match_digit(d, active);
            rank = lanes_below(peers);
            if (rank == 0) wave_cnt[wave_id()][d] = (uint32_t)__popcll(peers);
        }
        __syncthreads();
        {
            // per digit: exclusive prefix over waves, then advance the running offset
            const int dd = threadIdx.x;
            uint32_t acc = run[dd];
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = wave_cnt[w][dd];
                wave_cnt[w][dd] = acc;
                acc += c;
            }
            run[dd] = acc;
        }
        __syncthreads();
        if (valid) {
            const uint32_t dst = wave_cnt[wave_id()][d] + (uint32_t)rank;
#pragma unroll
            for (int w = 0; w < W; ++w) key_out[(uint64_t)w * stride + dst] = key_in[(uint64_t)w * stride + g];
            idx_out[dst] = idx_in ? idx_in[g] : (uint32_t)g;
        }
        __syncthreads();
    }
}

}  // namespace ccmc
