// primitives.h -- device-wide building blocks on gfx950 (64-lane wavefronts):
//   * exclusive / inclusive prefix scan of u32 / u64 arrays in one launch (LDS-staged tiles,
//     decoupled look-back between tiles)
//   * stable LSD radix sort of 64-bit keys with a u32 payload, 9-bit digits: one histogram
//     launch for all passes, then one single-sweep launch per digit; digit ranks from
//     wavefront ballots ("match" of equal digits) and LDS counters.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccmc {

constexpr int kThreads = 256;           // 4 wavefronts of 64
constexpr int kWaves = kThreads / 64;
constexpr int kScanItems = 8;           // items per thread in scans
constexpr int kScanTile = kThreads * kScanItems;
constexpr int kSortItems = 8;           // keys per thread of a radix tile
constexpr int kSortTile = kThreads * kSortItems;
constexpr int kRadixBits = 9;           // digit width of the radix sort
constexpr int kRadixBins = 1 << kRadixBits;

// ------------------------------------------------------------------ batched launches
// One launch serves the states of a batch: state s owns the blocks [off[s], off[s+1]) and
// reads its arguments from args[s].  Each kernel's body sees its block index within its state
// (blk) and its state's block count (nblk) in place of blockIdx.x and gridDim.x.  Every kernel
// also has a one-state form that takes its arguments by value: no argument table to copy to
// the device before the launches, and the pointers in the arguments are known to be global.
struct BatchMap {
    const uint32_t *off;  // n + 1 entries, off[0] = 0
    uint32_t n;
};

__device__ __forceinline__ uint32_t batch_state(const BatchMap &bm, uint32_t &blk, uint32_t &nblk)
{
    uint32_t lo = 0, hi = bm.n;  // last s with off[s] <= blockIdx.x
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (bm.off[mid] <= blockIdx.x)
            lo = mid;
        else
            hi = mid;
    }
    blk = blockIdx.x - bm.off[lo];
    nblk = bm.off[lo + 1] - bm.off[lo];
    return lo;
}

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

// Sum over a block of NW wavefronts (fixed order: lanes by shuffle tree, then waves 0..NW-1).
template <typename V, int NW = kWaves>
__device__ __forceinline__ V block_reduce_sum(V v)
{
    __shared__ V wave_tot[NW];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane_id() == 0) wave_tot[wave_id()] = v;
    __syncthreads();
    V all = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) all += wave_tot[w];
    __syncthreads();
    return all;
}

// -------------------------------------------------------------------------- scan
// Scans read their input through a source functor: a plain array, or a transform of
// another array (the selection weights are formed while being scanned).
// check(v) sees every loaded value once all loads of the tile are in flight.
template <typename V>
struct ArraySrc {
    const V *p;
    __device__ __forceinline__ V operator()(uint64_t i) const { return p[i]; }
    __device__ __forceinline__ void check(V) const {}
};

// n counts followed by a closing zero (scanned over n + 1 entries, so that the total lands
// at index n of the exclusive output).
template <typename V>
struct CountSrc {
    const V *p;
    uint64_t n;
    __device__ __forceinline__ V operator()(uint64_t i) const
    {
        const V v = p[i < n ? i : 0];  // unconditional load
        return i < n ? v : V(0);
    }
    __device__ __forceinline__ void check(V) const {}
};

// ------------------------------------------------------- single-pass scans and sorts
// Decoupled look-back (a tile publishes its total, then sums its predecessors' published
// totals until one carries an inclusive prefix).  Each status word holds a 2-bit flag and a
// 62-bit value, so relaxed agent-scope atomics suffice: release / acquire would write back
// or invalidate the XCD's whole L2 at every publish and poll.  Tiles are taken in ticket
// order, so every tile waited on belongs to a block that is already running.  The status
// words must be zero before the launch.
constexpr uint64_t kLbAggregate = 1ull << 62, kLbInclusive = 2ull << 62, kLbValue = (1ull << 62) - 1;

__device__ __forceinline__ void lb_publish(uint64_t *w, uint64_t flag, uint64_t v)
{
    __hip_atomic_store(w, flag | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of tile t from its predecessors' status words, by one wavefront.
__device__ __forceinline__ uint64_t lb_wave_lookback(uint64_t *status, uint64_t t)
{
    const int lane = lane_id();
    uint64_t excl = 0;
    int64_t base = (int64_t)t - 1;
    while (base >= 0) {
        const int64_t p = base - lane;
        const uint64_t w = p >= 0 ? __hip_atomic_load(&status[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kLbInclusive;
        const uint64_t flag = w & ~kLbValue;
        const uint64_t incl = __ballot(flag == kLbInclusive);
        const uint64_t pend = __ballot(flag == 0);
        const int first = incl ? __ffsll((long long)incl) - 1 : 64;
        const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1ull);
        if (pend & need) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        uint64_t v = lane <= first ? (w & kLbValue) : 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        excl += v;
        if (first < 64) break;
        base -= 64;
    }
    return excl;
}

// Fill dst[b] = v for b in [b0, b1), one range per lane; called by every lane of the wave.
// Short ranges are written by their own lane, long ones by the whole wavefront in turn, so
// that one long range does not serialise the wave.
template <typename D>
__device__ __forceinline__ void wave_fill_ranges(D *__restrict__ dst, uint64_t b0, uint64_t b1, D v)
{
    const bool big = b1 > b0 + 8;
    if (!big)
        for (uint64_t b = b0; b < b1; ++b) dst[b] = v;
    uint64_t m = __ballot(big);
    while (m) {
        const int l = __ffsll((long long)m) - 1;
        m &= m - 1;
        const uint64_t lb0 = __shfl(b0, l, 64), lb1 = __shfl(b1, l, 64);
        const D lv = __shfl(v, l, 64);
        for (uint64_t b = lb0 + (uint64_t)lane_id(); b < lb1; b += 64) dst[b] = lv;
    }
}

// Scan outputs: the array, plus a per-item hook that sees each item's exclusive prefix and
// value (called by every lane, in lockstep over the lane's items).
template <typename V>
struct ArrayOut {
    static constexpr int kItems = kScanItems;  // items per thread of the scan that writes it
    V *p;
    __device__ __forceinline__ void item(uint64_t, V, V, bool) const {}
};

// Single-launch scan of n values (n_tiles = ceil(n / tile) blocks, tile = 256 Out::kItems
// values); the grand total goes to *total when given.
template <typename V, typename Src, typename Out>
__device__ __forceinline__ void scan_lb_body(uint32_t blk, uint32_t nblk, Src in, Out out, uint64_t n, int inclusive,
                                                      uint64_t *__restrict__ status, uint64_t *__restrict__ ticket,
                                                      uint64_t *__restrict__ total)
{
    constexpr int kItems = Out::kItems;
    constexpr int kTile = kThreads * kItems;
    __shared__ V buf[kTile];
    __shared__ uint64_t s_tile, s_prefix;
    if (threadIdx.x == 0) s_tile = atomicAdd((unsigned long long *)ticket, 1ull);
    __syncthreads();
    const uint64_t t = s_tile;
    const uint64_t base = t * kTile;
    V ld[kItems];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        // clamped index: the loads are unconditional and all in flight at once (a guarded
        // load is compiled into a branch that waits for it)
        const uint64_t g = base + (uint64_t)i * kThreads + threadIdx.x;
        const V v = in(g < n ? g : n - 1);
        ld[i] = (g < n) ? v : V(0);
    }
#pragma unroll
    for (int i = 0; i < kItems; ++i) in.check(ld[i]);
#pragma unroll
    for (int i = 0; i < kItems; ++i) buf[i * kThreads + threadIdx.x] = ld[i];
    __syncthreads();
    V loc[kItems];
    V sum = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        loc[i] = buf[threadIdx.x * kItems + i];
        sum += loc[i];
    }
    V tile_total;
    const V excl_in_tile = block_exclusive_scan(sum, &tile_total);
    if (wave_id() == 0) {
        if (lane_id() == 0) lb_publish(&status[t], t == 0 ? kLbInclusive : kLbAggregate, (uint64_t)tile_total);
        const uint64_t prefix = t == 0 ? 0 : lb_wave_lookback(status, t);
        if (lane_id() == 0) {
            if (t > 0) lb_publish(&status[t], kLbInclusive, prefix + (uint64_t)tile_total);
            s_prefix = prefix;
            if (total && base + kTile >= n) *total = prefix + (uint64_t)tile_total;
        }
    }
    __syncthreads();
    V run = excl_in_tile + (V)s_prefix;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const V x = loc[i];
        const uint64_t g = base + (uint64_t)threadIdx.x * kItems + i;
        out.item(g, run, x, g < n);
        buf[threadIdx.x * kItems + i] = inclusive ? run + x : run;
        run += x;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const uint64_t g = base + (uint64_t)i * kThreads + threadIdx.x;
        if (g < n) out.p[g] = buf[i * kThreads + threadIdx.x];
    }
}

template <typename V, typename Src, typename Out>
struct ScanLbArgs {
    Src in;
    Out out;
    uint64_t n;
    int inclusive;
    uint64_t *status;
    uint64_t *ticket;
    uint64_t *total;
};

template <typename V, typename Src, typename Out>
__device__ __forceinline__ void k_scan_lb_entry(const ScanLbArgs<V, Src, Out> &A, uint32_t blk, uint32_t nblk)
{
    scan_lb_body<V, Src, Out>(blk, nblk, A.in, A.out, A.n, A.inclusive, A.status, A.ticket, A.total);
}

template <typename V, typename Src, typename Out>
__global__ void __launch_bounds__(kThreads) k_scan_lb(const ScanLbArgs<V, Src, Out> *__restrict__ args, BatchMap bm)
{
    uint32_t blk, nblk;
    k_scan_lb_entry<V, Src, Out>(args[batch_state(bm, blk, nblk)], blk, nblk);
}

template <typename V, typename Src, typename Out>
__global__ void __launch_bounds__(kThreads) k_scan_lb(const ScanLbArgs<V, Src, Out> A)
{
    k_scan_lb_entry<V, Src, Out>(A, blockIdx.x, gridDim.x);
}

// ----------------------------------------------------------------- radix sort
// Keys are W words in SoA layout (word w of item i at key[w * stride + i]).  One pass sorts
// by the 8-bit digit at bit `shift` of word `word`, stably.

// Digits of equal value among the active lanes of this wave.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active)
{
    uint64_t peers = active;
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const uint64_t m = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? m : ~m;
    }
    return peers;
}

// ------------------------------------------------------------ onesweep radix passes
// Keys are 64-bit, sorted by kRadixBits-bit digits from bit shift0 up (bits below shift0 are
// carried, not sorted on: the sort stays stable in the input order for equal sorted bits).
// Digit histograms of every pass in one read of the keys (they do not depend on the order):
// per-lane LDS atomics, except where a wavefront's digits are all equal (the top digits of
// narrow key ranges), which add once; then one global atomic per non-empty bin and block.
constexpr int kRadixMaxPasses = (64 + kRadixBits - 1) / kRadixBits;
// The histogram launch: each block adds its bins to the global histogram once, and on a large
// input those atomics are what the grid waits on, so large inputs take few fat blocks (NT =
// 1024 threads, at most one per CU); small ones take one 256-thread block per tile, to spread
// over more CUs.
constexpr int kGhistFat = 1024;
constexpr uint64_t kGhistFatFrom = 256;  // radix tiles from which the fat blocks are used
constexpr uint64_t kGhistBlocks = 1024;  // blocks of either kind at most
__host__ __device__ __forceinline__ uint64_t ghist_grid(uint64_t n, int nt)
{
    const uint64_t tile = (uint64_t)nt * kSortItems, t = (n + tile - 1) / tile;
    const uint64_t cap = nt == kGhistFat ? kGhistBlocks / 4 : kGhistBlocks;
    return t < cap ? (t ? t : 1) : cap;
}

template <int NT>
__device__ __forceinline__ void radix_ghist_body(uint32_t blk, uint32_t nblk, const uint64_t *__restrict__ key, const uint64_t *__restrict__ n_live,
                                                          int passes, int shift0, uint32_t *__restrict__ ghist)
{
    const uint64_t n = *n_live;
    __shared__ uint32_t h[kRadixMaxPasses][kRadixBins];
    for (int p = 0; p < passes; ++p)
        for (int d = threadIdx.x; d < kRadixBins; d += NT) h[p][d] = 0;
    __syncthreads();
    // tiles blk, blk + nblk, ...: few blocks, so that few atomics meet on each global bin
    for (uint64_t base = (uint64_t)blk * ((uint64_t)NT * kSortItems); base < n; base += (uint64_t)nblk * ((uint64_t)NT * kSortItems)) {
        uint64_t k[kSortItems];
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const uint64_t g = base + (uint64_t)r * NT + threadIdx.x;
            k[r] = key[g < n ? g : n - 1];  // clamped: unconditional loads
        }
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const uint64_t g = base + (uint64_t)r * NT + threadIdx.x;
            const bool valid = g < n;
            const uint64_t active = __ballot(valid);
            const int leader = active ? __ffsll((long long)active) - 1 : 0;
            for (int p = 0; p < passes; ++p) {
                const int sh = shift0 + kRadixBits * p;  // a batch's extra passes may lie past bit 63
                const uint32_t d = sh < 64 ? (uint32_t)((k[r] >> sh) & (kRadixBins - 1)) : 0u;
                const uint32_t d0 = (uint32_t)__shfl((int)d, leader, 64);
                const bool same = __ballot(valid && d != d0) == 0;  // every active lane holds d0
                if (same) {
                    if (lane_id() == leader && active) atomicAdd(&h[p][d0], (uint32_t)__popcll(active));
                } else if (valid) {
                    atomicAdd(&h[p][d], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int p = 0; p < passes; ++p)
        for (int d = threadIdx.x; d < kRadixBins; d += NT)
            if (h[p][d]) atomicAdd(&ghist[p * kRadixBins + d], h[p][d]);
}

struct RadixGhistArgs {
    const uint64_t *key;
    const uint64_t *n_live;
    int passes;
    int shift0;  // bit of the first digit (the sort key's low bits may carry other data)
    uint32_t *ghist;
};

template <int NT>
__device__ __forceinline__ void k_radix_ghist_entry(const RadixGhistArgs &A, uint32_t blk, uint32_t nblk)
{
    radix_ghist_body<NT>(blk, nblk, A.key, A.n_live, A.passes, A.shift0, A.ghist);
}

template <int NT>
__global__ void __launch_bounds__(NT) k_radix_ghist(const RadixGhistArgs *__restrict__ args, BatchMap bm)
{
    uint32_t blk, nblk;
    k_radix_ghist_entry<NT>(args[batch_state(bm, blk, nblk)], blk, nblk);
}

template <int NT>
__global__ void __launch_bounds__(NT) k_radix_ghist(const RadixGhistArgs A)
{
    k_radix_ghist_entry<NT>(A, blockIdx.x, gridDim.x);
}

// One stable pass by the digit at `shift`, carrying one value of type V per key (the record's
// amplitude in the annihilation sort; an index generated from the input position when
// val_in is null, for the processor partition).  Wavefront w of a tile owns the tile's keys
// [w * 64 * kSortItems, (w + 1) * 64 * kSortItems), 64 per round, and ranks them against its
// own LDS digit counters (no block barrier between rounds: a wavefront's LDS accesses are in
// order).  The tile then combines its wavefronts' counts, publishes its per-digit counts,
// looks back over the earlier tiles digit by digit, and places each key at
// digit base + earlier tiles + earlier wavefronts + rank in its wavefront.  The tile is
// staged in LDS in its sorted order first (keys, then values), so that consecutive lanes
// write consecutive addresses of a digit's run.  status holds kRadixBins words per tile and
// must be zero before the launch.  Thread x also owns the digits x + j * kThreads of the
// per-digit work.
constexpr int kDigitsPerThread = kRadixBins / kThreads;
constexpr int kRadixLbDepth = 4;  // predecessor tiles read per digit and look-back round

template <typename V>
__device__ __forceinline__ void radix_onesweep_body(uint32_t blk, uint32_t nblk, const uint64_t *__restrict__ key_in, const V *__restrict__ idx_in,
                                                             uint64_t *__restrict__ key_out, V *__restrict__ idx_out,
                                                             const uint64_t *__restrict__ n_live, int shift,
                                                             const uint32_t *__restrict__ ghist, uint64_t *__restrict__ status,
                                                             uint64_t *__restrict__ ticket)
{
    __shared__ uint32_t wave_cnt[kWaves][kRadixBins];  // per wavefront: digit counts, then offsets
    __shared__ uint32_t dig_base[kRadixBins];          // output position of the digit's run, less its tile start
    __shared__ uint32_t t_start[kRadixBins];           // the digit's start in the tile's sorted order
    __shared__ uint64_t s_stage[kSortTile];            // the tile in sorted order: keys, then values
    __shared__ uint64_t s_tile;
    const uint64_t n = *n_live;
    if (threadIdx.x == 0) s_tile = atomicAdd((unsigned long long *)ticket, 1ull);
    const int w = wave_id(), lane = lane_id();
#pragma unroll
    for (int j = 0; j < kRadixBins / 64; ++j) wave_cnt[w][lane + 64 * j] = 0;
    __syncthreads();
    const uint64_t t = s_tile;
    const uint64_t base = t * kSortTile;
    if (base >= n) return;  // tiles beyond the live count: nobody waits on them
    const uint64_t wbase = base + (uint64_t)w * 64 * kSortItems;
    uint64_t k[kSortItems];
    V ix[kSortItems];
    uint16_t rk[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {  // all loads in flight before the ranking rounds
        const uint64_t g = wbase + (uint64_t)r * 64 + lane;
        const uint64_t gc = g < n ? g : n - 1;  // clamped: unconditional loads
        k[r] = key_in[gc];
        ix[r] = idx_in ? idx_in[gc] : (V)g;
    }
    uint32_t gh[kDigitsPerThread];  // this thread's digits of the pass histogram
#pragma unroll
    for (int j = 0; j < kDigitsPerThread; ++j) gh[j] = ghist[threadIdx.x + j * kThreads];
    uint32_t *cnt = wave_cnt[w];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint64_t g = wbase + (uint64_t)r * 64 + lane;
        const bool valid = g < n;
        const uint32_t d = shift < 64 ? (uint32_t)((k[r] >> shift) & (kRadixBins - 1)) : 0u;
        const uint64_t active = __ballot(valid);
        uint32_t rank = 0;
        if (valid) {
            const uint64_t peers = match_digit(d, active);
            const uint32_t before = cnt[d];  // read by every peer before the leader's update
            const int below = lanes_below(peers);
            rank = before + (uint32_t)below;
            if (below == 0) cnt[d] = before + (uint32_t)__popcll(peers);
        }
        rk[r] = (uint16_t)rank;
    }
    __syncthreads();
    // per digit: exclusive prefix over the wavefronts, and the tile's count
    uint32_t tile_cnt[kDigitsPerThread];
#pragma unroll
    for (int j = 0; j < kDigitsPerThread; ++j) {
        const int dd = threadIdx.x + j * kThreads;
        uint32_t acc = 0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) {
            const uint32_t c = wave_cnt[ww][dd];
            wave_cnt[ww][dd] = acc;
            acc += c;
        }
        tile_cnt[j] = acc;
    }
    // publish this tile's counts first, so that later tiles' look-backs find them sooner
    uint64_t *st = status + t * kRadixBins;
#pragma unroll
    for (int j = 0; j < kDigitsPerThread; ++j)
        lb_publish(&st[threadIdx.x + j * kThreads], t == 0 ? kLbInclusive : kLbAggregate, tile_cnt[j]);
    // global base of each digit: exclusive prefix of the pass histogram over the digits; and
    // the digit's start in the tile: exclusive prefix of the tile's counts
    // (both in one scan: the histogram in the high half, the tile's counts in the low half,
    // which holds at most kSortTile and never carries; the histogram sums to the live count,
    // below 2^32)
    uint32_t gbase[kDigitsPerThread], tbase[kDigitsPerThread];
    {
        uint64_t carry = 0;
#pragma unroll
        for (int j = 0; j < kDigitsPerThread; ++j) {
            uint64_t tot;
            const uint64_t ex = carry + block_exclusive_scan(((uint64_t)gh[j] << 32) | tile_cnt[j], &tot);
            carry += tot;
            gbase[j] = (uint32_t)(ex >> 32);
            tbase[j] = (uint32_t)ex;
        }
    }
    // sum the earlier tiles' counts (the digit chains of a thread advance together)
    uint64_t excl[kDigitsPerThread];
    int64_t pp[kDigitsPerThread];
#pragma unroll
    for (int j = 0; j < kDigitsPerThread; ++j) {
        excl[j] = 0;
        pp[j] = (int64_t)t - 1;
    }
    for (;;) {
        bool busy = false;
#pragma unroll
        for (int j = 0; j < kDigitsPerThread; ++j) {
            if (pp[j] < 0) continue;
            // kRadixLbDepth predecessors per round, all loads in flight together; consumed
            // nearest first up to the first inclusive word, or up to an unpublished one, from
            // which the next round polls again
            uint64_t sw[kRadixLbDepth];
#pragma unroll
            for (int q = 0; q < kRadixLbDepth; ++q) {
                const int64_t p = pp[j] - q;
                sw[q] = p >= 0 ? __hip_atomic_load(&status[(uint64_t)p * kRadixBins + threadIdx.x + j * kThreads],
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                               : kLbInclusive;
            }
            bool stop = false;
#pragma unroll
            for (int q = 0; q < kRadixLbDepth; ++q) {
                if (stop) continue;
                const uint64_t flag = sw[q] & ~kLbValue;
                if (flag == 0) {
                    stop = true;  // not published yet: poll again from this tile
                    continue;
                }
                excl[j] += sw[q] & kLbValue;
                if (flag == kLbInclusive) {
                    pp[j] = -1;
                    stop = true;
                } else {
                    pp[j] -= 1;
                }
            }
            busy |= pp[j] >= 0;
        }
        if (!busy) break;
    }
#pragma unroll
    for (int j = 0; j < kDigitsPerThread; ++j) {
        const int d = threadIdx.x + j * kThreads;
        if (t > 0) lb_publish(&st[d], kLbInclusive, excl[j] + tile_cnt[j]);
        dig_base[d] = gbase[j] + (uint32_t)excl[j] - tbase[j];
        t_start[d] = tbase[j];
    }
    __syncthreads();
    // position of each key in the tile's sorted order; the keys staged there
    uint32_t lp[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint64_t g = wbase + (uint64_t)r * 64 + lane;
        const uint32_t d = shift < 64 ? (uint32_t)((k[r] >> shift) & (kRadixBins - 1)) : 0u;
        lp[r] = t_start[d] + wave_cnt[w][d] + rk[r];
        if (g < n) s_stage[lp[r]] = k[r];
    }
    __syncthreads();
    const uint32_t tn = n - base < (uint64_t)kSortTile ? (uint32_t)(n - base) : (uint32_t)kSortTile;
    uint32_t dst[kSortItems];  // output position of sorted slot threadIdx.x + m * kThreads
#pragma unroll
    for (int m = 0; m < kSortItems; ++m) {
        const uint32_t i = threadIdx.x + (uint32_t)m * kThreads;
        dst[m] = 0;
        if (i < tn) {
            const uint64_t key = s_stage[i];
            const uint32_t d = shift < 64 ? (uint32_t)((key >> shift) & (kRadixBins - 1)) : 0u;
            dst[m] = dig_base[d] + i;
            key_out[dst[m]] = key;
        }
    }
    __syncthreads();  // the keys are read: the stage takes the values
    V *sv = reinterpret_cast<V *>(s_stage);
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint64_t g = wbase + (uint64_t)r * 64 + lane;
        if (g < n) sv[lp[r]] = ix[r];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kSortItems; ++m) {
        const uint32_t i = threadIdx.x + (uint32_t)m * kThreads;
        if (i < tn) idx_out[dst[m]] = sv[i];
    }
}

template <typename V>
struct RadixOnesweepArgs {
    const uint64_t *key_in;
    const V *idx_in;
    uint64_t *key_out;
    V *idx_out;
    const uint64_t *n_live;
    int shift;
    const uint32_t *ghist;
    uint64_t *status;
    uint64_t *ticket;
};

template <typename V>
__device__ __forceinline__ void k_radix_onesweep_entry(const RadixOnesweepArgs<V> &A, uint32_t blk, uint32_t nblk)
{
    radix_onesweep_body<V>(blk, nblk, A.key_in, A.idx_in, A.key_out, A.idx_out, A.n_live, A.shift, A.ghist, A.status, A.ticket);
}

template <typename V>
__global__ void __launch_bounds__(kThreads) k_radix_onesweep(const RadixOnesweepArgs<V> *__restrict__ args, BatchMap bm)
{
    uint32_t blk, nblk;
    k_radix_onesweep_entry<V>(args[batch_state(bm, blk, nblk)], blk, nblk);
}

template <typename V>
__global__ void __launch_bounds__(kThreads) k_radix_onesweep(const RadixOnesweepArgs<V> A)
{
    k_radix_onesweep_entry<V>(A, blockIdx.x, gridDim.x);
}

}  // namespace ccmc
