// kernels.h -- the CCMC time-step kernels (Spencer et al., arXiv:1807.03749, Sec. II & IV).
//
// One step, in launch order (scans are single launches with decoupled look-back):
//   k_fill           clear the step scalars and look-back status words
//   weights scan     fixed-point selection weights q_i and their prefix          (a1)
//   k_guide          bucket table of the prefix for the excitor draws           (a2)
//   k_items          non-composite items (FNC): reference + every excitor        (a4, a5, a9, a10)
//                    and sampled clusters: size, excitor draws, collapse, amplitude  (a2, a3, a4, a9, a10)
//   slot scan        record slots per item (1 death + n attempts), first item per block
//   k_generate       one lane per record slot: death or spawning attempt        (a6, a7, a8)
//   region scan      records per generation block
//   k_gather         dense records and their truncated-space rank               (a8)
//   radix sort       stable LSD sort of (rank | position, amplitude)            (a11)
//   k_seg_fold       sum of each run in record order, store lookup, new         (a12)
//                    determinants numbered by look-back; k_seg_close for runs across tiles
//   k_merge          merge, occupation rounding and compaction into the other    (a12, a13)
//                    store buffer (look-back for the output positions)
//   k_final_part     FP64 population, projected-energy and count reductions    (a14)
#pragma once
#include "device.h"
#include "primitives.h"

namespace ccmc {

constexpr int kGenRounds = 4;                       // rounds of 256 slots per generation block
constexpr int kGenSlots = kThreads * kGenRounds;    // slots (and region capacity) per block

constexpr uint64_t kErrBlowup = 1, kErrAttempts = 2, kErrSlotCap = 4, kErrRecCap = 8;

// Device-side scalars of one step (all 64-bit words, cleared at the start of the step).
struct Scratch {
    uint64_t qtot;
    uint64_t err;             // kErr* bits; any bit fails the step (the current store is left as it was)
    uint64_t n_discarded;
    uint64_t n_attempts;
    uint64_t n_spawns;
    uint64_t n_deaths;
    uint64_t max_n;
    uint64_t n_slots;         // record slots of the step (deaths + attempts)
    uint64_t n_rec;           // records emitted by the step
    uint64_t n_live;          // records the annihilation works on (0 after an overflow)
    uint64_t n_place;         // excitors partitioned by virtual processor (the store size)
    uint64_t seq;             // host copy only: the batch's sequence number, written last
    uint64_t n_new;           // new determinants
    uint64_t hf_hit;
    uint64_t n_out;           // excitors after the step
    double hf_sum;
    double n_total;
    double num;
};

struct StepArgs {
    double tau, shift;
    double cutoff, theta;
    double thr_cluster, thr_nc;
    uint32_t kmin;
    uint32_t step;            // t & 0x0FFFFFFF
    uint32_t key0, key1;
    uint64_t n_sel;
    int fnc;
    uint32_t gsh;             // shift of the selection guide
    uint64_t gcap;            // entries of the selection guide
    uint32_t n_ranks;         // virtual processors (1: none)
};

// The store partitioned by virtual processor: perm[j] is the store index at position j of
// the partition (processors in order, store order within each) and processor r holds
// positions [seg[r], seg[r + 1]).  Unused with one processor.
struct Ranks {
    const uint32_t *perm;
    const uint32_t *seg;
};

// Per-block partial statistics of the item kernels, reduced by k_final_part.
struct ItemPartials {
    double *num;       // projected-energy numerator
    uint64_t *att;     // spawning attempts
    uint64_t *disc;    // discarded selections
    uint64_t *maxn;    // largest attempt count
};

// A block's four partials in one exchange: the shuffle tree of block_reduce_sum within each
// wavefront (the same order, so the same sums), then thread 0 adds the wavefronts in order and
// writes the block's entry.
__device__ __forceinline__ void store_item_partials(double num, uint64_t att, uint64_t disc, uint64_t mx, ItemPartials part,
                                                    uint32_t blk)
{
    __shared__ double s_num[kWaves];
    __shared__ uint64_t s_att[kWaves], s_disc[kWaves], s_mx[kWaves];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        num += __shfl_down(num, o, 64);
        att += __shfl_down(att, o, 64);
        disc += __shfl_down(disc, o, 64);
        const uint64_t m = __shfl_down(mx, o, 64);
        mx = m > mx ? m : mx;
    }
    if (lane_id() == 0) {
        s_num[wave_id()] = num;
        s_att[wave_id()] = att;
        s_disc[wave_id()] = disc;
        s_mx[wave_id()] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double n = 0.0;
        uint64_t a = 0, d = 0, m = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            n += s_num[w];
            a += s_att[w];
            d += s_disc[w];
            m = s_mx[w] > m ? s_mx[w] : m;
        }
        part.num[blk] = n;
        part.att[blk] = a;
        part.disc[blk] = d;
        part.maxn[blk] = m;
    }
}

template <typename V, int NW = kWaves>
__device__ __forceinline__ V block_reduce_max(V v)
{
    __shared__ V wave_max[NW];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const V o = __shfl_down(v, off, 64);
        v = o > v ? o : v;
    }
    if (lane_id() == 0) wave_max[wave_id()] = v;
    __syncthreads();
    V m = wave_max[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) m = wave_max[w] > m ? wave_max[w] : m;
    __syncthreads();
    return m;
}

// Items: one per cluster that may emit records.  SoA key layout with stride `stride`.
template <typename T>
struct Items {
    uint64_t *key;
    T *A;
    T *death;      // death amount -tau (K - S) A, 0 when none
    uint32_t *n;   // spawning attempts
    uint64_t *cnt; // record slots: n + 1 (slot 0 = death), 0 when discarded; a discarded
                   // item's other fields are not written (nothing reads an item without slots)
    uint64_t stride;
};

template <typename T>
__device__ __forceinline__ uint32_t attempt_count(T A, double thr, uint32_t kmin, uint64_t *err)
{
    uint32_t k = kmin;
    if (thr > 0) {
        const double f = floor(fabs((double)A) / thr);
        if (!(f <= (double)kMaxAttempts)) {
            atomicOr((unsigned long long *)err, (unsigned long long)kErrAttempts);
            return kMaxAttempts;
        }
        if ((uint32_t)f > k) k = (uint32_t)f;
    }
    return k;
}

// ------------------------------------------------------------------------ weights
// q_i = max(1, rint(|N_i| 2^24)), formed while the inclusive prefix P is scanned: the prefix
// is exact, so the excitor drawn for a given random number does not depend on the
// summation order (Sec. II: probability |t_i| / (N_tot - t_HF)).
constexpr uint64_t kWeightCap = 1ull << 52;  // |N_i| >= 2^28 (or NaN) is a blow-up

__device__ __forceinline__ uint64_t weight_of(double amp)
{
    double w = rint(fabs(amp) * 16777216.0);
    w = w < 1.0 ? 1.0 : w;
    return (uint64_t)fmin(w, (double)kWeightCap);  // NaN -> kWeightCap
}

template <typename T>
struct WeightSrc {
    const T *amp;
    Scratch *sc;
    const uint32_t *perm;  // weights in the order of the processor partition, or store order
    static constexpr uint64_t kCap = kWeightCap;
    __device__ __forceinline__ uint64_t operator()(uint64_t i) const { return weight_of((double)amp[perm ? perm[i] : i]); }
    __device__ __forceinline__ void check(uint64_t q) const
    {
        if (q >= kCap) atomicOr((unsigned long long *)&sc->err, (unsigned long long)kErrBlowup);
    }
};

// The guide of the excitor draws, one lane per excitor g (exclusive prefix lo = P[g-1],
// inclusive prefix hi = P[g]): a draw x in [0, Q) falls in bucket x >> gsh, and guide[b] is the
// first excitor whose prefix exceeds b << gsh, so the drawn excitor lies in
// [guide[b], guide[b+1]] -- a short search instead of one over the whole store.  Excitor g
// owns the buckets with lo <= b << gsh < hi (a large amplitude owns many: its wavefront writes
// them together); the last one also owns the two closing buckets.  The shift comes from the
// host (from the previous step's Q), so buckets past the capacity gcap may exist: draws there
// search from guide[gcap - 1] to the end.
//
// The same lanes write each excitor's draw record: everything a draw of it reads, in one
// place -- its inclusive prefix, its amplitude (the bits of T in the low bytes of a 64-bit
// word) and its bitstring (W words) -- so that a draw, after the guide, touches one or two
// lines instead of one per array.  Records follow the order of the prefix (the processor
// partition's, or the store's).
struct DrawRecs {
    uint64_t *rec;
    uint32_t stride;  // 64-bit words per record: 2 + W
};

template <typename T>
__device__ __forceinline__ T rec_amp(uint64_t bits)
{
    if constexpr (sizeof(T) == 8) {
        return __longlong_as_double((long long)bits);
    } else {
        return __int_as_float((int)(uint32_t)bits);
    }
}

struct GuideArgs {
    const uint64_t *P;
    uint32_t *guide;
    uint64_t gcap;
    uint32_t gsh;
    uint64_t n;
    // virtual processors: the sorted processor of each partition position, and the segment
    // starts to fill (seg[r] = first position whose processor is at least r, r <= n_ranks)
    const uint64_t *vsorted;
    uint32_t *seg;
    uint32_t n_ranks;
    // the draw records: store columns to copy (through perm in partition order)
    const void *amp;
    int amp8;  // amplitudes of 8 bytes (else 4)
    const uint64_t *skey;
    uint64_t sstride;
    int words;
    const uint32_t *perm;
    DrawRecs dr;
};

__device__ __forceinline__ void k_guide_entry(const GuideArgs &A, uint32_t blk, uint32_t nblk)
{
    const uint64_t g = (uint64_t)blk * kThreads + threadIdx.x;
    uint64_t b0 = 0, b1 = 0;
    if (g < A.n) {
        const uint64_t src = A.perm ? A.perm[g] : g;
        uint64_t *r = A.dr.rec + g * A.dr.stride;
        r[0] = A.P[g];
        r[1] = A.amp8 ? static_cast<const uint64_t *>(A.amp)[src] : (uint64_t) static_cast<const uint32_t *>(A.amp)[src];
        for (int w = 0; w < A.words; ++w) r[2 + w] = A.skey[(uint64_t)w * A.sstride + src];
    }
    if (g < A.n) {
        const uint64_t unit = 1ull << A.gsh, lo = g ? A.P[g - 1] : 0, hi = A.P[g];
        b0 = (lo + unit - 1) >> A.gsh;
        b1 = g + 1 == A.n ? (hi >> A.gsh) + 2 : (hi + unit - 1) >> A.gsh;
        b1 = b1 < A.gcap ? b1 : A.gcap;
        b0 = b0 < b1 ? b0 : b1;
    }
    wave_fill_ranges<uint32_t>(A.guide, b0, b1, (uint32_t)g);
    if (A.n_ranks > 1) {
        uint64_t r0 = 0, r1 = 0, e0 = 0, e1 = 0;
        if (g < A.n) {
            const uint64_t r = A.vsorted[g];
            r0 = g ? A.vsorted[g - 1] + 1 : 0;  // processors (previous, r] start at g
            r1 = r + 1;
            if (g + 1 == A.n) {  // processors after the last one start at n
                e0 = r + 1;
                e1 = (uint64_t)A.n_ranks + 1;
            }
        }
        wave_fill_ranges<uint32_t>(A.seg, r0, r1, (uint32_t)g);
        wave_fill_ranges<uint32_t>(A.seg, e0, e1, (uint32_t)A.n);
    }
}

__global__ void __launch_bounds__(kThreads) k_guide(const GuideArgs *__restrict__ args, BatchMap bm)
{
    uint32_t blk, nblk;
    k_guide_entry(args[batch_state(bm, blk, nblk)], blk, nblk);
}

__global__ void __launch_bounds__(kThreads) k_guide(const GuideArgs A)
{
    k_guide_entry(A, blockIdx.x, gridDim.x);
}

// Processor of every store entry this step (eq. 9), as the key of the one-pass radix
// partition; also the partition's length for the radix kernels.
template <int W>
struct PlaceArgs {
    const uint64_t *key;
    uint64_t stride;
    uint64_t ne;
    uint64_t i_tau;
    uint32_t n_ranks, move_shift, seed;
    uint64_t *vkey;
    Scratch *sc;
};

template <int W>
__device__ __forceinline__ void k_place_entry(const PlaceArgs<W> &A, uint32_t blk, uint32_t nblk)
{
    const uint64_t i = (uint64_t)blk * kThreads + threadIdx.x;
    if (i == 0) A.sc->n_place = A.ne;
    if (i >= A.ne) return;
    uint64_t d[W];
#pragma unroll
    for (int w = 0; w < W; ++w) d[w] = A.key[(uint64_t)w * A.stride + i];
    A.vkey[i] = placement<W>(d, A.i_tau, A.n_ranks, A.move_shift, A.seed);
}

template <int W>
__global__ void __launch_bounds__(kThreads) k_place(const PlaceArgs<W> *__restrict__ args, BatchMap bm)
{
    uint32_t blk, nblk;
    k_place_entry<W>(args[batch_state(bm, blk, nblk)], blk, nblk);
}

template <int W>
__global__ void __launch_bounds__(kThreads) k_place(const PlaceArgs<W> A)
{
    k_place_entry<W>(A, blockIdx.x, gridDim.x);
}

// The index of the store lookups, in two levels.  The fence holds every fs-th rank of the
// sorted store, fence[k] = rank[k fs] (k < nf): with fs = kFence a run of fs consecutive ranks
// is one 128-byte line; a store small enough to stay in the cache takes fs = 1 (the fence is the
// ranks themselves, and the lookup skips its second level).  The rank table
// rtab[c] = first k with fence[k] >= c << rsh (c < rt_n) narrows the fence search for a rank r
// to k in [rtab[r >> rsh], rtab[(r >> rsh) + 1]].  Both ride
// along in the items launch, which waits on memory: a lane per fence entry copies its rank, a
// lane per bucket searches the ranks at fence positions.  (Buckets that point into the whole
// store needed a binary search per bucket with a dependent line fetch per probe, about 10 GB
// per step at 5x10^6 excitors; lanes per store entry that fill the buckets above their rank
// make fills as long and uneven as the gaps between ranks in a space of 7x10^8 determinants.)
constexpr uint64_t kFence = 16;
constexpr uint64_t kFenceDirect = 1ull << 17;  // stores up to this many entries (1 MB of ranks) take fs = 1

__host__ __device__ __forceinline__ uint64_t fence_stride(uint64_t ne) { return ne <= kFenceDirect ? 1 : kFence; }
__host__ __device__ __forceinline__ uint64_t fence_count(uint64_t ne) { return (ne + fence_stride(ne) - 1) / fence_stride(ne); }

struct Fence {
    const uint64_t *srank;
    uint64_t ne;
    uint64_t *fence;
    uint32_t *rtab;
    uint64_t rt_n;
    uint32_t rsh;
};

// blocks [0, fence blocks): the fence (none with fs = 1); the blocks after them: the rank table
__device__ __forceinline__ void fence_block(unsigned blk, const Fence &f)
{
    const uint64_t fs = fence_stride(f.ne), nf = fence_count(f.ne);
    const unsigned nbf = fs > 1 ? (unsigned)((nf + kThreads - 1) / kThreads) : 0u;
    if (blk < nbf) {
        const uint64_t k = (uint64_t)blk * kThreads + threadIdx.x;
        if (k < nf) f.fence[k] = f.srank[k * fs];
        return;
    }
    const uint64_t c = (uint64_t)(blk - nbf) * kThreads + threadIdx.x;
    if (c >= f.rt_n) return;
    const uint64_t key = c << f.rsh;
    uint64_t l0 = 0, h0 = nf;
    while (l0 < h0) {
        const uint64_t mid = (l0 + h0) >> 1;
        if (f.srank[mid * fs] < key)
            l0 = mid + 1;
        else
            h0 = mid;
    }
    f.rtab[c] = (uint32_t)l0;
}

// ------------------------------------- co-location of excitors over iterations (Sec. III.B)
// pl[t * n + i] = processor of excitor i at iteration t, for t < T.
template <int W>
__global__ void __launch_bounds__(kThreads) k_codist_place(const uint64_t *__restrict__ keys, uint64_t n, uint64_t T,
                                                           uint32_t n_ranks, uint32_t move_shift, uint32_t seed,
                                                           uint16_t *__restrict__ pl)
{
    const uint64_t x = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (x >= n * T) return;
    const uint64_t t = x / n, i = x - t * n;
    uint64_t d[W];
#pragma unroll
    for (int w = 0; w < W; ++w) d[w] = keys[i * W + w];
    pl[x] = (uint16_t)placement<W>(d, t, n_ranks, move_shift, seed);
}

// Pair counts c_ij = #{t < T_c : pl[t][i] = pl[t][j]} for i < j, summed (c and c^2) at each
// checkpoint T_c.  A block holds kCoRows excitors i against 256 excitors j, one j per thread
// with a counter per i; blocks entirely on or below the diagonal exit.  Iterations run in
// chunks of up to kCoChunk that end at checkpoints: the chunk's i rows are staged in LDS
// (every thread reads the same word: a broadcast) and each thread loads its j's placements
// for the chunk before comparing.  Absent excitors carry values no placement takes.  Integer
// sums, so the result does not depend on the order of the atomic additions.
constexpr int kCoRows = 32, kCoChunk = 32;

__global__ void __launch_bounds__(kThreads) k_codist_pairs(const uint16_t *__restrict__ pl, uint64_t n,
                                                           const uint64_t *__restrict__ cps, int ncp,
                                                           unsigned long long *__restrict__ sums)
{
    __shared__ uint4 s_i[kCoChunk][kCoRows / 4];
    const uint64_t i0 = (uint64_t)blockIdx.y * kCoRows;
    const uint64_t jb = (uint64_t)blockIdx.x * kThreads;
    if (jb + kThreads <= i0 + 1) return;  // every j of the block is <= every i
    const uint64_t j = jb + threadIdx.x;
    const bool jv = j < n;
    const uint64_t jc = jv ? j : n - 1;
    uint32_t c[kCoRows];
#pragma unroll
    for (int r = 0; r < kCoRows; ++r) c[r] = 0;
    const uint64_t T = cps[ncp - 1];
    int next = 0;
    uint64_t t = 0;
    for (;;) {
        while (next < ncp && cps[next] == t) {
            uint64_t s1 = 0, s2 = 0;
#pragma unroll
            for (int r = 0; r < kCoRows; ++r) {
                const uint64_t i = i0 + r;
                if (jv && i < j) {
                    s1 += c[r];
                    s2 += (uint64_t)c[r] * c[r];
                }
            }
            s1 = block_reduce_sum(s1);
            s2 = block_reduce_sum(s2);
            if (threadIdx.x == 0) {
                atomicAdd(&sums[2 * next], (unsigned long long)s1);
                atomicAdd(&sums[2 * next + 1], (unsigned long long)s2);
            }
            ++next;
        }
        if (t >= T) break;
        const uint64_t end = cps[next] - t < (uint64_t)kCoChunk ? cps[next] : t + kCoChunk;  // next <= ncp - 1 here
        const int len = (int)(end - t);
        // stage rows i0 .. i0 + kCoRows of iterations t .. end - 1
        uint32_t *si = reinterpret_cast<uint32_t *>(&s_i[0][0]);
        for (int x = threadIdx.x; x < kCoChunk * kCoRows; x += kThreads) {
            const int tc = x / kCoRows, r = x - tc * kCoRows;
            const uint64_t i = i0 + r;
            const uint64_t ic = i < n ? i : n - 1;
            const uint32_t v = pl[(t + (tc < len ? tc : 0)) * n + ic];
            si[x] = (i < n && tc < len) ? v : 0xFFFFFFFFu;
        }
        uint32_t rj[kCoChunk];
#pragma unroll
        for (int tc = 0; tc < kCoChunk; ++tc) {
            const uint32_t v = pl[(t + (tc < len ? tc : 0)) * n + jc];
            rj[tc] = jv ? v : 0xFFFFFFFEu;
        }
        __syncthreads();
#pragma unroll
        for (int tc = 0; tc < kCoChunk; ++tc) {
            if (tc < len) {
#pragma unroll
                for (int q = 0; q < kCoRows / 4; ++q) {
                    const uint4 v = s_i[tc][q];
                    c[4 * q + 0] += v.x == rj[tc];
                    c[4 * q + 1] += v.y == rj[tc];
                    c[4 * q + 2] += v.z == rj[tc];
                    c[4 * q + 3] += v.w == rj[tc];
                }
            }
        }
        __syncthreads();
        t = end;
    }
}

// ------------------------------------------------------- non-composite items (FNC)
// Item 0 is the reference (A = N_0, K = 0), item i+1 the store entry i (A = N_i);
// p = 1 for all of them (Sec. IV.B).
template <int W, typename T>
__device__ __forceinline__ void noncomposite_block(unsigned blk, const SysDev &S, const uint64_t *__restrict__ skey, const T *__restrict__ samp,
                                                           const T *__restrict__ sK, uint64_t sstride, uint64_t ne, double n0,
                                                           StepArgs a, Items<T> it, ItemPartials part, Scratch *sc)
{
    const uint64_t k = (uint64_t)blk * kThreads + threadIdx.x;
    double num = 0.0;
    uint64_t att = 0, mx = 0;
    if (k <= ne) {
        uint64_t d[W];
        T A, K;
        int L;
        if (k == 0) {
#pragma unroll
            for (int w = 0; w < W; ++w) d[w] = S.hf[w];
            A = (T)n0;
            K = T(0);
            L = 0;
        } else {
#pragma unroll
            for (int w = 0; w < W; ++w) d[w] = skey[(uint64_t)w * sstride + (k - 1)];
            A = samp[k - 1];
            K = sK[k - 1];
            L = level_of<W>(S, d);
        }
        const uint32_t n = attempt_count<T>(A, a.thr_nc, a.kmin, &sc->err);
        T death = T(0);
        if (L <= S.l) death = -(T)a.tau * (K - (T)a.shift) * A;
        if (L == 1 || L == 2)
            num = (double)(reference_element<W, T>(S, d, L) * (T)excitor_sign<W>(S, d) * A);
#pragma unroll
        for (int w = 0; w < W; ++w) it.key[(uint64_t)w * it.stride + k] = d[w];
        it.A[k] = A;
        it.death[k] = death;
        it.n[k] = n;
        it.cnt[k] = (uint64_t)n + 1;
        att = n;
        mx = n;
    }
    store_item_partials(num, att, 0, mx, part, blk);
}

// --------------------------------------------------------------- sampled clusters
// Selection k draws s from p_size (s in [0, l+2], or [2, l+2] for the composite part of full
// non-composite sampling), then s excitors with probability q_i / Q each; repeats are
// discarded (Sec. II).  The product of the excitors is collapsed by applying them to the
// reference one operator at a time; a repeated hole or particle makes it vanish.
template <int W, typename T>
__device__ __forceinline__ void select_block(unsigned blk, const SysDev &S, const uint64_t *__restrict__ drec,
                                                     uint64_t ne, const uint64_t *__restrict__ P,
                                                     const uint32_t *__restrict__ guide, Ranks rk, double n0, StepArgs a,
                                                     Items<T> it, uint64_t item_base, ItemPartials part, Scratch *sc)
{
    constexpr uint32_t kRec = 2 + W;  // words of a draw record: prefix, amplitude, bitstring
    const uint64_t k = (uint64_t)blk * kThreads + threadIdx.x;
    double num = 0.0;
    uint64_t att = 0, disc = 0, mx = 0;
    if (k < a.n_sel) {
        // With N_p virtual processors selection k is made by processor k mod N_p, whose
        // excitors hold the prefix range [base, base + Q) of the partition's weights and
        // which makes `count` of the step's selections (Sec. III).
        uint64_t Q = sc->qtot, base = 0, count = a.n_sel;
        if (a.n_ranks > 1) {
            const uint32_t rank = (uint32_t)(k % a.n_ranks);
            const uint32_t s0 = ne ? rk.seg[rank] : 0, s1 = ne ? rk.seg[rank + 1] : 0;
            base = s0 ? P[s0 - 1] : 0;
            Q = (s1 ? P[s1 - 1] : 0) - base;
            count = a.n_sel / a.n_ranks + (rank < a.n_sel % a.n_ranks ? 1 : 0);
        }
        const uint32_t gsh = a.gsh;
        Draws r(a.key0, a.key1, kSelect, (uint32_t)k, 0u, a.step);
        const int lo = a.fnc ? 2 : 0, hi = S.l + 2;
        const int s = draw_size(uniform53(r.get(0)), lo, hi);
        bool ok = !(s > 0 && Q == 0);
        // Every draw of the cluster first; then the loads they need are issued together (one
        // latency chain per cluster instead of one per excitor).
        uint64_t xs[kMaxClusterSize];
        uint32_t l0[kMaxClusterSize], h0[kMaxClusterSize];
#pragma unroll
        for (int c = 0; c < kMaxClusterSize; ++c) {
            xs[c] = 0;
            l0[c] = h0[c] = 0;
            if (c < s && ok) xs[c] = base + below(r.get(1 + c), Q);
        }
#pragma unroll
        for (int c = 0; c < kMaxClusterSize; ++c) {
            if (c < s && ok) {
                // the drawn excitor lies in [guide[gb], guide[gb + 1]] (past the table: in
                // [guide[gcap - 1], ne - 1]); the last candidate's prefix exceeds x, so only the
                // others are probed, and a bucket inside one excitor's weight needs no probe
                const uint64_t gb = xs[c] >> gsh;
                if (gb + 1 < a.gcap) {
                    l0[c] = guide[gb];
                    h0[c] = guide[gb + 1];
                } else {
                    l0[c] = guide[a.gcap - 1];
                    h0[c] = (uint32_t)ne - 1u;
                }
            }
        }
        // lock-step binary searches: first i in [l0, h0) with P[i] > x (the prefix of the
        // draw records), else h0
        for (bool more = ok && s > 0; more;) {
            more = false;
#pragma unroll
            for (int c = 0; c < kMaxClusterSize; ++c) {
                if (c < s && l0[c] < h0[c]) {
                    const uint32_t mid = (l0[c] + h0[c]) >> 1;
                    if (drec[(uint64_t)mid * kRec] > xs[c])
                        h0[c] = mid;
                    else
                        l0[c] = mid + 1;
                    more |= l0[c] < h0[c];
                }
            }
        }
        // repeated excitors: discarded (Sec. II)
#pragma unroll
        for (int c = 1; c < kMaxClusterSize; ++c)
#pragma unroll
            for (int b = 0; b < c; ++b)
                if (c < s) ok &= (l0[b] != l0[c]);
        // selection probability and product of amplitudes, in draw order; each draw's weight
        // is its amplitude's (the prefix step P[i] - P[i-1] exactly)
        // The drawn records' amplitudes and bitstrings: for one- and two-word determinants every
        // load is issued before the first use (one latency instead of two); wider ones would
        // hold too many registers, and load each field where it is used.
        constexpr bool kPreload = W <= 2;
        uint64_t ab[kMaxClusterSize], kx[kMaxClusterSize][kPreload ? W : 1];
#pragma unroll
        for (int c = 0; c < kMaxClusterSize; ++c) {
            const uint64_t *rc = drec + (uint64_t)l0[c] * kRec;
            const bool use = c < s && ok;
            ab[c] = use ? rc[1] : 0ull;
            if constexpr (kPreload) {
#pragma unroll
                for (int w = 0; w < W; ++w) kx[c][w] = use ? rc[2 + w] : 0ull;
            }
        }
        double fact = 1.0;
        for (int c = 2; c <= s; ++c) fact *= (double)c;
        double p = (double)count * size_prob(s, lo, hi) * fact;
        T prod = (T)n0;
#pragma unroll
        for (int c = 0; c < kMaxClusterSize; ++c) {
            if (c < s && ok) {
                const T ni = rec_amp<T>(ab[c]);
                const uint64_t qi = weight_of((double)ni);
                p *= (double)qi / (double)Q;
                if (c == 0)
                    prod = ni;
                else
                    prod *= ni / (T)n0;
            }
        }
        // the s excitors share one of N_p processors: times N_p^(1-s) (Sec. III)
        if (a.n_ranks > 1) {
            if (s == 0) {
                p *= (double)a.n_ranks;
            } else {
                double dd = 1.0;
                for (int c = 1; c < s; ++c) dd *= (double)a.n_ranks;
                p /= dd;
            }
        }
        uint64_t d[W];
#pragma unroll
        for (int w = 0; w < W; ++w) d[w] = S.hf[w];
        int e = 0;
        // apply c_{X_s} first: annihilate holes ascending, then create particles descending
#pragma unroll
        for (int c = kMaxClusterSize - 1; c >= 0; --c) {
            if (c >= s || !ok) continue;
            uint64_t x[W];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                if constexpr (kPreload)
                    x[w] = kx[c][w];
                else
                    x[w] = drec[(uint64_t)l0[c] * kRec + 2 + w];
            }
#pragma unroll
            for (int w = 0; w < W; ++w) {
                uint64_t h = S.hf[w] & ~x[w];
                while (h) {
                    const int q = 64 * w + __ffsll((long long)h) - 1;
                    h &= h - 1;
                    if (!bit_test<W>(d, q)) ok = false;
                    e += count_below<W>(d, q);
                    bit_flip<W>(d, q);
                }
            }
#pragma unroll
            for (int w = W - 1; w >= 0; --w) {
                uint64_t pm = x[w] & ~S.hf[w];
                while (pm) {
                    const int q = 64 * w + 63 - __clzll((long long)pm);
                    pm &= ~(1ull << (q & 63));
                    if (bit_test<W>(d, q)) ok = false;
                    e += count_below<W>(d, q);
                    bit_flip<W>(d, q);
                }
            }
        }
        const int L = level_of<W>(S, d);
        if (L > S.l + 2) ok = false;
        uint32_t n = 0;
        uint64_t cnt = 0;
        T A = T(0), death = T(0);
        if (ok) {
            // sign of c_X1..c_Xs |HF> = sigma s_D(X) |D_X>; the cluster amplitude is
            // t_HF^(1-s) prod t_i with that sign (a sign flip is exact in either order)
            const int sigma = ((e & 1) ? -1 : 1) * excitor_sign<W>(S, d);
            const T Ac = (s == 0) ? (T)n0 : (sigma < 0 ? -prod : prod);
            // p is formed in FP64 and can fall below the FP32 range at large populations
            // (n_sel p_size s! prod q_i/Q): divide in FP64, then round to T
            A = (T)((double)Ac / p);
            n = attempt_count<T>(A, a.thr_cluster, a.kmin, &sc->err);
            cnt = (uint64_t)n + 1;
            if (L <= S.l) death = -(T)a.tau * (diagonal<W, T>(S, d) - (T)a.shift) * A;
            if (L == 1 || L == 2) num = (double)(reference_element<W, T>(S, d, L) * (T)excitor_sign<W>(S, d) * A);
            att = n;
            mx = n;
        } else {
            disc = 1;
        }
        const uint64_t j = item_base + k;
        if (ok) {
#pragma unroll
            for (int w = 0; w < W; ++w) it.key[(uint64_t)w * it.stride + j] = d[w];
            it.A[j] = A;
            it.death[j] = death;
            it.n[j] = n;
        }
        it.cnt[j] = cnt;
    }
    store_item_partials(num, att, disc, mx, part, blk);
    if (k == 0) it.cnt[item_base + a.n_sel] = 0;  // closing entry of the slot-count scan
}

// One launch for both kinds of item: blocks [0, nb_fnc) are the non-composite items, blocks
// [nb_fnc, nb_items) the sampled clusters (selection k = (block - nb_fnc) * 256 + thread), and
// the blocks after them build the store's rank table.
template <int W, typename T>
__device__ __forceinline__ void items_body(uint32_t blk, uint32_t nblk, SysDev S, const uint64_t *__restrict__ skey, const T *__restrict__ samp,
                                                    const T *__restrict__ sK, uint64_t sstride, uint64_t ne,
                                                    const uint64_t *__restrict__ P, const uint64_t *__restrict__ drec,
                                                    const uint32_t *__restrict__ guide,
                                                    Ranks rk, double n0, StepArgs a, Items<T> it, unsigned nb_fnc, uint64_t n_fnc,
                                                    unsigned nb_items, Fence rt, ItemPartials part, Scratch *sc)
{
    if (blk >= nb_items) {  // trailing blocks: the fence of the store lookups
        fence_block(blk - nb_items, rt);
        return;
    }
    // a prefix beyond 2^53 makes the selection probabilities inexact: refuse the step
    if (blk == 0 && threadIdx.x == 0 && sc->qtot > (1ull << 53))
        atomicOr((unsigned long long *)&sc->err, (unsigned long long)kErrBlowup);
    if (blk < nb_fnc) {
        noncomposite_block<W, T>(blk, S, skey, samp, sK, sstride, ne, n0, a, it, part, sc);
    } else {
        const unsigned b = blk - nb_fnc;
        ItemPartials ps{part.num + nb_fnc, part.att + nb_fnc, part.disc + nb_fnc, part.maxn + nb_fnc};
        select_block<W, T>(b, S, drec, ne, P, guide, rk, n0, a, it, n_fnc, ps, sc);
    }
}

template <int W, typename T>
struct ItemsArgs {
    SysDev S;
    const uint64_t *skey;
    const T *samp;
    const T *sK;
    uint64_t sstride;
    uint64_t ne;
    const uint64_t *P;
    const uint64_t *drec;
    const uint32_t *guide;
    Ranks rk;
    double n0;
    StepArgs a;
    Items<T> it;
    unsigned nb_fnc;
    uint64_t n_fnc;
    unsigned nb_items;
    Fence rt;
    ItemPartials part;
    Scratch *sc;
};

template <int W, typename T>
__device__ __forceinline__ void k_items_entry(const ItemsArgs<W, T> &A, uint32_t blk, uint32_t nblk)
{
    items_body<W, T>(blk, nblk, A.S, A.skey, A.samp, A.sK, A.sstride, A.ne, A.P, A.drec, A.guide, A.rk, A.n0, A.a, A.it, A.nb_fnc, A.n_fnc, A.nb_items, A.rt, A.part, A.sc);
}

template <int W, typename T>
__global__ void __launch_bounds__(kThreads) k_items(const ItemsArgs<W, T> *__restrict__ args, BatchMap bm)
{
    uint32_t blk, nblk;
    k_items_entry<W, T>(args[batch_state(bm, blk, nblk)], blk, nblk);
}

template <int W, typename T>
__global__ void __launch_bounds__(kThreads) k_items(const ItemsArgs<W, T> A)
{
    k_items_entry<W, T>(A, blockIdx.x, gridDim.x);
}

// ----------------------------------------------------------------- generation
// Records of one block of kGenSlots consecutive slots are compacted, in slot order, into
// the block's own region; a scan of the block counts and a gather then lay them out densely.
// Slot order is record-id order, so the stable sort that follows keeps every
// determinant's contributions in id order.
struct Records {
    uint64_t *rank;    // rank of the target in the truncated space
    uint64_t *key;     // SoA target bitstrings, stride `stride`
    void *amp;         // T
    uint64_t *id;      // optional record ids
    uint64_t stride;
};

// A spawning attempt in two halves.  gen_excitation draws the excitation of determinant d
// (Philox stream (purpose, k, m)) and applies it: false for a null draw or a target beyond
// the truncation level (Sec. II), else the target bitstring and the orbitals (j = tb = -1 for
// a single).  spawn_amount then evaluates the Slater-Condon element and the spawned amount
// -dtau H_tc s_D(c) s_D(t) A / (n p_gen) (Sec. II sign rule, Sec. IV.C), with the stochastic
// rounding of amounts below the spawn cutoff; false when nothing is spawned.
template <int W, int K>
__device__ __forceinline__ bool gen_excitation(const SysDev &S, const uint64_t *d, uint32_t purpose, uint32_t k,
                                               uint32_t m, const StepArgs &a, uint64_t *tgt, int &i, int &j, int &ta,
                                               int &tb)
{
    Draws r(a.key0, a.key1, purpose, k, m, a.step);
    const int N = S.nel;
    i = j = ta = tb = -1;
    if (is_ueg<K>(S)) {
        const uint32_t pr = (uint32_t)below(r.get(0), S.npairs);
        const int alpha = (int)below(r.get(1), S.half);
        const uint32_t xy = S.pairs[pr];  // the pair (x < y) of lexicographic rank pr, tabulated
        const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
        // The target's level is L(d) - [i virtual] - [j virtual] + [a virtual] + [b virtual].
        // When it exceeds the truncation whatever b is, the attempt ends early: the same
        // outcome as the level test below.  d's occupied orbitals in index order are its
        // N - L(d) reference ones, then its virtual ones, so i (the x-th) is virtual iff
        // x >= N - L(d); with N even, a = 2 alpha + spin is virtual iff alpha >= N / 2.  So
        // the test can run before the orbitals are selected.
        const int Ld = level_of<W>(S, d);
        if ((N & 1) == 0 && Ld - (x >= N - Ld) - (y >= N - Ld) + (alpha >= N / 2) > S.l) return false;
        i = select_bit<W>(d, x);
        j = select_bit<W>(d, y);
        ta = 2 * alpha + (i & 1);
        if (bit_test<W>(d, ta)) return false;
        if (Ld - (i >= N) - (j >= N) + (ta >= N) > S.l) return false;  // (odd N)
        // k_b = k_i + k_j - k_a, all three components in one integer sum of the packed fields
        // (each field stays inside its 10 bits: no carry or borrow crosses between them)
        const int G = S.G, D = 2 * G + 1;
        const int s3 = (int)S.kpack[i >> 1] + (int)S.kpack[j >> 1] - (int)S.kpack[ta >> 1];
        const int bx = (s3 & 1023) - 256 - G, by = ((s3 >> 10) & 1023) - 256 - G, bz = ((s3 >> 20) & 1023) - 256 - G;
        if (bx < -G || bx > G || by < -G || by > G || bz < -G || bz > G) return false;
        const int beta = S.grid[((bx + G) * D + (by + G)) * D + (bz + G)];
        if (beta < 0) return false;
        tb = 2 * beta + (j & 1);
        if (tb == ta || bit_test<W>(d, tb)) return false;
    } else {
        // the truncation test first, from the draws alone (as in the UEG generator: with N
        // even the target's level follows from the occupied ranks and the alphas)
        const bool single = uniform53(r.get(0)) < S.p_single;
        const int Ld = level_of<W>(S, d);
        if (single) {
            const int xa = (int)below(r.get(1), (uint64_t)N);
            const int aa = (int)below(r.get(2), S.half);
            if ((N & 1) == 0 && Ld - (xa >= N - Ld) + (aa >= N / 2) > S.l) return false;
            i = select_bit<W>(d, xa);
            ta = 2 * aa + (i & 1);
            if (bit_test<W>(d, ta)) return false;
        } else {
            const uint32_t xy = S.pairs[(uint32_t)below(r.get(1), S.npairs)];
            const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
            const int aa = (int)below(r.get(2), S.half), ab = (int)below(r.get(3), S.half);
            if ((N & 1) == 0 && Ld - (x >= N - Ld) - (y >= N - Ld) + (aa >= N / 2) + (ab >= N / 2) > S.l) return false;
            i = select_bit<W>(d, x);
            j = select_bit<W>(d, y);
            ta = 2 * aa + (i & 1);
            tb = 2 * ab + (j & 1);
            if (ta == tb || bit_test<W>(d, ta) || bit_test<W>(d, tb)) return false;
        }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) tgt[w] = d[w];
    bit_flip<W>(tgt, i);
    bit_flip<W>(tgt, ta);
    if (j >= 0) {
        bit_flip<W>(tgt, j);
        bit_flip<W>(tgt, tb);
    }
    // spawns beyond the truncation level are discarded (Sec. II)
    return level_of<W>(S, tgt) <= S.l;
}

template <int W, typename T, int K>
__device__ __forceinline__ bool spawn_amount(const SysDev &S, const uint64_t *d, const uint64_t *tgt, int i, int j, int ta,
                                             int tb, T A, uint32_t n, uint32_t purpose, uint32_t k, uint32_t m,
                                             const StepArgs &a, T &x)
{
    double pgen;
    int ridx;
    if (is_ueg<K>(S)) {
        pgen = (((i & 1) == (j & 1)) ? 2.0 : 1.0) / ((double)S.npairs * (double)S.half);
        ridx = 2;
    } else if (j < 0) {
        pgen = S.p_single / ((double)S.nel * (double)S.half);
        ridx = 4;
    } else {
        pgen = (1.0 - S.p_single) * (((i & 1) == (j & 1)) ? 2.0 : 1.0) /
               ((double)S.npairs * (double)S.half * (double)S.half);
        ridx = 4;
    }
    T H;
    if (j < 0) {
        H = single_element<W, T, K>(S, d, i, ta);
    } else {
        const int t1 = ta < tb ? ta : tb, t2 = ta < tb ? tb : ta;
        H = double_element<W, T, K>(S, d, i, j, t1, t2);
    }
    const int sc = excitor_sign<W>(S, d), st = excitor_sign<W>(S, tgt);
    // -dtau H_ij s_D(i) s_D(j) A / (n p_gen)  (Sec. II spawning sign, Sec. IV.C eq. 10)
    x = -(T)a.tau * H * (T)sc * (T)st * A / ((T)n * (T)pgen);
    if (x == T(0)) return false;
    if (fabs((double)x) < a.cutoff) {
        Draws r(a.key0, a.key1, purpose, k, m, a.step);
        const double u = uniform53(r.get(ridx));
        if (u < fabs((double)x) / a.cutoff)
            x = (T)copysign(a.cutoff, (double)x);
        else
            return false;
    }
    return true;
}

// Output of the record-slot scan: the slot offset of every item, and the first item of each
// generation block (the item whose slot range holds the block's first slot), scattered by
// the items themselves -- slots beyond the capacity belong to no block.
struct SlotOut {
    // 16 items per thread: half the tiles of the other scans, so half the look-back chain over
    // the ~10^6 item counts (19 -> 16 us at 1.2 M items; the small scans are faster at 8)
    static constexpr int kItems = 16;
    uint64_t *p;
    uint64_t *block_item;
    uint64_t slot_cap;
    __device__ __forceinline__ void item(uint64_t i, uint64_t excl, uint64_t x, bool valid) const
    {
        uint64_t b0 = 0, b1 = 0;
        if (valid && x) {
            const uint64_t end = excl + x < slot_cap ? excl + x : slot_cap;
            b0 = (excl + kGenSlots - 1) / kGenSlots;
            b1 = end > 0 ? (end - 1) / kGenSlots + 1 : 0;  // blocks whose first slot is < end
        }
        wave_fill_ranges<uint64_t>(block_item, b0, b1, i);
    }
};

// Items of a generation block whose offsets are staged in LDS (more: searched in HBM).  With
// 1024 the block's LDS is 22.5 KB, so 7 blocks fit in a CU's 160 KB; with the register budget
// of 7 waves per SIMD below, the kernel runs at 7 waves per SIMD instead of 6.
constexpr int kGenLdsItems = 1024;
constexpr int kGenWaveSlots = 64 * kGenRounds;  // consecutive slots of one wavefront

// Per-block statistics of the generation kernel (no single-address atomics).
struct GenStats {
    uint32_t *count;    // records of each block
    uint32_t *spawns;
    uint32_t *deaths;
};

// One block covers kGenSlots consecutive record slots, wavefront w the kGenWaveSlots slots
// from w * kGenWaveSlots.  The item of each slot comes from a slot map in LDS: every item with
// a slot marks its first slot in the block, and a running maximum over the slots fills the
// rest.  Pass 1, one lane per slot: keep the slot as a candidate if it is a non-zero death or an
// attempt whose excitation is valid, compacted per wavefront in slot order.  Pass 2, one lane
// per candidate: evaluate the element and the spawned amount, and write the records in slot
// order into the block's region.  Splitting the two halves keeps every lane of pass 2 busy:
// only a small fraction of the attempts survive pass 1.
constexpr uint32_t kCandDeath = 1u << 31;

template <int W, typename T, int K>
__device__ __forceinline__ void generate_body(uint32_t blk, uint32_t nblk, SysDev S, Items<T> it, const uint64_t *__restrict__ off,
                                                       const uint64_t *__restrict__ block_item, uint64_t n_fnc,
                                                       uint64_t n_items, uint64_t slot_cap, StepArgs a, Records rec,
                                                       int keep_ids, GenStats gs, Scratch *sc)
{
    __shared__ uint32_t s_off[kGenLdsItems + 1];  // item offsets relative to the first item's
    __shared__ uint16_t s_map[kGenSlots];         // item of each slot, relative to the first item
    __shared__ uint32_t wave_tot[kWaves];
    __shared__ uint32_t s_wpre[kWaves + 1];       // candidates of the wavefronts before each
    __shared__ uint32_t c_item[kGenSlots];  // candidate: item
    __shared__ uint32_t c_slot[kGenSlots];  // candidate: slot in its item (kCandDeath: the death)
    __shared__ uint64_t c_orb[kGenSlots];   // candidate: i, j, a, b (16 bits each)
    T *ramp = static_cast<T *>(rec.amp);
    const uint64_t g0 = (uint64_t)blk * kGenSlots;
    const uint64_t n_all = off[n_items];
    const uint64_t n_slots = n_all < slot_cap ? n_all : slot_cap;
    if (blk == 0 && threadIdx.x == 0) {
        gs.count[nblk] = 0;  // closing entry of the scan
        if (n_all > slot_cap) atomicOr((unsigned long long *)&sc->err, (unsigned long long)kErrSlotCap);
    }
    if (g0 >= n_slots) {  // idle block (the grid covers the capacity)
        if (threadIdx.x == 0) gs.count[blk] = gs.spawns[blk] = gs.deaths[blk] = 0;
        return;
    }
    // items of this block: from the one holding its first slot to the one holding the next
    // block's first slot (for the last block: every remaining item)
    const uint64_t lo = block_item[blk];
    const uint64_t hi = g0 + kGenSlots < n_slots ? block_item[blk + 1] : n_items - 1;
    const bool lds = hi - lo + 1 <= (uint64_t)kGenLdsItems;
    const uint64_t obase = off[lo];  // <= g0; every slot of the block is below obase + 2^31
    const int wv = wave_id(), lane = lane_id();
    if (lds) {
        for (uint64_t t = threadIdx.x; t <= hi - lo + 1; t += kThreads) {
            const uint64_t r = off[lo + t] - obase;
            s_off[t] = r < 0xFFFFFFFFull ? (uint32_t)r : 0xFFFFFFFFu;
        }
        for (int t = threadIdx.x; t < kGenSlots; t += kThreads) s_map[t] = 0;  // slot 0 is item lo's
        __syncthreads();
        const uint32_t g0r = (uint32_t)(g0 - obase);
        for (uint32_t r = 1 + threadIdx.x; r <= (uint32_t)(hi - lo); r += kThreads) {
            const uint32_t s0 = s_off[r];
            if (s_off[r + 1] > s0 && s0 - g0r < (uint32_t)kGenSlots) s_map[s0 - g0r] = (uint16_t)r;  // s0 > g0r
        }
        __syncthreads();
        // running maximum: kPer consecutive slots per thread, then over the threads
        constexpr int kPer = kGenSlots / kThreads;
        uint32_t m[kPer], run = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t x = s_map[threadIdx.x * kPer + j];
            run = x > run ? x : run;
            m[j] = run;
        }
        uint32_t inc = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o, 64);
            if (lane >= o) inc = t > inc ? t : inc;
        }
        if (lane == 63) wave_tot[wv] = inc;
        uint32_t before = __shfl_up(inc, 1, 64);
        before = lane ? before : 0u;
        __syncthreads();
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww)
            if (ww < wv) before = wave_tot[ww] > before ? wave_tot[ww] : before;
#pragma unroll
        for (int j = 0; j < kPer; ++j) s_map[threadIdx.x * kPer + j] = (uint16_t)(m[j] > before ? m[j] : before);
        __syncthreads();
    }
    // ---- pass 1: candidates, compacted into this wavefront's segment of the candidate lists
    uint32_t wcount = 0;
    const uint32_t wseg = (uint32_t)wv * kGenWaveSlots;
    for (int rd = 0; rd < kGenRounds; ++rd) {
        const uint32_t t = wseg + (uint32_t)rd * 64 + (uint32_t)lane;
        const uint64_t g = g0 + t;
        bool keep = false;
        uint32_t item32 = 0, slot = 0;
        uint64_t orb = 0;
        if (g < n_slots) {
            uint64_t item;
            if (lds) {
                const uint32_t rel = s_map[t];
                item = lo + rel;
                slot = (uint32_t)(g - obase) - s_off[rel];
            } else {  // last item in [lo, hi] whose offset is <= g, searched in HBM
                uint64_t l0 = lo, h0 = hi + 1;
                while (l0 < h0) {
                    const uint64_t mid = (l0 + h0) >> 1;
                    if (off[mid] > g)
                        h0 = mid;
                    else
                        l0 = mid + 1;
                }
                item = l0 - 1;
                slot = (uint32_t)(g - off[item]);
            }
            item32 = (uint32_t)item;
            if (slot == 0) {
                keep = it.death[item] != T(0);
                slot = kCandDeath;
            } else {
                const bool nc = item < n_fnc;
                const uint32_t k = (uint32_t)(nc ? item : item - n_fnc);
                uint64_t d[W], tgt[W];
#pragma unroll
                for (int ww = 0; ww < W; ++ww) d[ww] = it.key[(uint64_t)ww * it.stride + item];
                int i, j, ta, tb;
                keep = gen_excitation<W, K>(S, d, nc ? kSpawnNonComposite : kSpawnSampled, k, slot - 1, a, tgt, i, j, ta, tb);
                orb = (uint64_t)(uint16_t)i | ((uint64_t)(uint16_t)j << 16) | ((uint64_t)(uint16_t)ta << 32) |
                      ((uint64_t)(uint16_t)tb << 48);
            }
        }
        const uint64_t mk = __ballot(keep);
        if (keep) {
            const uint32_t q = wseg + wcount + (uint32_t)lanes_below(mk);
            c_item[q] = item32;
            c_slot[q] = slot;
            c_orb[q] = orb;
        }
        wcount += (uint32_t)__popcll(mk);
    }
    if (lane == 0) wave_tot[wv] = wcount;
    __syncthreads();
    if (threadIdx.x == 0) {  // candidates of the wavefronts before each
        uint32_t acc = 0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) {
            s_wpre[ww] = acc;
            acc += wave_tot[ww];
        }
        s_wpre[kWaves] = acc;
    }
    __syncthreads();
    const uint32_t nc_total = s_wpre[kWaves];
    // ---- pass 2: amounts of the candidates, records in slot order
    uint32_t base = 0, spawns = 0, deaths = 0;
    for (uint32_t e0 = 0; e0 < nc_total; e0 += kThreads) {
        const uint32_t e = e0 + threadIdx.x;
        bool emit = false;
        uint64_t tgt[W];
        T x = T(0);
        uint64_t id = 0;
        if (e < nc_total) {
            uint32_t q = e;  // position of candidate e: its wavefront's segment, then its rank there
#pragma unroll
            for (int ww = 0; ww < kWaves; ++ww) {
                const uint32_t p0 = s_wpre[ww];
                if (e >= p0) q = (uint32_t)ww * kGenWaveSlots + (e - p0);
            }
            const uint64_t item = c_item[q];
            const uint32_t cs = c_slot[q];
            const bool nc = item < n_fnc;
            const uint32_t k = (uint32_t)(nc ? item : item - n_fnc);
            uint64_t d[W];
#pragma unroll
            for (int w = 0; w < W; ++w) d[w] = it.key[(uint64_t)w * it.stride + item];
            if (cs == kCandDeath) {
                x = it.death[item];
#pragma unroll
                for (int w = 0; w < W; ++w) tgt[w] = d[w];
                emit = true;
                ++deaths;
                id = ((nc ? 0ull : 1ull) << 62) | ((uint64_t)k << 30);
            } else {
                const uint64_t orb = c_orb[q];
                const int i = (int16_t)(orb & 0xFFFF), j = (int16_t)((orb >> 16) & 0xFFFF);
                const int ta = (int16_t)((orb >> 32) & 0xFFFF), tb = (int16_t)((orb >> 48) & 0xFFFF);
#pragma unroll
                for (int w = 0; w < W; ++w) tgt[w] = d[w];
                bit_flip<W>(tgt, i);
                bit_flip<W>(tgt, ta);
                if (j >= 0) {
                    bit_flip<W>(tgt, j);
                    bit_flip<W>(tgt, tb);
                }
                emit = spawn_amount<W, T, K>(S, d, tgt, i, j, ta, tb, it.A[item], it.n[item],
                                          nc ? kSpawnNonComposite : kSpawnSampled, k, cs - 1, a, x);
                spawns += emit ? 1u : 0u;
                id = ((nc ? 0ull : 1ull) << 62) | ((uint64_t)k << 30) | (uint64_t)cs;
            }
        }
        const uint64_t mk = __ballot(emit);
        if (lane_id() == 0) wave_tot[wave_id()] = (uint32_t)__popcll(mk);
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            if (w < wave_id()) before += wave_tot[w];
            total += wave_tot[w];
        }
        if (emit) {
            const uint64_t dst = g0 + base + before + (uint32_t)lanes_below(mk);
#pragma unroll
            for (int w = 0; w < W; ++w) rec.key[(uint64_t)w * rec.stride + dst] = tgt[w];
            ramp[dst] = x;
            if (keep_ids) rec.id[dst] = id;
        }
        base += total;
        __syncthreads();
    }
    // spawns and deaths of the block in one exchange (16 bits each per wavefront suffice)
    uint32_t sd = spawns | deaths << 16;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sd += __shfl_down(sd, o, 64);
    if (lane_id() == 0) wave_tot[wave_id()] = sd;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t bs = 0, bd = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            bs += wave_tot[w] & 0xFFFFu;
            bd += wave_tot[w] >> 16;
        }
        gs.count[blk] = base;
        gs.spawns[blk] = bs;
        gs.deaths[blk] = bd;
    }
}

template <int W, typename T>
struct GenerateArgs {
    SysDev S;
    Items<T> it;
    const uint64_t *off;
    const uint64_t *block_item;
    uint64_t n_fnc;
    uint64_t n_items;
    uint64_t slot_cap;
    StepArgs a;
    Records rec;
    int keep_ids;
    GenStats gs;
    Scratch *sc;
};

template <int W, typename T, int K>
__device__ __forceinline__ void k_generate_entry(const GenerateArgs<W, T> &A, uint32_t blk, uint32_t nblk)
{
    generate_body<W, T, K>(blk, nblk, A.S, A.it, A.off, A.block_item, A.n_fnc, A.n_items, A.slot_cap, A.a, A.rec, A.keep_ids, A.gs, A.sc);
}

// One kernel per kind of system (K = kSystemUEG or kSystemMol): the other generator's code and
// registers are left out.
template <int W, typename T, int K>
__global__ void __launch_bounds__(kThreads) k_generate(const GenerateArgs<W, T> *__restrict__ args, BatchMap bm)
{
    uint32_t blk, nblk;
    k_generate_entry<W, T, K>(args[batch_state(bm, blk, nblk)], blk, nblk);
}

template <int W, typename T, int K>
__global__ void __launch_bounds__(kThreads) k_generate(const GenerateArgs<W, T> A)
{
    k_generate_entry<W, T, K>(A, blockIdx.x, gridDim.x);
}

// Determinants of one or two words fit the register budget of 7 waves per SIMD without
// spilling (at most 72 VGPRs), four words that of 6 (at most 80); wider ones keep the
// compiler's own budget.
#define CCMC_GENERATE_WAVES(W_, T_, K_, N_)                                                                            \
    template <>                                                                                                        \
    __global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(N_, N_)))                          \
    k_generate<W_, T_, K_>(const GenerateArgs<W_, T_> *__restrict__ args, BatchMap bm)                                 \
    {                                                                                                                  \
        uint32_t blk, nblk;                                                                                            \
        k_generate_entry<W_, T_, K_>(args[batch_state(bm, blk, nblk)], blk, nblk);                                     \
    }                                                                                                                  \
    template <>                                                                                                        \
    __global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(N_, N_)))                          \
    k_generate<W_, T_, K_>(const GenerateArgs<W_, T_> A)                                                               \
    {                                                                                                                  \
        k_generate_entry<W_, T_, K_>(A, blockIdx.x, gridDim.x);                                                        \
    }
#define CCMC_GENERATE_WAVES_BOTH(W_, T_, N_)                                                                           \
    CCMC_GENERATE_WAVES(W_, T_, kSystemUEG, N_)                                                                        \
    CCMC_GENERATE_WAVES(W_, T_, kSystemMol, N_)
CCMC_GENERATE_WAVES_BOTH(1, float, 7)
CCMC_GENERATE_WAVES_BOTH(1, double, 7)
CCMC_GENERATE_WAVES_BOTH(2, float, 7)
CCMC_GENERATE_WAVES_BOTH(2, double, 7)
CCMC_GENERATE_WAVES_BOTH(4, float, 6)
CCMC_GENERATE_WAVES_BOTH(4, double, 6)
#undef CCMC_GENERATE_WAVES_BOTH
#undef CCMC_GENERATE_WAVES

// Dense layout of the records.  Output position r belongs to the region q (generation block
// q) with boff[q] <= r < boff[q+1], at slot position r - boff[q] of that region.  Block b
// writes the outputs [b * kGatherTile, (b + 1) * kGatherTile): its first region comes from
// tile_region (scattered by the region scan), the region offsets of its range are staged in
// LDS and each output finds its region there.  The truncated-space rank of each record (the
// sort key) is computed on the way.
constexpr int kGatherTile = 256;
constexpr int kGatherLds = 2048;

// Output of the region scan: the record offset of every region, and the region holding the
// first output of each gather tile, scattered by the regions themselves.
struct RegionOut {
    static constexpr int kItems = kScanItems;
    uint32_t *p;
    uint32_t *tile_region;
    uint64_t cap;  // entries of tile_region (records past the dense capacity are never gathered)
    __device__ __forceinline__ void item(uint64_t q, uint32_t excl, uint32_t x, bool valid) const
    {
        uint64_t b0 = 0, b1 = 0;
        if (valid && x) {
            b0 = (excl + kGatherTile - 1) / kGatherTile;
            b1 = ((uint64_t)excl + x - 1) / kGatherTile + 1;  // tiles whose first output is < excl + x
            b1 = b1 < cap ? b1 : cap;
            b0 = b0 < b1 ? b0 : b1;
        }
        wave_fill_ranges<uint32_t>(tile_region, b0, b1, (uint32_t)q);
    }
};

// The sort key of a record: its rank, or with `packed` (ranks of at most 32 bits) the rank in the
// high half and the record's dense position in the low half, so that the sorted list also
// tells where each record's bitstring is.
template <int W, typename T>
__device__ __forceinline__ void gather_body(uint32_t blk, uint32_t nblk, const SysDev S, Records reg, const uint32_t *__restrict__ boff,
                                            const uint32_t *__restrict__ tile_region, uint64_t n_blocks, uint64_t rec_cap,
                                            Records out, int keep_ids, int packed, Scratch *sc)
{
    __shared__ uint32_t s_b[kGatherLds + 1];
    // records the annihilation works on: all of them, or none after a capacity overflow
    const uint64_t nr = sc->n_rec;
    const bool over = nr > rec_cap || (sc->err & kErrSlotCap);
    const uint64_t live = over ? 0 : nr;
    if (blk == 0 && threadIdx.x == 0) {
        sc->n_live = live;
        if (nr > rec_cap) atomicOr((unsigned long long *)&sc->err, (unsigned long long)kErrRecCap);
    }
    const uint64_t o0 = (uint64_t)blk * kGatherTile;
    if (o0 >= live) return;
    const uint64_t o1 = o0 + kGatherTile < live ? o0 + kGatherTile : live;
    const uint32_t qa = tile_region[blk];
    const uint32_t qb = o1 < live ? tile_region[blk + 1] : (uint32_t)(n_blocks - 1);
    const uint32_t nq = qb - qa + 1;  // regions [qa, qb] hold this tile's outputs
    const bool lds = nq + 1 <= (uint32_t)kGatherLds;
    if (lds)
        for (uint32_t t = threadIdx.x; t <= nq; t += kThreads) s_b[t] = boff[qa + t];
    __syncthreads();
    for (uint64_t r = o0 + threadIdx.x; r < o1; r += kThreads) {
        uint32_t l0, h0, q;
        if (lds) {  // last q in [qa, qb] with boff[q] <= r
            l0 = 0;
            h0 = nq;
            while (l0 < h0) {
                const uint32_t mid = (l0 + h0) >> 1;
                if (s_b[mid] > r)
                    h0 = mid;
                else
                    l0 = mid + 1;
            }
            q = qa + l0 - 1;
        } else {
            l0 = qa;
            h0 = qb + 1;
            while (l0 < h0) {
                const uint32_t mid = (l0 + h0) >> 1;
                if (boff[mid] > r)
                    h0 = mid;
                else
                    l0 = mid + 1;
            }
            q = l0 - 1;
        }
        const uint64_t src = (uint64_t)q * kGenSlots + (r - (lds ? s_b[q - qa] : boff[q]));
        uint64_t d[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            d[w] = reg.key[(uint64_t)w * reg.stride + src];
            if (packed || keep_ids) out.key[(uint64_t)w * out.stride + r] = d[w];
        }
        const uint64_t rk = space_rank<W>(S, d);
        out.rank[r] = packed ? (rk << 32 | r) : rk;
        static_cast<T *>(out.amp)[r] = static_cast<const T *>(reg.amp)[src];
        if (keep_ids) out.id[r] = reg.id[src];
    }
}

template <int W, typename T>
struct GatherArgs {
    const SysDev S;
    Records reg;
    const uint32_t *boff;
    const uint32_t *tile_region;
    uint64_t n_blocks;
    uint64_t rec_cap;
    Records out;
    int keep_ids;
    int packed;
    Scratch *sc;
};

template <int W, typename T>
__device__ __forceinline__ void k_gather_entry(const GatherArgs<W, T> &A, uint32_t blk, uint32_t nblk)
{
    gather_body<W, T>(blk, nblk, A.S, A.reg, A.boff, A.tile_region, A.n_blocks, A.rec_cap, A.out, A.keep_ids, A.packed, A.sc);
}

template <int W, typename T>
__global__ void __launch_bounds__(kThreads) k_gather(const GatherArgs<W, T> *__restrict__ args, BatchMap bm)
{
    uint32_t blk, nblk;
    k_gather_entry<W, T>(args[batch_state(bm, blk, nblk)], blk, nblk);
}

template <int W, typename T>
__global__ void __launch_bounds__(kThreads) k_gather(const GatherArgs<W, T> A)
{
    k_gather_entry<W, T>(A, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------- annihilation
// Records are sorted by rank (equal ranks = equal determinants, ascending rank = ascending
// key) and, within a determinant, by record id (the sort is stable).  The contributions to a
// determinant are summed in three levels: each thread left-folds the pieces of runs among its
// kFoldItems consecutive records; a segmented suffix scan over the threads of a tile sums the
// following threads' pieces of a run (a tree of log2(kThreads) rounds, so a run as long as the
// tile costs no serial walk); a run's head adds that sum, then the pieces of the following
// tiles in order.  The grouping is fixed by the tiling, so the sums are reproducible and equal
// the plain left fold up to rounding order.  The head of each run looks
// its rank up in the store: a hit adds to that entry, the reference (rank 0) adds to N_0, a
// miss becomes a new excitor at insertion point ins.  A run that continues past its tile is
// left "open" (its sum within the tile, rank and insertion point go to the tile's summary):
// k_seg_close finishes it once every tile's leading piece is known.
constexpr int kFoldItems = 8;
constexpr int kFoldTile = kThreads * kFoldItems;
constexpr uint64_t kNoOpen = ~0ull;

struct FoldTiles {
    double *lead;        // per tile: left fold of its records before its first run head
    uint32_t *has_head;  // per tile: any run head in the tile
    uint64_t *open;      // per tile: record index of its open head, or kNoOpen
    uint64_t *open_new;  // per tile: new-determinant index of its open head (if new)
    uint64_t *status;    // per tile: look-back status of the count of new determinants
    double *open_sum;    // per tile: the open run's sum within the tile
    uint64_t *open_pos;  // per tile: the open run's store insertion point
    uint64_t *open_rank; // per tile: the open run's rank
    uint64_t *ticket;
};

// The determinants that are not in the store, in rank order: bitstring, rank, insertion point
// in the store and summed amount.
struct NewDets {
    uint64_t *key;
    uint64_t *rank;
    uint64_t *ins;
    double *sum;
    uint64_t stride;
    const uint64_t *rkey;  // dense record bitstrings (stride rstride), read with packed sort keys
    uint64_t rstride;
};

// Rank of a sorted record key (see gather_body).
__device__ __forceinline__ uint64_t key_rank(uint64_t k, int packed) { return packed ? k >> 32 : k; }

// The records arrive sorted as (key, amplitude) pairs: the amplitudes are read in order.  A new
// determinant's bitstring is read from the dense records at the position the packed key
// carries, or (ranks above 32 bits) recovered from its rank.
template <int W, typename T>
__device__ __forceinline__ void seg_fold_body(uint32_t blk, uint32_t nblk, const SysDev &S, const uint64_t *__restrict__ rank,
                                                       const T *__restrict__ val, int packed, uint64_t cap,
                                                       const uint64_t *__restrict__ srank, uint64_t ne,
                                                       double *__restrict__ delta,
                                                       const uint64_t *__restrict__ fence, const uint32_t *__restrict__ rtab,
                                                       uint64_t rt_n, uint32_t rsh,
                                                       FoldTiles ft, NewDets nd, Scratch *sc)
{
    __shared__ double s_lead[kThreads];
    __shared__ uint32_t s_head[kThreads];
    __shared__ uint64_t s_open, s_open_new, s_open_pos, s_open_rank, s_tile, s_prefix;
    __shared__ double s_open_sum;
    const uint64_t n = sc->n_live;
    // tiles in ticket order: the look-back over the counts of new determinants only waits
    // for tiles that are already running
    if (threadIdx.x == 0) s_tile = atomicAdd((unsigned long long *)ft.ticket, 1ull);
    __syncthreads();
    const uint64_t tile = s_tile;
    const uint64_t base = tile * kFoldTile;
    const uint64_t r0 = base + (uint64_t)threadIdx.x * kFoldItems;
    if (base >= n) {
        if (threadIdx.x == 0) {
            ft.lead[tile] = 0.0;
            ft.has_head[tile] = 0;
            ft.open[tile] = kNoOpen;
        }
        return;
    }
    if (threadIdx.x == 0) s_open = kNoOpen;
    // this thread's records, the one before and the one after (clamped: unconditional loads)
    uint64_t rr[kFoldItems + 1];
    uint32_t pos_of[kFoldItems];  // dense position of each record (packed keys)
#pragma unroll
    for (int i = 0; i <= kFoldItems; ++i) {
        const uint64_t r = r0 + i;
        const uint64_t k = rank[r < n ? r : n - 1];
        if (i < kFoldItems) pos_of[i] = (uint32_t)k;
        rr[i] = r < n ? key_rank(k, packed) : ~0ull;
    }
    const uint64_t rprev = r0 ? key_rank(rank[r0 - 1 < n ? r0 - 1 : n - 1], packed) : ~0ull;
    double v[kFoldItems];
#pragma unroll
    for (int i = 0; i < kFoldItems; ++i) v[i] = (double)val[r0 + i < n ? r0 + i : n - 1];
    bool head[kFoldItems];
    uint32_t any = 0;
#pragma unroll
    for (int i = 0; i < kFoldItems; ++i) {
        const bool valid = r0 + i < n;
        head[i] = valid && (r0 + i == 0 || rr[i] != (i ? rr[i - 1] : (r0 + i - 1 < n ? rprev : ~0ull)));
        any |= head[i] ? 1u : 0u;
    }
    // leading piece: this thread's records before its first head (all of them if none)
    double lead = 0.0;
    {
        bool in_lead = true;
#pragma unroll
        for (int i = 0; i < kFoldItems; ++i) {
            in_lead = in_lead && !head[i] && (r0 + i < n);
            if (in_lead) lead += v[i];
        }
    }
    s_lead[threadIdx.x] = lead;
    s_head[threadIdx.x] = any;
    __syncthreads();
    // segmented suffix sums over the threads (Hillis-Steele, log2(kThreads) rounds): afterwards
    // s_lead[t] is the sum of the leading pieces of threads t .. e, e the first thread >= t
    // holding a head (or the last thread), and s_head[t] tells whether there is such a head
    {
        const uint32_t t = threadIdx.x;
        double rv = lead;
        uint32_t rf = any;
#pragma unroll
        for (uint32_t off = 1; off < (uint32_t)kThreads; off <<= 1) {
            const bool in = t + off < (uint32_t)kThreads;
            const double ov = in ? s_lead[t + off] : 0.0;
            const uint32_t of = in ? s_head[t + off] : 0u;
            __syncthreads();
            if (!rf && in) {
                rv += ov;
                rf = of;
            }
            s_lead[t] = rv;
            s_head[t] = rf;
            __syncthreads();
        }
    }
    // runs that start here: fold the rest of this thread's piece, then the following pieces
    double acc[kFoldItems];
    bool open[kFoldItems];
#pragma unroll
    for (int i = 0; i < kFoldItems; ++i) {
        acc[i] = 0.0;
        open[i] = false;
        if (!head[i]) continue;
        const uint64_t rk = rr[i];
        double sum = v[i];
        int m = i + 1;
        bool more = true;
#pragma unroll
        for (int q = 1; q < kFoldItems; ++q) {
            if (q <= i) continue;
            more = more && rr[q] == rk;
            if (more) {
                sum += v[q];
                m = q + 1;
            }
        }
        if (m == kFoldItems && rr[kFoldItems] == rk) {  // the run continues into the next thread
            bool to_end = true;  // no head after this thread: the run reaches the tile's end
            if (threadIdx.x + 1 < kThreads) {
                sum += s_lead[threadIdx.x + 1];
                to_end = !s_head[threadIdx.x + 1];
            }
            // past the tile end: continues if the next tile starts with the same rank
            open[i] = to_end && base + kFoldTile < n && key_rank(rank[base + kFoldTile], packed) == rk;
        }
        acc[i] = sum;
    }
    // store lookups of all heads of this thread in lock step: first entry with rank >= rk.
    // The fence first: the first chunk whose leading rank exceeds rk (f in [0, nf]); the entry
    // then lies in [(f-1) kFence, min(f kFence, ne)] (0 when f = 0).
    const uint32_t nf = (uint32_t)fence_count(ne), fs = (uint32_t)fence_stride(ne);
    uint32_t lo[kFoldItems], hi[kFoldItems];
#pragma unroll
    for (int i = 0; i < kFoldItems; ++i) {
        lo[i] = hi[i] = 0;
        if (head[i] && rr[i] != 0 && ne) {  // the fence range of the rank's bucket
            const uint64_t c = rr[i] >> rsh;
            lo[i] = rtab[c];
            hi[i] = c + 1 < rt_n ? rtab[c + 1] : nf;
        }
    }
    if (fs > 1) {
        // the first fence entry of the range with fence[k] > rk, else the range's end
        for (bool busy = true; busy;) {
            busy = false;
#pragma unroll
            for (int i = 0; i < kFoldItems; ++i) {
                if (lo[i] < hi[i]) {
                    const uint32_t mid = (lo[i] + hi[i]) >> 1;
                    if (fence[mid] > rr[i])
                        hi[i] = mid;
                    else
                        lo[i] = mid + 1;
                    busy |= lo[i] < hi[i];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < kFoldItems; ++i) {
            const uint32_t f = lo[i];
            if (head[i] && rr[i] != 0 && ne && f > 0) {
                lo[i] = (f - 1) * fs;
                hi[i] = f * fs < ne ? f * fs : (uint32_t)ne;
            } else {
                lo[i] = hi[i] = 0;
            }
        }
    }
    // with fs = 1 the bucket's range is already the range of store entries to search
    for (bool busy = true; busy;) {
        busy = false;
#pragma unroll
        for (int i = 0; i < kFoldItems; ++i) {
            if (lo[i] < hi[i]) {
                const uint32_t mid = (lo[i] + hi[i]) >> 1;
                if (srank[mid] < rr[i])
                    lo[i] = mid + 1;
                else
                    hi[i] = mid;
                busy |= lo[i] < hi[i];
            }
        }
    }
    // new determinants of this thread, numbered in record order across the tiles
    bool fresh[kFoldItems];
    uint32_t n_fresh = 0;
#pragma unroll
    for (int i = 0; i < kFoldItems; ++i) {
        const uint64_t rk = rr[i];
        const uint64_t pos = lo[i];
        fresh[i] = head[i] && rk != 0 && !(pos < ne && srank[pos] == rk);
        n_fresh += fresh[i] ? 1u : 0u;
    }
    uint32_t tile_fresh;
    uint32_t j = block_exclusive_scan(n_fresh, &tile_fresh);
    if (wave_id() == 0) {
        if (lane_id() == 0)
            lb_publish(&ft.status[tile], tile == 0 ? kLbInclusive : kLbAggregate, (uint64_t)tile_fresh);
        const uint64_t prefix = tile == 0 ? 0 : lb_wave_lookback(ft.status, tile);
        if (lane_id() == 0) {
            if (tile > 0) lb_publish(&ft.status[tile], kLbInclusive, prefix + tile_fresh);
            s_prefix = prefix;
            if (base + kFoldTile >= n) sc->n_new = prefix + tile_fresh;  // the last live tile
        }
    }
    __syncthreads();
    const uint64_t jbase = s_prefix;
#pragma unroll
    for (int i = 0; i < kFoldItems; ++i) {
        if (!head[i]) continue;
        const uint64_t rk = rr[i];
        const uint64_t r = r0 + i;
        const uint64_t pos = lo[i];
        if (fresh[i]) {
            const uint64_t jj = jbase + j++;
            uint64_t d[W];
            if (packed) {
#pragma unroll
                for (int w = 0; w < W; ++w) d[w] = nd.rkey[(uint64_t)w * nd.rstride + pos_of[i]];
            } else {
                space_unrank<W>(S, rk, d);
            }
#pragma unroll
            for (int w = 0; w < W; ++w) nd.key[(uint64_t)w * nd.stride + jj] = d[w];
            nd.rank[jj] = rk;
            nd.ins[jj] = pos;
            if (!open[i]) nd.sum[jj] = acc[i];  // an open run's sum is written when it is closed
            if (open[i]) s_open_new = jj;
        }
        if (open[i]) {  // at most one per tile: the run of the tile's last record
            s_open = r;
            s_open_sum = acc[i];
            s_open_pos = pos;
            s_open_rank = rk;
        } else if (rk == 0) {
            sc->hf_sum = acc[i];
            sc->hf_hit = 1;
        } else if (!fresh[i]) {
            delta[pos] = acc[i];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ft.lead[tile] = s_lead[0];  // the tile's leading piece
        ft.has_head[tile] = s_head[0];
        ft.open[tile] = s_open;
        ft.open_new[tile] = s_open_new;
        ft.open_sum[tile] = s_open_sum;
        ft.open_pos[tile] = s_open_pos;
        ft.open_rank[tile] = s_open_rank;
    }
}

template <int W, typename T>
struct SegFoldArgs {
    SysDev S;
    const uint64_t *rank;
    const T *val;
    int packed;
    uint64_t cap;
    const uint64_t *srank;
    uint64_t ne;
    double *delta;
    const uint64_t *fence;
    const uint32_t *rtab;
    uint64_t rt_n;
    uint32_t rsh;
    FoldTiles ft;
    NewDets nd;
    Scratch *sc;
};

template <int W, typename T>
__device__ __forceinline__ void k_seg_fold_entry(const SegFoldArgs<W, T> &A, uint32_t blk, uint32_t nblk)
{
    seg_fold_body<W, T>(blk, nblk, A.S, A.rank, A.val, A.packed, A.cap, A.srank, A.ne, A.delta, A.fence,
                        A.rtab, A.rt_n, A.rsh, A.ft, A.nd, A.sc);
}

template <int W, typename T>
__global__ void __launch_bounds__(kThreads) k_seg_fold(const SegFoldArgs<W, T> *__restrict__ args, BatchMap bm)
{
    uint32_t blk, nblk;
    k_seg_fold_entry<W, T>(args[batch_state(bm, blk, nblk)], blk, nblk);
}

template <int W, typename T>
__global__ void __launch_bounds__(kThreads) k_seg_fold(const SegFoldArgs<W, T> A)
{
    k_seg_fold_entry<W, T>(A, blockIdx.x, gridDim.x);
}

// Finish the open runs: add the leading pieces of the following tiles until one holds a head,
// then land on N_0, the store entry or the new determinant.  One lane per tile.
__device__ __forceinline__ void seg_close_body(uint32_t blk, uint32_t nblk, uint64_t n_tiles, const uint64_t *__restrict__ srank,
                                               uint64_t ne, double *__restrict__ delta, double *__restrict__ nsum,
                                               FoldTiles ft, Scratch *sc)
{
    const uint64_t t = (uint64_t)blk * kThreads + threadIdx.x;
    if (t >= n_tiles || ft.open[t] == kNoOpen) return;
    double acc = ft.open_sum[t];
    for (uint64_t k = t + 1; k < n_tiles; ++k) {
        acc += ft.lead[k];
        if (ft.has_head[k]) break;
    }
    const uint64_t rk = ft.open_rank[t];
    if (rk == 0) {
        sc->hf_sum = acc;
        sc->hf_hit = 1;
    } else {
        const uint64_t pos = ft.open_pos[t];
        if (pos < ne && srank[pos] == rk)
            delta[pos] = acc;
        else
            nsum[ft.open_new[t]] = acc;
    }
}

struct SegCloseArgs {
    uint64_t n_tiles;
    const uint64_t *srank;
    uint64_t ne;
    double *delta;
    double *nsum;
    FoldTiles ft;
    Scratch *sc;
};

__device__ __forceinline__ void k_seg_close_entry(const SegCloseArgs &A, uint32_t blk, uint32_t nblk)
{
    seg_close_body(blk, nblk, A.n_tiles, A.srank, A.ne, A.delta, A.nsum, A.ft, A.sc);
}

__global__ void __launch_bounds__(kThreads) k_seg_close(const SegCloseArgs *__restrict__ args, BatchMap bm)
{
    uint32_t blk, nblk;
    k_seg_close_entry(args[batch_state(bm, blk, nblk)], blk, nblk);
}

__global__ void __launch_bounds__(kThreads) k_seg_close(const SegCloseArgs A)
{
    k_seg_close_entry(A, blockIdx.x, gridDim.x);
}

// Merge the store (with its sums added) and the new determinants into key order, round, and
// compact into the other store buffer, in one pass over the merged positions.  Merged
// position p holds new determinant j when ins_j + j = p (new determinant j lands after the
// ins_j store entries below it and the j new ones before it), else store entry p - #(new
// before p).  Real-weight occupation rounding at merged position p: 0 < |N| < theta becomes
// +-theta with probability |N| / theta, else 0, from a Philox draw keyed by p (the reference
// is exempt).  Survivors get their output position from a scan over the tiles (decoupled
// look-back in ticket order) and are written compacted; the per-tile |N| sums feed the
// population total.  The current buffer is only read, so a failed step leaves it intact.
struct StoreCols {
    uint64_t *key;
    void *amp;
    void *K;
    uint64_t *rank;
    uint64_t stride;
};

constexpr int kMergeItems = 4;  // merged positions per thread, one per row of the tile
constexpr int kMergeTile = kThreads * kMergeItems;
constexpr unsigned kMergeBlocks = 1024;  // resident blocks of the merge (per state)

// #{j < n : ins[j] + j < P} by one wavefront.  ins[j] + j (the merged position of new
// determinant j) is strictly increasing, so a 64-way search narrows [lo, hi] by 64 per round.
__device__ __forceinline__ uint64_t wave_new_before(const uint64_t *__restrict__ ins, uint64_t n, uint64_t P)
{
    uint64_t lo = 0, hi = n;  // the answer lies in [lo, hi]
    while (hi > lo) {
        const uint64_t step = (hi - lo + 63) >> 6;
        const uint64_t idx = lo + (uint64_t)lane_id() * step;
        const uint64_t c = idx < hi ? idx : hi - 1;
        const bool below = idx < hi && ins[c] + c < P;
        const uint64_t nb = (uint64_t)__popcll(__ballot(below));
        if (nb == 0) break;  // the probe at lo fails: the answer is lo
        const uint64_t nhi = lo + nb * step;
        lo += (nb - 1) * step + 1;
        hi = nhi < hi ? nhi : hi;
    }
    return lo;
}

// Merged position p of a tile is row p / kThreads, thread p % kThreads, so every row is read
// and written with coalesced accesses.  The tile's new determinants are scattered into LDS by
// position; counts "before p" (new determinants, survivors) come from per-row ballots.
template <int W, typename T>
__device__ __forceinline__ void merge_body(uint32_t blk, uint32_t nblk, const SysDev S, StoreCols in, uint64_t ne,
                                           const double *__restrict__ delta, const uint64_t *__restrict__ nkey,
                                           const uint64_t *__restrict__ nrank, uint64_t nstride,
                                           const uint64_t *__restrict__ nins, const double *__restrict__ nsum, StoreCols out,
                                           StepArgs a, uint64_t *__restrict__ status, uint64_t *__restrict__ ticket,
                                           double *__restrict__ abs_part, Scratch *sc)
{
    __shared__ uint64_t s_tile, s_prefix, s_j[2];
    __shared__ uint16_t s_new[kMergeTile];                 // 1 + (j - j0) of the new determinant at a position, or 0
    __shared__ uint32_t s_cnt[kMergeItems][kWaves];        // per row and wave: new determinants, then survivors
    __shared__ T s_K[kMergeTile];                          // diagonal elements of the tile's new determinants
    const uint64_t nn = sc->n_new;
    const uint64_t total = ne + nn;
    // A step already in error (a capacity overflow upstream) is abandoned by every block
    // alike, before any index is formed from its possibly incomplete records.
    if (sc->err) return;
    const int w = wave_id(), lane = lane_id();
    // Blocks take tiles in ticket order until the merged store is covered: a tile waits
    // only on tiles taken before it, all held by running blocks.
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd((unsigned long long *)ticket, 1ull);
        for (int i = threadIdx.x; i < kMergeTile; i += kThreads) s_new[i] = 0;
        __syncthreads();
        const uint64_t tile = s_tile;
        const uint64_t P0 = tile * kMergeTile;
        if (P0 >= total) return;
        if (w < 2) {
            const uint64_t P = w == 0 ? P0 : (P0 + kMergeTile < total ? P0 + kMergeTile : total);
            const uint64_t j = wave_new_before(nins, nn, P);
            if (lane == 0) s_j[w] = j;
        }
        __syncthreads();
        const uint64_t j0 = s_j[0], j1 = s_j[1];
        // the new determinants, by one thread each: position and diagonal element
        for (uint64_t j = j0 + threadIdx.x; j < j1; j += kThreads) {
            const uint64_t o = nins[j] + j - P0;  // in [0, kMergeTile) by the choice of j0 and j1
            uint64_t d[W];
#pragma unroll
            for (int x = 0; x < W; ++x) d[x] = nkey[(uint64_t)x * nstride + j];
            if (o < kMergeTile && j - j0 < kMergeTile) {
                s_new[o] = (uint16_t)(j - j0 + 1);
                s_K[j - j0] = diagonal<W, T, true>(S, d);
            }
        }
        __syncthreads();
        uint32_t f[kMergeItems];
#pragma unroll
        for (int u = 0; u < kMergeItems; ++u) {
            f[u] = s_new[u * kThreads + threadIdx.x];
            const uint64_t m = __ballot(f[u] != 0);
            if (lane == 0) s_cnt[u][w] = (uint32_t)__popcll(m);
        }
        __syncthreads();
        T v[kMergeItems];
        uint64_t src[kMergeItems];
        double abs_sum = 0.0;
        {
            uint64_t nb = j0;  // new determinants in the rows before the current one
#pragma unroll
            for (int u = 0; u < kMergeItems; ++u) {
                uint64_t below_w = 0, in_row = 0;
#pragma unroll
                for (int x = 0; x < kWaves; ++x) {
                    if (x < w) below_w += s_cnt[u][x];
                    in_row += s_cnt[u][x];
                }
                const uint64_t m = __ballot(f[u] != 0);
                const uint64_t p = P0 + (uint64_t)u * kThreads + threadIdx.x;
                v[u] = T(0);
                src[u] = 0;
                if (f[u] != 0) {
                    src[u] = j0 + f[u] - 1;
                    v[u] = (T)nsum[src[u]];
                } else if (p < total) {
                    src[u] = p - (nb + below_w + (uint64_t)lanes_below(m));
                    v[u] = (T)((double)static_cast<const T *>(in.amp)[src[u]] + delta[src[u]]);
                }
                if (v[u] != T(0) && fabs((double)v[u]) < a.theta) {
                    Draws r(a.key0, a.key1, kRound, (uint32_t)p, 0u, a.step);
                    const double uu = uniform53(r.get(0));
                    v[u] = (uu < fabs((double)v[u]) / a.theta) ? (T)copysign(a.theta, (double)v[u]) : T(0);
                }
                abs_sum += fabs((double)v[u]);
                nb += in_row;
            }
        }
        __syncthreads();  // the new-determinant counts are read; s_cnt takes the survivor counts
#pragma unroll
        for (int u = 0; u < kMergeItems; ++u) {
            const uint64_t m = __ballot(v[u] != T(0));
            if (lane == 0) s_cnt[u][w] = (uint32_t)__popcll(m);
        }
        __syncthreads();  // the survivor counts are published
        uint64_t tile_keep = 0;
#pragma unroll
        for (int u = 0; u < kMergeItems; ++u)
#pragma unroll
            for (int x = 0; x < kWaves; ++x) tile_keep += s_cnt[u][x];
        // the tile's count goes out before the |N| sum, so that later tiles' look-backs find it sooner
        if (threadIdx.x == 0) lb_publish(&status[tile], tile == 0 ? kLbInclusive : kLbAggregate, tile_keep);
        const double tile_abs = block_reduce_sum(abs_sum);
        if (w == 0) {
            const uint64_t prefix = tile == 0 ? 0 : lb_wave_lookback(status, tile);
            if (lane == 0) {
                if (tile > 0) lb_publish(&status[tile], kLbInclusive, prefix + tile_keep);
                s_prefix = prefix;
                if (P0 + kMergeTile >= total) sc->n_out = prefix + tile_keep;  // the last tile
                abs_part[tile] = tile_abs;
            }
        }
        __syncthreads();
        // survivors' columns: every row's loads first, then the stores
        uint64_t dk[kMergeItems][W], rk[kMergeItems];
        T K[kMergeItems];
#pragma unroll
        for (int u = 0; u < kMergeItems; ++u) {
            const bool nw = f[u] != 0;
            const uint64_t *kb = nw ? nkey : in.key;
            const uint64_t ks = nw ? nstride : in.stride;
            const uint64_t c = v[u] != T(0) ? src[u] : 0;  // a row slot without a survivor loads entry 0
#pragma unroll
            for (int x = 0; x < W; ++x) dk[u][x] = kb[(uint64_t)x * ks + c];
            rk[u] = (nw ? nrank : in.rank)[c];
            const T k_new = s_K[nw ? f[u] - 1 : 0];
            K[u] = nw ? k_new : static_cast<const T *>(in.K)[c];
        }
        uint64_t q = s_prefix;  // survivors before the current row
#pragma unroll
        for (int u = 0; u < kMergeItems; ++u) {
            const uint64_t m = __ballot(v[u] != T(0));
            uint64_t before = 0, in_row = 0;
#pragma unroll
            for (int x = 0; x < kWaves; ++x) {
                if (x < w) before += s_cnt[u][x];
                in_row += s_cnt[u][x];
            }
            if (v[u] != T(0)) {
                const uint64_t o = q + before + (uint64_t)lanes_below(m);
#pragma unroll
                for (int x = 0; x < W; ++x) out.key[(uint64_t)x * out.stride + o] = dk[u][x];
                static_cast<T *>(out.amp)[o] = v[u];
                static_cast<T *>(out.K)[o] = K[u];
                out.rank[o] = rk[u];
            }
            q += in_row;
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

template <int W, typename T>
struct MergeArgs {
    SysDev S;
    StoreCols in;
    uint64_t ne;
    const double *delta;
    const uint64_t *nkey;
    const uint64_t *nrank;
    uint64_t nstride;
    const uint64_t *nins;
    const double *nsum;
    StoreCols out;
    StepArgs a;
    uint64_t *status;
    uint64_t *ticket;
    double *abs_part;
    Scratch *sc;
};

template <int W, typename T>
__device__ __forceinline__ void k_merge_entry(const MergeArgs<W, T> &A, uint32_t blk, uint32_t nblk)
{
    merge_body<W, T>(blk, nblk, A.S, A.in, A.ne, A.delta, A.nkey, A.nrank, A.nstride, A.nins, A.nsum, A.out, A.a, A.status,
                     A.ticket, A.abs_part, A.sc);
}

template <int W, typename T>
__global__ void __launch_bounds__(kThreads) k_merge(const MergeArgs<W, T> *__restrict__ args, BatchMap bm)
{
    uint32_t blk, nblk;
    k_merge_entry<W, T>(args[batch_state(bm, blk, nblk)], blk, nblk);
}

template <int W, typename T>
__global__ void __launch_bounds__(kThreads) k_merge(const MergeArgs<W, T> A)
{
    k_merge_entry<W, T>(A, blockIdx.x, gridDim.x);
}

// The step's statistics in a fixed-order two-stage reduction: block b of k_final_part sums
// the b-th contiguous chunk of every partial array (the item kernels' per-block partials, the
// generation blocks' spawn and death counts, the per-block |N| sums of the compacted store);
// the last block to finish adds the chunk sums in chunk order.
struct FinalPart {
    double num, tot;
    uint64_t att, disc, mx, sp, de, pad;
};

// Every field of a FinalPart over the block, in one exchange: a shuffle tree within each
// wavefront, then thread 0 adds the wavefronts in order (the result is valid in thread 0).
__device__ __forceinline__ FinalPart block_reduce_part(FinalPart a)
{
    __shared__ FinalPart s_w[kWaves];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a.num += __shfl_down(a.num, o, 64);
        a.tot += __shfl_down(a.tot, o, 64);
        a.att += __shfl_down(a.att, o, 64);
        a.disc += __shfl_down(a.disc, o, 64);
        a.sp += __shfl_down(a.sp, o, 64);
        a.de += __shfl_down(a.de, o, 64);
        const uint64_t m = __shfl_down(a.mx, o, 64);
        a.mx = m > a.mx ? m : a.mx;
    }
    if (lane_id() == 0) s_w[wave_id()] = a;
    __syncthreads();
    FinalPart r{};
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const FinalPart b = s_w[w];
            r.num += b.num;
            r.tot += b.tot;
            r.att += b.att;
            r.disc += b.disc;
            r.sp += b.sp;
            r.de += b.de;
            r.mx = b.mx > r.mx ? b.mx : r.mx;
        }
    }
    return r;
}

__device__ __forceinline__ void chunk_of(uint64_t n, uint64_t g, uint64_t nb, uint64_t &lo, uint64_t &hi)
{
    const uint64_t c = (n + nb - 1) / nb;
    lo = g * c < n ? g * c : n;
    hi = lo + c < n ? lo + c : n;
}

// The block's part of the first stage (valid in thread 0).
__device__ __forceinline__ FinalPart final_part_body(uint32_t blk, uint32_t nblk, ItemPartials part, uint64_t n_parts, GenStats gs,
                                                     uint64_t n_gen, const double *__restrict__ abs_part, uint64_t n_abs,
                                                     const Scratch *sc, uint64_t ne)
{
    {  // the merge wrote the absolute sums of the tiles covering the merged store only
        const uint64_t live = (ne + sc->n_new + kMergeTile - 1) / kMergeTile;
        n_abs = live < n_abs ? live : n_abs;
    }
    constexpr int U = 4;  // loads in flight per array and thread
    double num = 0.0, tot = 0.0;
    uint64_t att = 0, disc = 0, mx = 0, sp = 0, de = 0;
    uint64_t lo, hi;
    chunk_of(n_parts, blk, nblk, lo, hi);
    for (uint64_t i0 = lo; i0 < hi; i0 += U * kThreads) {
        double a[U];
        uint64_t b[U], c[U], d[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {  // clamped indices: unconditional loads, then select
            const uint64_t i = i0 + (uint64_t)u * kThreads + threadIdx.x;
            const bool in = i < hi;
            const uint64_t ic = in ? i : hi - 1;
            a[u] = part.num[ic];
            b[u] = part.att[ic];
            c[u] = part.disc[ic];
            d[u] = part.maxn[ic];
            a[u] = in ? a[u] : 0.0;
            b[u] = in ? b[u] : 0;
            c[u] = in ? c[u] : 0;
            d[u] = in ? d[u] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            num += a[u];
            att += b[u];
            disc += c[u];
            mx = d[u] > mx ? d[u] : mx;
        }
    }
    chunk_of(n_gen, blk, nblk, lo, hi);
    for (uint64_t i0 = lo; i0 < hi; i0 += 2 * U * kThreads) {
        uint32_t x[2 * U], y[2 * U];
#pragma unroll
        for (int u = 0; u < 2 * U; ++u) {
            const uint64_t i = i0 + (uint64_t)u * kThreads + threadIdx.x;
            const uint64_t ic = i < hi ? i : hi - 1;
            x[u] = gs.spawns[ic];
            y[u] = gs.deaths[ic];
            x[u] = i < hi ? x[u] : 0u;
            y[u] = i < hi ? y[u] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 2 * U; ++u) {
            sp += x[u];
            de += y[u];
        }
    }
    chunk_of(n_abs, blk, nblk, lo, hi);
    for (uint64_t i0 = lo; i0 < hi; i0 += 2 * U * kThreads) {
        double x[2 * U];
#pragma unroll
        for (int u = 0; u < 2 * U; ++u) {
            const uint64_t i = i0 + (uint64_t)u * kThreads + threadIdx.x;
            x[u] = abs_part[i < hi ? i : hi - 1];
            x[u] = i < hi ? x[u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 2 * U; ++u) tot += x[u];
    }
    FinalPart r{};
    r.num = num;
    r.tot = tot;
    r.att = att;
    r.disc = disc;
    r.sp = sp;
    r.de = de;
    r.mx = mx;
    return block_reduce_part(r);
}

// The step's scalars from the reduced statistics, by one thread.
__device__ __forceinline__ void final_write(const FinalPart &a, Scratch *sc, Scratch *copy, uint64_t seq)
{
    sc->num = a.num;
    sc->n_total = a.tot;
    sc->n_attempts = a.att;
    sc->n_discarded = a.disc;
    sc->max_n = a.mx;
    sc->n_spawns = a.sp;
    sc->n_deaths = a.de;
    // The step's scalars go straight to the host's pinned copy; the batch's sequence number is
    // stored last, behind a system-scope release, so the host that sees it sees the rest.
    Scratch c = *sc;
    c.seq = 0;  // no batch has number 0: the host waits for the release below
    *copy = c;
    __hip_atomic_store(&copy->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The second stage, by the whole last block: thread t sums parts t, t + kThreads, ... (in that
// order), then the block reduces in its fixed tree order.  All loads of a thread are issued
// before its first add.
constexpr int kFinalPerThread = 2;  // parts per thread: n <= kThreads * kFinalPerThread

__device__ __forceinline__ void final_body(uint32_t blk, uint32_t nblk, const FinalPart *__restrict__ in, uint64_t n, Scratch *sc,
                                           Scratch *copy, uint64_t seq)
{
    FinalPart b[kFinalPerThread];
#pragma unroll
    for (int u = 0; u < kFinalPerThread; ++u) {
        const uint64_t i = (uint64_t)u * kThreads + threadIdx.x;
        b[u] = in[i < n ? i : 0];
        if (i >= n) b[u] = FinalPart{};
    }
    FinalPart a{};
#pragma unroll
    for (int u = 0; u < kFinalPerThread; ++u) {
        a.num += b[u].num;
        a.tot += b[u].tot;
        a.att += b[u].att;
        a.disc += b[u].disc;
        a.sp += b[u].sp;
        a.de += b[u].de;
        a.mx = b[u].mx > a.mx ? b[u].mx : a.mx;
    }
    a = block_reduce_part(a);
    if (threadIdx.x == 0) final_write(a, sc, copy, seq);
}

struct FinalPartArgs {
    ItemPartials part;
    uint64_t n_parts;
    GenStats gs;
    uint64_t n_gen;
    const double *abs_part;
    uint64_t n_abs;
    Scratch *sc;
    uint64_t ne;
    FinalPart *out;
    uint64_t *done;  // blocks of this state finished (zero before the launch)
    Scratch *copy;   // device address of the host's pinned copy of the scalars
    uint64_t seq;
};

// Both stages of the reduction in one launch: each block publishes its part and counts
// itself done (a release atomic); the block that finishes last acquires, sums the parts in
// block order and hands the scalars to the host.  A state with one block hands its sum over
// directly.
__device__ __forceinline__ void k_final_part_entry(const FinalPartArgs &A, uint32_t blk, uint32_t nblk)
{
    const FinalPart r = final_part_body(blk, nblk, A.part, A.n_parts, A.gs, A.n_gen, A.abs_part, A.n_abs, A.sc, A.ne);
    if (nblk == 1) {  // the only block holds the whole sum: no hand-over between blocks
        if (threadIdx.x == 0) final_write(r, A.sc, A.copy, A.seq);
        return;
    }
    if (threadIdx.x == 0) A.out[blk] = r;
    __shared__ bool s_last;
    if (threadIdx.x == 0) {
        const uint64_t before = __hip_atomic_fetch_add(A.done, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        s_last = before + 1 == nblk;
    }
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // only the last block reads the others' parts
    final_body(blk, nblk, A.out, nblk, A.sc, A.copy, A.seq);
}

__global__ void __launch_bounds__(kThreads) k_final_part(const FinalPartArgs *__restrict__ args, BatchMap bm)
{
    uint32_t blk, nblk;
    k_final_part_entry(args[batch_state(bm, blk, nblk)], blk, nblk);
}

__global__ void __launch_bounds__(kThreads) k_final_part(const FinalPartArgs A)
{
    k_final_part_entry(A, blockIdx.x, gridDim.x);
}

// Clear each state's step area and the per-entry sums of its store.
struct ClearArgs {
    uint64_t *p;
    uint64_t n;
    double *delta;
    uint64_t ne;
};

__device__ __forceinline__ void k_clear_entry(const ClearArgs &A, uint32_t blk, uint32_t nblk)
{
    const uint64_t i = (uint64_t)blk * kThreads + threadIdx.x;
    if (i < A.n)
        A.p[i] = 0;
    else if (i - A.n < A.ne)
        A.delta[i - A.n] = 0.0;
}

__global__ void __launch_bounds__(kThreads) k_clear(const ClearArgs *__restrict__ args, BatchMap bm)
{
    uint32_t blk, nblk;
    k_clear_entry(args[batch_state(bm, blk, nblk)], blk, nblk);
}

__global__ void __launch_bounds__(kThreads) k_clear(const ClearArgs A)
{
    k_clear_entry(A, blockIdx.x, gridDim.x);
}

template <typename V>
__global__ void k_fill(V *p, uint64_t n, V v)
{
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) p[i] = v;
}

// Diagonal and truncated-space rank of imported store entries.
template <int W, typename T>
__global__ void __launch_bounds__(kThreads) k_store_init(const SysDev S, const uint64_t *__restrict__ key, uint64_t stride,
                                                         uint64_t n, T *__restrict__ K, uint64_t *__restrict__ rank)
{
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    uint64_t d[W];
#pragma unroll
    for (int w = 0; w < W; ++w) d[w] = key[(uint64_t)w * stride + i];
    K[i] = diagonal<W, T>(S, d);
    rank[i] = space_rank<W>(S, d);
}

// (PQ|RS) = sum_L B_LPQ B_LRS (the Cholesky-built two-electron table), summed over L in order.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_build_eri(const double *__restrict__ B, int n, int nchol, T *__restrict__ eri)
{
    const uint64_t t = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    const uint64_t nn = (uint64_t)n * n;
    if (t >= nn * nn) return;
    const uint64_t pq = t / nn, rs = t % nn;
    double v = 0.0;
    for (int L = 0; L < nchol; ++L) v += B[(uint64_t)L * nn + pq] * B[(uint64_t)L * nn + rs];
    eri[t] = (T)v;
}

}  // namespace ccmc
