// device.h -- device-side building blocks of the CCMC step on gfx950: Philox4x32-10,
// multi-word bitstring operations (popcount / select), fermionic signs by popcount,
// Slater-Condon elements for the UEG and molecule-like Hamiltonians, and the diagonal
// relative to E_HF.
//
// Paper: Spencer et al., arXiv:1807.03749, Sec. II (excitors, s_D, spawning sign).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccmc {

constexpr int kMaxWords = 8;
constexpr int kMaxClusterSize = 8;   // l + 2 with l <= 6
constexpr uint32_t kMaxAttempts = (1u << 30) - 2;
constexpr int kSystemUEG = 1;
constexpr int kSystemMol = 2;

enum Purpose : uint32_t { kSelect = 0, kSpawnSampled = 1, kSpawnNonComposite = 2, kRound = 3 };

// Constant description of the system, passed by value to every kernel.
struct SysDev {
    int kind, nel, M, nsp, l;
    uint32_t npairs, half;
    uint64_t hf[kMaxWords];
    // UEG
    int G;                 // half-width of the momentum lookup grid
    const int *grid;       // [(2G+1)^3] spatial index of a wavevector or -1
    const int *nvec;       // [nsp][3] integer wavevectors
    const void *vq;        // [dmax+1] Coulomb kernel 4 pi / (Omega |k|^2) by |dn|^2 (T)
    // molecular
    const void *h;         // [nsp][nsp] (T)
    const void *eri;       // [nsp^4] chemists' (PQ|RS) (T)
    // both
    const void *fock;      // [M] f_p = h_pp + sum_{j in HF} <pj||pj> (T)
    const void *vpair;     // [M][M] <pq||pq> (T)
    double p_single;
    // ranks in the truncated space (see space_rank)
    const uint64_t *binom_v;  // [(M+1) * 9]: C(n, j), j <= 8
    const uint64_t *binom_o;  // [(N+1) * (N+1)]: C(n, k), saturating
    const uint64_t *rank_v;   // [(M-N+1) * (l+1)]: rank term of a virtual orbital (see space_rank)
    // excitation generators
    const uint32_t *pairs;    // [N (N-1) / 2]: the pair (x < y) of each rank, x | y << 16 (lexicographic)
    const uint32_t *kpack;    // UEG [nsp]: wavevector components + G + 256 in 10-bit fields (x, y, z)
};

// Kernels specialised for one kind of system pass K = kSystemUEG or kSystemMol (the other
// kind's code is then dropped at compile time); K = 0 decides at run time.
template <int K>
__device__ __forceinline__ bool is_ueg(const SysDev &S)
{
    return K == kSystemUEG || (K == 0 && S.kind == kSystemUEG);
}

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror & Shaw (SC'11): ten rounds, two 32x32->64 products per round,
// Weyl key schedule.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32x32->64 multiply per product (both halves from a single instruction)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// A stream of 64-bit draws for (purpose, item k, attempt m) at step t: Philox block j
// uses counter (j, m, k, purpose << 28 | t); block words (x0..x3) give draws 2j and 2j+1 as
// x0 | x1 << 32 and x2 | x3 << 32.
struct Draws {
    uint32_t k0, k1, m, k, w;
    int have = -1;
    uint4 blk;
    __device__ Draws(uint32_t key0, uint32_t key1, uint32_t purpose, uint32_t item, uint32_t att, uint32_t step)
        : k0(key0), k1(key1), m(att), k(item), w((purpose << 28) | (step & 0x0FFFFFFFu)) {}
    __device__ __forceinline__ uint64_t get(int idx)
    {
        const int j = idx >> 1;
        if (j != have) {
            blk = philox4x32_10(make_uint4((uint32_t)j, m, k, w), k0, k1);
            have = j;
        }
        return (idx & 1) ? ((uint64_t)blk.z | ((uint64_t)blk.w << 32)) : ((uint64_t)blk.x | ((uint64_t)blk.y << 32));
    }
};

__device__ __forceinline__ double uniform53(uint64_t v) { return (double)(v >> 11) * 0x1.0p-53; }
// integer uniform in [0, n): high word of v * n
__device__ __forceinline__ uint64_t below(uint64_t v, uint64_t n) { return __umul64hi(v, n); }

// --------------------------------------------------------------- bitstring helpers
template <int W>
__device__ __forceinline__ bool bit_test(const uint64_t *d, int p)
{
    return (d[p >> 6] >> (p & 63)) & 1ull;
}
template <int W>
__device__ __forceinline__ void bit_flip(uint64_t *d, int p)
{
    d[p >> 6] ^= 1ull << (p & 63);
}
// number of set bits strictly below orbital p
template <int W>
__device__ __forceinline__ int count_below(const uint64_t *d, int p)
{
    int c = 0;
    const int wp = p >> 6;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        if (w < wp) c += __popcll(d[w]);
        if (w == wp) c += __popcll(d[w] & ((1ull << (p & 63)) - 1ull));
    }
    return c;
}
// position of the n-th set bit (0-based) of a 64-bit word
__device__ __forceinline__ int select64(uint64_t x, int n)
{
    // the half first, then five halving rounds on 32-bit words
    const uint32_t lo = (uint32_t)x;
    const int c0 = __popc(lo);
    const bool up = n >= c0;
    uint32_t v = up ? (uint32_t)(x >> 32) : lo;
    n = up ? n - c0 : n;
    int pos = up ? 32 : 0;
#pragma unroll
    for (int s = 16; s > 0; s >>= 1) {
        const int c = __popc(v & ((1u << s) - 1u));
        const bool g = n >= c;
        n = g ? n - c : n;
        v = g ? v >> s : v;
        pos += g ? s : 0;
    }
    return pos;
}
// orbital of the n-th occupied spin orbital of d (-1 if d has at most n): the word is chosen
// by running popcounts, then one select within it
template <int W>
__device__ __forceinline__ int select_bit(const uint64_t *d, int n)
{
    uint64_t x = d[0];
    int base = 0;
    bool found = false;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int c = __popcll(d[w]);
        const bool here = !found && n < c;
        x = here ? d[w] : x;
        base = here ? 64 * w : base;
        n = (found || here) ? n : n - c;
        found = found || here;
    }
    return found ? base + select64(x, n) : -1;
}
template <int W>
__device__ __forceinline__ int popcount(const uint64_t *d)
{
    int c = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) c += __popcll(d[w]);
    return c;
}
// excitation level relative to the reference: number of occupied non-reference orbitals
template <int W>
__device__ __forceinline__ int level_of(const SysDev &S, const uint64_t *d)
{
    int c = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) c += __popcll(d[w] & ~S.hf[w]);
    return c;
}
template <int W>
__device__ __forceinline__ bool key_equal(const uint64_t *a, const uint64_t *b)
{
    bool e = true;
#pragma unroll
    for (int w = 0; w < W; ++w) e &= (a[w] == b[w]);
    return e;
}
// -1, 0, 1 ordering as W-word unsigned integers, most significant word first
template <int W>
__device__ __forceinline__ int key_cmp(const uint64_t *a, const uint64_t *b)
{
#pragma unroll
    for (int w = W - 1; w >= 0; --w) {
        if (a[w] != b[w]) return a[w] < b[w] ? -1 : 1;
    }
    return 0;
}

// s_D(i) = <D_i| c_i |D_HF> (Sec. II, eq. 6).  With the reference on orbitals 0..N-1,
// annihilating the holes i_1 < .. < i_L in turn gives (-1)^(sum_k i_k - L(L-1)/2), and each
// creator passes the N-L remaining reference electrons: (-1)^(L(N-L)).  The parity of
// sum_k i_k is the parity of the number of odd-numbered holes.
template <int W>
__device__ __forceinline__ int excitor_sign(const SysDev &S, const uint64_t *d)
{
    int L = 0, odd = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint64_t holes = S.hf[w] & ~d[w];
        L += __popcll(holes);
        odd += __popcll(holes & 0xAAAAAAAAAAAAAAAAull);
    }
    const int e = odd - (L * (L - 1)) / 2 + L * (S.nel - L);
    return (e & 1) ? -1 : 1;
}

// ------------------------------------------------------------------- integrals
// <pq|rs> with spin deltas; momentum conservation is guaranteed by the callers (UEG).
template <typename T, int K = 0>
__device__ __forceinline__ T u2(const SysDev &S, int p, int q, int r, int s)
{
    if (((p ^ r) & 1) | ((q ^ s) & 1)) return T(0);
    const int P = p >> 1, Q = q >> 1, R = r >> 1, X = s >> 1;
    if (is_ueg<K>(S)) {
        const int *np = S.nvec + 3 * P, *nr = S.nvec + 3 * R;
        const int dx = np[0] - nr[0], dy = np[1] - nr[1], dz = np[2] - nr[2];
        const int d2 = dx * dx + dy * dy + dz * dz;
        if (d2 == 0) return T(0);
        return static_cast<const T *>(S.vq)[d2];
    }
    const size_t n = (size_t)S.nsp;
    return static_cast<const T *>(S.eri)[((P * n + R) * n + Q) * n + X];
}
template <typename T, int K = 0>
__device__ __forceinline__ T anti(const SysDev &S, int p, int q, int r, int s)
{
    return u2<T, K>(S, p, q, r, s) - u2<T, K>(S, p, q, s, r);
}
template <typename T, int K = 0>
__device__ __forceinline__ T h1(const SysDev &S, int p, int q)
{
    if ((p ^ q) & 1) return T(0);
    if (is_ueg<K>(S)) return T(0);  // only used off-diagonal (singles)
    return static_cast<const T *>(S.h)[(size_t)(p >> 1) * S.nsp + (q >> 1)];
}

// <D'| H |D> for D' = D with f1 < f2 replaced by t1 < t2 (a double excitation):
// gamma <t1 t2 || f1 f2> with gamma = <D'| c+_t1 c+_t2 c_f2 c_f1 |D> from popcounts.
template <int W, typename T, int K = 0>
__device__ __forceinline__ T double_element(const SysDev &S, const uint64_t *d, int f1, int f2, int t1, int t2)
{
    uint64_t x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = d[w];
    int e = count_below<W>(x, f1);
    bit_flip<W>(x, f1);
    e += count_below<W>(x, f2);
    bit_flip<W>(x, f2);
    e += count_below<W>(x, t2);
    bit_flip<W>(x, t2);
    e += count_below<W>(x, t1);
    const T v = anti<T, K>(S, t1, t2, f1, f2);
    return (e & 1) ? -v : v;
}

// <D'| H |D> for D' = D with f replaced by t (a single excitation):
// gamma (h_tf + sum_{k in D} <tk||fk>) with gamma = <D'| c+_t c_f |D>.
template <int W, typename T, int K = 0>
__device__ __forceinline__ T single_element(const SysDev &S, const uint64_t *d, int f, int t)
{
    uint64_t x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = d[w];
    int e = count_below<W>(x, f);
    bit_flip<W>(x, f);
    e += count_below<W>(x, t);
    T v = h1<T, K>(S, t, f);
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint64_t m = d[w];
        while (m) {
            const int k = 64 * w + __ffsll((long long)m) - 1;
            m &= m - 1;
            v += anti<T, K>(S, t, k, f, k);
        }
    }
    return (e & 1) ? -v : v;
}

// <D_HF| H |D> for an excitor of level 1 or 2 (projected energy, Sec. II eq. 7).
template <int W, typename T>
__device__ __forceinline__ T reference_element(const SysDev &S, const uint64_t *d, int L)
{
    int parts[2], holes[2], np = 0, nh = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint64_t p = d[w] & ~S.hf[w], h = S.hf[w] & ~d[w];
        while (p && np < 2) {
            parts[np++] = 64 * w + __ffsll((long long)p) - 1;
            p &= p - 1;
        }
        while (h && nh < 2) {
            holes[nh++] = 64 * w + __ffsll((long long)h) - 1;
            h &= h - 1;
        }
    }
    if (L == 1) return single_element<W, T>(S, d, parts[0], holes[0]);
    return double_element<W, T>(S, d, parts[0], parts[1], holes[0], holes[1]);
}

// ------------------------------------------------ virtual processors (Sec. III)
// MurmurHash2 (A. Appleby, 32-bit) of the W words of d read as 8W little-endian bytes: two
// 4-byte blocks per word, low half first.  8W is a multiple of 4, so there is no tail.
template <int W>
__device__ __forceinline__ uint32_t murmur2_det(const uint64_t *d, uint32_t seed)
{
    constexpr uint32_t m = 0x5bd1e995u;
    uint32_t h = seed ^ (uint32_t)(8 * W);
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            uint32_t k = (uint32_t)(d[w] >> (32 * half));
            k *= m;
            k ^= k >> 24;
            k *= m;
            h *= m;
            h ^= k;
        }
    h ^= h >> 13;
    h *= m;
    h ^= h >> 15;
    return h;
}

constexpr uint32_t kMaxRanks = 512;  // one radix pass partitions the store by processor

// eq. 9: o = (hash(D) + i_tau) >> nu_move, p = hash(D xor o) mod N_p, with o xored
// into word 0; nu_move >= 64 leaves o = 0 (the static placement hash(D) mod N_p).
template <int W>
__device__ __forceinline__ uint32_t placement(const uint64_t *d, uint64_t i_tau, uint32_t n_ranks,
                                              uint32_t move_shift, uint32_t seed)
{
    if (n_ranks <= 1) return 0;
    const uint64_t o = move_shift >= 64 ? 0 : ((uint64_t)murmur2_det<W>(d, seed) + i_tau) >> move_shift;
    uint64_t x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = d[w];
    x[0] ^= o;
    return murmur2_det<W>(x, seed) % n_ranks;
}

// K_D = H_DD - E_HF from the holes I and particles A of D:
// sum_A f_a - sum_I f_i + sum_{a<b} <ab||ab> + sum_{i<j} <ij||ij> - sum_{a,i} <ai||ai>.
// With IssueAll, up to kDiagFast holes and particles every table load is issued before the
// first add (clamped indices, absent terms added as zero, so the sum and its order are those
// of the plain loops): for callers with few waves to hide the latency of dependent loads.
// Callers at full occupancy keep the plain loops, which hold fewer registers.
constexpr int kDiagFast = 4;

template <int W, typename T, bool IssueAll = false>
__device__ __forceinline__ T diagonal(const SysDev &S, const uint64_t *d)
{
    int hole[kMaxClusterSize], part[kMaxClusterSize], nh = 0, np = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint64_t p = d[w] & ~S.hf[w], h = S.hf[w] & ~d[w];
        while (p && np < kMaxClusterSize) {
            part[np++] = 64 * w + __ffsll((long long)p) - 1;
            p &= p - 1;
        }
        while (h && nh < kMaxClusterSize) {
            hole[nh++] = 64 * w + __ffsll((long long)h) - 1;
            h &= h - 1;
        }
    }
    const T *f = static_cast<const T *>(S.fock);
    const T *V = static_cast<const T *>(S.vpair);
    const size_t M = (size_t)S.M;
    T k = T(0);
    if (IssueAll && np <= kDiagFast && nh <= kDiagFast) {
        constexpr int F = kDiagFast;
        int pa[F], ho[F];
#pragma unroll
        for (int x = 0; x < F; ++x) {
            pa[x] = x < np ? part[x] : 0;
            ho[x] = x < nh ? hole[x] : 0;
        }
        T fp[F], fh[F], vpp[F * (F - 1) / 2], vhh[F * (F - 1) / 2], vph[F * F];
#pragma unroll
        for (int x = 0; x < F; ++x) {
            fp[x] = f[pa[x]];
            fh[x] = f[ho[x]];
        }
#pragma unroll
        for (int a = 0, c = 0; a < F; ++a)
#pragma unroll
            for (int b = a + 1; b < F; ++b, ++c) {
                vpp[c] = V[pa[a] * M + pa[b]];
                vhh[c] = V[ho[a] * M + ho[b]];
            }
#pragma unroll
        for (int a = 0; a < F; ++a)
#pragma unroll
            for (int i = 0; i < F; ++i) vph[a * F + i] = V[pa[a] * M + ho[i]];
#pragma unroll
        for (int a = 0; a < F; ++a) k += a < np ? fp[a] : T(0);
#pragma unroll
        for (int i = 0; i < F; ++i) k -= i < nh ? fh[i] : T(0);
#pragma unroll
        for (int a = 0, c = 0; a < F; ++a)
#pragma unroll
            for (int b = a + 1; b < F; ++b, ++c) k += b < np ? vpp[c] : T(0);
#pragma unroll
        for (int a = 0, c = 0; a < F; ++a)
#pragma unroll
            for (int b = a + 1; b < F; ++b, ++c) k += b < nh ? vhh[c] : T(0);
#pragma unroll
        for (int a = 0; a < F; ++a)
#pragma unroll
            for (int i = 0; i < F; ++i) k -= (a < np && i < nh) ? vph[a * F + i] : T(0);
        return k;
    }
    for (int a = 0; a < np; ++a) k += f[part[a]];
    for (int i = 0; i < nh; ++i) k -= f[hole[i]];
    for (int a = 0; a < np; ++a)
        for (int b = a + 1; b < np; ++b) k += V[part[a] * M + part[b]];
    for (int i = 0; i < nh; ++i)
        for (int j = i + 1; j < nh; ++j) k += V[hole[i] * M + hole[j]];
    for (int a = 0; a < np; ++a)
        for (int i = 0; i < nh; ++i) k -= V[part[a] * M + hole[i]];
    return k;
}

// Rank of a determinant among all determinants with N electrons and excitation level <= l,
// in ascending bitstring order: the number of such D' < D.  Walking the set bits of D from
// the top, D' agrees with D above bit p, has p empty, and places the remaining k electrons
// below p: j of them in the virtual orbitals [N, p) and k - j in [0, min(p, N)), with at most
// l - v virtual ones in total (v = virtual electrons of D above p).  The rank is monotone in
// the key order, so sorting records by rank groups equal determinants and keeps the store's
// key order, with ceil(log2(space)) bits instead of M.
template <int W>
__device__ __forceinline__ uint64_t space_rank(const SysDev &S, const uint64_t *d)
{
    // Above the reference orbitals every electron placed so far is virtual (a = v, k = N - v),
    // and the sum over j is tabulated per (p - N, v) in rank_v.  Below them D' has no
    // virtual electron left to place below p (nv = 0): only j = 0 counts, C(p, k).
    const int N = S.nel, l = S.l;
    uint64_t r = 0;
    int a = 0;
#pragma unroll
    for (int w = W - 1; w >= 0; --w) {
        uint64_t m = d[w] & ~S.hf[w];
        while (m) {
            const int p = 64 * w + 63 - __clzll((long long)m);
            m &= ~(1ull << (p & 63));
            if (a <= l) r += S.rank_v[(p - N) * (l + 1) + a];
            ++a;
        }
    }
#pragma unroll
    for (int w = W - 1; w >= 0; --w) {
        uint64_t m = d[w] & S.hf[w];
        while (m) {
            const int p = 64 * w + 63 - __clzll((long long)m);
            m &= ~(1ull << (p & 63));
            const int k = N - a;
            if (k <= p) r += S.binom_o[p * (N + 1) + k];
            ++a;
        }
    }
    return r;
}

// The determinant of rank r (the inverse of space_rank): orbitals are decided from the top.
// With the bits above p fixed (a electrons placed, v of them virtual), the determinants that
// leave p empty number S(p) = sum_j C(virtual orbitals below p, j) C(reference orbitals below
// p, k - j) over j <= l - v (k = N - a electrons still to place), and they all come before the
// ones that fill p: p is filled iff r >= S(p), and then r drops by S(p).  As in space_rank,
// S(p) is rank_v[p - N][v] above the reference orbitals and C(p, k) below them.
template <int W>
__device__ __forceinline__ void space_unrank(const SysDev &S, uint64_t r, uint64_t *d)
{
    const int N = S.nel, l = S.l;
#pragma unroll
    for (int w = 0; w < W; ++w) d[w] = 0;
    int a = 0;
    for (int p = S.M - 1; p >= N && a < N; --p) {
        const uint64_t empty = a <= l ? S.rank_v[(p - N) * (l + 1) + a] : 0;
        if (r >= empty) {
            r -= empty;
            d[p >> 6] |= 1ull << (p & 63);
            ++a;
        }
    }
    for (int p = (N < S.M ? N : S.M) - 1; p >= 0 && a < N; --p) {
        const int k = N - a;
        const uint64_t empty = k <= p ? S.binom_o[p * (N + 1) + k] : 0;
        if (r >= empty) {
            r -= empty;
            d[p >> 6] |= 1ull << (p & 63);
            ++a;
        }
    }
}

// Cluster-size distribution: p(s) = 2^-(s-lo+1) for lo <= s < hi, the remainder at hi.
__device__ __forceinline__ int draw_size(double u, int lo, int hi)
{
    double c = 0.0;
    for (int s = lo; s < hi; ++s) {
        c += ldexp(1.0, -(s - lo + 1));
        if (u < c) return s;
    }
    return hi;
}
__device__ __forceinline__ double size_prob(int s, int lo, int hi)
{
    return (s < hi) ? ldexp(1.0, -(s - lo + 1)) : ldexp(1.0, -(hi - lo));
}

}  // namespace ccmc
