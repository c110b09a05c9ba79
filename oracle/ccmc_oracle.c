/*
 * ccmc_oracle.c -- plain, serial, FP64 CPU oracle of one CCMC time step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the CPU
 * baseline of the benchmark; never by the product path.  It shares no code with the HIP
 * library.  It is deliberately slow: fermionic signs come from applying operators one by
 * one to sorted orbital lists, matrix elements from the general Slater-Condon rules,
 * annihilation from a sort of all records followed by a left fold.
 *
 * Paper: Spencer et al., arXiv:1807.03749 (section / equation named at each function).
 */
#include "ccmc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXW ORC_MAXW
#define MAXM (64 * MAXW)
#define MAX_SLOT ((uint64_t)1 << 30)          /* record slot field width */
#define MAX_ATTEMPTS (MAX_SLOT - 2)          /* slot 0 is the death record */

enum { KIND_UEG = 1, KIND_MOL = 2 };

struct orc_system {
    int kind;
    int nel, M, W, nsp;
    double L, omega;  /* UEG box length and volume */
    int *nvec;        /* UEG: integer wavevector per spatial orbital, [nsp][3] */
    double *h;        /* molecular: one-electron integrals [nsp][nsp] */
    double *eri;      /* molecular: chemists' (PQ|RS), [nsp^4] */
    uint64_t hf[MAXW];
    double ehf;
};

typedef struct {
    uint64_t key[MAXW];
    double amp;
    uint64_t id;
} record;

struct orc_run {
    const orc_system *sys;
    int l;  /* truncation level */
    orc_options opt;
    uint64_t step;
    double n0;
    uint64_t n;        /* store size */
    uint64_t cap;
    uint64_t *keys;    /* [cap][W] */
    double *amps;      /* [cap] */
    uint64_t *q;       /* fixed-point weights of the current store */
    uint64_t *pref;    /* inclusive prefix of q */
    uint64_t qtot;
    record *rec;
    uint64_t nrec, caprec;
};

/* ------------------------------------------------------------------------- bits */

static int getbit(const uint64_t *d, int p) { return (int)((d[p >> 6] >> (p & 63)) & 1u); }
static void setbit(uint64_t *d, int p) { d[p >> 6] |= (uint64_t)1 << (p & 63); }
static void clrbit(uint64_t *d, int p) { d[p >> 6] &= ~((uint64_t)1 << (p & 63)); }

/* Sorted list of occupied spin orbitals. */
static int occ_list(const orc_system *S, const uint64_t *d, int *occ)
{
    int n = 0;
    for (int p = 0; p < S->M; ++p)
        if (getbit(d, p)) occ[n++] = p;
    return n;
}

static int count_bits(const orc_system *S, const uint64_t *d)
{
    int n = 0;
    for (int p = 0; p < S->M; ++p) n += getbit(d, p);
    return n;
}

/* Keys compare as W-word unsigned integers, most significant word first. */
static int key_cmp(int W, const uint64_t *a, const uint64_t *b)
{
    for (int w = W - 1; w >= 0; --w) {
        if (a[w] < b[w]) return -1;
        if (a[w] > b[w]) return 1;
    }
    return 0;
}

/* ------------------------------------------------ operators on sorted orbital lists */
/* |occ> = c+_{occ[0]} c+_{occ[1]} ... |0>, occ ascending (Sec. II, determinant string). */

/* Apply c_p.  Moving c_p to the position of c+_p passes k creators: sign (-1)^k. */
static int op_annihilate(int *occ, int *n, int p)
{
    for (int k = 0; k < *n; ++k) {
        if (occ[k] == p) {
            memmove(occ + k, occ + k + 1, (size_t)(*n - k - 1) * sizeof(int));
            (*n)--;
            return (k & 1) ? -1 : 1;
        }
    }
    return 0;
}

/* Apply c+_p.  Moving c+_p into ascending position passes k creators: sign (-1)^k. */
static int op_create(int *occ, int *n, int p)
{
    int k = 0;
    while (k < *n && occ[k] < p) ++k;
    if (k < *n && occ[k] == p) return 0;
    memmove(occ + k + 1, occ + k, (size_t)(*n - k) * sizeof(int));
    occ[k] = p;
    (*n)++;
    return (k & 1) ? -1 : 1;
}

/* Holes (HF orbitals absent from det) and particles (non-HF orbitals present), ascending. */
static int holes_particles(const orc_system *S, const uint64_t *d, int *holes, int *parts)
{
    int nh = 0, np = 0;
    for (int p = 0; p < S->M; ++p) {
        int in_hf = getbit(S->hf, p), in_d = getbit(d, p);
        if (in_hf && !in_d) holes[nh++] = p;
        if (!in_hf && in_d) parts[np++] = p;
    }
    return (nh == np) ? nh : -1;
}

/* Apply the excitor c^{a1..aL}_{i1..iL} = c+_{a1} .. c+_{aL} c_{iL} .. c_{i1} (Sec. II, eq. 4):
 * the rightmost operator c_{i1} acts first.  Returns the accumulated sign, 0 if it vanishes. */
static int apply_excitor(int *occ, int *n, const int *holes, const int *parts, int L)
{
    int sign = 1;
    for (int k = 0; k < L; ++k) {
        int sg = op_annihilate(occ, n, holes[k]);
        if (!sg) return 0;
        sign *= sg;
    }
    for (int k = L - 1; k >= 0; --k) {
        int sg = op_create(occ, n, parts[k]);
        if (!sg) return 0;
        sign *= sg;
    }
    return sign;
}

int orc_excitation_level(const orc_system *S, const uint64_t *det)
{
    int holes[MAXM], parts[MAXM];
    return holes_particles(S, det, holes, parts);
}

/* s_D(i) = <D_i| c_i |D_HF> (Sec. II, eq. 6). */
int orc_excitor_sign(const orc_system *S, const uint64_t *det)
{
    int holes[MAXM], parts[MAXM], occ[MAXM];
    int L = holes_particles(S, det, holes, parts);
    if (L < 0) return 0;
    int n = occ_list(S, S->hf, occ);
    int sign = apply_excitor(occ, &n, holes, parts, L);
    /* the result must be det itself */
    uint64_t chk[MAXW] = {0};
    for (int k = 0; k < n; ++k) setbit(chk, occ[k]);
    if (key_cmp(S->W, chk, det) != 0) return 0;
    return sign;
}

/* Collapse c_{X1} c_{X2} .. c_{Xs} to sigma * c_{X} (Sec. II, text after eq. 5): write out the
 * whole operator string, then bubble it into canonical order (creators ascending, then
 * annihilators descending), one transposition of two distinct fermion operators at a time. */
int orc_collapse(const orc_system *S, int s, const uint64_t *keys, uint64_t *out, int *sign)
{
    int rank[2 * MAXM];
    int nops = 0;
    int used_h[MAXM] = {0}, used_p[MAXM] = {0};
    for (int r = 0; r < s; ++r) {
        int holes[MAXM], parts[MAXM];
        int L = holes_particles(S, keys + (size_t)r * S->W, holes, parts);
        if (L < 0) return 0;
        for (int k = 0; k < L; ++k) {
            if (used_h[holes[k]] || used_p[parts[k]]) return 0; /* c_i c_i = 0, c+_a c+_a = 0 */
            used_h[holes[k]] = 1;
            used_p[parts[k]] = 1;
        }
        /* creators a1 < .. < aL written left to right: canonical rank = orbital */
        for (int k = 0; k < L; ++k) rank[nops++] = parts[k];
        /* annihilators written c_{iL} .. c_{i1}: canonical rank M + (M - 1 - orbital) */
        for (int k = L - 1; k >= 0; --k) rank[nops++] = S->M + (S->M - 1 - holes[k]);
    }
    int sg = 1;
    for (int pass = 0; pass < nops; ++pass)
        for (int k = 0; k + 1 < nops; ++k)
            if (rank[k] > rank[k + 1]) {
                int tmp = rank[k];
                rank[k] = rank[k + 1];
                rank[k + 1] = tmp;
                sg = -sg;
            }
    memcpy(out, S->hf, sizeof(uint64_t) * (size_t)S->W);
    for (int p = 0; p < S->M; ++p) {
        if (used_h[p]) clrbit(out, p);
        if (used_p[p]) setbit(out, p);
    }
    *sign = sg;
    return 1;
}

/* ------------------------------------------------------------------- integrals */

/* h_pq (spin orbitals).  UEG: kinetic energy |k|^2/2 with k = 2 pi n / L. */
double orc_h1(const orc_system *S, int p, int q)
{
    if ((p & 1) != (q & 1)) return 0.0;
    int P = p >> 1, Q = q >> 1;
    if (S->kind == KIND_UEG) {
        if (P != Q) return 0.0;
        const int *n = S->nvec + 3 * P;
        double kf = 2.0 * M_PI / S->L;
        return 0.5 * kf * kf * (double)(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    }
    return S->h[(size_t)P * S->nsp + Q];
}

/* <pq|rs> (physicists').  UEG: 4 pi / (Omega |k_p - k_r|^2) when momentum is conserved and
 * spins match, with the q = 0 term omitted.  Molecular: (PR|QS) with spin deltas. */
double orc_u2(const orc_system *S, int p, int q, int r, int s)
{
    if ((p & 1) != (r & 1) || (q & 1) != (s & 1)) return 0.0;
    int P = p >> 1, Q = q >> 1, R = r >> 1, Sx = s >> 1;
    if (S->kind == KIND_UEG) {
        const int *np = S->nvec + 3 * P, *nq = S->nvec + 3 * Q, *nr = S->nvec + 3 * R,
                  *ns = S->nvec + 3 * Sx;
        for (int c = 0; c < 3; ++c)
            if (np[c] + nq[c] != nr[c] + ns[c]) return 0.0;
        int d2 = 0;
        for (int c = 0; c < 3; ++c) d2 += (np[c] - nr[c]) * (np[c] - nr[c]);
        if (d2 == 0) return 0.0;
        double kf = 2.0 * M_PI / S->L;
        return 4.0 * M_PI / (S->omega * (kf * kf * (double)d2));
    }
    size_t n = (size_t)S->nsp;
    return S->eri[((P * n + R) * n + Q) * n + Sx];
}

static double anti(const orc_system *S, int p, int q, int r, int s)
{
    return orc_u2(S, p, q, r, s) - orc_u2(S, p, q, s, r);
}

/* ------------------------------------------------------------- Slater-Condon rules */

double orc_hamiltonian(const orc_system *S, const uint64_t *bra, const uint64_t *ket)
{
    int occ[MAXM];
    int nk = occ_list(S, ket, occ);
    int holes[4], parts[4], nh = 0, np = 0;  /* holes: in ket only; parts: in bra only */
    for (int p = 0; p < S->M; ++p) {
        int b = getbit(bra, p), k = getbit(ket, p);
        if (k && !b) {
            if (nh == 2) return 0.0;
            holes[nh++] = p;
        }
        if (b && !k) {
            if (np == 2) return 0.0;
            parts[np++] = p;
        }
    }
    if (nh != np) return 0.0;
    if (nh == 0) {
        double e1 = 0.0, e2 = 0.0;
        for (int a = 0; a < nk; ++a) e1 += orc_h1(S, occ[a], occ[a]);
        for (int a = 0; a < nk; ++a)
            for (int b = 0; b < nk; ++b) e2 += anti(S, occ[a], occ[b], occ[a], occ[b]);
        return e1 + 0.5 * e2;
    }
    int work[MAXM], n = nk, sign = 1;
    memcpy(work, occ, sizeof(int) * (size_t)nk);
    if (nh == 1) {
        int i = holes[0], a = parts[0];
        sign *= op_annihilate(work, &n, i);
        sign *= op_create(work, &n, a);
        double v = orc_h1(S, a, i);
        for (int k = 0; k < nk; ++k) v += anti(S, a, occ[k], i, occ[k]);
        return sign * v;
    }
    /* double: <bra| c+_a c+_b c_j c_i |ket> <ab||ij>, i < j, a < b */
    int i = holes[0], j = holes[1], a = parts[0], b = parts[1];
    sign *= op_annihilate(work, &n, i);
    sign *= op_annihilate(work, &n, j);
    sign *= op_create(work, &n, b);
    sign *= op_create(work, &n, a);
    return sign * anti(S, a, b, i, j);
}

double orc_ehf(const orc_system *S) { return S->ehf; }

/* ------------------------------------------------------------------------ systems */

static int cmp_nvec(const void *x, const void *y)
{
    const int *a = (const int *)x, *b = (const int *)y;
    int na = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    int nb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    if (na != nb) return na < nb ? -1 : 1;
    for (int c = 0; c < 3; ++c)
        if (a[c] != b[c]) return a[c] < b[c] ? -1 : 1;
    return 0;
}

static void finish_system(orc_system *S)
{
    S->W = (S->M + 63) / 64;
    memset(S->hf, 0, sizeof S->hf);
    for (int p = 0; p < S->nel; ++p) setbit(S->hf, p);
    S->ehf = orc_hamiltonian(S, S->hf, S->hf);
}

/* 3D UEG in a cubic box of volume Omega = N (4 pi / 3) r_s^3; plane waves with
 * |n|^2 <= n2max, ordered by (|n|^2, n_x, n_y, n_z). */
int orc_system_ueg(int n_el, int n2max, double rs, orc_system **out)
{
    if (n_el < 2 || (n_el & 1) || n2max < 0 || !(rs > 0)) return ORC_EINVAL;
    int nmax = 0;
    while ((nmax + 1) * (nmax + 1) <= n2max) ++nmax;
    int cap = (2 * nmax + 1) * (2 * nmax + 1) * (2 * nmax + 1);
    int *nv = (int *)malloc(sizeof(int) * 3 * (size_t)cap);
    if (!nv) return ORC_ENOMEM;
    int cnt = 0;
    for (int x = -nmax; x <= nmax; ++x)
        for (int y = -nmax; y <= nmax; ++y)
            for (int z = -nmax; z <= nmax; ++z)
                if (x * x + y * y + z * z <= n2max) {
                    nv[3 * cnt] = x;
                    nv[3 * cnt + 1] = y;
                    nv[3 * cnt + 2] = z;
                    ++cnt;
                }
    qsort(nv, (size_t)cnt, 3 * sizeof(int), cmp_nvec);
    int nocc = n_el / 2;
    if (2 * cnt > MAXM || nocc > cnt) {
        free(nv);
        return ORC_EINVAL;
    }
    if (nocc < cnt) {
        /* open shell if the last occupied and the first virtual share |n|^2 */
        const int *a = nv + 3 * (nocc - 1), *b = nv + 3 * nocc;
        if (a[0] * a[0] + a[1] * a[1] + a[2] * a[2] == b[0] * b[0] + b[1] * b[1] + b[2] * b[2]) {
            free(nv);
            return ORC_EINVAL;
        }
    }
    orc_system *S = (orc_system *)calloc(1, sizeof *S);
    if (!S) {
        free(nv);
        return ORC_ENOMEM;
    }
    S->kind = KIND_UEG;
    S->nel = n_el;
    S->nsp = cnt;
    S->M = 2 * cnt;
    S->nvec = nv;
    S->L = rs * cbrt(4.0 * M_PI * n_el / 3.0);
    S->omega = S->L * S->L * S->L;
    finish_system(S);
    *out = S;
    return 0;
}

/* Molecule-like system: (PQ|RS) = sum_L B_LPQ B_LRS built from the Cholesky vectors. */
int orc_system_mol(int n_el, int n_spatial, const double *h, const double *chol, int n_chol,
                   orc_system **out)
{
    if (n_el < 2 || (n_el & 1) || n_spatial < 1 || 2 * n_spatial > MAXM || n_el > 2 * n_spatial ||
        n_chol < 0 || !h || (n_chol > 0 && !chol))
        return ORC_EINVAL;
    orc_system *S = (orc_system *)calloc(1, sizeof *S);
    if (!S) return ORC_ENOMEM;
    size_t n = (size_t)n_spatial;
    S->kind = KIND_MOL;
    S->nel = n_el;
    S->nsp = n_spatial;
    S->M = 2 * n_spatial;
    S->h = (double *)malloc(sizeof(double) * n * n);
    S->eri = (double *)calloc(n * n * n * n, sizeof(double));
    if (!S->h || !S->eri) {
        orc_system_free(S);
        return ORC_ENOMEM;
    }
    memcpy(S->h, h, sizeof(double) * n * n);
    for (size_t P = 0; P < n; ++P)
        for (size_t Q = 0; Q < n; ++Q)
            for (size_t R = 0; R < n; ++R)
                for (size_t T = 0; T < n; ++T) {
                    double v = 0.0;
                    for (int L = 0; L < n_chol; ++L)
                        v += chol[((size_t)L * n + P) * n + Q] * chol[((size_t)L * n + R) * n + T];
                    S->eri[((P * n + Q) * n + R) * n + T] = v;
                }
    finish_system(S);
    *out = S;
    return 0;
}

void orc_system_free(orc_system *S)
{
    if (!S) return;
    free(S->nvec);
    free(S->h);
    free(S->eri);
    free(S);
}

int orc_system_dims(const orc_system *S, int *n_el, int *n_so, int *n_words)
{
    if (!S) return ORC_EINVAL;
    if (n_el) *n_el = S->nel;
    if (n_so) *n_so = S->M;
    if (n_words) *n_words = S->W;
    return 0;
}

int orc_ueg_nvec(const orc_system *S, int *out)
{
    if (!S || S->kind != KIND_UEG) return ORC_EINVAL;
    memcpy(out, S->nvec, sizeof(int) * 3 * (size_t)S->nsp);
    return 0;
}

double orc_ueg_box_length(const orc_system *S) { return S->kind == KIND_UEG ? S->L : 0.0; }

/* ------------------------------------------------------------------------ Philox */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two 32x32->64
 * multiplications, with a Weyl-sequence key schedule. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

enum { PURPOSE_SELECT = 0, PURPOSE_SPAWN_SAMPLED = 1, PURPOSE_SPAWN_NONCOMP = 2, PURPOSE_ROUND = 3 };

/* The idx-th 64-bit draw of item k, attempt m, for a purpose at step t.  Philox block
 * j = idx / 2 uses counter (j, m, k, purpose << 28 | t) and key (seed lo, seed hi); the
 * block's words (x0, x1, x2, x3) give the draws x0 | x1 << 32 and x2 | x3 << 32. */
static uint64_t draw(const orc_run *R, int purpose, uint64_t k, uint64_t m, int idx)
{
    uint32_t ctr[4] = {(uint32_t)(idx / 2), (uint32_t)m, (uint32_t)k,
                       ((uint32_t)purpose << 28) | (uint32_t)(R->step & 0x0FFFFFFFu)};
    uint32_t key[2] = {(uint32_t)R->opt.seed, (uint32_t)(R->opt.seed >> 32)};
    uint32_t x[4];
    orc_philox(ctr, key, x);
    if (idx % 2 == 0) return (uint64_t)x[0] | ((uint64_t)x[1] << 32);
    return (uint64_t)x[2] | ((uint64_t)x[3] << 32);
}

static double uniform(uint64_t v) { return (double)(v >> 11) * 0x1.0p-53; }

/* Integer uniform in [0, n): the high word of v * n. */
static uint64_t below(uint64_t v, uint64_t n)
{
    return (uint64_t)(((unsigned __int128)v * (unsigned __int128)n) >> 64);
}

/* ------------------------------------------------------------ virtual processors */
/* MurmurHash2 (Austin Appleby; 32-bit, public domain): 4-byte little-endian blocks, each
 * mixed by multiply-xorshift-multiply and folded into h = h * m ^ k; the 1-3 tail bytes; a
 * final avalanche. */
uint32_t orc_murmur2(const void *key, int len, uint32_t seed)
{
    const uint32_t m = 0x5bd1e995u;
    const unsigned char *b = (const unsigned char *)key;
    uint32_t h = seed ^ (uint32_t)len;
    while (len >= 4) {
        uint32_t k = (uint32_t)b[0] | (uint32_t)b[1] << 8 | (uint32_t)b[2] << 16 | (uint32_t)b[3] << 24;
        k *= m;
        k ^= k >> 24;
        k *= m;
        h *= m;
        h ^= k;
        b += 4;
        len -= 4;
    }
    if (len == 3) h ^= (uint32_t)b[2] << 16;
    if (len >= 2) h ^= (uint32_t)b[1] << 8;
    if (len >= 1) {
        h ^= (uint32_t)b[0];
        h *= m;
    }
    h ^= h >> 13;
    h *= m;
    h ^= h >> 15;
    return h;
}

static uint32_t hash_det(int W, const uint64_t *d, uint32_t seed)
{
    unsigned char buf[8 * MAXW];
    for (int w = 0; w < W; ++w)
        for (int c = 0; c < 8; ++c) buf[8 * w + c] = (unsigned char)(d[w] >> (8 * c));
    return orc_murmur2(buf, 8 * W, seed);
}

/* eq. 9 (Sec. III). */
uint32_t orc_placement(int W, const uint64_t *det, uint64_t i_tau, uint32_t n_ranks, uint32_t move_shift,
                       uint32_t seed)
{
    if (n_ranks <= 1) return 0;
    uint64_t o = move_shift >= 64 ? 0 : ((uint64_t)hash_det(W, det, seed) + i_tau) >> move_shift;
    uint64_t d[MAXW];
    memcpy(d, det, sizeof(uint64_t) * (size_t)W);
    d[0] ^= o;
    return hash_det(W, d, seed) % n_ranks;
}

int orc_codistribution(int W, const uint64_t *keys, uint64_t n, uint32_t n_ranks, uint32_t move_shift,
                       uint32_t seed, const uint64_t *checkpoints, int n_checkpoints, uint64_t *sum_c,
                       uint64_t *sum_c2)
{
    if (W < 1 || W > MAXW || n_checkpoints < 1) return ORC_EINVAL;
    for (int c = 1; c < n_checkpoints; ++c)
        if (checkpoints[c] < checkpoints[c - 1]) return ORC_EINVAL;
    uint64_t T = checkpoints[n_checkpoints - 1];
    uint32_t *pl = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    uint64_t *cnt = (uint64_t *)calloc((size_t)(n * (n ? n - 1 : 0) / 2 + 1), sizeof(uint64_t));
    if (!pl || !cnt) {
        free(pl);
        free(cnt);
        return ORC_ENOMEM;
    }
    for (int c = 0; c < n_checkpoints; ++c) sum_c[c] = sum_c2[c] = 0;
    int next = 0;
    for (uint64_t t = 0; t <= T && next < n_checkpoints; ++t) {
        while (next < n_checkpoints && checkpoints[next] == t) {  /* iterations 0 .. t-1 counted */
            uint64_t k = 0;
            for (uint64_t i = 0; i < n; ++i)
                for (uint64_t j = i + 1; j < n; ++j, ++k) {
                    sum_c[next] += cnt[k];
                    sum_c2[next] += cnt[k] * cnt[k];
                }
            ++next;
        }
        if (t == T) break;
        for (uint64_t i = 0; i < n; ++i) pl[i] = orc_placement(W, keys + i * W, t, n_ranks, move_shift, seed);
        uint64_t k = 0;
        for (uint64_t i = 0; i < n; ++i)
            for (uint64_t j = i + 1; j < n; ++j, ++k) cnt[k] += pl[i] == pl[j];
    }
    free(pl);
    free(cnt);
    return 0;
}

/* --------------------------------------------------------------------------- runs */

uint64_t orc_weight(double amp)
{
    double q = rint(fabs(amp) * 16777216.0);
    if (q < 1.0) q = 1.0;
    return (uint64_t)q;
}

static int reserve(orc_run *R, uint64_t cap)
{
    if (cap <= R->cap) return 0;
    uint64_t nc = R->cap ? R->cap : 64;
    while (nc < cap) nc *= 2;
    uint64_t *k = (uint64_t *)realloc(R->keys, sizeof(uint64_t) * nc * (size_t)R->sys->W);
    if (!k) return ORC_ENOMEM;
    R->keys = k;
    double *a = (double *)realloc(R->amps, sizeof(double) * nc);
    if (!a) return ORC_ENOMEM;
    R->amps = a;
    uint64_t *q = (uint64_t *)realloc(R->q, sizeof(uint64_t) * nc);
    if (!q) return ORC_ENOMEM;
    R->q = q;
    uint64_t *p = (uint64_t *)realloc(R->pref, sizeof(uint64_t) * nc);
    if (!p) return ORC_ENOMEM;
    R->pref = p;
    R->cap = nc;
    return 0;
}

/* Selection weights of the current store (Sec. II: probability |t_i| / (N_tot - t_HF)),
 * in fixed point so that every prefix is exact. */
static int compute_weights(orc_run *R)
{
    uint64_t acc = 0;
    for (uint64_t i = 0; i < R->n; ++i) {
        if (!(fabs(R->amps[i]) < 0x1.0p28)) return ORC_EOVERFLOW;
        R->q[i] = orc_weight(R->amps[i]);
        acc += R->q[i];
        R->pref[i] = acc;
    }
    if (acc > ((uint64_t)1 << 53)) return ORC_EOVERFLOW;
    R->qtot = acc;
    return 0;
}

int orc_run_create(const orc_system *S, int truncation, const orc_options *opt, orc_run **out)
{
    if (!S || !opt || !out || truncation < 1 || truncation > 6 || truncation > S->nel ||
        opt->min_spawn_attempts < 1 || !(opt->spawn_cutoff >= 0) ||
        !(opt->occupation_threshold >= 0) || !(opt->p_single >= 0 && opt->p_single <= 1))
        return ORC_EINVAL;
    orc_run *R = (orc_run *)calloc(1, sizeof *R);
    if (!R) return ORC_ENOMEM;
    R->sys = S;
    R->l = truncation;
    R->opt = *opt;
    R->n0 = opt->init_pop;
    R->qtot = 0;
    if (reserve(R, 64)) {
        orc_run_free(R);
        return ORC_ENOMEM;
    }
    *out = R;
    return 0;
}

void orc_run_free(orc_run *R)
{
    if (!R) return;
    free(R->keys);
    free(R->amps);
    free(R->q);
    free(R->pref);
    free(R->rec);
    free(R);
}

int orc_import(orc_run *R, const uint64_t *keys, const double *amps, uint64_t n, double n_ref,
               uint64_t step)
{
    const orc_system *S = R->sys;
    int W = S->W;
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t *k = keys + i * (uint64_t)W;
        if (i > 0 && key_cmp(W, keys + (i - 1) * (uint64_t)W, k) >= 0) return ORC_EINVAL;
        if (count_bits(S, k) != S->nel) return ORC_EINVAL;
        for (int p = S->M; p < 64 * W; ++p)
            if (getbit(k, p)) return ORC_EINVAL;
        int L = orc_excitation_level(S, k);
        if (L < 1 || L > R->l) return ORC_EINVAL;
        if (!(amps[i] != 0.0) || !isfinite(amps[i])) return ORC_EINVAL;
    }
    if (!isfinite(n_ref)) return ORC_EINVAL;
    if (reserve(R, n)) return ORC_ENOMEM;
    memcpy(R->keys, keys, sizeof(uint64_t) * (size_t)(n * (uint64_t)W));
    memcpy(R->amps, amps, sizeof(double) * (size_t)n);
    R->n = n;
    R->n0 = n_ref;
    R->step = step;
    R->nrec = 0;
    return compute_weights(R);
}

int orc_export_size(const orc_run *R, uint64_t *n)
{
    *n = R->n;
    return 0;
}

int orc_export(const orc_run *R, uint64_t *keys, double *amps, double *n_ref, uint64_t *step)
{
    if (keys) memcpy(keys, R->keys, sizeof(uint64_t) * (size_t)(R->n * (uint64_t)R->sys->W));
    if (amps) memcpy(amps, R->amps, sizeof(double) * (size_t)R->n);
    if (n_ref) *n_ref = R->n0;
    if (step) *step = R->step;
    return 0;
}

/* Position of det in the store, or -1. */
static int64_t store_find(const orc_run *R, const uint64_t *det)
{
    int W = R->sys->W;
    int64_t lo = 0, hi = (int64_t)R->n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        int c = key_cmp(W, R->keys + (uint64_t)mid * W, det);
        if (c == 0) return mid;
        if (c < 0)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

/* Cluster-size distribution: p(s) = 2^-(s-lo+1) for lo <= s < hi, the remainder at hi
 * (Sec. II with its footnote; lo = 0 for the original algorithm, lo = 2 for the composite
 * clusters of full non-composite sampling, Sec. IV.B). */
static double size_prob(int s, int lo, int hi)
{
    if (s < lo || s > hi) return 0.0;
    if (s < hi) return ldexp(1.0, -(s - lo + 1));
    return ldexp(1.0, -(hi - lo));
}

static int draw_size(double u, int lo, int hi)
{
    double c = 0.0;
    for (int s = lo; s < hi; ++s) {
        c += ldexp(1.0, -(s - lo + 1));
        if (u < c) return s;
    }
    return hi;
}

/* Multi-spawn attempt count (Sec. IV.C, eq. 11) with a floor of k_min. */
int orc_attempts(const orc_run *R, double A, int noncomposite, uint64_t *n)
{
    double thr = noncomposite ? R->opt.noncomposite_threshold : R->opt.multispawn_threshold;
    uint64_t k = (uint64_t)R->opt.min_spawn_attempts;
    if (thr > 0) {
        double f = floor(fabs(A) / thr);
        if (!(f <= (double)MAX_ATTEMPTS)) return ORC_EOVERFLOW;
        if ((uint64_t)f > k) k = (uint64_t)f;
    }
    if (k > MAX_ATTEMPTS) return ORC_EOVERFLOW;
    *n = k;
    return 0;
}

int orc_cluster_ranked(const orc_run *R, int s, const uint64_t *idx, uint64_t count, uint64_t qnorm,
                       uint32_t n_ranks, int composite, uint64_t *det, double *A, int *level,
                       uint64_t *n_attempts)
{
    const orc_system *S = R->sys;
    int W = S->W;
    int lo = composite ? 2 : 0, hi = R->l + 2;
    if (s < lo || s > hi) return 0;
    if (s > 0 && R->n == 0) return 0;
    for (int a = 0; a < s; ++a) {
        if (idx[a] >= R->n) return 0;
        for (int b = 0; b < a; ++b)
            if (idx[a] == idx[b]) return 0; /* repeated excitor: discarded (Sec. II) */
    }
    int sign = 1;
    if (s == 0) {
        memcpy(det, S->hf, sizeof(uint64_t) * (size_t)W);
    } else {
        uint64_t keys[8 * MAXW];
        for (int a = 0; a < s; ++a) memcpy(keys + a * W, R->keys + idx[a] * W, sizeof(uint64_t) * W);
        if (!orc_collapse(S, s, keys, det, &sign)) return 0;
    }
    int L = orc_excitation_level(S, det);
    if (L > R->l + 2) return 0;
    /* expected number of times this cluster is drawn in `count` selections */
    double fact = 1.0;
    for (int a = 2; a <= s; ++a) fact *= (double)a;
    double p = (double)count * size_prob(s, lo, hi) * fact;
    for (int a = 0; a < s; ++a) p *= (double)R->q[idx[a]] / (double)qnorm;
    /* N_p processors (Sec. III): times N_p^(1-s) */
    if (n_ranks > 1) {
        if (s == 0) {
            p *= (double)n_ranks;
        } else {
            double d = 1.0;
            for (int a = 1; a < s; ++a) d *= (double)n_ranks;
            p /= d;
        }
    }
    /* cluster amplitude t_HF^(1-s) prod t_i with the collapse sign (Sec. II, eq. 2) */
    double Ac;
    if (s == 0) {
        Ac = R->n0;
    } else {
        Ac = (double)sign * R->amps[idx[0]];
        for (int a = 1; a < s; ++a) Ac *= R->amps[idx[a]] / R->n0;
    }
    *A = Ac / p;
    *level = L;
    if (orc_attempts(R, *A, 0, n_attempts)) return ORC_EOVERFLOW;
    return 1;
}

int orc_cluster(const orc_run *R, int s, const uint64_t *idx, uint64_t n_sel, int composite,
                uint64_t *det, double *A, int *level, uint64_t *n_attempts)
{
    return orc_cluster_ranked(R, s, idx, n_sel, R->qtot, 1, composite, det, A, level, n_attempts);
}

double orc_death(const orc_run *R, const uint64_t *det, double A, double tau, double shift)
{
    double K = orc_hamiltonian(R->sys, det, det) - R->sys->ehf;
    return -tau * (K - shift) * A;
}

static uint64_t n_pairs(int n) { return (uint64_t)n * (uint64_t)(n - 1) / 2; }

/* Pair (x < y) of rank r in lexicographic order. */
static void unrank_pair(int n, uint64_t r, int *x, int *y)
{
    for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b) {
            if (r == 0) {
                *x = a;
                *y = b;
                return;
            }
            --r;
        }
    *x = *y = -1;
}

/* Uniform excitation generators (readings; the paper cites but does not define its own).
 * UEG, doubles only: pair (i<j) of occupied orbitals uniformly, a uniformly among the
 * spatial orbitals with the spin of i, b fixed by momentum conservation with the spin of j.
 * Molecular: a single with probability p_single (i uniform among occupied, a among the
 * spatial orbitals with the spin of i), else a double (pair uniformly, a with the spin of
 * i, b with the spin of j).  Null on an occupied target orbital or a == b. */
int orc_attempt(const orc_run *R, const uint64_t *det, double A, uint64_t n, const uint64_t *choice,
                double tau, uint64_t *target, double *x)
{
    const orc_system *S = R->sys;
    int occ[MAXM];
    int N = occ_list(S, det, occ);
    int half = S->M / 2;
    uint64_t np = n_pairs(N);
    int i = -1, j = -1, a = -1, b = -1;
    double pgen;
    memcpy(target, det, sizeof(uint64_t) * (size_t)S->W);
    if (S->kind == KIND_UEG) {
        int xa, ya;
        if (choice[0] >= np || choice[1] >= (uint64_t)half) return 0;
        unrank_pair(N, choice[0], &xa, &ya);
        i = occ[xa];
        j = occ[ya];
        a = 2 * (int)choice[1] + (i & 1);
        if (getbit(det, a)) return 0;
        const int *ni = S->nvec + 3 * (i >> 1), *nj = S->nvec + 3 * (j >> 1), *na = S->nvec + 3 * (a >> 1);
        int nb[3] = {ni[0] + nj[0] - na[0], ni[1] + nj[1] - na[1], ni[2] + nj[2] - na[2]};
        int beta = -1;
        for (int c = 0; c < S->nsp; ++c) {
            const int *nc = S->nvec + 3 * c;
            if (nc[0] == nb[0] && nc[1] == nb[1] && nc[2] == nb[2]) beta = c;
        }
        if (beta < 0) return 0;
        b = 2 * beta + (j & 1);
        if (b == a || getbit(det, b)) return 0;
        pgen = (((i & 1) == (j & 1)) ? 2.0 : 1.0) / ((double)np * (double)half);
    } else {
        if (choice[0] == 0) {
            if (choice[1] >= (uint64_t)N || choice[2] >= (uint64_t)half) return 0;
            i = occ[choice[1]];
            a = 2 * (int)choice[2] + (i & 1);
            if (getbit(det, a)) return 0;
            pgen = R->opt.p_single / ((double)N * (double)half);
        } else {
            int xa, ya;
            if (choice[1] >= np || choice[2] >= (uint64_t)half || choice[3] >= (uint64_t)half) return 0;
            unrank_pair(N, choice[1], &xa, &ya);
            i = occ[xa];
            j = occ[ya];
            a = 2 * (int)choice[2] + (i & 1);
            b = 2 * (int)choice[3] + (j & 1);
            if (a == b || getbit(det, a) || getbit(det, b)) return 0;
            pgen = (1.0 - R->opt.p_single) * (((i & 1) == (j & 1)) ? 2.0 : 1.0) /
                   ((double)np * (double)half * (double)half);
        }
    }
    clrbit(target, i);
    setbit(target, a);
    if (j >= 0) {
        clrbit(target, j);
        setbit(target, b);
    }
    /* spawns beyond the truncation level are discarded (Sec. II) */
    if (orc_excitation_level(S, target) > R->l) return 0;
    double H = orc_hamiltonian(S, target, det);
    int sc = orc_excitor_sign(S, det), st = orc_excitor_sign(S, target);
    /* spawned amplitude -dtau H_ij s_D(i) s_D(j) A / (n p_gen) (Sec. II and Sec. IV.C) */
    *x = -tau * H * (double)sc * (double)st * A / ((double)n * pgen);
    return 1;
}

static int push_record(orc_run *R, const uint64_t *key, double amp, uint64_t id)
{
    if (R->nrec == R->caprec) {
        uint64_t nc = R->caprec ? 2 * R->caprec : 1024;
        record *r = (record *)realloc(R->rec, sizeof(record) * nc);
        if (!r) return ORC_ENOMEM;
        R->rec = r;
        R->caprec = nc;
    }
    record *r = R->rec + R->nrec++;
    memset(r->key, 0, sizeof r->key);
    memcpy(r->key, key, sizeof(uint64_t) * (size_t)R->sys->W);
    r->amp = amp;
    r->id = id;
    return 0;
}

/* Record id: (class << 62) | (item << 30) | slot; slot 0 is the death, slot m + 1 attempt m.
 * Class 0 = non-composite items of full non-composite sampling, class 1 = sampled clusters. */
static uint64_t record_id(int cls, uint64_t k, uint64_t slot)
{
    return ((uint64_t)cls << 62) | (k << 30) | slot;
}

typedef struct {
    double num;
    uint64_t attempts, spawns, deaths, maxn;
} step_acc;

/* Projected-energy term, death and n spawning attempts of one item (Sec. II). */
static int process_item(orc_run *R, int cls, int purpose, uint64_t k, const uint64_t *det, double A,
                        int L, uint64_t n, double tau, double shift, step_acc *acc)
{
    const orc_system *S = R->sys;
    int rc;
    if (L == 1 || L == 2) /* projected energy (Sec. II, eq. 7) */
        acc->num += orc_hamiltonian(S, S->hf, det) * (double)orc_excitor_sign(S, det) * A;
    if (L <= R->l) {
        double d = orc_death(R, det, A, tau, shift);
        if (d != 0.0) {
            if ((rc = push_record(R, det, d, record_id(cls, k, 0)))) return rc;
            acc->deaths++;
        }
    }
    if (n > acc->maxn) acc->maxn = n;
    acc->attempts += n;
    int N = S->nel, half = S->M / 2;
    uint64_t np = n_pairs(N);
    for (uint64_t m = 0; m < n; ++m) {
        uint64_t choice[4] = {0, 0, 0, 0};
        int ridx;
        if (S->kind == KIND_UEG) {
            choice[0] = below(draw(R, purpose, k, m, 0), np);
            choice[1] = below(draw(R, purpose, k, m, 1), (uint64_t)half);
            ridx = 2;
        } else {
            choice[0] = uniform(draw(R, purpose, k, m, 0)) < R->opt.p_single ? 0 : 1;
            choice[1] = below(draw(R, purpose, k, m, 1), choice[0] == 0 ? (uint64_t)N : np);
            choice[2] = below(draw(R, purpose, k, m, 2), (uint64_t)half);
            choice[3] = below(draw(R, purpose, k, m, 3), (uint64_t)half);
            ridx = 4;
        }
        uint64_t target[MAXW];
        double x;
        if (!orc_attempt(R, det, A, n, choice, tau, target, &x)) continue;
        if (x == 0.0) continue;
        if (fabs(x) < R->opt.spawn_cutoff) {
            /* unbiased stochastic rounding of small spawns to +-cutoff */
            double u = uniform(draw(R, purpose, k, m, ridx));
            if (u < fabs(x) / R->opt.spawn_cutoff)
                x = copysign(R->opt.spawn_cutoff, x);
            else
                continue;
        }
        if ((rc = push_record(R, target, x, record_id(cls, k, m + 1)))) return rc;
        acc->spawns++;
    }
    return 0;
}

static int g_sort_w; /* word count for the record comparator */

static int cmp_record(const void *x, const void *y)
{
    const record *a = (const record *)x, *b = (const record *)y;
    int c = key_cmp(g_sort_w, a->key, b->key);
    if (c) return c;
    return a->id < b->id ? -1 : (a->id > b->id ? 1 : 0);
}

typedef struct {
    uint64_t key[MAXW];
    double amp;
} entry;

static int cmp_entry(const void *x, const void *y)
{
    const entry *a = (const entry *)x, *b = (const entry *)y;
    return key_cmp(g_sort_w, a->key, b->key);
}

int orc_step(orc_run *R, double tau, double shift, uint64_t n_sel, orc_stats *st)
{
    const orc_system *S = R->sys;
    int W = S->W, rc;
    if (n_sel > 0xFFFFFFFFull || R->n + 1 > 0xFFFFFFFFull) return ORC_EINVAL;
    if ((rc = compute_weights(R))) return rc;
    R->nrec = 0;
    step_acc acc = {0.0, 0, 0, 0, 0};
    double den = R->n0;
    uint64_t discarded = 0;
    int fnc = R->opt.full_noncomposite;

    if (fnc) {
        /* full non-composite sampling (Sec. IV.B): the reference and every excitor, p = 1 */
        uint64_t n;
        if ((rc = orc_attempts(R, R->n0, 1, &n))) return rc;
        if ((rc = process_item(R, 0, PURPOSE_SPAWN_NONCOMP, 0, S->hf, R->n0, 0, n, tau, shift, &acc)))
            return rc;
        for (uint64_t i = 0; i < R->n; ++i) {
            const uint64_t *det = R->keys + i * W;
            if ((rc = orc_attempts(R, R->amps[i], 1, &n))) return rc;
            if ((rc = process_item(R, 0, PURPOSE_SPAWN_NONCOMP, i + 1, det, R->amps[i],
                                   orc_excitation_level(S, det), n, tau, shift, &acc)))
                return rc;
        }
    }
    /* virtual processors (Sec. III): where each excitor sits this step, and the total
     * weight of each processor's excitors */
    const uint32_t np = R->opt.n_ranks > 1 ? R->opt.n_ranks : 1;
    uint32_t *where = NULL;
    uint64_t *qrank = NULL;
    if (np > 1) {
        where = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(R->n + 1));
        qrank = (uint64_t *)calloc(np, sizeof(uint64_t));
        if (!where || !qrank) {
            free(where);
            free(qrank);
            return ORC_ENOMEM;
        }
        for (uint64_t i = 0; i < R->n; ++i) {
            where[i] = orc_placement(W, R->keys + i * W, R->step, np, R->opt.move_shift, R->opt.hash_seed);
            qrank[where[i]] += R->q[i];
        }
    }
    for (uint64_t k = 0; k < n_sel; ++k) {
        int lo = fnc ? 2 : 0, hi = R->l + 2;
        int s = draw_size(uniform(draw(R, PURPOSE_SELECT, k, 0, 0)), lo, hi);
        uint64_t idx[8];
        int ok = 1;
        /* one processor: selection k is made by processor k mod N_p from its own excitors,
         * which make count = the number of selections on that processor */
        const uint32_t rank = (uint32_t)(k % np);
        const uint64_t qnorm = np > 1 ? qrank[rank] : R->qtot;
        const uint64_t count = np > 1 ? n_sel / np + (rank < n_sel % np ? 1 : 0) : n_sel;
        for (int a = 0; a < s; ++a) {
            if (qnorm == 0) {
                ok = 0;
                break;
            }
            uint64_t r = below(draw(R, PURPOSE_SELECT, k, 0, 1 + a), qnorm);
            if (np == 1) {
                /* excitor with P[i-1] <= r < P[i] */
                uint64_t lo_i = 0, hi_i = R->n;
                while (lo_i < hi_i) {
                    uint64_t mid = (lo_i + hi_i) / 2;
                    if (R->pref[mid] > r)
                        hi_i = mid;
                    else
                        lo_i = mid + 1;
                }
                idx[a] = lo_i;
            } else {
                /* the processor's excitors in store order, each owning q_i values of r */
                uint64_t acc = 0, i = 0;
                for (; i < R->n; ++i) {
                    if (where[i] != rank) continue;
                    acc += R->q[i];
                    if (acc > r) break;
                }
                idx[a] = i;
            }
        }
        uint64_t det[MAXW], n = 0;
        double A = 0.0;
        int L = 0;
        if (ok) {
            ok = orc_cluster_ranked(R, s, idx, count, qnorm, np, fnc, det, &A, &L, &n);
            if (ok < 0) {
                free(where);
                free(qrank);
                return ok;
            }
        }
        if (!ok) {
            ++discarded;
            continue;
        }
        if ((rc = process_item(R, 1, PURPOSE_SPAWN_SAMPLED, k, det, A, L, n, tau, shift, &acc))) {
            free(where);
            free(qrank);
            return rc;
        }
    }
    free(where);
    free(qrank);

    /* annihilation (Sec. II): group records by key, sum each group in id order */
    g_sort_w = W;
    qsort(R->rec, (size_t)R->nrec, sizeof(record), cmp_record);
    entry *ent = (entry *)malloc(sizeof(entry) * (size_t)(R->n + R->nrec + 1));
    if (!ent) return ORC_ENOMEM;
    for (uint64_t i = 0; i < R->n; ++i) {
        memset(ent[i].key, 0, sizeof ent[i].key);
        memcpy(ent[i].key, R->keys + i * W, sizeof(uint64_t) * W);
        ent[i].amp = R->amps[i];
    }
    uint64_t nent = R->n;
    double n0 = R->n0;
    for (uint64_t r = 0; r < R->nrec;) {
        uint64_t e = r + 1;
        while (e < R->nrec && key_cmp(W, R->rec[e].key, R->rec[r].key) == 0) ++e;
        double sum = R->rec[r].amp;
        for (uint64_t t = r + 1; t < e; ++t) sum += R->rec[t].amp;
        if (key_cmp(W, R->rec[r].key, S->hf) == 0) {
            n0 = n0 + sum;
        } else {
            int64_t pos = store_find(R, R->rec[r].key);
            if (pos >= 0) {
                ent[pos].amp = ent[pos].amp + sum;
            } else {
                memcpy(ent[nent].key, R->rec[r].key, sizeof ent[nent].key);
                ent[nent].amp = sum;
                ++nent;
            }
        }
        r = e;
    }
    qsort(ent, (size_t)nent, sizeof(entry), cmp_entry);

    /* real-weight occupation rounding: |N| < theta becomes +-theta with probability
     * |N| / theta, else 0; the reference is exempt.  Then drop zeros. */
    double theta = R->opt.occupation_threshold;
    uint64_t nout = 0;
    for (uint64_t k = 0; k < nent; ++k) {
        double v = ent[k].amp;
        if (v != 0.0 && fabs(v) < theta) {
            double u = uniform(draw(R, PURPOSE_ROUND, k, 0, 0));
            v = (u < fabs(v) / theta) ? copysign(theta, v) : 0.0;
        }
        if (v != 0.0) {
            ent[nout] = ent[k];
            ent[nout].amp = v;
            ++nout;
        }
    }
    if ((rc = reserve(R, nout))) {
        free(ent);
        return rc;
    }
    double ntot = fabs(n0);
    for (uint64_t k = 0; k < nout; ++k) {
        memcpy(R->keys + k * W, ent[k].key, sizeof(uint64_t) * W);
        R->amps[k] = ent[k].amp;
        ntot += fabs(ent[k].amp);
    }
    free(ent);
    R->n = nout;
    R->n0 = n0;
    R->step += 1;
    if ((rc = compute_weights(R))) return rc;

    if (st) {
        st->step = R->step;
        st->n_selections = n_sel;
        st->n_discarded = discarded;
        st->n_spawn_attempts = acc.attempts;
        st->n_spawns = acc.spawns;
        st->n_deaths = acc.deaths;
        st->n_excitors = nout;
        st->max_attempts_per_cluster = acc.maxn;
        st->n_total = ntot;
        st->n_ref = n0;
        st->eproj_num = acc.num;
        st->eproj_den = den;
    }
    return 0;
}

int orc_records_size(const orc_run *R, uint64_t *n)
{
    *n = R->nrec;
    return 0;
}

/* Records of the last step in id order (they are kept sorted by key after annihilation,
 * so sort a copy by id). */
static int cmp_id(const void *x, const void *y)
{
    const record *a = (const record *)x, *b = (const record *)y;
    return a->id < b->id ? -1 : (a->id > b->id ? 1 : 0);
}

int orc_records(const orc_run *R, uint64_t *keys, double *amps, uint64_t *ids)
{
    int W = R->sys->W;
    record *c = (record *)malloc(sizeof(record) * (size_t)(R->nrec ? R->nrec : 1));
    if (!c) return ORC_ENOMEM;
    memcpy(c, R->rec, sizeof(record) * (size_t)R->nrec);
    qsort(c, (size_t)R->nrec, sizeof(record), cmp_id);
    for (uint64_t r = 0; r < R->nrec; ++r) {
        if (keys) memcpy(keys + r * W, c[r].key, sizeof(uint64_t) * W);
        if (amps) amps[r] = c[r].amp;
        if (ids) ids[r] = c[r].id;
    }
    free(c);
    return 0;
}
