// ccmc.hip -- host side of the MI355X CCMC step library: system tables, device buffers,
// the launch sequence of one time step, and the C ABI declared in include/ccmc.h.
//
// Paper: Spencer, Neufeld, Vigor, Franklin & Thom, arXiv:1807.03749 (Sec. II, Sec. IV).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "ccmc.h"
#include "kernels.h"

using namespace ccmc;

namespace {

thread_local std::string g_init_error;

// ------------------------------------------------------------------ device buffers
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// A timed launch; its work is unit_bytes x the count it covers, known when it is resolved
// (a count produced on the device is read back at the end of the step).
// Work of one launch for the profile: algorithmic bytes = unit_bytes x count, work units =
// *items (or the same count).  Counts produced on the device are read after the step's
// synchronisation, through pointers to the host copies of the step's sizes.
struct Work {
    double unit_bytes;
    const uint64_t *count;  // live count, or null for `fixed`
    uint64_t fixed;
    const uint64_t *items = nullptr;
    double unit_bytes2 = 0;  // plus unit_bytes2 x *count2
    const uint64_t *count2 = nullptr;
};

struct Pending {
    const char *name;
    hipEvent_t a, b;
    Work w;
};

struct Accum {
    uint64_t launches = 0;
    double ms = 0, bytes = 0, items = 0;
};

// Host description of the system.
struct HostSys {
    int kind = 0, nel = 0, M = 0, W = 0, nsp = 0;
    std::vector<int> nvec;   // [nsp][3]
    double L = 0, omega = 0, kf = 0;
    int n2max = 0, G = 0;
    std::vector<int> grid;
    std::vector<double> vq;
    std::vector<double> h;   // molecular [nsp][nsp]
    std::vector<double> fock, vpair;
    double ehf = 0;
};

}  // namespace

struct ccmc_state {
    ccmc_system sys{};
    ccmc_options opt{};
    int l = 0;
    int W = 0, WP = 0;
    bool fp32 = false;
    size_t es = 8;  // amplitude element size
    hipStream_t stream = nullptr;
    bool own_stream = false;
    HostSys hs;
    SysDev sd{};
    std::vector<DevBuf *> all;
    DevBuf t_grid, t_nvec, t_vq, t_h, t_eri, t_fock, t_vpair, t_binv, t_bino;
    int rank_bits = 0;  // bits of the largest truncated-space rank
    // the store: current buffer cur, merge target 1 - cur
    DevBuf skey[2], samp[2], sK[2], srank[2];
    uint64_t scap = 0;
    int cur = 0;
    uint64_t ne = 0;
    double n0 = 0;
    uint64_t step = 0;
    double last_num = 0, last_den = 0;
    // per-step buffers
    DevBuf P, guide, delta, rtab;
    uint64_t rt_n = 0;   // rank-table buckets
    uint32_t rsh = 0;    // rank-table shift
    uint64_t last_q = 0; // Q of the last step (sizes the next selection guide)
    DevBuf ikey, iA, ideath, in, ilevel, icnt, ioff;
    uint64_t icap = 0;
    DevBuf num_part, att_part, disc_part, max_part, abs_part;
    DevBuf block_item, gcount, gspawn, gdeath, boff;
    DevBuf rkey, ramp, rid;  // per-block record regions
    uint64_t rcap = 0;              // region slots
    DevBuf drank, dkey, damp, did, sr[2], sidx[2];
    DevBuf is_new, new_pos, ins, seg_sum, nkey, nrank, nins, nsum, keep, pos;
    uint64_t dcap = 0;  // dense record capacity
    uint64_t slot_hint = 1 << 16, rec_hint = 1 << 14;  // capacities planned for the next step
    uint64_t cnt_slots = 0, cnt_rec = 0, cnt_merged = 0, cnt_new = 0, cnt_att = 0, cnt_live_items = 0;  // live counts of the last step
    DevBuf lb;  // step scalars, tickets, radix histograms and look-back status words
    Scratch *hscratch = nullptr;  // pinned
    // last step's spawn list (keep_spawn_ids)
    uint64_t last_nrec = 0;
    int last_rec_buf = -1;
    size_t bytes_held = 0;
    std::string err;
    bool prof = false;
    std::string prof_names;  // "*" or ",name,name,": the launches timed
    std::vector<Pending> pending;
    std::vector<hipEvent_t> ev_pool;
    std::map<std::string, Accum> accum;
};

namespace {

#define HIP_TRY(...)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (__VA_ARGS__);                                                        \
        if (e_ != hipSuccess) {                                                               \
            st->err = std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_);               \
            return CCMC_EDEVICE;                                                              \
        }                                                                                     \
    } while (0)

#define TRY(...)                                                                              \
    do {                                                                                      \
        ccmc_status s_ = (__VA_ARGS__);                                                       \
        if (s_ != CCMC_OK) return s_;                                                         \
    } while (0)

ccmc_status ensure(ccmc_state *st, DevBuf &b, size_t bytes)
{
    if (bytes <= b.bytes) return CCMC_OK;
    size_t nb = std::max<size_t>(bytes, 256);
    nb = std::max(nb, b.bytes + b.bytes / 2);
    if (st->opt.hbm_budget_bytes && st->bytes_held - b.bytes + nb > st->opt.hbm_budget_bytes) {
        nb = bytes;
        if (st->bytes_held - b.bytes + nb > st->opt.hbm_budget_bytes) {
            st->err = "HBM budget of " + std::to_string(st->opt.hbm_budget_bytes) + " bytes exceeded";
            return CCMC_ENOMEM;
        }
    }
    void *p = nullptr;
    if (hipMalloc(&p, nb) != hipSuccess) {
        (void)hipGetLastError();
        st->err = "hipMalloc of " + std::to_string(nb) + " bytes failed";
        return CCMC_ENOMEM;
    }
    if (b.p) {
        (void)hipStreamSynchronize(st->stream);
        (void)hipFree(b.p);
    }
    st->bytes_held += nb - b.bytes;
    b.p = p;
    b.bytes = nb;
    return CCMC_OK;
}

void release(ccmc_state *st, DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    st->bytes_held -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
}

template <class X>
X *ptr(DevBuf &b)
{
    return static_cast<X *>(b.p);
}

unsigned grid_for(uint64_t n, uint64_t per_block = kThreads)
{
    return (unsigned)std::max<uint64_t>(1, (n + per_block - 1) / per_block);
}

// --------------------------------------------------------------------- profiling
hipEvent_t take_event(ccmc_state *st)
{
    if (!st->ev_pool.empty()) {
        hipEvent_t e = st->ev_pool.back();
        st->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
}

bool profiled(const ccmc_state *st, const char *name)
{
    return st->prof_names == "*" || st->prof_names.find("," + std::string(name) + ",") != std::string::npos;
}

template <class F>
void launch(ccmc_state *st, const char *name, Work w, F &&f)
{
    if (!st->prof || !profiled(st, name)) {
        f();
        return;
    }
    Pending p{name, take_event(st), take_event(st), w};
    (void)hipEventRecord(p.a, st->stream);
    f();
    (void)hipEventRecord(p.b, st->stream);
    st->pending.push_back(p);
}

void resolve_profile(ccmc_state *st)
{
    for (auto &p : st->pending) {
        float ms = 0;
        (void)hipEventSynchronize(p.b);
        (void)hipEventElapsedTime(&ms, p.a, p.b);
        const double n = (double)(p.w.count ? *p.w.count : p.w.fixed);
        Accum &a = st->accum[p.name];
        a.launches++;
        a.ms += ms;
        a.bytes += p.w.unit_bytes * n + (p.w.count2 ? p.w.unit_bytes2 * (double)*p.w.count2 : 0.0);
        a.items += p.w.items ? (double)*p.w.items : n;
        st->ev_pool.push_back(p.a);
        st->ev_pool.push_back(p.b);
    }
    st->pending.clear();
}

// --------------------------------------------------------------------------- scan
// Single-launch look-back scan; status must hold ceil(n / kScanTile) zeroed words.
template <typename V, typename Src, typename Out>
void scan_lb(ccmc_state *st, Src in, Out out, uint64_t n, bool inclusive, uint64_t *status, uint64_t *ticket,
             uint64_t *total)
{
    if (!n) return;
    const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
    k_scan_lb<V, Src, Out><<<(unsigned)tiles, kThreads, 0, st->stream>>>(in, out, n, inclusive ? 1 : 0, status, ticket,
                                                                         total);
}

uint64_t scan_tiles(uint64_t n) { return (n + kScanTile - 1) / kScanTile; }

// ------------------------------------------------------------------------ systems
int words_for(int M) { return (M + 63) / 64; }
int padded_words(int W)
{
    static const int ws[] = {1, 2, 3, 4, 6, 8};
    for (int w : ws)
        if (w >= W) return w;
    return -1;
}

bool build_ueg(HostSys &hs, int nel, int n2max, double rs, std::string &err)
{
    int nmax = 0;
    while ((nmax + 1) * (nmax + 1) <= n2max) ++nmax;
    std::vector<std::array<int, 4>> v;
    for (int x = -nmax; x <= nmax; ++x)
        for (int y = -nmax; y <= nmax; ++y)
            for (int z = -nmax; z <= nmax; ++z) {
                const int n2 = x * x + y * y + z * z;
                if (n2 <= n2max) v.push_back({n2, x, y, z});
            }
    std::sort(v.begin(), v.end());  // by |n|^2, then n_x, n_y, n_z
    const int nocc = nel / 2;
    if (nel < 2 || (nel & 1) || nocc > (int)v.size() || 2 * (int)v.size() > 64 * kMaxWords) {
        err = "UEG: need an even number of electrons that fits the basis (M <= 512)";
        return false;
    }
    if (nocc < (int)v.size() && v[nocc - 1][0] == v[nocc][0]) {
        err = "UEG: open shell (the last occupied and first virtual plane waves share |n|^2)";
        return false;
    }
    hs.kind = CCMC_UEG;
    hs.nel = nel;
    hs.nsp = (int)v.size();
    hs.M = 2 * hs.nsp;
    hs.n2max = n2max;
    hs.nvec.resize(3 * hs.nsp);
    for (int i = 0; i < hs.nsp; ++i)
        for (int c = 0; c < 3; ++c) hs.nvec[3 * i + c] = v[i][1 + c];
    hs.L = rs * std::cbrt(4.0 * M_PI * nel / 3.0);
    hs.omega = hs.L * hs.L * hs.L;
    hs.kf = 2.0 * M_PI / hs.L;
    // Coulomb kernel 4 pi / (Omega |k|^2), |k|^2 = kf^2 |dn|^2, |dn|^2 <= 4 n2max
    hs.vq.assign(4 * n2max + 1, 0.0);
    for (int d = 1; d <= 4 * n2max; ++d) hs.vq[d] = 4.0 * M_PI / (hs.omega * (hs.kf * hs.kf * (double)d));
    hs.G = 3 * nmax;
    const int D = 2 * hs.G + 1;
    hs.grid.assign((size_t)D * D * D, -1);
    for (int i = 0; i < hs.nsp; ++i) {
        const int *n = &hs.nvec[3 * i];
        hs.grid[((size_t)(n[0] + hs.G) * D + (n[1] + hs.G)) * D + (n[2] + hs.G)] = i;
    }
    const int M = hs.M;
    auto u_exch = [&](int p, int q) -> double {  // <pq|qp>, p != q
        if ((p ^ q) & 1) return 0.0;
        const int *a = &hs.nvec[3 * (p >> 1)], *b = &hs.nvec[3 * (q >> 1)];
        const int d = (a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) + (a[2] - b[2]) * (a[2] - b[2]);
        return d ? hs.vq[d] : 0.0;
    };
    hs.vpair.assign((size_t)M * M, 0.0);
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q)
            if (p != q) hs.vpair[(size_t)p * M + q] = -u_exch(p, q);  // direct term is q = 0
    hs.fock.assign(M, 0.0);
    double e1 = 0, e2 = 0;
    for (int p = 0; p < M; ++p) {
        const int *n = &hs.nvec[3 * (p >> 1)];
        const double t = 0.5 * hs.kf * hs.kf * (double)(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        double f = t;
        for (int j = 0; j < nel; ++j) f += hs.vpair[(size_t)p * M + j];
        hs.fock[p] = f;
        if (p < nel) {
            e1 += t;
            for (int j = 0; j < nel; ++j) e2 += hs.vpair[(size_t)p * M + j];
        }
    }
    hs.ehf = e1 + 0.5 * e2;
    return true;
}

bool build_mol(HostSys &hs, int nel, const ccmc_integrals *ints, std::string &err)
{
    const int n = ints->n_spatial;
    if (nel < 2 || (nel & 1) || n < 1 || nel > 2 * n || 2 * n > 64 * kMaxWords || !ints->h ||
        ints->n_chol < 0 || (ints->n_chol > 0 && !ints->chol)) {
        err = "molecular: invalid sizes or null integral arrays";
        return false;
    }
    hs.kind = CCMC_MOLECULAR;
    hs.nel = nel;
    hs.nsp = n;
    hs.M = 2 * n;
    hs.h.assign(ints->h, ints->h + (size_t)n * n);
    const int M = hs.M;
    const size_t nn = (size_t)n * n;
    auto eri = [&](int P, int Q, int R, int S) {  // (PQ|RS), summed over L in order
        double v = 0.0;
        for (int L = 0; L < ints->n_chol; ++L) v += ints->chol[L * nn + (size_t)P * n + Q] * ints->chol[L * nn + (size_t)R * n + S];
        return v;
    };
    hs.vpair.assign((size_t)M * M, 0.0);
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q) {
            if (p == q) continue;
            const int P = p >> 1, Q = q >> 1;
            double v = eri(P, P, Q, Q);  // <pq|pq> = (PP|QQ)
            if (((p ^ q) & 1) == 0) v -= eri(P, Q, Q, P);  // <pq|qp> = (PQ|QP)
            hs.vpair[(size_t)p * M + q] = v;
        }
    hs.fock.assign(M, 0.0);
    double e1 = 0, e2 = 0;
    for (int p = 0; p < M; ++p) {
        const double hp = hs.h[(size_t)(p >> 1) * n + (p >> 1)];
        double f = hp;
        for (int j = 0; j < nel; ++j) f += hs.vpair[(size_t)p * M + j];
        hs.fock[p] = f;
        if (p < nel) {
            e1 += hp;
            for (int j = 0; j < nel; ++j) e2 += hs.vpair[(size_t)p * M + j];
        }
    }
    hs.ehf = e1 + 0.5 * e2;
    return true;
}

template <typename T>
ccmc_status upload_table(ccmc_state *st, DevBuf &b, const std::vector<double> &v)
{
    std::vector<T> t(v.begin(), v.end());
    TRY(ensure(st, b, std::max<size_t>(1, t.size()) * sizeof(T)));
    if (!t.empty()) HIP_TRY(hipMemcpy(b.p, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice));
    return CCMC_OK;
}

template <typename T>
ccmc_status upload_system(ccmc_state *st, const ccmc_integrals *ints)
{
    HostSys &hs = st->hs;
    SysDev &S = st->sd;
    S.kind = hs.kind;
    S.nel = hs.nel;
    S.M = hs.M;
    S.nsp = hs.nsp;
    S.l = st->l;
    S.npairs = (uint32_t)(hs.nel * (hs.nel - 1) / 2);
    S.half = (uint32_t)(hs.M / 2);
    for (int w = 0; w < kMaxWords; ++w) S.hf[w] = 0;
    for (int p = 0; p < hs.nel; ++p) S.hf[p >> 6] |= 1ull << (p & 63);
    S.p_single = st->opt.p_single;
    {
        // C(n, j) for the virtual part (j <= 8) and C(n, k) for the occupied part, both
        // saturating at 2^63; the truncated space itself must stay below 2^62.
        const int M = hs.M, N = hs.nel;
        const uint64_t sat = 1ull << 63;
        auto binom = [&](int n, int k) -> uint64_t {
            if (k < 0 || k > n) return 0;
            unsigned __int128 v = 1;
            for (int i = 1; i <= k; ++i) {
                v = v * (unsigned)(n - k + i) / (unsigned)i;
                if (v > sat) return sat;
            }
            return (uint64_t)v;
        };
        std::vector<uint64_t> bv((size_t)(M + 1) * 9), bo((size_t)(N + 1) * (N + 1));
        for (int n = 0; n <= M; ++n)
            for (int j = 0; j <= 8; ++j) bv[(size_t)n * 9 + j] = binom(n, j);
        for (int n = 0; n <= N; ++n)
            for (int k = 0; k <= N; ++k) bo[(size_t)n * (N + 1) + k] = binom(n, k);
        unsigned __int128 space = 0;
        for (int j = 0; j <= st->l; ++j) space += (unsigned __int128)binom(N, j) * binom(M - N, j);
        if (space >= ((unsigned __int128)1 << 62)) {
            st->err = "truncated space too large for 64-bit determinant ranks";
            return CCMC_EINVAL;
        }
        int bits = 0;
        while (((unsigned __int128)1 << bits) < space) ++bits;
        st->rank_bits = bits;
        TRY(ensure(st, st->t_binv, bv.size() * 8));
        TRY(ensure(st, st->t_bino, bo.size() * 8));
        HIP_TRY(hipMemcpy(st->t_binv.p, bv.data(), bv.size() * 8, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(st->t_bino.p, bo.data(), bo.size() * 8, hipMemcpyHostToDevice));
        S.binom_v = ptr<uint64_t>(st->t_binv);
        S.binom_o = ptr<uint64_t>(st->t_bino);
    }
    TRY(upload_table<T>(st, st->t_fock, hs.fock));
    TRY(upload_table<T>(st, st->t_vpair, hs.vpair));
    S.fock = st->t_fock.p;
    S.vpair = st->t_vpair.p;
    if (hs.kind == CCMC_UEG) {
        S.G = hs.G;
        TRY(ensure(st, st->t_grid, hs.grid.size() * sizeof(int)));
        HIP_TRY(hipMemcpy(st->t_grid.p, hs.grid.data(), hs.grid.size() * sizeof(int), hipMemcpyHostToDevice));
        TRY(ensure(st, st->t_nvec, hs.nvec.size() * sizeof(int)));
        HIP_TRY(hipMemcpy(st->t_nvec.p, hs.nvec.data(), hs.nvec.size() * sizeof(int), hipMemcpyHostToDevice));
        TRY(upload_table<T>(st, st->t_vq, hs.vq));
        S.grid = ptr<int>(st->t_grid);
        S.nvec = ptr<int>(st->t_nvec);
        S.vq = st->t_vq.p;
    } else {
        TRY(upload_table<T>(st, st->t_h, hs.h));
        S.h = st->t_h.p;
        const uint64_t n = hs.nsp, n4 = n * n * n * n;
        DevBuf chol;
        const size_t cb = std::max<size_t>(1, (size_t)ints->n_chol * n * n) * sizeof(double);
        TRY(ensure(st, chol, cb));
        if (ints->n_chol > 0)
            HIP_TRY(hipMemcpy(chol.p, ints->chol, (size_t)ints->n_chol * n * n * sizeof(double), hipMemcpyHostToDevice));
        TRY(ensure(st, st->t_eri, n4 * sizeof(T)));
        k_build_eri<T><<<grid_for(n4), kThreads, 0, st->stream>>>(ptr<double>(chol), (int)n, ints->n_chol, ptr<T>(st->t_eri));
        HIP_TRY(hipStreamSynchronize(st->stream));
        release(st, chol);
        S.eri = st->t_eri.p;
    }
    return CCMC_OK;
}

// ------------------------------------------------------------------------ the store
// Entries of the selection guide for a store capacity: several times the buckets the shift
// aims at, so that Q may grow between steps before draws fall past the table.
uint64_t guide_cap(uint64_t scap) { return 2 * scap + 8; }

// Grow the store (both buffers) to hold n entries, keeping the current contents.
template <int W, typename T>
ccmc_status ensure_store(ccmc_state *st, uint64_t n)
{
    if (n <= st->scap) return CCMC_OK;
    uint64_t nc = std::max<uint64_t>(n, std::max<uint64_t>(1024, st->scap + st->scap / 2));
    DevBuf k, a, K, r;
    TRY(ensure(st, k, nc * W * sizeof(uint64_t)));
    TRY(ensure(st, a, nc * sizeof(T)));
    TRY(ensure(st, K, nc * sizeof(T)));
    TRY(ensure(st, r, nc * sizeof(uint64_t)));
    const int c = st->cur;
    if (st->ne) {
        HIP_TRY(hipMemcpy2DAsync(k.p, nc * sizeof(uint64_t), st->skey[c].p, st->scap * sizeof(uint64_t),
                                 st->ne * sizeof(uint64_t), W, hipMemcpyDeviceToDevice, st->stream));
        HIP_TRY(hipMemcpyAsync(a.p, st->samp[c].p, st->ne * sizeof(T), hipMemcpyDeviceToDevice, st->stream));
        HIP_TRY(hipMemcpyAsync(K.p, st->sK[c].p, st->ne * sizeof(T), hipMemcpyDeviceToDevice, st->stream));
        HIP_TRY(hipMemcpyAsync(r.p, st->srank[c].p, st->ne * sizeof(uint64_t), hipMemcpyDeviceToDevice, st->stream));
        HIP_TRY(hipStreamSynchronize(st->stream));
    }
    for (int b = 0; b < 2; ++b) {
        release(st, st->skey[b]);
        release(st, st->samp[b]);
        release(st, st->sK[b]);
        release(st, st->srank[b]);
    }
    st->skey[c] = k;
    st->samp[c] = a;
    st->sK[c] = K;
    st->srank[c] = r;
    TRY(ensure(st, st->skey[1 - c], nc * W * sizeof(uint64_t)));
    TRY(ensure(st, st->samp[1 - c], nc * sizeof(T)));
    TRY(ensure(st, st->sK[1 - c], nc * sizeof(T)));
    TRY(ensure(st, st->srank[1 - c], nc * sizeof(uint64_t)));
    TRY(ensure(st, st->P, nc * sizeof(uint64_t)));
    TRY(ensure(st, st->guide, guide_cap(nc) * sizeof(uint32_t)));
    TRY(ensure(st, st->delta, nc * sizeof(double)));
    // rank table: about one bucket per store entry, at most one per rank
    int rt_bits = 1;
    while (rt_bits < 40 && (1ull << rt_bits) < nc) ++rt_bits;
    rt_bits = std::min(rt_bits, std::max(st->rank_bits, 1));
    st->rt_n = 1ull << rt_bits;
    st->rsh = (uint32_t)std::max(0, st->rank_bits - rt_bits);
    TRY(ensure(st, st->rtab, (st->rt_n + 1) * sizeof(uint32_t)));
    st->scap = nc;
    return CCMC_OK;
}

// ---------------------------------------------------------------------- the step
constexpr uint64_t kMaxFinalParts = 512;
  // blocks of the first stage of the final reduction

// One attempt at a step.  Sizes produced on the device (record slots, records, new
// determinants, survivors) are never read back in the middle: kernels read them from device
// memory, and grids cover capacities planned from the previous step.  If a count exceeds
// its capacity, the overflow bit turns the final compaction into a no-op; the host then
// grows the buffers and the step is replayed with the same Philox counters (*replay).
template <int W, typename T>
ccmc_status step_once(ccmc_state *st, double tau, double shift, uint64_t n_sel, ccmc_stats *out, bool *replay)
{
    *replay = false;
    hipStream_t s = st->stream;
    const uint64_t ne = st->ne;
    const bool fnc = st->opt.full_noncomposite != 0;
    const uint64_t n_fnc = fnc ? ne + 1 : 0;
    const uint64_t n_items = n_fnc + n_sel;
    const int c = st->cur;
    const double kb = (double)(W * 8);  // bytes of one bitstring
    const double tb = (double)sizeof(T);
    const bool ids = st->opt.keep_spawn_ids != 0;

    StepArgs a;
    a.tau = tau;
    a.shift = shift;
    a.cutoff = st->opt.spawn_cutoff;
    a.theta = st->opt.occupation_threshold;
    a.thr_cluster = st->opt.multispawn_threshold;
    a.thr_nc = st->opt.noncomposite_threshold;
    a.kmin = (uint32_t)st->opt.min_spawn_attempts;
    a.step = (uint32_t)(st->step & 0x0FFFFFFFu);
    a.key0 = (uint32_t)st->opt.seed;
    a.key1 = (uint32_t)(st->opt.seed >> 32);
    a.n_sel = n_sel;
    a.fnc = fnc ? 1 : 0;
    {
        // guide shift from the last step's Q (any shift gives the same draws; this one keeps
        // about one bucket per two excitors, so that large amplitudes own few buckets)
        const uint64_t q_est = st->last_q ? st->last_q : (ne << 24);
        uint32_t sh = 0;
        while (sh < 63 && (q_est >> sh) + 2 > ne / 2 + 2) ++sh;
        a.gsh = sh;
        a.gcap = guide_cap(st->scap);
    }

    // ---- capacities for this step (all allocation happens here, before any launch)
    const uint64_t slot_cap = std::max<uint64_t>(kGenSlots, (st->slot_hint + kGenSlots - 1) / kGenSlots * kGenSlots);
    const uint64_t nblk_cap = slot_cap / kGenSlots;
    const uint64_t rec_cap = std::max<uint64_t>(1, std::min<uint64_t>(st->rec_hint, slot_cap));
    if (slot_cap + ne + 1 >= (1ull << 32)) {
        st->err = "more than 2^32 record slots in one step";
        return CCMC_EOVERFLOW;
    }
    if (n_items + 1 > st->icap) {
        const uint64_t nc = std::max<uint64_t>(n_items + 1, st->icap + st->icap / 2);
        TRY(ensure(st, st->ikey, nc * W * sizeof(uint64_t)));
        TRY(ensure(st, st->iA, nc * sizeof(T)));
        TRY(ensure(st, st->ideath, nc * sizeof(T)));
        TRY(ensure(st, st->in, nc * sizeof(uint32_t)));
        TRY(ensure(st, st->ilevel, nc));
        TRY(ensure(st, st->icnt, nc * sizeof(uint64_t)));
        TRY(ensure(st, st->ioff, nc * sizeof(uint64_t)));
        st->icap = nc;
    }
    if (slot_cap > st->rcap) {
        const uint64_t nc = slot_cap;
        const uint64_t nb = nc / kGenSlots + 2;
        TRY(ensure(st, st->rkey, nc * W * sizeof(uint64_t)));
        TRY(ensure(st, st->ramp, nc * sizeof(T)));
        TRY(ensure(st, st->block_item, nb * sizeof(uint64_t)));
        for (DevBuf *b : {&st->gcount, &st->gspawn, &st->gdeath, &st->boff}) TRY(ensure(st, *b, nb * sizeof(uint32_t)));
        st->rcap = nc;
    }
    if (ids && st->rid.bytes < st->rcap * sizeof(uint64_t)) TRY(ensure(st, st->rid, st->rcap * sizeof(uint64_t)));
    if (rec_cap + 1 > st->dcap) {
        const uint64_t nc = rec_cap + 1;
        for (DevBuf *b : {&st->dkey, &st->nkey}) TRY(ensure(st, *b, nc * W * sizeof(uint64_t)));
        TRY(ensure(st, st->damp, nc * sizeof(T)));
        for (DevBuf *b : {&st->drank, &st->sr[0], &st->sr[1], &st->ins, &st->nins, &st->nrank})
            TRY(ensure(st, *b, nc * sizeof(uint64_t)));
        for (DevBuf *b : {&st->sidx[0], &st->sidx[1], &st->is_new, &st->new_pos}) TRY(ensure(st, *b, nc * sizeof(uint32_t)));
        for (DevBuf *b : {&st->seg_sum, &st->nsum}) TRY(ensure(st, *b, nc * sizeof(double)));
        st->dcap = nc;
    }
    if (ids && st->did.bytes < st->dcap * sizeof(uint64_t)) TRY(ensure(st, st->did, st->dcap * sizeof(uint64_t)));
    const uint64_t mcap = ne + rec_cap;  // merged store capacity of this step
    TRY(ensure_store<W, T>(st, mcap + 1));
    TRY(ensure(st, st->keep, (mcap + 1) * sizeof(uint32_t)));
    TRY(ensure(st, st->pos, (mcap + 1) * sizeof(uint32_t)));
    const uint64_t tiles = (rec_cap + kSortTile - 1) / kSortTile;
    const int passes = std::max(1, (st->rank_bits + kRadixBits - 1) / kRadixBits);
    const unsigned nb_fnc = fnc ? grid_for(n_fnc) : 0, nb_sel = n_sel ? grid_for(n_sel) : 0;
    const size_t nparts = (size_t)(nb_fnc + nb_sel + 1);
    TRY(ensure(st, st->num_part, nparts * sizeof(double)));
    TRY(ensure(st, st->att_part, nparts * sizeof(uint64_t)));
    TRY(ensure(st, st->disc_part, nparts * sizeof(uint64_t)));
    TRY(ensure(st, st->max_part, nparts * sizeof(uint64_t)));
    const unsigned nb_abs = grid_for(mcap);
    TRY(ensure(st, st->abs_part, (nb_abs + 1) * sizeof(double)));

    // One zeroed area per step: the step scalars, the scan tickets, the look-back status
    // words of every scan and radix pass, and the radix histograms (64-bit words).
    enum { kTkWeights, kTkOff, kTkBoff, kTkNew, kTkKeep, kTkRadix, kTickets = kTkRadix + 8 };
    const uint64_t w_scratch = (sizeof(Scratch) + 7) / 8;
    const uint64_t o_tick = w_scratch;
    const uint64_t o_weights = o_tick + kTickets;
    const uint64_t o_off = o_weights + scan_tiles(ne);
    const uint64_t o_boff = o_off + scan_tiles(n_items + 1);
    const uint64_t o_new = o_boff + scan_tiles(nblk_cap + 1);
    const uint64_t o_keep = o_new + scan_tiles(rec_cap);
    const uint64_t o_ghist = o_keep + scan_tiles(mcap);
    const uint64_t o_rstat = o_ghist + (uint64_t)passes * kRadixBins / 2;
    const uint64_t o_fold = o_rstat + (uint64_t)passes * tiles * kRadixBins;
    const uint64_t fold_tiles = (rec_cap + kFoldTile - 1) / kFoldTile;
    const uint64_t o_fin = o_fold + 3 * fold_tiles;
    const uint64_t lb_words = o_fin + kMaxFinalParts * (sizeof(FinalPart) / 8);
    TRY(ensure(st, st->lb, lb_words * sizeof(uint64_t)));
    uint64_t *lb = ptr<uint64_t>(st->lb);
    uint64_t *tick = lb + o_tick;
    Scratch *sc = reinterpret_cast<Scratch *>(lb);
    launch(st, "clear", Work{8.0, nullptr, lb_words}, [&] {
        k_fill<uint64_t><<<grid_for(lb_words), kThreads, 0, s>>>(lb, lb_words, 0ull);
    });

    const uint64_t scap = st->scap;
    const uint64_t *skey = ptr<uint64_t>(st->skey[c]);
    const T *samp = ptr<T>(st->samp[c]);
    const T *sK = ptr<T>(st->sK[c]);
    const uint64_t *srank = ptr<uint64_t>(st->srank[c]);

    // ---- (a1) selection weights, formed inside the scan of their prefix, with the
    // excitor-draw guide and the store's rank table
    if (ne) {
        const WeightOut wo{ptr<uint64_t>(st->P), ptr<uint32_t>(st->guide), a.gcap, a.gsh, ne};
        // bytes: amplitude read, prefix written, about two guide entries
        launch(st, "weights_scan", Work{tb + 16.0, nullptr, ne}, [&] {
            scan_lb<uint64_t>(st, WeightSrc<T>{samp, sc}, wo, ne, true, lb + o_weights, tick + kTkWeights, &sc->qtot);
        });
    }

    // ---- (a2-a5, a9, a10) items: non-composite (FNC) then sampled clusters
    Items<T> it{ptr<uint64_t>(st->ikey), ptr<T>(st->iA), ptr<T>(st->ideath), ptr<uint32_t>(st->in),
                ptr<uint8_t>(st->ilevel), ptr<uint64_t>(st->icnt), st->icap};
    ItemPartials part{ptr<double>(st->num_part), ptr<uint64_t>(st->att_part), ptr<uint64_t>(st->disc_part),
                      ptr<uint64_t>(st->max_part)};
    const double item_bytes = kb + 2 * tb + 13.0;  // key, A, death, n, level, slot count
    // the store's rank table for the lookups of the annihilation (built only with a store)
    const RankTable rt{srank, ne, ptr<uint32_t>(st->rtab), st->rt_n, st->rsh};
    const unsigned nb_rt = ne ? grid_for(st->rt_n) : 0;
    if (n_items || nb_rt) {
        // bytes: each item written (plus, for the non-composite ones, the store entry read)
        launch(st, "items", Work{item_bytes, nullptr, n_items}, [&] {
            k_items<W, T><<<nb_fnc + nb_sel + nb_rt, kThreads, 0, s>>>(st->sd, skey, samp, sK, scap, ne,
                                                                       ptr<uint64_t>(st->P), ptr<uint32_t>(st->guide),
                                                                       st->n0, a, it, nb_fnc, n_fnc, nb_fnc + nb_sel, rt,
                                                                       part, sc);
        });
    }
    if (!n_sel) k_fill<uint64_t><<<1, 1, 0, s>>>(it.cnt + n_items, 1, 0ull);
    launch(st, "slot_scan", Work{16.0, nullptr, n_items + 1}, [&] {
        scan_lb<uint64_t>(st, ArraySrc<uint64_t>{it.cnt},
                          SlotOut{ptr<uint64_t>(st->ioff), ptr<uint64_t>(st->block_item), slot_cap}, n_items + 1, false,
                          lb + o_off, tick + kTkOff, &sc->n_slots);
    });

    // ---- (a6-a8) records: death and spawning attempts, one lane per slot, compacted per block
    Records reg{nullptr, ptr<uint64_t>(st->rkey), st->ramp.p, ptr<uint64_t>(st->rid), st->rcap};
    GenStats gst{ptr<uint32_t>(st->gcount), ptr<uint32_t>(st->gspawn), ptr<uint32_t>(st->gdeath)};
    // bytes: the records written and each live item read once (key, A, death, n, offset);
    // work units: spawning attempts
    launch(st, "generate", Work{kb + tb + (ids ? 8.0 : 0.0), &st->cnt_rec, 0, &st->cnt_att, kb + 2 * tb + 12.0,
                                &st->cnt_live_items}, [&] {
        k_generate<W, T><<<(unsigned)nblk_cap, kThreads, 0, s>>>(st->sd, it, ptr<uint64_t>(st->ioff),
                                                                 ptr<uint64_t>(st->block_item), n_fnc, n_items, slot_cap, a,
                                                                 reg, ids ? 1 : 0, gst, sc);
    });
    launch(st, "region_scan", Work{8.0, nullptr, nblk_cap + 1}, [&] {
        scan_lb<uint32_t>(st, ArraySrc<uint32_t>{gst.count}, ArrayOut<uint32_t>{ptr<uint32_t>(st->boff)}, nblk_cap + 1,
                          false, lb + o_boff, tick + kTkBoff, &sc->n_rec);
    });
    const uint64_t dc = st->dcap;
    Records rec{ptr<uint64_t>(st->drank), ptr<uint64_t>(st->dkey), st->damp.p, ptr<uint64_t>(st->did), dc};
    launch(st, "gather", Work{2.0 * (kb + tb + (ids ? 8.0 : 0.0)) + 8.0, &st->cnt_rec, 0}, [&] {
        k_gather<W, T><<<grid_for(rec_cap), kThreads, 0, s>>>(st->sd, reg, ptr<uint32_t>(st->boff), nblk_cap, rec_cap, rec,
                                                              ids ? 1 : 0, sc);
    });

    // ---- (a11) stable LSD radix sort of (rank, record index): one histogram launch for all
    // passes, then one single-sweep launch per digit
    const uint64_t *n_live = &sc->n_live;
    uint32_t *ghist = reinterpret_cast<uint32_t *>(lb + o_ghist);
    launch(st, "radix_ghist", Work{8.0, &st->cnt_rec, 0}, [&] {
        k_radix_ghist<<<(unsigned)tiles, kThreads, 0, s>>>(ptr<uint64_t>(st->drank), n_live, passes, ghist);
    });
    const uint64_t *kin = ptr<uint64_t>(st->drank);
    const uint32_t *iin = nullptr;
    int ob = 0;
    for (int p = 0; p < passes; ++p) {
        uint64_t *kout = ptr<uint64_t>(st->sr[ob]);
        uint32_t *iout = ptr<uint32_t>(st->sidx[ob]);
        launch(st, "radix_onesweep", Work{2 * 8.0 + (iin ? 8.0 : 4.0), &st->cnt_rec, 0}, [&] {
            k_radix_onesweep<<<(unsigned)tiles, kThreads, 0, s>>>(kin, iin, kout, iout, n_live, kRadixBits * p,
                                                                  ghist + kRadixBins * p,
                                                                  lb + o_rstat + (uint64_t)p * tiles * kRadixBins,
                                                                  tick + kTkRadix + p);
        });
        kin = kout;
        iin = iout;
        ob ^= 1;
    }
    const uint64_t *sorted_rank = kin;
    const uint32_t *sorted_idx = iin;

    // ---- (a12) runs of equal determinants: left fold in record order, store lookup by rank
    double *delta = ptr<double>(st->delta);
    FoldTiles ft{reinterpret_cast<double *>(lb + o_fold), reinterpret_cast<uint32_t *>(lb + o_fold + fold_tiles),
                 lb + o_fold + 2 * fold_tiles};
    launch(st, "seg_fold", Work{8.0 + 4.0 + tb + 4.0, &st->cnt_rec, 0}, [&] {
        k_seg_fold<T><<<(unsigned)fold_tiles, kThreads, 0, s>>>(sorted_rank, sorted_idx, ptr<T>(st->damp), rec_cap, srank, ne,
                                                               delta, ptr<uint32_t>(st->is_new), ptr<uint64_t>(st->ins),
                                                               ptr<double>(st->seg_sum), ptr<uint32_t>(st->rtab), st->rt_n,
                                                               st->rsh, ft, sc);
    });
    launch(st, "seg_close", Work{24.0, nullptr, fold_tiles}, [&] {
        k_seg_close<<<grid_for(fold_tiles), kThreads, 0, s>>>(sorted_rank, fold_tiles, srank, ne, delta,
                                                             ptr<uint64_t>(st->ins), ptr<double>(st->seg_sum), ft, sc);
    });
    launch(st, "new_scan", Work{8.0, &st->cnt_rec, 0}, [&] {
        scan_lb<uint32_t>(st, ArraySrc<uint32_t>{ptr<uint32_t>(st->is_new)}, ArrayOut<uint32_t>{ptr<uint32_t>(st->new_pos)},
                          rec_cap, false, lb + o_new, tick + kTkNew, &sc->n_new);
    });
    launch(st, "new_compact", Work{2.0 * (kb + 24.0) + 8.0, &st->cnt_new, 0}, [&] {
        k_new_compact<W><<<grid_for(rec_cap), kThreads, 0, s>>>(sorted_rank, sorted_idx, ptr<uint64_t>(st->dkey), dc, rec_cap,
                                                                ptr<uint32_t>(st->is_new), ptr<uint32_t>(st->new_pos),
                                                                ptr<uint64_t>(st->ins), ptr<double>(st->seg_sum),
                                                                ptr<uint64_t>(st->nkey), ptr<uint64_t>(st->nrank), dc,
                                                                ptr<uint64_t>(st->nins), ptr<double>(st->nsum), sc);
    });

    // ---- (a12, a13) merge and round into the other store buffer, compact back into this one
    const int m = 1 - c;
    const uint64_t S2 = st->scap;
    uint64_t *mkey = ptr<uint64_t>(st->skey[m]);
    T *mamp = ptr<T>(st->samp[m]);
    T *mK = ptr<T>(st->sK[m]);
    uint64_t *mrank = ptr<uint64_t>(st->srank[m]);
    uint32_t *keep = ptr<uint32_t>(st->keep), *pos = ptr<uint32_t>(st->pos);
    const double eb = kb + 2 * tb + 8.0;  // one store entry: key, amplitude, diagonal, rank
    launch(st, "merge", Work{2.0 * eb + 12.0, &st->cnt_merged, 0}, [&] {
        k_merge<W, T><<<grid_for(mcap), kThreads, 0, s>>>(st->sd, skey, samp, sK, srank, S2, ne, delta,
                                                          ptr<uint64_t>(st->nkey), ptr<uint64_t>(st->nrank), dc,
                                                          ptr<uint64_t>(st->nins), ptr<double>(st->nsum), mkey, mamp, mK, mrank,
                                                          S2, mcap, a, keep, sc);
    });
    launch(st, "keep_scan", Work{8.0, &st->cnt_merged, 0}, [&] {
        scan_lb<uint32_t>(st, ArraySrc<uint32_t>{keep}, ArrayOut<uint32_t>{pos}, mcap, false, lb + o_keep, tick + kTkKeep,
                          &sc->n_out);
    });
    launch(st, "compact", Work{2.0 * eb + 8.0, &st->cnt_merged, 0}, [&] {
        k_compact<W, T><<<nb_abs, kThreads, 0, s>>>(mkey, mamp, mK, mrank, S2, mcap, keep, pos,
                                                    ptr<uint64_t>(st->skey[c]), ptr<T>(st->samp[c]), ptr<T>(st->sK[c]),
                                                    ptr<uint64_t>(st->srank[c]), S2, delta, ptr<double>(st->abs_part), sc);
    });

    // ---- (a14) the step's statistics in one fixed-order reduction
    const uint64_t n_parts = nb_fnc + nb_sel;
    const uint64_t fin_blocks = std::min<uint64_t>(
        kMaxFinalParts, std::max<uint64_t>(1, (std::max({n_parts, nblk_cap, (uint64_t)nb_abs}) + 1023) / 1024));
    FinalPart *fin = reinterpret_cast<FinalPart *>(lb + o_fin);
    launch(st, "final", Work{0.0, nullptr, 0}, [&] {
        k_final_part<<<(unsigned)fin_blocks, kThreads, 0, s>>>(part, n_parts, gst, nblk_cap, ptr<double>(st->abs_part), nb_abs,
                                                               fin);
        k_final<<<1, kThreads, 0, s>>>(fin, fin_blocks, sc);
    });

    // ---- (a14) the one synchronisation of the step
    HIP_TRY(hipMemcpyAsync(st->hscratch, sc, sizeof(Scratch), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const Scratch scr = *st->hscratch;
    st->last_q = scr.qtot;
    st->cnt_slots = scr.n_slots;
    st->cnt_rec = scr.n_live;
    st->cnt_merged = ne + scr.n_new;
    st->cnt_new = scr.n_new;
    st->cnt_att = scr.n_attempts;
    st->cnt_live_items = scr.n_slots - scr.n_attempts;
    if (st->prof) resolve_profile(st);
    // plan the next step's capacities from this one
    st->slot_hint = std::max(st->slot_hint, scr.n_slots + scr.n_slots / 4 + 4096);
    st->rec_hint = std::max(st->rec_hint, scr.n_rec + scr.n_rec / 4 + 4096);
    if (scr.err) {
        // the compaction did not run; clear the sums the fold may have left behind
        if (ne) k_fill<double><<<grid_for(ne), kThreads, 0, s>>>(delta, ne, 0.0);
        HIP_TRY(hipStreamSynchronize(s));
        if (scr.err & kErrBlowup) {
            st->err = "population beyond the fixed-point range of the selection weights";
            return CCMC_EBLOWUP;
        }
        if (scr.err & kErrAttempts) {
            st->err = "more than 2^30-2 spawning attempts on one cluster";
            return CCMC_EOVERFLOW;
        }
        *replay = true;  // a capacity was exceeded: grow and replay
        return CCMC_OK;
    }
    const uint64_t nrec = scr.n_live;
    const double n0_old = st->n0;
    if (scr.hf_hit) st->n0 = st->n0 + scr.hf_sum;
    st->ne = scr.n_out;
    st->step += 1;
    st->last_num = scr.num;
    st->last_den = n0_old;
    st->last_nrec = nrec;
    st->last_rec_buf = ids ? 1 : -1;
    if (out) {
        out->step = st->step;
        out->n_selections = n_sel;
        out->n_discarded = scr.n_discarded;
        out->n_spawn_attempts = scr.n_attempts;
        out->n_spawns = scr.n_spawns;
        out->n_deaths = scr.n_deaths;
        out->n_excitors = st->ne;
        out->max_attempts_per_cluster = scr.max_n;
        out->n_total = scr.n_total + std::fabs(st->n0);
        out->n_ref = st->n0;
        out->eproj_num = scr.num;
        out->eproj_den = n0_old;
    }
    return CCMC_OK;
}

template <int W, typename T>
ccmc_status step_impl(ccmc_state *st, double tau, double shift, uint64_t n_sel, ccmc_stats *out)
{
    for (int attempt = 0; attempt < 8; ++attempt) {
        bool replay = false;
        TRY(step_once<W, T>(st, tau, shift, n_sel, out, &replay));
        if (!replay) return CCMC_OK;
    }
    st->err = "step capacity did not converge";
    return CCMC_ENOMEM;
}

template <int W, typename T>
ccmc_status import_impl(ccmc_state *st, const uint64_t *keys, const double *amps, uint64_t n, double n_ref, uint64_t step)
{
    const int Wt = st->W, M = st->hs.M;
    std::vector<uint64_t> hf(W, 0);
    for (int p = 0; p < st->hs.nel; ++p) hf[p >> 6] |= 1ull << (p & 63);
    auto cmp = [&](const uint64_t *x, const uint64_t *y) {
        for (int w = Wt - 1; w >= 0; --w)
            if (x[w] != y[w]) return x[w] < y[w] ? -1 : 1;
        return 0;
    };
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t *k = keys + i * Wt;
        if (i && cmp(keys + (i - 1) * Wt, k) >= 0) {
            st->err = "import: keys not strictly ascending at entry " + std::to_string(i);
            return CCMC_EINVAL;
        }
        int cnt = 0, lev = 0;
        for (int w = 0; w < Wt; ++w) {
            uint64_t v = k[w];
            if (64 * (w + 1) > M) {
                const int keepb = M - 64 * w;
                const uint64_t mask = keepb >= 64 ? ~0ull : ((1ull << keepb) - 1ull);
                if (v & ~mask) {
                    st->err = "import: bits at or above M in entry " + std::to_string(i);
                    return CCMC_EINVAL;
                }
            }
            cnt += __builtin_popcountll(v);
            lev += __builtin_popcountll(v & ~hf[w]);
        }
        if (cnt != st->hs.nel || lev < 1 || lev > st->l) {
            st->err = "import: entry " + std::to_string(i) + " has the wrong electron count or level";
            return CCMC_EINVAL;
        }
        if (!(amps[i] != 0.0) || !std::isfinite(amps[i])) {
            st->err = "import: amplitude " + std::to_string(i) + " is zero or not finite";
            return CCMC_EINVAL;
        }
    }
    if (!std::isfinite(n_ref)) {
        st->err = "import: N_0 not finite";
        return CCMC_EINVAL;
    }
    st->ne = 0;
    TRY(ensure_store<W, T>(st, n + 1));
    const int c = st->cur;
    const uint64_t cap = st->scap;
    std::vector<uint64_t> soa((size_t)W * std::max<uint64_t>(n, 1), 0);
    for (uint64_t i = 0; i < n; ++i)
        for (int w = 0; w < Wt; ++w) soa[(size_t)w * n + i] = keys[i * Wt + w];
    std::vector<T> ta(amps, amps + n);
    if (n) {
        HIP_TRY(hipMemcpy2D(st->skey[c].p, cap * sizeof(uint64_t), soa.data(), n * sizeof(uint64_t), n * sizeof(uint64_t), W,
                            hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(st->samp[c].p, ta.data(), n * sizeof(T), hipMemcpyHostToDevice));
        k_store_init<W, T><<<grid_for(n), kThreads, 0, st->stream>>>(st->sd, ptr<uint64_t>(st->skey[c]), cap, n,
                                                                     ptr<T>(st->sK[c]), ptr<uint64_t>(st->srank[c]));
        k_fill<double><<<grid_for(n), kThreads, 0, st->stream>>>(ptr<double>(st->delta), n, 0.0);
        HIP_TRY(hipStreamSynchronize(st->stream));
    }
    st->ne = n;
    st->n0 = n_ref;
    st->step = step;
    st->last_q = 0;
    st->last_rec_buf = -1;
    st->last_nrec = 0;
    return CCMC_OK;
}

template <int W, typename T>
ccmc_status export_impl(const ccmc_state *cst, uint64_t *keys, double *amps)
{
    ccmc_state *st = const_cast<ccmc_state *>(cst);
    const uint64_t n = st->ne;
    if (!n) return CCMC_OK;
    const int c = st->cur, Wt = st->W;
    std::vector<uint64_t> soa((size_t)W * n);
    std::vector<T> ta(n);
    HIP_TRY(hipMemcpy2D(soa.data(), n * sizeof(uint64_t), st->skey[c].p, st->scap * sizeof(uint64_t), n * sizeof(uint64_t), W,
                        hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ta.data(), st->samp[c].p, n * sizeof(T), hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < n; ++i) {
        if (keys)
            for (int w = 0; w < Wt; ++w) keys[i * Wt + w] = soa[(size_t)w * n + i];
        if (amps) amps[i] = (double)ta[i];
    }
    return CCMC_OK;
}

template <int W, typename T>
ccmc_status export_spawns_impl(const ccmc_state *cst, uint64_t *keys, double *amps, uint64_t *ids)
{
    ccmc_state *st = const_cast<ccmc_state *>(cst);
    const uint64_t n = st->last_nrec;
    if (!n) return CCMC_OK;
    const int Wt = st->W;
    std::vector<uint64_t> soa((size_t)W * n), id(n);
    std::vector<T> ta(n);
    HIP_TRY(hipMemcpy2D(soa.data(), n * sizeof(uint64_t), st->dkey.p, st->dcap * sizeof(uint64_t), n * sizeof(uint64_t), W,
                        hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ta.data(), st->damp.p, n * sizeof(T), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(id.data(), st->did.p, n * sizeof(uint64_t), hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < n; ++i) {
        if (keys)
            for (int w = 0; w < Wt; ++w) keys[i * Wt + w] = soa[(size_t)w * n + i];
        if (amps) amps[i] = (double)ta[i];
        if (ids) ids[i] = id[i];
    }
    return CCMC_OK;
}

// Dispatch on (padded words, precision).
template <template <int, typename> class F, typename... Args>
ccmc_status dispatch(const ccmc_state *st, Args... args)
{
#define CCMC_CASE(WW)                                                                   \
    case WW:                                                                            \
        return st->fp32 ? F<WW, float>::run(args...) : F<WW, double>::run(args...);
    switch (st->WP) {
        CCMC_CASE(1)
        CCMC_CASE(2)
        CCMC_CASE(3)
        CCMC_CASE(4)
        CCMC_CASE(6)
        CCMC_CASE(8)
    }
#undef CCMC_CASE
    return CCMC_EINVAL;
}

template <int W, typename T>
struct StepF {
    static ccmc_status run(ccmc_state *st, double tau, double shift, uint64_t n, ccmc_stats *out)
    {
        return step_impl<W, T>(st, tau, shift, n, out);
    }
};
template <int W, typename T>
struct ImportF {
    static ccmc_status run(ccmc_state *st, const uint64_t *k, const double *a, uint64_t n, double r, uint64_t s)
    {
        return import_impl<W, T>(st, k, a, n, r, s);
    }
};
template <int W, typename T>
struct ExportF {
    static ccmc_status run(const ccmc_state *st, uint64_t *k, double *a) { return export_impl<W, T>(st, k, a); }
};
template <int W, typename T>
struct SpawnsF {
    static ccmc_status run(const ccmc_state *st, uint64_t *k, double *a, uint64_t *i)
    {
        return export_spawns_impl<W, T>(st, k, a, i);
    }
};
template <int W, typename T>
struct StoreF {
    static ccmc_status run(ccmc_state *st, uint64_t n) { return ensure_store<W, T>(st, n); }
};
template <int W, typename T>
struct SystemF {
    static ccmc_status run(ccmc_state *st, const ccmc_integrals *ints) { return upload_system<T>(st, ints); }
};

void destroy(ccmc_state *st)
{
    if (!st) return;
    if (st->stream) (void)hipStreamSynchronize(st->stream);
    DevBuf *bufs[] = {&st->t_grid, &st->t_nvec, &st->t_vq, &st->t_h, &st->t_eri, &st->t_fock, &st->t_vpair,
                      &st->t_binv, &st->t_bino, &st->skey[0], &st->skey[1], &st->samp[0], &st->samp[1], &st->sK[0],
                      &st->sK[1], &st->srank[0], &st->srank[1], &st->P, &st->guide, &st->delta, &st->rtab, &st->ikey,
                      &st->iA, &st->ideath, &st->in, &st->ilevel, &st->icnt, &st->ioff, &st->num_part, &st->att_part, &st->disc_part, &st->max_part, &st->abs_part,
                      &st->block_item, &st->gcount, &st->gspawn, &st->gdeath, &st->boff, &st->rkey, &st->ramp, &st->rid, &st->drank, &st->dkey, &st->damp, &st->did, &st->sr[0], &st->sr[1],
                      &st->sidx[0], &st->sidx[1], &st->is_new,
                      &st->new_pos, &st->ins, &st->seg_sum, &st->nkey, &st->nrank, &st->nins, &st->nsum, &st->keep,
                      &st->pos, &st->lb};
    for (DevBuf *b : bufs) release(st, *b);
    for (auto &p : st->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : st->ev_pool) (void)hipEventDestroy(e);
    if (st->hscratch) (void)hipHostFree(st->hscratch);
    if (st->own_stream && st->stream) (void)hipStreamDestroy(st->stream);
    delete st;
}

}  // namespace

// =========================================================================== C ABI
extern "C" {

ccmc_status ccmc_options_default(ccmc_options *opt)
{
    if (!opt) return CCMC_EINVAL;
    std::memset(opt, 0, sizeof *opt);
    opt->precision = CCMC_FP64;
    opt->full_noncomposite = 0;
    opt->min_spawn_attempts = 1;
    opt->multispawn_threshold = 0.0;
    opt->noncomposite_threshold = 1.0;
    opt->spawn_cutoff = 0.01;
    opt->occupation_threshold = 1.0;
    opt->init_pop = 10.0;
    opt->p_single = 0.1;
    opt->seed = 1234;
    return CCMC_OK;
}

ccmc_status ccmc_init(const ccmc_system *sys, const ccmc_integrals *ints, int truncation, const ccmc_options *opt,
                      ccmc_state **out)
{
    g_init_error.clear();
    if (!sys || !opt || !out) {
        g_init_error = "ccmc_init: null argument";
        return CCMC_EINVAL;
    }
    *out = nullptr;
    if (opt->precision != CCMC_FP64 && opt->precision != CCMC_FP32) {
        g_init_error = "ccmc_init: precision must be CCMC_FP64 or CCMC_FP32";
        return CCMC_EINVAL;
    }
    if (opt->min_spawn_attempts < 1 || !(opt->spawn_cutoff >= 0) || !(opt->occupation_threshold >= 0) ||
        !(opt->p_single >= 0 && opt->p_single <= 1) || !std::isfinite(opt->init_pop)) {
        g_init_error = "ccmc_init: invalid sampling options";
        return CCMC_EINVAL;
    }
    ccmc_state *st = new ccmc_state();
    st->opt = *opt;
    st->sys = *sys;
    st->l = truncation;
    st->fp32 = opt->precision == CCMC_FP32;
    st->es = st->fp32 ? 4 : 8;
    std::string err;
    bool ok = false;
    if (sys->kind == CCMC_UEG)
        ok = build_ueg(st->hs, sys->n_electrons, sys->n2_max, sys->rs, err) && sys->rs > 0;
    else if (sys->kind == CCMC_MOLECULAR && ints)
        ok = build_mol(st->hs, sys->n_electrons, ints, err);
    else
        err = "ccmc_init: unknown system kind or missing integrals";
    if (ok && (truncation < 1 || truncation > 6 || truncation > sys->n_electrons)) {
        ok = false;
        err = "ccmc_init: truncation must be in [1, min(6, N)]";
    }
    if (!ok) {
        g_init_error = err.empty() ? "ccmc_init: invalid system" : err;
        delete st;
        return CCMC_EINVAL;
    }
    st->sys.n_spin_orbitals = st->hs.M;
    st->W = words_for(st->hs.M);
    st->WP = padded_words(st->W);
    if (opt->hip_stream) {
        st->stream = (hipStream_t)opt->hip_stream;
    } else {
        if (hipStreamCreate(&st->stream) != hipSuccess) {
            g_init_error = "ccmc_init: hipStreamCreate failed (no GPU?)";
            delete st;
            return CCMC_EDEVICE;
        }
        st->own_stream = true;
    }
    ccmc_status rc = CCMC_OK;
    if (hipHostMalloc((void **)&st->hscratch, sizeof(Scratch)) != hipSuccess) {
        st->err = "hipHostMalloc failed";
        rc = CCMC_EDEVICE;
    }
    if (rc == CCMC_OK) rc = dispatch<SystemF>(st, st, ints);
    if (rc == CCMC_OK) rc = dispatch<StoreF>(st, st, (uint64_t)1024);
    if (rc != CCMC_OK) {
        g_init_error = st->err;
        destroy(st);
        return rc;
    }
    st->n0 = opt->init_pop;
    *out = st;
    return CCMC_OK;
}

ccmc_status ccmc_step(ccmc_state *st, double tau, double shift, uint64_t n_attempts, ccmc_stats *out)
{
    if (!st) return CCMC_EINVAL;
    st->err.clear();
    if (!(tau > 0) || !std::isfinite(tau) || !std::isfinite(shift) || n_attempts > 0xFFFFFFFFull) {
        st->err = "ccmc_step: need tau > 0, finite shift and n_attempts < 2^32";
        return CCMC_EINVAL;
    }
    if (st->ne + 1 > 0xFFFFFFFFull) {
        st->err = "ccmc_step: store too large for 32-bit item indices";
        return CCMC_EOVERFLOW;
    }
    return dispatch<StepF>(st, st, tau, shift, n_attempts, out);
}

ccmc_status ccmc_energy(const ccmc_state *st, double *e_hf, double *eproj_num, double *eproj_den)
{
    if (!st) return CCMC_EINVAL;
    if (e_hf) *e_hf = st->hs.ehf;
    if (eproj_num) *eproj_num = st->last_num;
    if (eproj_den) *eproj_den = st->last_den;
    return CCMC_OK;
}

void ccmc_free(ccmc_state *st) { destroy(st); }

const char *ccmc_last_error(const ccmc_state *st) { return st ? st->err.c_str() : g_init_error.c_str(); }

ccmc_status ccmc_export_size(const ccmc_state *st, uint64_t *n)
{
    if (!st || !n) return CCMC_EINVAL;
    *n = st->ne;
    return CCMC_OK;
}

ccmc_status ccmc_export(const ccmc_state *st, uint64_t *keys, double *amps, uint64_t capacity, uint64_t *n, double *n_ref,
                        uint64_t *step)
{
    if (!st) return CCMC_EINVAL;
    ccmc_state *m = const_cast<ccmc_state *>(st);
    m->err.clear();
    if (capacity < st->ne) {
        m->err = "ccmc_export: capacity smaller than the store";
        return CCMC_EINVAL;
    }
    ccmc_status rc = dispatch<ExportF>(st, st, keys, amps);
    if (rc != CCMC_OK) return rc;
    if (n) *n = st->ne;
    if (n_ref) *n_ref = st->n0;
    if (step) *step = st->step;
    return CCMC_OK;
}

ccmc_status ccmc_import(ccmc_state *st, const uint64_t *keys, const double *amps, uint64_t n, double n_ref, uint64_t step)
{
    if (!st || (n && (!keys || !amps))) return CCMC_EINVAL;
    st->err.clear();
    return dispatch<ImportF>(st, st, keys, amps, n, n_ref, step);
}

ccmc_status ccmc_spawns_size(const ccmc_state *st, uint64_t *n)
{
    if (!st || !n) return CCMC_EINVAL;
    *n = st->last_rec_buf >= 0 ? st->last_nrec : 0;
    return CCMC_OK;
}

ccmc_status ccmc_export_spawns(const ccmc_state *st, uint64_t *keys, double *amps, uint64_t *ids, uint64_t capacity,
                               uint64_t *n)
{
    if (!st) return CCMC_EINVAL;
    ccmc_state *m = const_cast<ccmc_state *>(st);
    m->err.clear();
    if (!st->opt.keep_spawn_ids) {
        m->err = "ccmc_export_spawns: keep_spawn_ids is off";
        return CCMC_EINVAL;
    }
    const uint64_t nr = st->last_rec_buf >= 0 ? st->last_nrec : 0;
    if (capacity < nr) {
        m->err = "ccmc_export_spawns: capacity too small";
        return CCMC_EINVAL;
    }
    if (nr) {
        ccmc_status rc = dispatch<SpawnsF>(st, st, keys, amps, ids);
        if (rc != CCMC_OK) return rc;
    }
    if (n) *n = nr;
    return CCMC_OK;
}

ccmc_status ccmc_profile(ccmc_state *st, const char *kernels)
{
    if (!st) return CCMC_EINVAL;
    st->prof = kernels != nullptr && kernels[0] != 0;
    if (!st->prof) {
        st->prof_names.clear();
    } else if (std::string(kernels) == "*") {
        st->prof_names = "*";
    } else {
        std::string k;
        for (const char *c = kernels; *c; ++c)
            if (*c != ' ') k += *c;
        st->prof_names = "," + k + ",";
    }
    return CCMC_OK;
}

ccmc_status ccmc_profile_read(ccmc_state *st, ccmc_kernel_time *out, int capacity, int *n)
{
    if (!st || !n) return CCMC_EINVAL;
    resolve_profile(st);
    int k = 0;
    for (auto &kv : st->accum) {
        if (k < capacity && out) {
            std::memset(&out[k], 0, sizeof(ccmc_kernel_time));
            std::strncpy(out[k].name, kv.first.c_str(), sizeof(out[k].name) - 1);
            out[k].launches = kv.second.launches;
            out[k].ms = kv.second.ms;
            out[k].bytes = kv.second.bytes;
            out[k].items = kv.second.items;
        }
        ++k;
    }
    *n = std::min(k, capacity);
    st->accum.clear();
    return CCMC_OK;
}

ccmc_status ccmc_dims(const ccmc_state *st, int *n_electrons, int *n_spin_orbitals, int *n_words)
{
    if (!st) return CCMC_EINVAL;
    if (n_electrons) *n_electrons = st->hs.nel;
    if (n_spin_orbitals) *n_spin_orbitals = st->hs.M;
    if (n_words) *n_words = st->W;
    return CCMC_OK;
}

ccmc_status ccmc_memory(const ccmc_state *st, uint64_t *bytes)
{
    if (!st || !bytes) return CCMC_EINVAL;
    *bytes = st->bytes_held;
    return CCMC_OK;
}

}  // extern "C"
