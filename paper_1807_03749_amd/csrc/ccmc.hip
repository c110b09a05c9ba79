// ccmc.hip -- host side of the MI355X CCMC step library: system tables, device buffers,
// the launch sequence of one time step, and the C ABI declared in include/ccmc.h.
//
// Paper: Spencer, Neufeld, Vigor, Franklin & Thom, arXiv:1807.03749 (Sec. II, Sec. IV).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ccmc.h"
#include "kernels.h"

using namespace ccmc;

// The step area of ccmc_step_noalloc: a fixed device array, one copy per GPU, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the host it is only a
// stand-in for the symbol); it uses the device address hipGetSymbolAddress gives for each GPU.
static __device__ __align__(256) uint64_t scratch[CCMC_NOALLOC_AREA_BYTES / sizeof(uint64_t)];

namespace {

thread_local std::string g_init_error;

// Device address of the fixed step area (`scratch`, above) on each GPU.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint64_t *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on GPU dev, looked up once per GPU with that GPU current.
ccmc_status noalloc_area(int dev, uint64_t **out, std::string &err)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) {
        err = "ccmc_init: device index beyond the no-allocation area table";
        return CCMC_EDEVICE;
    }
    if (!g_scratch_dev[dev]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) {
            err = "ccmc_init: hipGetDevice failed";
            return CCMC_EDEVICE;
        }
        if (cur != dev && hipSetDevice(dev) != hipSuccess) {
            err = "ccmc_init: hipSetDevice failed";
            return CCMC_EDEVICE;
        }
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) {
            err = std::string("ccmc_init: hipGetSymbolAddress of the no-allocation area failed: ") + hipGetErrorString(e);
            return CCMC_EDEVICE;
        }
        g_scratch_dev[dev] = static_cast<uint64_t *>(p);
    }
    *out = g_scratch_dev[dev];
    return CCMC_OK;
}

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
    std::vector<Work> w;  // one per state of the launch
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
    double e_core = 0;  // constant added to reported absolute energies
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
    DevBuf t_grid, t_nvec, t_vq, t_h, t_eri, t_fock, t_vpair, t_binv, t_bino, t_rankv, t_pairs, t_kpack;
    int rank_bits = 0;  // bits of the largest truncated-space rank
    // the store: current buffer cur, merge target 1 - cur
    DevBuf skey[2], samp[2], sK[2], srank[2];
    uint64_t scap = 0;
    int cur = 0;
    uint64_t ne = 0;
    double n0 = 0;
    double last_ntot = 0;  // N_tot after the last step (or at init / import): the blow-up bound's base
    uint64_t step = 0;
    double last_num = 0, last_den = 0;
    // per-step buffers
    DevBuf P, guide, delta, fence, rtab;
    DevBuf drec;  // draw records: prefix, amplitude and bitstring of each excitor, (2 + W) words
    DevBuf vkey[2], perm, seg;  // virtual processors: placement keys, the partition, its segments
    uint64_t last_q = 0; // Q of the last step (sizes the next selection guide)
    DevBuf ikey, iA, ideath, in, icnt, ioff;
    uint64_t icap = 0;
    DevBuf num_part, att_part, disc_part, max_part, abs_part;
    DevBuf block_item, gcount, gspawn, gdeath, boff;
    DevBuf rkey, ramp, rid;  // per-block record regions
    uint64_t rcap = 0;              // region slots
    DevBuf drank, dkey, damp, did, sr[2], sval[2], tile_region;
    DevBuf nkey, nrank, nins, nsum;
    uint64_t dcap = 0;  // dense record capacity
    uint64_t slot_hint = 1 << 16, rec_hint = 1 << 14;  // capacities planned for the next step
    uint64_t cnt_slots = 0, cnt_rec = 0, cnt_merged = 0, cnt_new = 0, cnt_att = 0, cnt_live_items = 0;  // live counts of the last step
    DevBuf lb;  // step scalars, tickets, radix histograms and look-back status words
    size_t lb_clean_bytes = 0;  // leading bytes of lb (and the fold sums) known to be zero
    // batched steps led by this state: argument tables and the batch's step scalars
    DevBuf arg_dev;
    uint8_t *arg_host = nullptr;  // pinned
    size_t arg_hcap = 0;
    Scratch *batch_hscr = nullptr;  // pinned, coherent: written by k_final_part
    Scratch *batch_hdev = nullptr;  // its device address
    size_t batch_hcap = 0;
    uint64_t batch_seq = 0;         // sequence number of the last batch this state led
    // last step's spawn list (keep_spawn_ids)
    uint64_t last_nrec = 0;
    int last_rec_buf = -1;
    size_t bytes_held = 0;
    // ccmc_step_noalloc: the GPU of the state's stream, that GPU's copy of the fixed step area,
    // and the flag that turns every buffer growth of the call into CCMC_ENOMEM
    int device = 0;
    uint64_t *noalloc_area = nullptr;
    bool no_grow = false;
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
    if (st->no_grow) {
        st->err = "ccmc_step_noalloc: the step needs a buffer of " + std::to_string(bytes) + " bytes where the state holds " +
                  std::to_string(b.bytes) + "; step once with ccmc_step to reserve it";
        return CCMC_ENOMEM;
    }
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
void launch(ccmc_state *st, const char *name, const std::vector<Work> &w, F &&f)
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
        Accum &a = st->accum[p.name];
        a.launches++;
        a.ms += ms;
        for (const Work &w : p.w) {
            const double n = (double)(w.count ? *w.count : w.fixed);
            a.bytes += w.unit_bytes * n + (w.count2 ? w.unit_bytes2 * (double)*w.count2 : 0.0);
            a.items += w.items ? (double)*w.items : n;
        }
        st->ev_pool.push_back(p.a);
        st->ev_pool.push_back(p.b);
    }
    st->pending.clear();
}

// --------------------------------------------------------------------------- scan
// Tiles of a single-launch look-back scan of n values.
uint64_t scan_tiles(uint64_t n, int items = kScanItems) { return (n + (uint64_t)kThreads * items - 1) / ((uint64_t)kThreads * items); }

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
        ints->n_chol < 0 || (ints->n_chol > 0 && !ints->chol) || (!ints->eri && ints->n_chol == 0) ||
        !std::isfinite(ints->e_core)) {
        err = "molecular: invalid sizes or null integral arrays";
        return false;
    }
    hs.e_core = ints->e_core;
    hs.kind = CCMC_MOLECULAR;
    hs.nel = nel;
    hs.nsp = n;
    hs.M = 2 * n;
    hs.h.assign(ints->h, ints->h + (size_t)n * n);
    const int M = hs.M;
    const size_t nn = (size_t)n * n;
    auto eri = [&](int P, int Q, int R, int S) {  // (PQ|RS): given, or summed over L in order
        if (ints->eri) return ints->eri[((size_t)P * n + Q) * nn + (size_t)R * n + S];
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
        // the rank's term of a virtual orbital p with v virtual electrons above it (all the
        // electrons above p are then virtual): sum_j C(p - N, j) C(N, N - v - j), j <= l - v
        const int L = st->l;
        std::vector<uint64_t> rv((size_t)(M - N + 1) * (L + 1), 0);
        for (int nv = 0; nv <= M - N; ++nv)
            for (int v = 0; v <= L && v <= N; ++v) {
                uint64_t t = 0;
                for (int j = 0; j <= L - v && j <= N - v; ++j) t += bv[(size_t)nv * 9 + j] * bo[(size_t)N * (N + 1) + (N - v - j)];
                rv[(size_t)nv * (L + 1) + v] = t;
            }
        TRY(ensure(st, st->t_rankv, rv.size() * 8));
        HIP_TRY(hipMemcpy(st->t_rankv.p, rv.data(), rv.size() * 8, hipMemcpyHostToDevice));
        S.rank_v = ptr<uint64_t>(st->t_rankv);
    }
    TRY(upload_table<T>(st, st->t_fock, hs.fock));
    TRY(upload_table<T>(st, st->t_vpair, hs.vpair));
    S.fock = st->t_fock.p;
    S.vpair = st->t_vpair.p;
    {  // occupied pairs (x < y) in lexicographic rank order, for the generators' pair draws
        std::vector<uint32_t> pr;
        for (int x = 0; x < hs.nel; ++x)
            for (int y = x + 1; y < hs.nel; ++y) pr.push_back((uint32_t)x | ((uint32_t)y << 16));
        pr.push_back(0);
        TRY(ensure(st, st->t_pairs, pr.size() * sizeof(uint32_t)));
        HIP_TRY(hipMemcpy(st->t_pairs.p, pr.data(), pr.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        S.pairs = ptr<uint32_t>(st->t_pairs);
    }
    if (hs.kind == CCMC_UEG) {
        if (hs.G > 127) {
            st->err = "UEG basis too wide for the packed wavevectors (|n_i| > 127)";
            return CCMC_EINVAL;
        }
        std::vector<uint32_t> kp((size_t)hs.nsp + 1, 0);
        for (int p = 0; p < hs.nsp; ++p)
            for (int c = 0; c < 3; ++c) kp[p] |= (uint32_t)(hs.nvec[3 * p + c] + hs.G + 256) << (10 * c);
        TRY(ensure(st, st->t_kpack, kp.size() * sizeof(uint32_t)));
        HIP_TRY(hipMemcpy(st->t_kpack.p, kp.data(), kp.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        S.kpack = ptr<uint32_t>(st->t_kpack);
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
        if (ints->eri) {  // the full table as given
            TRY(upload_table<T>(st, st->t_eri, std::vector<double>(ints->eri, ints->eri + n4)));
        } else {          // built on the device from the Cholesky vectors
            DevBuf chol;
            const size_t cb = std::max<size_t>(1, (size_t)ints->n_chol * n * n) * sizeof(double);
            TRY(ensure(st, chol, cb));
            HIP_TRY(hipMemcpy(chol.p, ints->chol, (size_t)ints->n_chol * n * n * sizeof(double), hipMemcpyHostToDevice));
            TRY(ensure(st, st->t_eri, n4 * sizeof(T)));
            k_build_eri<T><<<grid_for(n4), kThreads, 0, st->stream>>>(ptr<double>(chol), (int)n, ints->n_chol,
                                                                      ptr<T>(st->t_eri));
            HIP_TRY(hipStreamSynchronize(st->stream));
            release(st, chol);
        }
        S.eri = st->t_eri.p;
    }
    return CCMC_OK;
}

// ------------------------------------------------------------------------ the store
// Entries of the selection guide for a store capacity: several times the buckets the shift
// aims at, so that Q may grow between steps before draws fall past the table.
uint64_t guide_cap(uint64_t scap) { return 16 * scap + 8; }

// The buffers sized by the store capacity whose contents do not outlive a step: the merge's
// output store, the draw and guide arrays, the per-entry sums and the lookup index.  Ensured on
// every call, so that a call that failed for memory after the store itself grew finds them again.
template <int W, typename T>
ccmc_status ensure_store_companions(ccmc_state *st, uint64_t nc)
{
    const int m = 1 - st->cur;
    TRY(ensure(st, st->skey[m], nc * W * sizeof(uint64_t)));
    TRY(ensure(st, st->samp[m], nc * sizeof(T)));
    TRY(ensure(st, st->sK[m], nc * sizeof(T)));
    TRY(ensure(st, st->srank[m], nc * sizeof(uint64_t)));
    TRY(ensure(st, st->P, nc * sizeof(uint64_t)));
    TRY(ensure(st, st->drec, nc * (2 + W) * sizeof(uint64_t)));
    TRY(ensure(st, st->guide, guide_cap(nc) * sizeof(uint32_t)));
    if (st->opt.n_ranks > 1) {
        for (DevBuf *b : {&st->vkey[0], &st->vkey[1]}) TRY(ensure(st, *b, nc * sizeof(uint64_t)));
        TRY(ensure(st, st->perm, nc * sizeof(uint32_t)));
        TRY(ensure(st, st->seg, (kMaxRanks + 2) * sizeof(uint32_t)));
    }
    // the per-entry sums start at zero: a reallocated buffer holds no contents
    const void *held = st->delta.p;
    TRY(ensure(st, st->delta, nc * sizeof(double)));
    if (st->delta.p != held)
        k_fill<double><<<grid_for(st->delta.bytes / sizeof(double)), kThreads, 0, st->stream>>>(
            ptr<double>(st->delta), st->delta.bytes / sizeof(double), 0.0);
    // the lookup index: every kFence-th rank (for a store too large for the cache), and the
    // rank table, at most one bucket per fence entry rounded up to a power of two (planned per step)
    TRY(ensure(st, st->fence, (nc / kFence + 2) * sizeof(uint64_t)));
    TRY(ensure(st, st->rtab, (8 * std::min<uint64_t>(nc, kFenceDirect) + 2 * (nc / kFence) + 2) * sizeof(uint32_t)));
    return CCMC_OK;
}

// Grow the store to hold n entries, keeping the current contents.  The key words are stored
// one row per word with the capacity as the row pitch, so the capacity changes together with
// the current buffers or not at all: a call that fails for memory leaves the store as it was.
template <int W, typename T>
ccmc_status ensure_store(ccmc_state *st, uint64_t n)
{
    if (n > st->scap) {
        const uint64_t nc = std::max<uint64_t>(n, std::max<uint64_t>(1024, st->scap + st->scap / 2));
        DevBuf nb[4];
        const size_t bytes[4] = {nc * W * sizeof(uint64_t), nc * sizeof(T), nc * sizeof(T), nc * sizeof(uint64_t)};
        for (int b = 0; b < 4; ++b) {
            const ccmc_status rc = ensure(st, nb[b], bytes[b]);
            if (rc != CCMC_OK) {
                for (DevBuf &x : nb) release(st, x);
                return rc;
            }
        }
        const int c = st->cur;
        if (st->ne) {
            HIP_TRY(hipMemcpy2DAsync(nb[0].p, nc * sizeof(uint64_t), st->skey[c].p, st->scap * sizeof(uint64_t),
                                     st->ne * sizeof(uint64_t), W, hipMemcpyDeviceToDevice, st->stream));
            HIP_TRY(hipMemcpyAsync(nb[1].p, st->samp[c].p, st->ne * sizeof(T), hipMemcpyDeviceToDevice, st->stream));
            HIP_TRY(hipMemcpyAsync(nb[2].p, st->sK[c].p, st->ne * sizeof(T), hipMemcpyDeviceToDevice, st->stream));
            HIP_TRY(hipMemcpyAsync(nb[3].p, st->srank[c].p, st->ne * sizeof(uint64_t), hipMemcpyDeviceToDevice, st->stream));
            HIP_TRY(hipStreamSynchronize(st->stream));
        }
        for (int b = 0; b < 2; ++b) {
            release(st, st->skey[b]);
            release(st, st->samp[b]);
            release(st, st->sK[b]);
            release(st, st->srank[b]);
        }
        st->skey[c] = nb[0];
        st->samp[c] = nb[1];
        st->sK[c] = nb[2];
        st->srank[c] = nb[3];
        st->scap = nc;
    }
    return ensure_store_companions<W, T>(st, st->scap);
}

// ---------------------------------------------------------------------- the step
constexpr uint64_t kMaxFinalParts = kThreads * kFinalPerThread;  // blocks of the first stage of the final reduction

// Per-state plan of one batched step: sizes, capacities, the layout of the step area and
// every pointer the kernels need.  Planning allocates; nothing is launched before every state
// of the batch has been planned.
template <int W, typename T>
struct Plan {
    ccmc_state *st = nullptr;
    double tau = 0, shift = 0;
    uint64_t n_sel = 0;
    ccmc_stats *out = nullptr;
    StepArgs a{};
    bool fnc = false, ids = false;
    int c = 0, passes = 1;
    uint64_t ne = 0, n_fnc = 0, n_items = 0, slot_cap = 0, nblk_cap = 0, rec_cap = 0, mcap = 0, tiles = 0;
    uint64_t fold_tiles = 0, fin_blocks = 1, n_parts = 0, lb_words = 0;
    uint64_t gentries = 0;   // selection-guide buckets the step fills (from the last step's Q)
    unsigned nb_fnc = 0, nb_sel = 0, nb_rt = 0, nb_abs = 0;
    uint64_t o_tick = 0, o_weights = 0, o_off = 0, o_boff = 0, o_merge = 0, o_ghist = 0, o_rstat = 0;
    uint64_t o_fold = 0, o_fin = 0;
    bool packed = false;     // sort keys carry the rank in their high half and the record's position below
    uint64_t rt_n = 1;       // rank-table buckets of the store lookups, and their shift in rank space
    uint32_t rsh = 0;
    bool ranked = false;     // virtual processors: the store is partitioned by processor
    uint64_t ptiles = 0;     // radix tiles of the partition
    uint64_t o_pghist = 0, o_pstat = 0;
    uint64_t *lb = nullptr;
    Scratch *sc = nullptr;
    ccmc_status rc = CCMC_OK;  // this state's outcome
    bool replay = false;       // a capacity overflowed: grow and step again
};

enum { kTkWeights, kTkOff, kTkBoff, kTkFold, kTkMerge, kTkPlace, kTkFinal, kTkRadix, kTickets = kTkRadix + kRadixMaxPasses };

// Sizes and capacities of one state's step (all allocation happens here).
template <int W, typename T>
ccmc_status plan_sizes(Plan<W, T> &p)
{
    ccmc_state *st = p.st;
    const uint64_t ne = st->ne;
    p.ne = ne;
    p.fnc = st->opt.full_noncomposite != 0;
    p.ids = st->opt.keep_spawn_ids != 0;
    p.n_fnc = p.fnc ? ne + 1 : 0;
    p.n_items = p.n_fnc + p.n_sel;
    p.c = st->cur;
    StepArgs &a = p.a;
    a.tau = p.tau;
    a.shift = p.shift;
    a.cutoff = st->opt.spawn_cutoff;
    a.theta = st->opt.occupation_threshold;
    a.thr_cluster = st->opt.multispawn_threshold;
    a.thr_nc = st->opt.noncomposite_threshold;
    a.kmin = (uint32_t)st->opt.min_spawn_attempts;
    a.step = (uint32_t)(st->step & 0x0FFFFFFFu);
    a.key0 = (uint32_t)st->opt.seed;
    a.key1 = (uint32_t)(st->opt.seed >> 32);
    a.n_sel = p.n_sel;
    a.fnc = p.fnc ? 1 : 0;
    p.packed = st->rank_bits <= 32;
    p.ranked = st->opt.n_ranks > 1;
    a.n_ranks = p.ranked ? st->opt.n_ranks : 1;
    p.ptiles = p.ranked ? (ne + kSortTile - 1) / kSortTile : 0;
    {
        // guide shift from the last step's Q (any shift gives the same draws).  A store beyond
        // about 10^6 excitors takes about eight buckets per excitor, so that most draws land in
        // a bucket inside one excitor's weight and need no prefix probe in HBM (16e/92so items
        // 947 -> 779 us, guide 100 -> 139 us); a smaller one, whose probes hit the cache, two,
        // because there the fill of the finer guide costs more than the probes it saves.
        const uint64_t per = ne > (1ull << 20) ? 8 : 2;
        const uint64_t q_est = st->last_q ? st->last_q : (ne << 24);
        uint32_t sh = 0;
        while (sh < 63 && (q_est >> sh) + 2 > per * ne + 2) ++sh;
        a.gsh = sh;
        p.gentries = (q_est >> sh) + 2;
    }
    p.slot_cap = std::max<uint64_t>(kGenSlots, (st->slot_hint + kGenSlots - 1) / kGenSlots * kGenSlots);
    p.rec_cap = std::max<uint64_t>(1, std::min<uint64_t>(st->rec_hint, p.slot_cap));
    if (st->no_grow) {
        // ccmc_step_noalloc: the capacities are what the state's buffers hold (a count beyond
        // them is found on the device and fails the call); nothing is planned beyond them
        const uint64_t slots_held = st->rcap / kGenSlots * kGenSlots;
        const uint64_t abs_held = st->abs_part.bytes / sizeof(double);
        const uint64_t merged_held = std::min<uint64_t>(st->scap ? st->scap - 1 : 0,
                                                        abs_held ? (abs_held - 1) * kMergeTile : 0);
        p.slot_cap = std::min(p.slot_cap, slots_held);
        p.rec_cap = std::min({p.rec_cap, p.slot_cap, st->dcap ? st->dcap - 1 : 0, merged_held > ne ? merged_held - ne : 0});
        if (p.slot_cap < kGenSlots || p.rec_cap < 1) {
            st->err = "ccmc_step_noalloc: the state holds no record buffers for this step; step once with ccmc_step to reserve them";
            return CCMC_ENOMEM;
        }
    }
    p.nblk_cap = p.slot_cap / kGenSlots;
    if (p.slot_cap + ne + 1 >= (1ull << 32)) {
        st->err = "more than 2^32 record slots in one step";
        return CCMC_EOVERFLOW;
    }
    if (p.n_items + 1 > st->icap) {
        const uint64_t nc = std::max<uint64_t>(p.n_items + 1, st->icap + st->icap / 2);
        TRY(ensure(st, st->ikey, nc * W * sizeof(uint64_t)));
        TRY(ensure(st, st->iA, nc * sizeof(T)));
        TRY(ensure(st, st->ideath, nc * sizeof(T)));
        TRY(ensure(st, st->in, nc * sizeof(uint32_t)));
        TRY(ensure(st, st->icnt, nc * sizeof(uint64_t)));
        TRY(ensure(st, st->ioff, nc * sizeof(uint64_t)));
        st->icap = nc;
    }
    if (p.slot_cap > st->rcap) {
        const uint64_t nc = p.slot_cap;
        const uint64_t nb = nc / kGenSlots + 2;
        TRY(ensure(st, st->rkey, nc * W * sizeof(uint64_t)));
        TRY(ensure(st, st->ramp, nc * sizeof(T)));
        TRY(ensure(st, st->block_item, nb * sizeof(uint64_t)));
        for (DevBuf *b : {&st->gcount, &st->gspawn, &st->gdeath, &st->boff}) TRY(ensure(st, *b, nb * sizeof(uint32_t)));
        st->rcap = nc;
    }
    if (p.ids && st->rid.bytes < st->rcap * sizeof(uint64_t)) TRY(ensure(st, st->rid, st->rcap * sizeof(uint64_t)));
    if (p.rec_cap + 1 > st->dcap) {
        const uint64_t nc = p.rec_cap + 1;
        for (DevBuf *b : {&st->dkey, &st->nkey}) TRY(ensure(st, *b, nc * W * sizeof(uint64_t)));
        TRY(ensure(st, st->damp, nc * sizeof(T)));
        for (DevBuf *b : {&st->drank, &st->sr[0], &st->sr[1], &st->nins, &st->nrank})
            TRY(ensure(st, *b, nc * sizeof(uint64_t)));
        for (DevBuf *b : {&st->sval[0], &st->sval[1]}) TRY(ensure(st, *b, nc * sizeof(T)));
        TRY(ensure(st, st->nsum, nc * sizeof(double)));
        TRY(ensure(st, st->tile_region, (nc / kGatherTile + 2) * sizeof(uint32_t)));
        st->dcap = nc;
    }
    if (p.ids && st->did.bytes < st->dcap * sizeof(uint64_t)) TRY(ensure(st, st->did, st->dcap * sizeof(uint64_t)));
    p.mcap = ne + p.rec_cap;  // merged store capacity of this step
    TRY(ensure_store<W, T>(st, p.mcap + 1));
    p.a.gcap = guide_cap(st->scap);
    p.tiles = (p.rec_cap + kSortTile - 1) / kSortTile;
    p.fold_tiles = (p.rec_cap + kFoldTile - 1) / kFoldTile;
    p.passes = std::max(1, (st->rank_bits + kRadixBits - 1) / kRadixBits);
    p.nb_fnc = p.fnc ? grid_for(p.n_fnc) : 0;
    p.nb_sel = p.n_sel ? grid_for(p.n_sel) : 0;
    {  // about one rank-space bucket per fence entry; four per entry for a store in the cache
        const uint64_t want = fence_stride(ne) > 1 ? fence_count(ne) : 4 * ne;
        int rt_bits = 1;
        while (rt_bits < 40 && (1ull << rt_bits) < want) ++rt_bits;
        rt_bits = std::min(rt_bits, std::max(st->rank_bits, 1));
        p.rt_n = 1ull << rt_bits;
        p.rsh = (uint32_t)std::max(0, st->rank_bits - rt_bits);
    }
    p.nb_rt = ne ? (fence_stride(ne) > 1 ? grid_for(fence_count(ne)) : 0) + grid_for(p.rt_n) : 0;
    p.n_parts = p.nb_fnc + p.nb_sel;
    const size_t nparts = (size_t)(p.n_parts + 1);
    TRY(ensure(st, st->num_part, nparts * sizeof(double)));
    TRY(ensure(st, st->att_part, nparts * sizeof(uint64_t)));
    TRY(ensure(st, st->disc_part, nparts * sizeof(uint64_t)));
    TRY(ensure(st, st->max_part, nparts * sizeof(uint64_t)));
    p.nb_abs = grid_for(p.mcap, kMergeTile);
    TRY(ensure(st, st->abs_part, (p.nb_abs + 1) * sizeof(double)));
    p.fin_blocks = std::min<uint64_t>(
        kMaxFinalParts, std::max<uint64_t>(1, (std::max({p.n_parts, p.nblk_cap, (uint64_t)p.nb_abs}) + 1023) / 1024));
    return CCMC_OK;
}

// The zeroed step area of one state (64-bit words): the step scalars, the scan tickets, the
// look-back status words of every scan and radix pass (the batch's number of passes), the
// radix histograms, the fold's tile summaries and the first stage of the final reduction.
template <int W, typename T>
ccmc_status plan_area(Plan<W, T> &p, int passes)
{
    ccmc_state *st = p.st;
    p.passes = passes;
    const uint64_t w_scratch = (sizeof(Scratch) + 7) / 8;
    p.o_tick = w_scratch;
    p.o_weights = p.o_tick + kTickets;
    p.o_off = p.o_weights + scan_tiles(p.ne);
    p.o_boff = p.o_off + scan_tiles(p.n_items + 1);
    p.o_merge = p.o_boff + scan_tiles(p.nblk_cap + 1);
    p.o_ghist = p.o_merge + grid_for(p.mcap, kMergeTile);
    p.o_rstat = p.o_ghist + (uint64_t)passes * kRadixBins / 2;
    p.o_fold = p.o_rstat + (uint64_t)passes * p.tiles * kRadixBins;
    p.o_pghist = p.o_fold + 8 * p.fold_tiles;  // lead, has_head, open, open_new, look-back status, open run
    p.o_pstat = p.o_pghist + kRadixBins / 2;
    p.o_fin = p.o_pstat + p.ptiles * kRadixBins;
    p.lb_words = p.o_fin + kMaxFinalParts * (sizeof(FinalPart) / 8);
    if (st->no_grow) {  // ccmc_step_noalloc: the GPU's fixed area, cleared by the step's first kernel
        if (p.lb_words * sizeof(uint64_t) > CCMC_NOALLOC_AREA_BYTES) {
            st->err = "ccmc_step_noalloc: the step area needs " + std::to_string(p.lb_words * sizeof(uint64_t)) +
                      " bytes, above the fixed " + std::to_string((unsigned long long)CCMC_NOALLOC_AREA_BYTES);
            return CCMC_ENOMEM;
        }
        p.lb = st->noalloc_area;
        p.sc = reinterpret_cast<Scratch *>(p.lb);
        return CCMC_OK;
    }
    const void *lb_was = st->lb.p;
    TRY(ensure(st, st->lb, p.lb_words * sizeof(uint64_t)));
    if (st->lb.p != lb_was) st->lb_clean_bytes = 0;  // a new area holds no known contents
    p.lb = ptr<uint64_t>(st->lb);
    p.sc = reinterpret_cast<Scratch *>(p.lb);
    return CCMC_OK;
}

// Argument tables of a batched step: per kernel, the states' argument structs and the
// block map, staged in host memory and copied to the device in one transfer.
struct ArgArena {
    ccmc_state *now = nullptr;  // one state: each kernel is launched as soon as it is staged
    std::vector<uint8_t> host;
    size_t add(const void *src, size_t bytes)
    {
        const size_t off = (host.size() + 63) & ~size_t(63);
        host.resize(off + bytes);
        std::memcpy(host.data() + off, src, bytes);
        return off;
    }
};

struct LaunchRec {
    const char *name;
    uint32_t blocks;
    size_t off_args, off_map;
    uint32_t n;
    std::vector<Work> works;
    std::function<void(const void *, BatchMap, unsigned)> go;
};

// Stage one batched kernel: per-state arguments and block counts (states with no blocks are
// kept in the map with an empty range).
template <class A, class K>
void stage(ArgArena &ar, std::vector<LaunchRec> &recs, const char *name, const std::vector<A> &args,
           const std::vector<uint32_t> &blocks, std::vector<Work> works, K kernel)
{
    std::vector<uint32_t> off(blocks.size() + 1, 0);
    for (size_t i = 0; i < blocks.size(); ++i) off[i + 1] = off[i] + blocks[i];
    if (off.back() == 0) return;
    static_assert(sizeof(A) <= 2048, "kernel arguments by value must stay well inside the 4 KB limit");
    if (ar.now) {  // one state: launch now with the arguments by value, while the host stages the next
        const A one = args[0];
        launch(ar.now, name, works, [&] { kernel(one, off.back()); });
        return;
    }
    LaunchRec r;
    r.name = name;
    r.blocks = off.back();
    r.off_args = ar.add(args.data(), args.size() * sizeof(A));
    r.off_map = ar.add(off.data(), off.size() * sizeof(uint32_t));
    r.n = (uint32_t)blocks.size();
    r.works = std::move(works);
    r.go = [kernel](const void *a, BatchMap bm, unsigned g) { kernel(static_cast<const A *>(a), g, bm); };
    recs.push_back(std::move(r));
}

// A batch of states: the argument tables and block maps in one copy to the device, then the
// launches in order.
ccmc_status launch_tables(ccmc_state *st, const ArgArena &ar, std::vector<LaunchRec> &recs, hipStream_t s)
{
    TRY(ensure(st, st->arg_dev, ar.host.size()));
    if (st->arg_hcap < ar.host.size()) {
        if (st->arg_host) (void)hipHostFree(st->arg_host);
        st->arg_host = nullptr;
        const size_t cap = ar.host.size() + ar.host.size() / 2 + 4096;
        if (hipHostMalloc((void **)&st->arg_host, cap) != hipSuccess) {
            st->arg_hcap = 0;
            st->err = "hipHostMalloc failed";
            return CCMC_EDEVICE;
        }
        st->arg_hcap = cap;
    }
    std::memcpy(st->arg_host, ar.host.data(), ar.host.size());
    HIP_TRY(hipMemcpyAsync(st->arg_dev.p, st->arg_host, ar.host.size(), hipMemcpyHostToDevice, s));
    const uint8_t *dev = static_cast<const uint8_t *>(st->arg_dev.p);
    for (auto &r : recs) {
        const BatchMap bm{reinterpret_cast<const uint32_t *>(dev + r.off_map), r.n};
        launch(st, r.name, r.works, [&] { r.go(dev + r.off_args, bm, r.blocks); });
    }
    return CCMC_OK;
}

// Pinned, coherent host memory for the step scalars of n states, which k_final_part writes.
ccmc_status host_scalars(ccmc_state *lead, size_t n)
{
    if (lead->batch_hcap >= n) return CCMC_OK;
    if (lead->no_grow) {
        lead->err = "ccmc_step_noalloc: no pinned memory for the step scalars";
        return CCMC_ENOMEM;
    }
    if (lead->batch_hscr) (void)hipHostFree(lead->batch_hscr);
    lead->batch_hscr = lead->batch_hdev = nullptr;
    lead->batch_hcap = 0;
    if (hipHostMalloc((void **)&lead->batch_hscr, n * sizeof(Scratch), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void **)&lead->batch_hdev, lead->batch_hscr, 0) != hipSuccess) {
        lead->err = "hipHostMalloc failed";
        return CCMC_EDEVICE;
    }
    std::memset(lead->batch_hscr, 0, n * sizeof(Scratch));
    lead->batch_hcap = n;
    return CCMC_OK;
}

// One attempt at a step of every state in `ps` (same words and precision), in shared
// launches.  Sizes produced on the device (record slots, records, new determinants,
// survivors) are never read back in the middle: kernels read them from device memory, and
// grids cover capacities planned from each state's previous step.  If a count exceeds its
// capacity, the overflow bit turns that state's final compaction into a no-op; the host
// then grows its buffers and replays its step with the same Philox counters (replay[i]).
// A batch whose launches are queued and whose scalars are still to be collected.
template <int W, typename T>
struct Launched {
    std::vector<Plan<W, T>> ps;
    std::vector<Plan<W, T> *> src;
    ccmc_state *lead = nullptr;
    uint64_t seq = 0;
};

template <int W, typename T>
ccmc_status batch_launch(std::vector<Plan<W, T> *> &all, Launched<W, T> &L)
{
    // plan every state; a state that cannot be planned (no memory, too many slots) drops out
    // of the batch unchanged
    std::vector<Plan<W, T>> ps;
    std::vector<Plan<W, T> *> src;
    for (Plan<W, T> *q : all) {
        q->replay = false;
        q->rc = plan_sizes<W, T>(*q);
        if (q->rc == CCMC_OK) {
            ps.push_back(*q);
            src.push_back(q);
        }
    }
    if (ps.empty()) return CCMC_OK;
    const size_t n = ps.size();
    ccmc_state *lead = ps[0].st;
    ccmc_state *const st = lead;  // errors of the batch's HIP calls are reported on its first state
    hipStream_t s = lead->stream;
    int passes = 1;
    for (auto &p : ps) passes = std::max(passes, p.passes);
    for (size_t i = 0; i < n; ++i) {
        src[i]->rc = plan_area<W, T>(ps[i], passes);
        if (src[i]->rc != CCMC_OK) {  // no memory for its step area: nothing ran; the others go again
            for (size_t j = 0; j < n; ++j)
                if (j != i) src[j]->replay = true;
            return CCMC_OK;
        }
    }
    TRY(host_scalars(lead, n));
    Scratch *scr_copy = lead->batch_hdev;
    const uint64_t seq = ++lead->batch_seq;
    const double kb = (double)(W * 8);  // bytes of one bitstring
    const double tb = (double)sizeof(T);
    ArgArena ar;
    ar.now = n == 1 ? lead : nullptr;
    std::vector<LaunchRec> recs;
    std::vector<uint32_t> blk(n);
    auto works = [&](auto f) {
        std::vector<Work> w;
        for (auto &p : ps) w.push_back(f(p));
        return w;
    };

    // ---- clear the step areas (a single state's area was cleared at the end of its last step,
    // unless the area has been reallocated since)
    {
        std::vector<ClearArgs> args;
        for (size_t i = 0; i < n; ++i) {
            const bool clean = n == 1 && !ps[i].st->no_grow && ps[i].st->lb_clean_bytes >= ps[i].lb_words * sizeof(uint64_t);
            args.push_back(ClearArgs{ps[i].lb, ps[i].lb_words, ptr<double>(ps[i].st->delta), ps[i].ne});
            blk[i] = clean ? 0 : grid_for(ps[i].lb_words + ps[i].ne);
            ps[i].st->lb_clean_bytes = 0;
        }
        stage(ar, recs, "clear", args, blk, works([&](auto &p) { return Work{8.0, nullptr, p.lb_words + p.ne}; }),
              [s](const auto &a, unsigned g, auto... bm) { k_clear<<<g, kThreads, 0, s>>>(a, bm...); });
    }
    // ---- virtual processors (Sec. III): place every excitor, then partition the store by
    // processor with one stable radix pass (store order within each processor)
    {
        std::vector<PlaceArgs<W>> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            ccmc_state *st = p.st;
            args.push_back(PlaceArgs<W>{ptr<uint64_t>(st->skey[p.c]), st->scap, p.ne, st->step, st->opt.n_ranks,
                                        st->opt.move_shift, st->opt.hash_seed, ptr<uint64_t>(st->vkey[0]), p.sc});
            blk[i] = p.ranked ? grid_for(p.ne) : 0;
        }
        stage(ar, recs, "place", args, blk, works([&](auto &p) { return Work{kb + 8.0, nullptr, p.ranked ? p.ne : 0}; }),
              [s](const auto &a, unsigned g, auto... bm) { k_place<W><<<g, kThreads, 0, s>>>(a, bm...); });
    }
    {
        std::vector<RadixGhistArgs> args;
        uint64_t most = 0;
        for (auto &p : ps) most = std::max(most, p.ptiles);
        const bool fat = most >= kGhistFatFrom;
        const int nt = fat ? kGhistFat : kThreads;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            args.push_back(RadixGhistArgs{ptr<uint64_t>(p.st->vkey[0]), &p.sc->n_place, 1, 0,
                                          reinterpret_cast<uint32_t *>(p.lb + p.o_pghist)});
            blk[i] = p.ptiles ? (uint32_t)ghist_grid(p.ptiles * kSortTile, nt) : 0u;
        }
        stage(ar, recs, "place_ghist", args, blk, works([&](auto &p) { return Work{8.0, nullptr, p.ranked ? p.ne : 0}; }),
              [s, fat](const auto &a, unsigned g, auto... bm) {
                  if (fat)
                      k_radix_ghist<kGhistFat><<<g, kGhistFat, 0, s>>>(a, bm...);
                  else
                      k_radix_ghist<kThreads><<<g, kThreads, 0, s>>>(a, bm...);
              });
    }
    {
        std::vector<RadixOnesweepArgs<uint32_t>> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            ccmc_state *st = p.st;
            args.push_back(RadixOnesweepArgs<uint32_t>{ptr<uint64_t>(st->vkey[0]), nullptr, ptr<uint64_t>(st->vkey[1]),
                                             ptr<uint32_t>(st->perm), &p.sc->n_place, 0,
                                             reinterpret_cast<const uint32_t *>(p.lb + p.o_pghist), p.lb + p.o_pstat,
                                             p.lb + p.o_tick + kTkPlace});
            blk[i] = (uint32_t)p.ptiles;
        }
        stage(ar, recs, "place_sweep", args, blk, works([&](auto &p) { return Work{20.0, nullptr, p.ranked ? p.ne : 0}; }),
              [s](const auto &a, unsigned g, auto... bm) { k_radix_onesweep<uint32_t><<<g, kThreads, 0, s>>>(a, bm...); });
    }
    // ---- (a1) selection weights, formed inside the scan of their prefix; the draw guide
    {
        using A = ScanLbArgs<uint64_t, WeightSrc<T>, ArrayOut<uint64_t>>;
        std::vector<A> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            ccmc_state *st = p.st;
            const uint32_t *perm = p.ranked ? ptr<uint32_t>(st->perm) : nullptr;
            args.push_back(A{WeightSrc<T>{ptr<T>(st->samp[p.c]), p.sc, perm}, ArrayOut<uint64_t>{ptr<uint64_t>(st->P)}, p.ne, 1,
                             p.lb + p.o_weights, p.lb + p.o_tick + kTkWeights, &p.sc->qtot});
            blk[i] = (uint32_t)scan_tiles(p.ne);
        }
        // bytes: amplitude read, prefix written
        stage(ar, recs, "weights_scan", args, blk, works([&](auto &p) { return Work{tb + 8.0, nullptr, p.ne}; }),
              [s](const auto &a, unsigned g, auto... bm) {
                  k_scan_lb<uint64_t, WeightSrc<T>, ArrayOut<uint64_t>><<<g, kThreads, 0, s>>>(a, bm...);
              });
    }
    {
        std::vector<GuideArgs> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            ccmc_state *st = p.st;
            args.push_back(GuideArgs{ptr<uint64_t>(st->P), ptr<uint32_t>(st->guide), p.a.gcap, p.a.gsh, p.ne,
                                     p.ranked ? ptr<uint64_t>(st->vkey[1]) : nullptr,
                                     p.ranked ? ptr<uint32_t>(st->seg) : nullptr, p.a.n_ranks, st->samp[p.c].p,
                                     sizeof(T) == 8 ? 1 : 0, ptr<uint64_t>(st->skey[p.c]), st->scap, W,
                                     p.ranked ? ptr<uint32_t>(st->perm) : nullptr,
                                     DrawRecs{ptr<uint64_t>(st->drec), (uint32_t)(2 + W)}});
            blk[i] = p.n_sel && p.ne ? grid_for(p.ne) : 0;
        }
        // bytes: prefix, amplitude and bitstring read, the draw record written, and the guide's
        // buckets (one to two per excitor, four to eight beyond 2^20 excitors)
        stage(ar, recs, "guide", args, blk, works([&](auto &p) {
                  const double guide = p.ne ? 4.0 * (double)p.gentries / (double)p.ne : 0.0;
                  return Work{guide + 8.0 + tb + kb + 8.0 * (2 + W), nullptr, p.ne};
              }),
              [s](const auto &a, unsigned g, auto... bm) { k_guide<<<g, kThreads, 0, s>>>(a, bm...); });
    }
    // ---- (a2-a5, a9, a10) items: non-composite (FNC) then sampled clusters; then the rank table
    auto items_of = [&](Plan<W, T> &p) {
        ccmc_state *st = p.st;
        return Items<T>{ptr<uint64_t>(st->ikey), ptr<T>(st->iA), ptr<T>(st->ideath), ptr<uint32_t>(st->in),
                        ptr<uint64_t>(st->icnt), st->icap};
    };
    auto parts_of = [&](Plan<W, T> &p) {
        ccmc_state *st = p.st;
        return ItemPartials{ptr<double>(st->num_part), ptr<uint64_t>(st->att_part), ptr<uint64_t>(st->disc_part),
                            ptr<uint64_t>(st->max_part)};
    };
    auto gen_of = [&](Plan<W, T> &p) {
        ccmc_state *st = p.st;
        return GenStats{ptr<uint32_t>(st->gcount), ptr<uint32_t>(st->gspawn), ptr<uint32_t>(st->gdeath)};
    };
    {
        using A = ItemsArgs<W, T>;
        std::vector<A> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            ccmc_state *st = p.st;
            const uint64_t *srank = ptr<uint64_t>(st->srank[p.c]);
            const Fence rt{srank, p.ne, ptr<uint64_t>(st->fence), ptr<uint32_t>(st->rtab), p.rt_n, p.rsh};
            // with fs = 1 the fence is the store's ranks themselves
            args.push_back(A{st->sd, ptr<uint64_t>(st->skey[p.c]), ptr<T>(st->samp[p.c]), ptr<T>(st->sK[p.c]), st->scap,
                             p.ne, ptr<uint64_t>(st->P), ptr<uint64_t>(st->drec), ptr<uint32_t>(st->guide),
                             Ranks{p.ranked ? ptr<uint32_t>(st->perm) : nullptr, p.ranked ? ptr<uint32_t>(st->seg) : nullptr},
                             st->n0, p.a, items_of(p), p.nb_fnc,
                             p.n_fnc, p.nb_fnc + p.nb_sel, rt, parts_of(p), p.sc});
            blk[i] = p.nb_fnc + p.nb_sel + p.nb_rt;
        }
        // bytes: every item's slot count, and key, A, death and n of each live item
        stage(ar, recs, "items", args, blk, works([&](auto &p) {
                  return Work{8.0, nullptr, p.n_items, nullptr, kb + 2 * tb + 4.0, &p.st->cnt_live_items};
              }),
              [s](const auto &a, unsigned g, auto... bm) { k_items<W, T><<<g, kThreads, 0, s>>>(a, bm...); });
    }
    {
        using A = ScanLbArgs<uint64_t, CountSrc<uint64_t>, SlotOut>;
        std::vector<A> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            ccmc_state *st = p.st;
            args.push_back(A{CountSrc<uint64_t>{ptr<uint64_t>(st->icnt), p.n_items},
                             SlotOut{ptr<uint64_t>(st->ioff), ptr<uint64_t>(st->block_item), p.slot_cap}, p.n_items + 1, 0,
                             p.lb + p.o_off, p.lb + p.o_tick + kTkOff, &p.sc->n_slots});
            blk[i] = (uint32_t)scan_tiles(p.n_items + 1, SlotOut::kItems);
        }
        stage(ar, recs, "slot_scan", args, blk, works([&](auto &p) { return Work{16.0, nullptr, p.n_items + 1}; }),
              [s](const auto &a, unsigned g, auto... bm) { k_scan_lb<uint64_t, CountSrc<uint64_t>, SlotOut><<<g, kThreads, 0, s>>>(a, bm...); });
    }
    // ---- (a6-a8) records: death and spawning attempts, one lane per slot, compacted per block
    auto regions_of = [&](Plan<W, T> &p) {
        ccmc_state *st = p.st;
        return Records{nullptr, ptr<uint64_t>(st->rkey), st->ramp.p, ptr<uint64_t>(st->rid), st->rcap};
    };
    {
        using A = GenerateArgs<W, T>;
        std::vector<A> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            ccmc_state *st = p.st;
            args.push_back(A{st->sd, items_of(p), ptr<uint64_t>(st->ioff), ptr<uint64_t>(st->block_item), p.n_fnc,
                             p.n_items, p.slot_cap, p.a, regions_of(p), p.ids ? 1 : 0, gen_of(p), p.sc});
            blk[i] = (uint32_t)p.nblk_cap;
        }
        // bytes: the records written and each live item read once (key, A, death, n, offset);
        // work units: spawning attempts
        stage(ar, recs, "generate", args, blk, works([&](auto &p) {
                  return Work{kb + tb + (p.ids ? 8.0 : 0.0), &p.st->cnt_rec, 0, &p.st->cnt_att, kb + 2 * tb + 12.0,
                              &p.st->cnt_live_items};
              }),
              [s, ueg = ps[0].st->hs.kind == CCMC_UEG](const auto &a, unsigned g, auto... bm) {
                  if (ueg)
                      k_generate<W, T, kSystemUEG><<<g, kThreads, 0, s>>>(a, bm...);
                  else
                      k_generate<W, T, kSystemMol><<<g, kThreads, 0, s>>>(a, bm...);
              });
    }
    {
        using A = ScanLbArgs<uint32_t, CountSrc<uint32_t>, RegionOut>;
        std::vector<A> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            ccmc_state *st = p.st;
            args.push_back(A{CountSrc<uint32_t>{ptr<uint32_t>(st->gcount), p.nblk_cap},
                             RegionOut{ptr<uint32_t>(st->boff), ptr<uint32_t>(st->tile_region), st->dcap / kGatherTile + 2},
                             p.nblk_cap + 1, 0,
                             p.lb + p.o_boff, p.lb + p.o_tick + kTkBoff, &p.sc->n_rec});
            blk[i] = (uint32_t)scan_tiles(p.nblk_cap + 1);
        }
        stage(ar, recs, "region_scan", args, blk, works([&](auto &p) { return Work{8.0, nullptr, p.nblk_cap + 1}; }),
              [s](const auto &a, unsigned g, auto... bm) {
                  k_scan_lb<uint32_t, CountSrc<uint32_t>, RegionOut><<<g, kThreads, 0, s>>>(a, bm...);
              });
    }
    auto dense_of = [&](Plan<W, T> &p) {
        ccmc_state *st = p.st;
        return Records{ptr<uint64_t>(st->drank), ptr<uint64_t>(st->dkey), st->damp.p, ptr<uint64_t>(st->did), st->dcap};
    };
    {
        using A = GatherArgs<W, T>;
        std::vector<A> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            ccmc_state *st = p.st;
            args.push_back(A{st->sd, regions_of(p), ptr<uint32_t>(st->boff), ptr<uint32_t>(st->tile_region), p.nblk_cap,
                             p.rec_cap, dense_of(p), p.ids ? 1 : 0, p.packed ? 1 : 0, p.sc});
            blk[i] = grid_for(p.rec_cap, kGatherTile);
        }
        // bytes: each record's region key and amplitude read, its sort key, amplitude and
        // bitstring written (with spawn ids kept: also its id read and written)
        stage(ar, recs, "gather", args, blk, works([&](auto &p) {
                  return Work{2.0 * (kb + tb) + 8.0 + (p.ids ? 16.0 : 0.0), &p.st->cnt_rec, 0};
              }),
              [s](const auto &a, unsigned g, auto... bm) { k_gather<W, T><<<g, kThreads, 0, s>>>(a, bm...); });
    }
    // ---- (a11) stable LSD radix sort of (rank, amplitude): one histogram launch for all
    // passes, then one single-sweep launch per digit
    {
        std::vector<RadixGhistArgs> args;
        uint64_t most = 0;
        for (auto &p : ps) most = std::max(most, p.tiles);
        const bool fat = most >= kGhistFatFrom;
        const int nt = fat ? kGhistFat : kThreads;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            args.push_back(RadixGhistArgs{ptr<uint64_t>(p.st->drank), &p.sc->n_live, passes, p.packed ? 32 : 0,
                                          reinterpret_cast<uint32_t *>(p.lb + p.o_ghist)});
            blk[i] = p.tiles ? (uint32_t)ghist_grid(p.tiles * kSortTile, nt) : 0u;
        }
        stage(ar, recs, "radix_ghist", args, blk, works([&](auto &p) { return Work{8.0, &p.st->cnt_rec, 0}; }),
              [s, fat](const auto &a, unsigned g, auto... bm) {
                  if (fat)
                      k_radix_ghist<kGhistFat><<<g, kGhistFat, 0, s>>>(a, bm...);
                  else
                      k_radix_ghist<kThreads><<<g, kThreads, 0, s>>>(a, bm...);
              });
    }
    for (int pass = 0; pass < passes; ++pass) {
        std::vector<RadixOnesweepArgs<T>> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            ccmc_state *st = p.st;
            const int ob = pass & 1;
            const uint64_t *kin = pass == 0 ? ptr<uint64_t>(st->drank) : ptr<uint64_t>(st->sr[ob ^ 1]);
            const T *vin = pass == 0 ? ptr<T>(st->damp) : ptr<T>(st->sval[ob ^ 1]);
            args.push_back(RadixOnesweepArgs<T>{kin, vin, ptr<uint64_t>(st->sr[ob]), ptr<T>(st->sval[ob]), &p.sc->n_live,
                                             (p.packed ? 32 : 0) + kRadixBits * pass,
                                             reinterpret_cast<const uint32_t *>(p.lb + p.o_ghist) + kRadixBins * pass,
                                             p.lb + p.o_rstat + (uint64_t)pass * p.tiles * kRadixBins,
                                             p.lb + p.o_tick + kTkRadix + pass});
            blk[i] = (uint32_t)p.tiles;
        }
        // bytes: each (rank, amplitude) pair read and written
        stage(ar, recs, "radix_onesweep", args, blk, works([&](auto &p) { return Work{2.0 * (8.0 + tb), &p.st->cnt_rec, 0}; }),
              [s](const auto &a, unsigned g, auto... bm) { k_radix_onesweep<T><<<g, kThreads, 0, s>>>(a, bm...); });
    }
    const int sorted = (passes - 1) & 1;  // buffer of the last pass
    // ---- (a12) runs of equal determinants: fold in record order, store lookup by rank
    auto fold_of = [&](Plan<W, T> &p) {
        uint64_t *f = p.lb + p.o_fold;
        const uint64_t nt = p.fold_tiles;
        return FoldTiles{reinterpret_cast<double *>(f), reinterpret_cast<uint32_t *>(f + nt), f + 2 * nt, f + 3 * nt,
                         f + 4 * nt, reinterpret_cast<double *>(f + 5 * nt), f + 6 * nt, f + 7 * nt,
                         p.lb + p.o_tick + kTkFold};
    };
    {
        using A = SegFoldArgs<W, T>;
        std::vector<A> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            ccmc_state *st = p.st;
            const NewDets nd{ptr<uint64_t>(st->nkey), ptr<uint64_t>(st->nrank), ptr<uint64_t>(st->nins), ptr<double>(st->nsum),
                             st->dcap, ptr<uint64_t>(st->dkey), st->dcap};
            args.push_back(A{st->sd, ptr<uint64_t>(st->sr[sorted]), ptr<T>(st->sval[sorted]), p.packed ? 1 : 0, p.rec_cap,
                             ptr<uint64_t>(st->srank[p.c]), p.ne, ptr<double>(st->delta),
                             fence_stride(p.ne) > 1 ? ptr<uint64_t>(st->fence) : ptr<uint64_t>(st->srank[p.c]),
                             ptr<uint32_t>(st->rtab), p.rt_n, p.rsh, fold_of(p), nd, p.sc});
            blk[i] = (uint32_t)p.fold_tiles;
        }
        // bytes: each sorted (rank, amplitude) pair and (per head) the new-determinant entry
        stage(ar, recs, "seg_fold", args, blk, works([&](auto &p) { return Work{8.0 + tb, &p.st->cnt_rec, 0, nullptr, kb + 24.0, &p.st->cnt_new}; }),
              [s](const auto &a, unsigned g, auto... bm) { k_seg_fold<W, T><<<g, kThreads, 0, s>>>(a, bm...); });
    }
    {
        std::vector<SegCloseArgs> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            ccmc_state *st = p.st;
            args.push_back(SegCloseArgs{p.fold_tiles, ptr<uint64_t>(st->srank[p.c]), p.ne, ptr<double>(st->delta),
                                        ptr<double>(st->nsum), fold_of(p), p.sc});
            blk[i] = grid_for(p.fold_tiles);
        }
        stage(ar, recs, "seg_close", args, blk, works([&](auto &p) { return Work{48.0, nullptr, p.fold_tiles}; }),
              [s](const auto &a, unsigned g, auto... bm) { k_seg_close<<<g, kThreads, 0, s>>>(a, bm...); });
    }
    // ---- (a12, a13) merge, round and compact into the other store buffer
    const double eb = kb + 2 * tb + 8.0;  // one store entry: key, amplitude, diagonal, rank
    {
        using A = MergeArgs<W, T>;
        std::vector<A> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            ccmc_state *st = p.st;
            const int m = 1 - p.c;
            const StoreCols in{ptr<uint64_t>(st->skey[p.c]), st->samp[p.c].p, st->sK[p.c].p, ptr<uint64_t>(st->srank[p.c]),
                               st->scap};
            const StoreCols out{ptr<uint64_t>(st->skey[m]), st->samp[m].p, st->sK[m].p, ptr<uint64_t>(st->srank[m]), st->scap};
            args.push_back(A{st->sd, in, p.ne, ptr<double>(st->delta), ptr<uint64_t>(st->nkey), ptr<uint64_t>(st->nrank),
                             st->dcap, ptr<uint64_t>(st->nins), ptr<double>(st->nsum), out, p.a, p.lb + p.o_merge,
                             p.lb + p.o_tick + kTkMerge, ptr<double>(st->abs_part), p.sc});
            blk[i] = std::min(p.nb_abs, kMergeBlocks);
        }
        // bytes: each merged entry read (store entry and its sum, or a new determinant) and
        // each survivor written
        stage(ar, recs, "merge", args, blk, works([&](auto &p) { return Work{2.0 * eb + 8.0, &p.st->cnt_merged, 0}; }),
              [s](const auto &a, unsigned g, auto... bm) { k_merge<W, T><<<g, kThreads, 0, s>>>(a, bm...); });
    }
    // ---- (a14) the step's statistics in a fixed-order two-stage reduction
    {
        std::vector<FinalPartArgs> args;
        for (size_t i = 0; i < n; ++i) {
            auto &p = ps[i];
            args.push_back(FinalPartArgs{parts_of(p), p.n_parts, gen_of(p), p.nblk_cap, ptr<double>(p.st->abs_part), p.nb_abs,
                                         p.sc, p.ne, reinterpret_cast<FinalPart *>(p.lb + p.o_fin),
                                         p.lb + p.o_tick + kTkFinal, scr_copy + i, seq});
            blk[i] = (uint32_t)p.fin_blocks;
        }
        stage(ar, recs, "final", args, blk, works([&](auto &) { return Work{0.0, nullptr, 0}; }),
              [s](const auto &a, unsigned g, auto... bm) { k_final_part<<<g, kThreads, 0, s>>>(a, bm...); });
    }
    // ---- a single state clears its whole area and fold sums for the next step now, while the
    // host reads this step's scalars and plans the next one (the scalars went to host memory)
    if (n == 1 && !ps[0].st->no_grow) {
        ccmc_state *const one = ps[0].st;
        const uint64_t words = one->lb.bytes / sizeof(uint64_t);
        const std::vector<ClearArgs> args{ClearArgs{ps[0].lb, words, ptr<double>(one->delta), one->scap}};
        const std::vector<uint32_t> b1{(uint32_t)grid_for(words + one->scap)};
        stage(ar, recs, "clear", args, b1, std::vector<Work>{Work{8.0, nullptr, words + one->scap}},
              [s](const auto &a, unsigned g, auto... bm) { k_clear<<<g, kThreads, 0, s>>>(a, bm...); });
        one->lb_clean_bytes = words * sizeof(uint64_t);
    }

    // ---- a batch: the argument tables in one copy, then the launches (a single state has
    // launched each kernel as it was staged)
    if (n > 1) TRY(launch_tables(lead, ar, recs, s));
    L.ps = std::move(ps);
    L.src = std::move(src);
    L.lead = lead;
    L.seq = seq;
    return CCMC_OK;
}

// Collect a launched batch: wait for its scalars, then commit (or roll back) each state.
template <int W, typename T>
ccmc_status batch_finish(Launched<W, T> &L)
{
    if (L.ps.empty()) return CCMC_OK;
    auto &ps = L.ps;
    auto &src = L.src;
    const size_t n = ps.size();
    ccmc_state *lead = L.lead;
    ccmc_state *const st = lead;  // errors of the batch's HIP calls are reported on its first state
    hipStream_t s = lead->stream;
    const uint64_t seq = L.seq;

    // ---- (a14) the one synchronisation of the step: k_final_part writes each state's scalars into
    // pinned host memory and then the batch's sequence number; the host polls for it (and,
    // every few thousand polls, asks whether the stream has ended without writing it)
    for (size_t i = 0; i < n; ++i) {
        const volatile uint64_t *flag = &lead->batch_hscr[i].seq;
        for (uint32_t polls = 1; *flag != seq; ++polls) {
            if ((polls & 4095) == 0) {
                const hipError_t q = hipStreamQuery(s);
                if (q == hipErrorNotReady) continue;
                HIP_TRY(q);
                if (*flag != seq) {
                    lead->err = "the step's scalars did not reach the host";
                    return CCMC_EDEVICE;
                }
            }
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    for (size_t i = 0; i < n; ++i) {
        auto &p = ps[i];
        ccmc_state *st = p.st;
        const Scratch scr = lead->batch_hscr[i];
        st->last_q = scr.qtot;
        st->cnt_slots = scr.n_slots;
        st->cnt_rec = scr.n_live;
        st->cnt_merged = p.ne + scr.n_new;
        st->cnt_new = scr.n_new;
        st->cnt_att = scr.n_attempts;
        st->cnt_live_items = scr.n_slots - scr.n_attempts;
        // plan the next step's capacities from this one
        st->slot_hint = std::max(st->slot_hint, scr.n_slots + scr.n_slots / 4 + 4096);
        st->rec_hint = std::max(st->rec_hint, scr.n_rec + scr.n_rec / 4 + 4096);
        if (scr.err) {
            // the compaction did not run; clear the sums the fold may have left behind
            if (p.ne) k_fill<double><<<grid_for(p.ne), kThreads, 0, s>>>(ptr<double>(st->delta), p.ne, 0.0);
            HIP_TRY(hipStreamSynchronize(s));
            if (scr.err & kErrBlowup) {
                st->err = "population beyond the fixed-point range of the selection weights";
                src[i]->rc = CCMC_EBLOWUP;
            } else if (scr.err & kErrAttempts) {
                st->err = "more than 2^30-2 spawning attempts on one cluster";
                src[i]->rc = CCMC_EOVERFLOW;
            } else {
                src[i]->replay = true;  // a capacity was exceeded: grow and replay
            }
            continue;
        }
        const double n0_old = st->n0;
        const double n0_new = scr.hf_hit ? st->n0 + scr.hf_sum : st->n0;
        const double ntot_new = scr.n_total + std::fabs(n0_new);
        if (st->opt.blowup_factor > 0 && st->last_ntot > 0 && !(ntot_new <= st->opt.blowup_factor * st->last_ntot)) {
            // the growth bound: the merged store is left unused, so the state stays as it was
            if (p.ne) k_fill<double><<<grid_for(p.ne), kThreads, 0, s>>>(ptr<double>(st->delta), p.ne, 0.0);
            HIP_TRY(hipStreamSynchronize(s));
            char msg[160];
            std::snprintf(msg, sizeof msg, "blow-up: the step took N_tot from %.6g to %.6g, above %.6g times", st->last_ntot,
                          ntot_new, st->opt.blowup_factor);
            st->err = msg;
            st->last_rec_buf = -1;
            src[i]->rc = CCMC_EBLOWUP;
            continue;
        }
        st->n0 = n0_new;
        st->last_ntot = ntot_new;
        st->ne = scr.n_out;
        st->cur = 1 - p.c;  // the merged store was written into the other buffer
        st->step += 1;
        st->last_num = scr.num;
        st->last_den = n0_old;
        st->last_nrec = scr.n_live;
        st->last_rec_buf = p.ids ? 1 : -1;
        if (p.out) {
            ccmc_stats *out = p.out;
            *out = ccmc_stats{};
            out->step = st->step;
            out->n_selections = p.n_sel;
            out->n_discarded = scr.n_discarded;
            out->n_spawn_attempts = scr.n_attempts;
            out->n_spawns = scr.n_spawns;
            out->n_deaths = scr.n_deaths;
            out->n_excitors = st->ne;
            out->max_attempts_per_cluster = scr.max_n;
            out->n_total = ntot_new;
            out->n_ref = st->n0;
            out->eproj_num = scr.num;
            out->eproj_den = n0_old;
        }
    }
    if (lead->prof) resolve_profile(lead);
    return CCMC_OK;
}

template <int W, typename T>
ccmc_status step_batch_once(std::vector<Plan<W, T> *> &all)
{
    Launched<W, T> L;
    TRY(batch_launch<W, T>(all, L));
    return batch_finish<W, T>(L);
}

// Steps of several states (same words and precision) in shared launches, in two halves so
// that the groups of one ccmc_step_batch call (one per words and precision) are all queued
// before the host waits for any: launch() plans and queues the first attempt; complete()
// collects it, then steps again, alone, the states whose capacities overflowed (after
// growing).  A state whose step fails is left unchanged with its error text set; the others
// complete their step.  complete() returns the first failure's status.
struct GroupStep {
    virtual ~GroupStep() = default;
    virtual void launch() = 0;
    virtual ccmc_status complete() = 0;
};

template <int W, typename T>
struct GroupStepT final : GroupStep {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    std::vector<Plan<W, T>> ps;
    std::vector<Plan<W, T> *> live;
    Launched<W, T> L;
    ccmc_status launch_rc = CCMC_OK;

    GroupStepT(ccmc_state *const *sts, size_t n, const double *tau, const double *shift, const uint64_t *n_sel,
               ccmc_stats *const *outs)
        : ps(n)
    {
        for (size_t i = 0; i < n; ++i) {
            ps[i].st = sts[i];
            ps[i].tau = tau[i];
            ps[i].shift = shift[i];
            ps[i].n_sel = n_sel[i];
            ps[i].out = outs ? outs[i] : nullptr;
            live.push_back(&ps[i]);
        }
    }

    void launch() override { launch_rc = batch_launch<W, T>(live, L); }

    ccmc_status complete() override
    {
        ccmc_status rb = launch_rc == CCMC_OK ? batch_finish<W, T>(L) : launch_rc;
        for (int attempt = 1;; ++attempt) {
            if (rb != CCMC_OK) {  // a HIP failure of the shared launches: every state still in the batch fails
                for (auto *p : live) {
                    if (p->st != live[0]->st) p->st->err = live[0]->st->err;
                    p->rc = rb;
                }
                break;
            }
            std::vector<Plan<W, T> *> again;
            for (auto *p : live) {
                if (p->rc != CCMC_OK || !p->replay) continue;
                if (p->st->no_grow) {  // ccmc_step_noalloc cannot grow the buffers a replay needs
                    p->st->err = "ccmc_step_noalloc: a count of the step exceeded the buffers the state holds; step once "
                                 "with ccmc_step to grow them";
                    p->rc = CCMC_ENOMEM;
                    continue;
                }
                again.push_back(p);
            }
            live.swap(again);
            if (live.empty()) break;
            if (attempt == 8) {
                for (auto *p : live) {
                    p->st->err = "step capacity did not converge";
                    p->rc = CCMC_ENOMEM;
                }
                break;
            }
            rb = step_batch_once<W, T>(live);
        }
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        ccmc_status first = CCMC_OK;
        for (auto &p : ps) {
            if (p.out) {
                if (p.rc != CCMC_OK) *p.out = ccmc_stats{};
                p.out->ms = ms;
                p.out->status = p.rc;
            }
            if (p.rc != CCMC_OK && first == CCMC_OK) first = p.rc;
        }
        return first;
    }
};

template <int W, typename T>
ccmc_status step_impl(ccmc_state *const *sts, size_t n, const double *tau, const double *shift, const uint64_t *n_sel,
                      ccmc_stats *const *outs)
{
    GroupStepT<W, T> g(sts, n, tau, shift, n_sel, outs);
    g.launch();
    return g.complete();
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
    // a grown store keeps the old contents, so that a growth refused part way (the store's own
    // buffers grown, the arrays sized by it not) leaves the state as it was
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
    {
        double tot = std::fabs(n_ref);
        for (uint64_t i = 0; i < n; ++i) tot += std::fabs(amps[i]);
        st->last_ntot = tot;
    }
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
    static ccmc_status run(ccmc_state *const *sts, size_t n, const double *tau, const double *shift, const uint64_t *n_sel,
                           ccmc_stats *const *outs)
    {
        return step_impl<W, T>(sts, n, tau, shift, n_sel, outs);
    }
};
template <int W, typename T>
struct GroupF {
    static ccmc_status run(std::unique_ptr<GroupStep> *out, ccmc_state *const *sts, size_t n, const double *tau,
                           const double *shift, const uint64_t *n_sel, ccmc_stats *const *outs)
    {
        out->reset(new GroupStepT<W, T>(sts, n, tau, shift, n_sel, outs));
        return CCMC_OK;
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
    DevBuf *bufs[] = {&st->t_rankv, &st->t_pairs, &st->t_kpack, &st->t_grid, &st->t_nvec, &st->t_vq, &st->t_h, &st->t_eri, &st->t_fock, &st->t_vpair,
                      &st->t_binv, &st->t_bino, &st->skey[0], &st->skey[1], &st->samp[0], &st->samp[1], &st->sK[0],
                      &st->sK[1], &st->srank[0], &st->srank[1], &st->P, &st->drec, &st->guide, &st->delta, &st->fence, &st->rtab, &st->ikey,
                      &st->iA, &st->ideath, &st->in, &st->icnt, &st->ioff, &st->num_part, &st->att_part, &st->disc_part, &st->max_part, &st->abs_part,
                      &st->block_item, &st->gcount, &st->gspawn, &st->gdeath, &st->boff, &st->rkey, &st->ramp, &st->rid, &st->drank, &st->dkey, &st->damp, &st->did, &st->sr[0], &st->sr[1],
                      &st->sval[0], &st->sval[1], &st->tile_region,
                      &st->nkey, &st->nrank, &st->nins, &st->nsum, &st->lb, &st->arg_dev,
                      &st->vkey[0], &st->vkey[1], &st->perm, &st->seg};
    for (DevBuf *b : bufs) release(st, *b);
    for (auto &p : st->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : st->ev_pool) (void)hipEventDestroy(e);
    if (st->arg_host) (void)hipHostFree(st->arg_host);
    if (st->batch_hscr) (void)hipHostFree(st->batch_hscr);
    if (st->own_stream && st->stream) (void)hipStreamDestroy(st->stream);
    delete st;
}

}  // namespace

// =========================================================================== C ABI
namespace {
template <int W>
void codist_launch(const uint64_t *keys, uint64_t n, uint64_t T, uint32_t n_ranks, uint32_t move_shift, uint32_t seed,
                   uint16_t *pl, const uint64_t *cps, int ncp, unsigned long long *sums, hipStream_t s)
{
    const uint64_t m = n * T;
    if (m) k_codist_place<W><<<(unsigned)((m + kThreads - 1) / kThreads), kThreads, 0, s>>>(keys, n, T, n_ranks, move_shift, seed, pl);
    const dim3 g((unsigned)((n + kThreads - 1) / kThreads), (unsigned)((n + kCoRows - 1) / kCoRows));
    if (n) k_codist_pairs<<<g, kThreads, 0, s>>>(pl, n, cps, ncp, sums);
}
}  // namespace

extern "C" {


ccmc_status ccmc_codistribution(int n_words, const uint64_t *keys, uint64_t n, uint32_t n_ranks, uint32_t move_shift,
                                uint32_t hash_seed, const uint64_t *checkpoints, int n_checkpoints, uint64_t *sum_c,
                                uint64_t *sum_c2)
{
    g_init_error.clear();
    if (n_words < 1 || n_words > kMaxWords || n_checkpoints < 1 || n_checkpoints > 64 || n_ranks < 1 ||
        n_ranks > 65535 || !checkpoints || !sum_c || !sum_c2 || (n && !keys)) {
        g_init_error = "ccmc_codistribution: invalid argument";
        return CCMC_EINVAL;
    }
    for (int c = 1; c < n_checkpoints; ++c)
        if (checkpoints[c] < checkpoints[c - 1]) {
            g_init_error = "ccmc_codistribution: checkpoints must ascend";
            return CCMC_EINVAL;
        }
    const uint64_t T = checkpoints[n_checkpoints - 1];
    if (T > (1ull << 24) || (n && T > (1ull << 31) / n) || n > (1ull << 31)) {
        g_init_error = "ccmc_codistribution: more than 2^31 placements or 2^24 iterations";
        return CCMC_EINVAL;
    }
    hipStream_t s = nullptr;
    void *dk = nullptr, *dpl = nullptr, *dcp = nullptr, *dsum = nullptr;
    auto fail = [&](hipError_t e) {
        g_init_error = std::string("ccmc_codistribution: ") + hipGetErrorString(e);
        (void)hipFree(dk);
        (void)hipFree(dpl);
        (void)hipFree(dcp);
        (void)hipFree(dsum);
        return e == hipErrorOutOfMemory ? CCMC_ENOMEM : CCMC_EDEVICE;
    };
    hipError_t e;
    const size_t kbytes = (size_t)(n ? n : 1) * n_words * sizeof(uint64_t);
    if ((e = hipMalloc(&dk, kbytes)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&dpl, (size_t)(n * T ? n * T : 1) * sizeof(uint16_t))) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&dcp, n_checkpoints * sizeof(uint64_t))) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&dsum, 2 * n_checkpoints * sizeof(uint64_t))) != hipSuccess) return fail(e);
    if (n && (e = hipMemcpy(dk, keys, n * n_words * sizeof(uint64_t), hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
    if ((e = hipMemcpy(dcp, checkpoints, n_checkpoints * sizeof(uint64_t), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
    if ((e = hipMemset(dsum, 0, 2 * n_checkpoints * sizeof(uint64_t))) != hipSuccess) return fail(e);
    auto *K = static_cast<const uint64_t *>(dk);
    auto *PL = static_cast<uint16_t *>(dpl);
    auto *CP = static_cast<const uint64_t *>(dcp);
    auto *SU = static_cast<unsigned long long *>(dsum);
    switch (n_words) {
    case 1: codist_launch<1>(K, n, T, n_ranks, move_shift, hash_seed, PL, CP, n_checkpoints, SU, s); break;
    case 2: codist_launch<2>(K, n, T, n_ranks, move_shift, hash_seed, PL, CP, n_checkpoints, SU, s); break;
    case 3: codist_launch<3>(K, n, T, n_ranks, move_shift, hash_seed, PL, CP, n_checkpoints, SU, s); break;
    case 4: codist_launch<4>(K, n, T, n_ranks, move_shift, hash_seed, PL, CP, n_checkpoints, SU, s); break;
    case 5: codist_launch<5>(K, n, T, n_ranks, move_shift, hash_seed, PL, CP, n_checkpoints, SU, s); break;
    case 6: codist_launch<6>(K, n, T, n_ranks, move_shift, hash_seed, PL, CP, n_checkpoints, SU, s); break;
    case 7: codist_launch<7>(K, n, T, n_ranks, move_shift, hash_seed, PL, CP, n_checkpoints, SU, s); break;
    default: codist_launch<8>(K, n, T, n_ranks, move_shift, hash_seed, PL, CP, n_checkpoints, SU, s); break;
    }
    if ((e = hipGetLastError()) != hipSuccess) return fail(e);
    std::vector<uint64_t> h(2 * n_checkpoints);
    if ((e = hipMemcpy(h.data(), dsum, h.size() * sizeof(uint64_t), hipMemcpyDeviceToHost)) != hipSuccess) return fail(e);
    for (int c = 0; c < n_checkpoints; ++c) {
        sum_c[c] = h[2 * c];
        sum_c2[c] = h[2 * c + 1];
    }
    (void)hipFree(dk);
    (void)hipFree(dpl);
    (void)hipFree(dcp);
    (void)hipFree(dsum);
    return CCMC_OK;
}

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
    opt->n_ranks = 1;
    opt->move_shift = 5;
    opt->hash_seed = 0;
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
    if (!(opt->blowup_factor <= 0 || (opt->blowup_factor > 1 && std::isfinite(opt->blowup_factor)))) {
        g_init_error = "ccmc_init: blowup_factor must be <= 0 (off) or a finite factor above 1";
        return CCMC_EINVAL;
    }
    if (opt->n_ranks > kMaxRanks) {
        g_init_error = "ccmc_init: n_ranks above 512";
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
    {
        int dev = 0;
        if (hipStreamGetDevice(st->stream, &dev) != hipSuccess) {
            (void)hipGetLastError();
            if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        }
        st->device = dev;
        std::string e;
        if (noalloc_area(dev, &st->noalloc_area, e) != CCMC_OK) {
            g_init_error = e;
            destroy(st);
            return CCMC_EDEVICE;
        }
    }
    ccmc_status rc = host_scalars(st, 1);
    if (rc == CCMC_OK) rc = dispatch<SystemF>(st, st, ints);
    if (rc == CCMC_OK) rc = dispatch<StoreF>(st, st, (uint64_t)1024);
    if (rc != CCMC_OK) {
        g_init_error = st->err;
        destroy(st);
        return rc;
    }
    st->n0 = opt->init_pop;
    st->last_ntot = std::fabs(opt->init_pop);
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
    ccmc_state *const sts[1] = {st};
    ccmc_stats *const outs[1] = {out};
    return dispatch<StepF>(st, sts, (size_t)1, &tau, &shift, &n_attempts, outs);
}

ccmc_status ccmc_step_noalloc(ccmc_state *st, double tau, double shift, uint64_t n_attempts, ccmc_stats *out)
{
    if (!st) return CCMC_EINVAL;
    if (!st->noalloc_area || st->batch_hcap < 1) {
        st->err = "ccmc_step_noalloc: the state has no fixed step area";
        return CCMC_EDEVICE;
    }
    // every buffer growth of this call fails instead of allocating; profiling (which takes
    // events) is off for the call
    struct Restore {
        ccmc_state *s;
        bool prof;
        ~Restore()
        {
            s->no_grow = false;
            s->prof = prof;
        }
    } restore{st, st->prof};
    st->no_grow = true;
    st->prof = false;
    return ccmc_step(st, tau, shift, n_attempts, out);
}

ccmc_status ccmc_shift_update(ccmc_shift_control *ctl, double n_total, double tau)
{
    if (!ctl || ctl->period < 1 || ctl->period > 63 || !(tau > 0) || !std::isfinite(tau) || !(n_total > 0) ||
        !std::isfinite(n_total))
        return CCMC_EINVAL;
    const int ring = ctl->period + 1;
    if (!ctl->varying) {
        if (n_total < ctl->target) return CCMC_OK;
        ctl->varying = 1;
        ctl->since = 0;
        ctl->n_hist[0] = n_total;
        return CCMC_OK;
    }
    ctl->since += 1;
    ctl->n_hist[ctl->since % ring] = n_total;
    if (ctl->since % ctl->period == 0) {
        const double prev = ctl->n_hist[(ctl->since - ctl->period) % ring];
        ctl->shift -= ctl->damping / ((double)ctl->period * tau) * std::log(n_total / prev);
    }
    return CCMC_OK;
}

ccmc_status ccmc_run(ccmc_state *st, int n_steps, double tau, ccmc_shift_control *ctl, uint64_t *n_attempts,
                     ccmc_stats *out, int *n_done)
{
    if (!st) return CCMC_EINVAL;
    if (n_done) *n_done = 0;
    if (!ctl || !n_attempts || n_steps < 0 || ctl->period < 1 || ctl->period > 63) {
        st->err = "ccmc_run: need a control with period in [1, 63], n_attempts and n_steps >= 0";
        return CCMC_EINVAL;
    }
    for (int i = 0; i < n_steps; ++i) {
        ccmc_stats s{};
        const ccmc_status rc = ccmc_step(st, tau, ctl->shift, *n_attempts, &s);
        if (rc != CCMC_OK) return rc;
        if (out) out[i] = s;
        if (n_done) *n_done = i + 1;
        if (ccmc_shift_update(ctl, s.n_total, tau) != CCMC_OK) {
            st->err = "ccmc_run: the population vanished or is not finite";
            return CCMC_EINVAL;
        }
        const double next = std::floor(s.n_total + 0.5);
        if (!(next < 4294967296.0)) {
            st->err = "ccmc_run: the next step would need 2^32 or more selections";
            return CCMC_EOVERFLOW;
        }
        *n_attempts = (uint64_t)next;
    }
    return CCMC_OK;
}

ccmc_status ccmc_step_batch(ccmc_state *const *states, int n, const double *tau, const double *shift,
                            const uint64_t *n_attempts, ccmc_stats *out)
{
    if (n < 0 || (n > 0 && (!states || !tau || !shift || !n_attempts))) return CCMC_EINVAL;
    for (int i = 0; i < n; ++i) {
        ccmc_state *st = states[i];
        if (!st) return CCMC_EINVAL;
        st->err.clear();
        for (int j = 0; j < i; ++j)
            if (states[j] == st) {
                st->err = "ccmc_step_batch: a state appears twice";
                return CCMC_EINVAL;
            }
        if (!(tau[i] > 0) || !std::isfinite(tau[i]) || !std::isfinite(shift[i]) || n_attempts[i] > 0xFFFFFFFFull) {
            st->err = "ccmc_step_batch: need tau > 0, finite shift and n_attempts < 2^32";
            return CCMC_EINVAL;
        }
        if (st->ne + 1 > 0xFFFFFFFFull) {
            st->err = "ccmc_step_batch: store too large for 32-bit item indices";
            return CCMC_EOVERFLOW;
        }
    }
    // one batch per (words, precision, kind of system); each runs on the stream of its first state, after the
    // work already queued on the others' streams.  Every group is queued before the host
    // waits for any, so groups on different streams run on the device together.
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<char> done(n, 0);
    std::vector<std::unique_ptr<GroupStep>> groups;
    ccmc_status rc = CCMC_OK;
    for (int i = 0; i < n; ++i) {
        if (done[i]) continue;
        std::vector<ccmc_state *> g;
        std::vector<double> gt, gs;
        std::vector<uint64_t> ga;
        std::vector<ccmc_stats *> go;
        for (int j = i; j < n; ++j) {
            if (done[j] || states[j]->WP != states[i]->WP || states[j]->fp32 != states[i]->fp32 ||
                states[j]->hs.kind != states[i]->hs.kind)
                continue;
            done[j] = 1;
            g.push_back(states[j]);
            gt.push_back(tau[j]);
            gs.push_back(shift[j]);
            ga.push_back(n_attempts[j]);
            go.push_back(out ? out + j : nullptr);
        }
        bool waits = true;
        for (size_t k = 1; k < g.size() && waits; ++k) {
            if (g[k]->stream == g[0]->stream) continue;
            hipEvent_t ev;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                waits = false;
                break;
            }
            (void)hipEventRecord(ev, g[k]->stream);
            (void)hipStreamWaitEvent(g[0]->stream, ev, 0);
            (void)hipEventDestroy(ev);
        }
        std::unique_ptr<GroupStep> gp;
        const ccmc_status r =
            waits ? dispatch<GroupF>(g[0], &gp, g.data(), g.size(), gt.data(), gs.data(), ga.data(), go.data()) : CCMC_EDEVICE;
        if (r != CCMC_OK || !gp) {  // this group and the ones after it do not step; the queued ones finish
            rc = r != CCMC_OK ? r : CCMC_EINVAL;
            for (ccmc_state *x : g) x->err = "ccmc_step_batch: the group of this state could not be queued";
            break;
        }
        gp->launch();
        groups.push_back(std::move(gp));
    }
    for (auto &gp : groups) {
        const ccmc_status r = gp->complete();
        if (r != CCMC_OK && rc == CCMC_OK) rc = r;
    }
    if (out) {  // every state's statistics carry the wall time of the whole batch
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int i = 0; i < n; ++i) out[i].ms = ms;
    }
    return rc;
}

ccmc_status ccmc_energy(const ccmc_state *st, double *e_hf, double *eproj_num, double *eproj_den)
{
    if (!st) return CCMC_EINVAL;
    if (e_hf) *e_hf = st->hs.ehf + st->hs.e_core;
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

ccmc_status ccmc_set_budget(ccmc_state *st, uint64_t hbm_budget_bytes)
{
    if (!st) return CCMC_EINVAL;
    st->opt.hbm_budget_bytes = hbm_budget_bytes;
    return CCMC_OK;
}

}  // extern "C"
