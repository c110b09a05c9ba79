/*
 * ccmc.h -- C ABI of the MI355X (gfx950) coupled cluster Monte Carlo step library.
 *
 * The library runs the data-parallel hot path of coupled cluster Monte Carlo (CCMC) as
 * described by Spencer, Neufeld, Vigor, Franklin & Thom, "Large Scale Parallelization in
 * Stochastic Coupled Cluster", arXiv:1807.03749: one call of ccmc_step performs one time
 * step of eq. (CCMC) (Sec. II, eq. 3) -- cluster-size draw, excitor selection in
 * proportion to |t_i|, collapse with its fermionic sign, spawning (with full
 * non-composite and multi-spawn sampling, Sec. IV), death against the shift, and
 * annihilation into the device-resident sorted excitor store -- entirely in HIP kernels
 * on one GPU.
 *
 * Conventions shared by every entry point:
 *   - Determinants are bitstrings of W = ceil(M/64) 64-bit words; spin orbital p is bit
 *     (p & 63) of word (p >> 6); word 0 is least significant.  Keys order as W-word
 *     unsigned integers, most significant word first.  Spin orbital p = 2*spatial + sigma
 *     (sigma 0 = alpha, 1 = beta).  The Hartree-Fock reference occupies spin orbitals
 *     0 .. N-1.  Host key arrays are entry-major: keys[i*W + w].
 *   - Energies are relative to the Hartree-Fock energy E_HF; the shift S passed to
 *     ccmc_step is relative to E_HF as well.
 *   - Pointers in these signatures are HOST pointers, owned by the caller and only read
 *     or written during the call.  The state owns all device memory until ccmc_free.
 *   - Every call returns a ccmc_status; nothing throws across the ABI.  A failing call
 *     leaves the state as it was before the call, and ccmc_last_error(state) explains it.
 *   - One state is used by one host thread at a time.  Several states may share a HIP
 *     stream.  ccmc_step is asynchronous to the host except for the statistics copy.
 */
#ifndef CCMC_H
#define CCMC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ccmc_state ccmc_state;

typedef enum {
    CCMC_OK = 0,
    CCMC_EINVAL = -1,    /* invalid argument (bad size, unsorted keys, NaN, ...) */
    CCMC_ENOMEM = -2,    /* device memory or the HBM budget exhausted */
    CCMC_EOVERFLOW = -3, /* a count exceeded a field width (e.g. > 2^30-2 attempts on one
                            cluster, > 2^32-1 selections); the step was rolled back */
    CCMC_EDEVICE = -4,   /* HIP runtime error */
    CCMC_EBLOWUP = -5    /* population beyond the fixed-point range of the selection weights, or
                            (with ccmc_options.blowup_factor > 0) a step that multiplied N_tot by
                            more than that factor; the step was rolled back */
} ccmc_status;

enum { CCMC_UEG = 1, CCMC_MOLECULAR = 2 };
enum { CCMC_FP64 = 0, CCMC_FP32 = 1 };

/* The system (Sec. III.B uses the 3D uniform electron gas; Sec. III.B and IV use
 * molecules).  UEG: closed-shell N electrons in the plane waves with |n|^2 <= n2_max of a
 * cubic box of volume N (4 pi / 3) r_s^3; n_spin_orbitals is derived and ignored on input.
 * Molecular: n_spin_orbitals = 2 * n_spatial of the integrals. */
typedef struct {
    int kind;            /* CCMC_UEG or CCMC_MOLECULAR */
    int n_electrons;     /* even, closed shell */
    int n_spin_orbitals; /* molecular: 2 * n_spatial; UEG: output only */
    double rs;           /* UEG Wigner-Seitz radius (bohr) */
    int n2_max;          /* UEG kinetic cut-off |n|^2 <= n2_max */
} ccmc_system;

/* Molecular integrals (host, copied at init): h[n][n] symmetric one-electron integrals and
 * the chemists' two-electron integrals (pq|rs), either as the full table eri[n][n][n][n]
 * (8-fold symmetric) or as Cholesky vectors chol[n_chol][n][n] (each symmetric) with
 * (pq|rs) = sum_L chol[L][p][q] chol[L][r][s], which the library contracts on the device.
 * eri takes precedence when both are given; give at least one.  e_core is a constant (e.g.
 * nuclear repulsion) added to the reference energy that ccmc_energy reports; every other
 * energy is relative to E_HF.  Pass NULL for the UEG. */
typedef struct {
    int n_spatial;
    const double *h;
    const double *chol;
    int n_chol;
    const double *eri;
    double e_core;
} ccmc_integrals;

/* Sampling options.  Defaults (ccmc_options_default): FP64, original selection, k_min 1,
 * multi-spawn off, non-composite threshold 1, spawn cutoff 0.01, occupation threshold 1,
 * init_pop 10, p_single 0.1, seed 1234, no budget, default stream, no spawn ids, one
 * processor (n_ranks 1, move_shift 5, hash_seed 0), no growth bound (blowup_factor 0). */
typedef struct {
    int precision;                 /* CCMC_FP64 or CCMC_FP32 (amplitudes, spawns, integrals) */
    int full_noncomposite;         /* 1: full non-composite sampling (Sec. IV.B) */
    int min_spawn_attempts;        /* k_min >= 1: attempts per cluster are at least this */
    double multispawn_threshold;   /* A_thresh of Sec. IV.C for sampled clusters; <= 0: off */
    double noncomposite_threshold; /* A_thresh for the non-composite items; <= 0: off */
    double spawn_cutoff;           /* |spawn| below it is rounded to +-cutoff or 0, unbiased */
    double occupation_threshold;   /* |N_i| below it is rounded to +-threshold or 0, unbiased */
    double init_pop;               /* initial reference amplitude N_0 */
    double p_single;               /* molecular generator: probability of a single */
    uint64_t seed;                 /* Philox4x32-10 key */
    uint64_t hbm_budget_bytes;     /* 0: no limit; else device memory the state may hold */
    void *hip_stream;              /* hipStream_t to run on; NULL: the library's own stream */
    int keep_spawn_ids;            /* 1: keep the last step's spawn list for ccmc_export_spawns */
    /* Virtual processors (Sec. III, eq. 9), emulated on the one GPU.  With
     * n_ranks = N_p > 1 excitor D sits on processor p(D, i_tau) = hash(D xor o) mod N_p with
     * o = (hash(D) + i_tau) >> move_shift (hash: MurmurHash2 with hash_seed over the W words of
     * D as 8W little-endian bytes, o xored into word 0; i_tau the step index), and selection k
     * of a step is made by processor k mod N_p from its own excitors, with its selection
     * probability scaled by N_p^(1-s).  Non-composite items (full non-composite sampling),
     * spawning and annihilation are unchanged.  n_ranks 0 or 1: one processor; at most 512.
     * move_shift >= 64: excitors never move (eq. 8). */
    uint32_t n_ranks;
    uint32_t move_shift;
    uint32_t hash_seed;
    /* Blow-up detector (Sec. IV.A: runs below the shoulder population can blow up): a step
     * whose N_tot after the step exceeds blowup_factor times N_tot before it is rolled back
     * and fails with CCMC_EBLOWUP (state unchanged).  <= 0: off.  N_tot before the first step
     * is |init_pop|, after an import |N_0| + sum |N_i| of the imported store. */
    double blowup_factor;
} ccmc_options;

typedef struct {
    uint64_t step;                     /* step index after the step */
    uint64_t n_selections;             /* sampled cluster selections (n_attempts argument) */
    uint64_t n_discarded;              /* selections discarded (repeat, overlap, level) */
    uint64_t n_spawn_attempts;         /* excitation-generator calls, null ones included */
    uint64_t n_spawns;                 /* spawn records emitted (deaths excluded) */
    uint64_t n_deaths;                 /* death records emitted */
    uint64_t n_excitors;               /* excitors in the store after the step */
    uint64_t max_attempts_per_cluster;
    double n_total;                    /* |N_0| + sum |N_i| after the step (FP64) */
    double n_ref;                      /* N_0 after the step (FP64) */
    double eproj_num;                  /* sum over sampled clusters of <D_HF|H|D_c> s_D(c) A (FP64) */
    double eproj_den;                  /* N_0 before the step (FP64) */
    double ms;                         /* host wall time of the call that took the step, in ms
                                          (for ccmc_step_batch: of the whole batch) */
    int32_t status;                    /* this state's outcome: CCMC_OK, or the failure that left
                                          it unchanged (ccmc_step_batch reports each state's own);
                                          on failure the other fields are zero */
    int32_t reserved;
} ccmc_stats;

/* Per-kernel timing collected with HIP events on the state's stream (ccmc_profile). */
typedef struct {
    char name[40];
    uint64_t launches;
    double ms;        /* summed event time over the launches */
    double bytes;     /* algorithmic bytes moved by those launches (model in the design notes) */
    double items;     /* work units processed by those launches */
} ccmc_kernel_time;

/* Fill *opt with the defaults listed above. */
ccmc_status ccmc_options_default(ccmc_options *opt);

/* Create a state: builds the basis (UEG) or the two-electron table from the Cholesky
 * vectors (molecular) on the device, and starts from N_0 = init_pop on the reference with an
 * empty excitor store (Sec. II: the walk starts from unit-weight particles on the reference).
 * truncation l: 1 <= l <= 6 (2 = CCSD, 3 = CCSDT, 4 = CCSDTQ), l <= n_electrons; M <= 512.
 * On success *out owns device memory until ccmc_free.  Errors: EINVAL, ENOMEM, EDEVICE. */
ccmc_status ccmc_init(const ccmc_system *sys, const ccmc_integrals *ints, int truncation,
                      const ccmc_options *opt, ccmc_state **out);

/* One time step of eq. (CCMC) (Sec. II, eq. 3) with time step tau > 0 and shift S:
 *   - original selection: n_attempts cluster selections with p_size(s) = 2^-(s+1) over
 *     s in [0, l+2] (Sec. II and its footnote);
 *   - full non-composite (Sec. IV.B): the reference and every excitor are evolved
 *     explicitly, plus n_attempts composite selections with s in [2, l+2];
 *   - each cluster makes max(k_min, floor(|A| / A_thresh)) spawning attempts (Sec. IV.C);
 *   - annihilation sums every contribution to a determinant in record-id order and adds
 *     it to the store (or to N_0), then rounds small amplitudes and compacts.
 * n_attempts <= 2^32 - 1.  *out (may be NULL) receives the step statistics.
 * Errors: EINVAL, ENOMEM, EOVERFLOW, EBLOWUP, EDEVICE; on error the state is unchanged. */
ccmc_status ccmc_step(ccmc_state *st, double tau, double shift, uint64_t n_attempts,
                      ccmc_stats *out);

/* The same step as ccmc_step, for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): it calls no hipMalloc, hipFree,
 * hipHostMalloc or other allocating routine.  The step's zeroed area -- the step scalars,
 * scan tickets, look-back status words, radix histograms, fold tile summaries and the first
 * stage of the final reduction -- lives in a fixed device array of CCMC_NOALLOC_AREA_BYTES
 * (16 MiB) per GPU, which each GPU holds until the process ends; every other buffer is the
 * state's own, sized by earlier ccmc_step calls (or ccmc_import) and never grown here.
 * Results are those of ccmc_step (same kernels, same Philox counters).
 * Errors (state unchanged): CCMC_ENOMEM when the step needs a larger buffer than the state
 * holds -- planned from its earlier steps, or found on the device when a count exceeds the
 * planned capacity -- or a step area above the array's size (step once with ccmc_step to
 * reserve, then retry), and the other errors of ccmc_step.  The array is shared by every call on its GPU and keeps the last
 * call's contents (each call clears the part it uses): calls that overlap in time on one GPU,
 * e.g. from two host threads, race.  Profiling (ccmc_profile) is ignored by this call. */
#define CCMC_NOALLOC_AREA_BYTES (16u << 20)
ccmc_status ccmc_step_noalloc(ccmc_state *st, double tau, double shift, uint64_t n_attempts, ccmc_stats *out);

/* Population control of a run of steps (the log-growth shift update the paper's method is used
 * with; the paper cites it without a formula).  The shift stays fixed until N_tot first reaches
 * `target`; from then on, every `period` steps, S <- S - damping / (period tau) *
 * ln(N_tot(t) / N_tot(t - period)).  The struct carries the control's whole state, so runs can
 * be chained; set varying = 0 and shift to the starting shift for a fresh control.
 * 1 <= period <= 63. */
typedef struct {
    double target;
    double damping;
    int period;
    int varying;       /* in/out: 1 once N_tot has reached target */
    double shift;      /* in/out */
    int since;         /* in/out: steps since the shift started to vary */
    double n_hist[64]; /* in/out: N_tot of the last period + 1 steps since then, a ring */
} ccmc_shift_control;

/* The control's update after a step that ended with N_tot = n_total (host only, no device
 * call): starts the control at the first n_total >= target, and at every period-th step after
 * that moves the shift.  CCMC_EINVAL for a NULL control, a period outside [1, 63], tau <= 0
 * or a non-positive or non-finite n_total. */
ccmc_status ccmc_shift_update(ccmc_shift_control *ctl, double n_total, double tau);

/* n_steps consecutive steps of one state in a native loop (no return to the caller in between):
 * step i is ccmc_step(st, tau, ctl->shift, n, out + i) with n = *n_attempts for the first step
 * and floor(N_tot + 1/2) of the step before for the others (Sec. IV.B: as many selections as
 * the total amplitude), followed by ccmc_shift_update(ctl, N_tot, tau).  On return
 * *n_attempts is the selection count of the next step and *n_done the number of steps taken;
 * out (host, n_steps entries, may be NULL) receives each step's statistics.  Stops at the
 * first failing step and returns its status (that step leaves the state unchanged). */
ccmc_status ccmc_run(ccmc_state *st, int n_steps, double tau, ccmc_shift_control *ctl,
                     uint64_t *n_attempts, ccmc_stats *out, int *n_done);

/* Steps of n states in shared launches, for serving many solves at once: state i takes one
 * step exactly as ccmc_step(states[i], tau[i], shift[i], n_attempts[i], out + i) would alone
 * (each block of a launch works on one state's data with that state's Philox key), and
 * out[i] (out may be NULL) receives its statistics.  States with the same bitstring words
 * and precision share every launch; each such group runs on the stream of its first state
 * after the work already queued on the others' streams.  A state may appear once.
 * Errors: EINVAL for bad arguments (no state changes).  Otherwise each state succeeds or
 * fails on its own, with ccmc_step's errors: a failed state is unchanged and
 * ccmc_last_error(states[i]) is non-empty exactly for the failed states; the others complete
 * their step.  The first failure's status is returned. */
ccmc_status ccmc_step_batch(ccmc_state *const *states, int n, const double *tau, const double *shift,
                            const uint64_t *n_attempts, ccmc_stats *out);

/* Projected-energy estimator terms of the last step (Sec. II, eq. 7): E_proj is the ratio of
 * the means of eproj_num and eproj_den over the equilibrated steps.  e_hf receives the
 * Hartree-Fock energy (plus e_core for molecular systems).  Any output pointer may be NULL. */
ccmc_status ccmc_energy(const ccmc_state *st, double *e_hf, double *eproj_num, double *eproj_den);

/* Release the state and all its device memory.  NULL is ignored. */
void ccmc_free(ccmc_state *st);

/* Text of the last error on this state ("" if none); valid until the next call on it.
 * With st == NULL: the last error of a failed ccmc_init or ccmc_codistribution on this
 * thread. */
const char *ccmc_last_error(const ccmc_state *st);

/* Co-location statistics of the placement eq. 9 (Sec. III; the analysis of the
 * co-distribution figure).  keys: host array [n][n_words] of distinct determinants (word 0
 * least significant).  For iterations i_tau = 0 .. T-1 (T = the last checkpoint) every
 * excitor is placed on one of n_ranks processors (move_shift, hash_seed as in
 * ccmc_options); c_ij counts the iterations before a checkpoint T_c at which excitors i and
 * j share a processor.  For each checkpoint (host array, ascending, 1 to 64 of them) the
 * host outputs receive sum over pairs i < j of c_ij and of c_ij^2 (exact integers): the mean
 * co-location probability is sum_c / (T_c n (n-1) / 2).  Runs on the current device and
 * allocates n T 2-byte placements there (n T <= 2^31, T <= 2^24, 1 <= n_ranks <= 65535);
 * CCMC_EINVAL on bad arguments, CCMC_ENOMEM / CCMC_EDEVICE from HIP, with
 * ccmc_last_error(NULL) explaining. */
ccmc_status ccmc_codistribution(int n_words, const uint64_t *keys, uint64_t n, uint32_t n_ranks,
                                uint32_t move_shift, uint32_t hash_seed, const uint64_t *checkpoints,
                                int n_checkpoints, uint64_t *sum_c, uint64_t *sum_c2);

/* Number of excitors in the store; then ccmc_export copies the store (keys[n][W] in key
 * order and amplitudes as FP64), N_0 and the step index into host arrays of `capacity`
 * entries.  EINVAL if capacity is too small. */
ccmc_status ccmc_export_size(const ccmc_state *st, uint64_t *n);
ccmc_status ccmc_export(const ccmc_state *st, uint64_t *keys, double *amps, uint64_t capacity,
                        uint64_t *n, double *n_ref, uint64_t *step);

/* Replace the store: keys strictly ascending, each with N electrons, excitation level in
 * [1, l], no bits at or above M, amplitudes finite and non-zero; N_0 finite; the next step
 * uses Philox counters of step index `step`.  EINVAL on any violation, ENOMEM when the store
 * cannot grow to n entries within the budget (the state unchanged in both cases). */
ccmc_status ccmc_import(ccmc_state *st, const uint64_t *keys, const double *amps, uint64_t n,
                        double n_ref, uint64_t step);

/* With keep_spawn_ids set: the last step's spawn and death records (key, amplitude as FP64,
 * id) in id order, id = (class << 62) | (item << 30) | slot, class 0 for the non-composite
 * items of full non-composite sampling (item 0 = reference, item i+1 = store entry i) and 1
 * for sampled clusters (item = selection index); slot 0 is the death and slot m+1 attempt m.
 * EINVAL if keep_spawn_ids is off or capacity is too small. */
ccmc_status ccmc_spawns_size(const ccmc_state *st, uint64_t *n);
ccmc_status ccmc_export_spawns(const ccmc_state *st, uint64_t *keys, double *amps, uint64_t *ids,
                               uint64_t capacity, uint64_t *n);

/* Kernel timing with HIP events recorded on the state's stream around each timed launch.
 * kernels: NULL or "" turns timing off; "*" times every launch of the step; otherwise a
 * comma-separated list of the kernel names that ccmc_profile_read reports (e.g. "generate")
 * times those only, so that the rest of the step runs without events.  ccmc_profile_read
 * copies up to `capacity` accumulated entries and resets them. */
ccmc_status ccmc_profile(ccmc_state *st, const char *kernels);
ccmc_status ccmc_profile_read(ccmc_state *st, ccmc_kernel_time *out, int capacity, int *n);

/* Sizes of the state's system: electrons N, spin orbitals M (for the UEG derived from
 * n2_max at init) and bitstring words W = ceil(M/64).  Any output pointer may be NULL. */
ccmc_status ccmc_dims(const ccmc_state *st, int *n_electrons, int *n_spin_orbitals, int *n_words);

/* Device memory currently held by the state, in bytes. */
ccmc_status ccmc_memory(const ccmc_state *st, uint64_t *bytes);

/* Change the state's device-memory budget (hbm_budget_bytes; 0 = no limit).  A step that
 * failed with CCMC_ENOMEM left the state unchanged, so a caller with memory to spare can raise
 * the budget and step again.  A budget below ccmc_memory is accepted: it only stops further
 * growth.  CCMC_EINVAL for a NULL state. */
ccmc_status ccmc_set_budget(ccmc_state *st, uint64_t hbm_budget_bytes);

#ifdef __cplusplus
}
#endif
#endif
