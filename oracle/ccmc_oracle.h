/*
 * ccmc_oracle.h -- plain, serial, FP64 CPU oracle for one coupled cluster Monte Carlo
 * (CCMC) time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU baseline
 * leg of the benchmark may load this library.  The product path never calls it.  It
 * shares no code, header, table or constant generator with the HIP library.
 *
 * What it follows (Spencer, Neufeld, Vigor, Franklin & Thom, "Large Scale
 * Parallelization in Stochastic Coupled Cluster", arXiv:1807.03749):
 *   - the rescaled ansatz  Psi = t_HF exp(T / t_HF) |D_HF>            (Sec. II, eq. 2)
 *   - the linearised propagator, eq. (CCMC)                              (Sec. II, eq. 3)
 *   - cluster size p_size(s) = 2^-(s+1), last size takes the remainder,
 *     excitors drawn with probability |t_i| / (N_tot - t_HF)            (Sec. II + footnote)
 *   - excitor / determinant operator strings and s_D                     (Sec. II, eqs. 4-6)
 *   - spawning sign -sgn(H_ij s_D(i) s_D(j)), death, annihilation,
 *     truncation discard                                                 (Sec. II)
 *   - projected energy                                                   (Sec. II, eq. 7)
 *   - full non-composite sampling                                        (Sec. IV.B)
 *   - multi-spawn: n_attempts = max(1, floor(A / A_thresh))              (Sec. IV.C, eqs. 10-11)
 *
 * Readings where the paper is silent (all listed in the design notes of the repository):
 * fixed-point selection weights, the Philox counter layout, the uniform excitation
 * generators, the spawn cutoff and occupation rounding, the record ids and the summation
 * order of annihilation.
 *
 * Bitstring layout: a determinant over M spin orbitals is W = ceil(M/64) words of 64 bits;
 * spin orbital p is bit (p & 63) of word (p >> 6); word 0 is least significant.  Keys
 * compare as W-word unsigned integers, most significant word first.  Spin orbital
 * p = 2*spatial + sigma (sigma 0 = alpha, 1 = beta).  The HF determinant occupies spin
 * orbitals 0 .. N-1.
 *
 * All functions return 0 on success and a negative code on error (see ORC_E*).
 */
#ifndef CCMC_ORACLE_H
#define CCMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXW 8
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EOVERFLOW (-3)

typedef struct orc_system orc_system;
typedef struct orc_run orc_run;

typedef struct {
    int full_noncomposite;          /* 0: original cluster selection; 1: full non-composite */
    int min_spawn_attempts;         /* k_min >= 1 */
    double multispawn_threshold;    /* A_thresh for sampled clusters; <= 0: n = k_min */
    double noncomposite_threshold;  /* A_thresh for non-composite items; <= 0: n = k_min */
    double spawn_cutoff;            /* spawns below this magnitude are stochastically rounded */
    double occupation_threshold;    /* excitor amplitudes below this are stochastically rounded */
    double init_pop;                /* initial reference amplitude N_0 */
    double p_single;                /* molecular generator: probability of a single */
    uint64_t seed;                  /* Philox key */
    /* Virtual processors (Sec. III, eq. 9): 0 or 1 = one processor.  With
     * n_ranks = N_p > 1 every excitor sits on processor p(D, i_tau) and each selection
     * builds its cluster from the excitors of one processor only. */
    uint32_t n_ranks;
    uint32_t move_shift;            /* nu_move: an excitor may move every 2^nu_move steps;
                                       >= 64 never (the static eq. 8) */
    uint32_t hash_seed;             /* MurmurHash2 seed of the placement */
} orc_options;

typedef struct {
    uint64_t step;                  /* step index after the step */
    uint64_t n_selections;
    uint64_t n_discarded;
    uint64_t n_spawn_attempts;
    uint64_t n_spawns;              /* spawn records emitted (deaths excluded) */
    uint64_t n_deaths;              /* death records emitted */
    uint64_t n_excitors;            /* store size after the step */
    uint64_t max_attempts_per_cluster;
    double n_total;                 /* |N_0| + sum |N_i| after the step */
    double n_ref;                   /* N_0 after the step */
    double eproj_num;               /* sum of <D_HF|H|D_c> s_D(c) A over sampled items */
    double eproj_den;               /* N_0 before the step */
} orc_stats;

/* ---- systems ---- */
/* Uniform electron gas: closed shell, n_el electrons, plane waves |n|^2 <= n2max, r_s. */
int orc_system_ueg(int n_el, int n2max, double rs, orc_system **out);
/* Molecule-like: h[n][n] (symmetric), chol[n_chol][n][n] (each symmetric), n_el electrons. */
int orc_system_mol(int n_el, int n_spatial, const double *h, const double *chol, int n_chol,
                   orc_system **out);
void orc_system_free(orc_system *);
int orc_system_dims(const orc_system *, int *n_el, int *n_spin_orbitals, int *n_words);
/* UEG only: integer wavevector of each spatial orbital, out[n_spatial][3]. */
int orc_ueg_nvec(const orc_system *, int *out);
double orc_ueg_box_length(const orc_system *);
/* Spin-orbital integrals <pq|rs> (physicists' notation) and h_pq. */
double orc_h1(const orc_system *, int p, int q);
double orc_u2(const orc_system *, int p, int q, int r, int s);
/* Slater-Condon matrix element <bra|H|ket>. */
double orc_hamiltonian(const orc_system *, const uint64_t *bra, const uint64_t *ket);
double orc_ehf(const orc_system *);
/* s_D(i) = <D_i| c_i |D_HF> for the excitor that creates det from D_HF. */
int orc_excitor_sign(const orc_system *, const uint64_t *det);
int orc_excitation_level(const orc_system *, const uint64_t *det);
/* Collapse of the product c_1 c_2 ... c_s (keys[s][W], draw order).  Returns 1 and
 * fills out / *sign when the product is non-zero, 0 when it vanishes. */
int orc_collapse(const orc_system *, int s, const uint64_t *keys, uint64_t *out, int *sign);

/* ---- runs ---- */
int orc_run_create(const orc_system *, int truncation, const orc_options *, orc_run **out);
void orc_run_free(orc_run *);
int orc_import(orc_run *, const uint64_t *keys, const double *amps, uint64_t n, double n_ref,
               uint64_t step);
int orc_export_size(const orc_run *, uint64_t *n);
int orc_export(const orc_run *, uint64_t *keys, double *amps, double *n_ref, uint64_t *step);
int orc_step(orc_run *, double tau, double shift, uint64_t n_sel, orc_stats *st);
/* Records (key, amplitude, id) emitted by the last step, in id order. */
int orc_records_size(const orc_run *, uint64_t *n);
int orc_records(const orc_run *, uint64_t *keys, double *amps, uint64_t *ids);

/* ---- placement of excitors on virtual processors (Sec. III) ---- */
/* MurmurHash2 (Austin Appleby, 32-bit, public domain) of len bytes. */
uint32_t orc_murmur2(const void *key, int len, uint32_t seed);
/* eq. 9: o = (hash(D) + i_tau) >> nu_move; p = hash(D xor o) mod N_p, hashing the
 * W words of D as 8W little-endian bytes (word 0 first) and xoring o into word 0. */
uint32_t orc_placement(int W, const uint64_t *det, uint64_t i_tau, uint32_t n_ranks, uint32_t move_shift,
                       uint32_t seed);
/* Co-location of n excitors (keys[n][W]) over iterations i_tau = 0 .. T-1: for each
 * checkpoint T_c (ascending, <= T), the sums over pairs i < j of c_ij and c_ij^2, where
 * c_ij counts the iterations before T_c with p(D_i) = p(D_j). */
int orc_codistribution(int W, const uint64_t *keys, uint64_t n, uint32_t n_ranks, uint32_t move_shift,
                       uint32_t seed, const uint64_t *checkpoints, int n_checkpoints, uint64_t *sum_c,
                       uint64_t *sum_c2);

/* ---- components, exposed so that tests can enumerate every random outcome ---- */
/* Fixed-point selection weight of a store amplitude. */
uint64_t orc_weight(double amp);
/* Cluster from explicit draws idx[s] (store positions, draw order) of the current store.
 * composite = 1 uses the full non-composite size distribution over [2, l+2].
 * Returns 1 with det/A/level/n filled, or 0 when the cluster is discarded. */
int orc_cluster(const orc_run *, int s, const uint64_t *idx, uint64_t n_sel, int composite,
                uint64_t *det, double *A, int *level, uint64_t *n_attempts);
/* The same cluster drawn on one of N_p processors: `count` selections were made on that
 * processor and its excitors' weights sum to qnorm; the selection probability carries the
 * factor N_p^(1-s) (the s excitors share the processor with probability N_p^(1-s), and each
 * processor makes 1/N_p of the selections: N_p^-s relative to one processor's own draws). */
int orc_cluster_ranked(const orc_run *, int s, const uint64_t *idx, uint64_t count, uint64_t qnorm,
                       uint32_t n_ranks, int composite, uint64_t *det, double *A, int *level,
                       uint64_t *n_attempts);
/* Attempt counts: cluster rule and non-composite rule. */
int orc_attempts(const orc_run *, double A, int noncomposite, uint64_t *n);
/* One spawning attempt from det with effective amplitude A and n attempts, given explicit
 * generator choices (UEG: {pair, a}; molecular: {type, first, a, b}).  Returns 1 with the
 * target and the unrounded spawn amplitude, or 0 for a null attempt (including a target
 * beyond the truncation level). */
int orc_attempt(const orc_run *, const uint64_t *det, double A, uint64_t n, const uint64_t *choice,
                double tau, uint64_t *target, double *x);
/* Death amount -tau (K_c - S) A for a cluster collapsing onto det. */
double orc_death(const orc_run *, const uint64_t *det, double A, double tau, double shift);

/* ---- Philox4x32-10 ---- */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

#ifdef __cplusplus
}
#endif
#endif
