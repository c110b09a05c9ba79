"""Seeded synthetic inputs shared by the HIP path's callers and the oracle's tests.

This module only draws numbers: it holds none of the CCMC arithmetic (no sampling, no
matrix elements, no annihilation).  Everything here is seeded and reproducible.

Molecule-like integrals follow the recipe of the molecule-like benchmark system
(16 electrons in 46 spatial orbitals, 138 Cholesky vectors): orbital energies drawn
uniformly in [-1.5, 2.0] Eh and sorted; one-electron off-diagonals ~ N(0, 0.05) damped by
exp(-|p-q|/8); Cholesky vectors B_Lpq ~ N(0, 0.1) damped by exp(-|p-q|/6) and
symmetrised, so that (pq|rs) = sum_L B_Lpq B_Lrs has 8-fold symmetry and a positive
semidefinite supermatrix.  The diagonal of h is chosen so that the closed-shell Fock
diagonal equals the drawn orbital energies, which makes the lowest determinant a sensible
reference.  The paper's own molecular integrals (water dimer, three waters, benzene) are
not available; these systems stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

INTEGRAL_SEED = 20180710
PHILOX_SEED = 1234


def molecule_like(n_spatial: int = 46, n_electrons: int = 16, n_chol: int = 138,
                  seed: int = INTEGRAL_SEED, eps_range=(-1.5, 2.0), h_sigma: float = 0.05,
                  h_decay: float = 8.0, b_sigma: float = 0.1, b_decay: float = 6.0):
    """Return (h[n][n], chol[n_chol][n][n]) in float64."""
    rng = np.random.default_rng(seed)
    n = n_spatial
    eps = np.sort(rng.uniform(eps_range[0], eps_range[1], size=n))
    dist = np.abs(np.subtract.outer(np.arange(n), np.arange(n))).astype(np.float64)
    h = rng.normal(0.0, h_sigma, size=(n, n)) * np.exp(-dist / h_decay)
    h = 0.5 * (h + h.T)
    B = rng.normal(0.0, b_sigma, size=(n_chol, n, n)) * np.exp(-dist / b_decay)[None]
    B = 0.5 * (B + B.transpose(0, 2, 1))
    occ = n_electrons // 2
    # closed-shell Fock diagonal f_pp = h_pp + sum_j^occ [2 (pp|jj) - (pj|jp)] set to eps_p
    diag_j = np.einsum("lpp,ljj->p", B, B[:, :occ, :occ])
    diag_k = np.einsum("lpj,ljp->p", B[:, :, :occ], B[:, :occ, :])
    np.fill_diagonal(h, eps - (2.0 * diag_j - diag_k))
    return np.ascontiguousarray(h), np.ascontiguousarray(B)


@dataclass
class Workload:
    """One benchmark / test workload (system, truncation and sampling options)."""
    name: str
    system: str                    # "ueg" or "mol"
    n_electrons: int
    truncation: int
    tau: float
    target_population: float
    n2_max: int = 0                # UEG
    rs: float = 1.0                # UEG
    n_spatial: int = 0             # molecular
    n_chol: int = 0                # molecular
    full_noncomposite: bool = False
    min_spawn_attempts: int = 1
    multispawn_threshold: float = 0.0
    noncomposite_threshold: float = 1.0
    precision: str = "fp64"
    steps: int = 1000
    seed: int = PHILOX_SEED
    extra: dict = field(default_factory=dict)

    @property
    def n_spin_orbitals(self) -> int:
        if self.system == "ueg":
            return {2: 38, 4: 66, 5: 114, 8: 186, 9: 246, 12: 358}[self.n2_max]
        return 2 * self.n_spatial


# The five workloads of the benchmark plan.  UEG sizes: 19, 57 and 123 plane waves for
# |n|^2 <= 2, 5 and 9.
WORKLOADS = {
    "ueg14_38_ccsd_fp64": Workload(
        name="ueg14_38_ccsd_fp64", system="ueg", n_electrons=14, n2_max=2, rs=1.0, truncation=2,
        tau=0.005, target_population=5e4, steps=1000,
        extra=dict(shift_from_growth=True, bench_steps=400, bench_warmup=100)),
    "ueg14_114_ccsdt_fnc": Workload(
        name="ueg14_114_ccsdt_fnc", system="ueg", n_electrons=14, n2_max=5, rs=1.0, truncation=3,
        tau=0.002, target_population=1e6, full_noncomposite=True, min_spawn_attempts=4,
        multispawn_threshold=1.0, noncomposite_threshold=1.0, steps=20000),
    "mol16_92_ccsdtq_fp32": Workload(
        name="mol16_92_ccsdtq_fp32", system="mol", n_electrons=16, n_spatial=46, n_chol=138,
        truncation=4, tau=5e-4, target_population=5e6, full_noncomposite=True, min_spawn_attempts=8,
        multispawn_threshold=1.0, noncomposite_threshold=1.0, precision="fp32", steps=2000,
        # below its shoulder at this target: grown at tau itself, the shift started from the
        # growth rate and held with a strong damping (see the benchmark's population control)
        extra=dict(grow_factor=1.0, shift_from_growth=True, control_damping=0.5, bench_steps=30, bench_warmup=10)),
    "ueg54_246_ccsd_fp32": Workload(
        name="ueg54_246_ccsd_fp32", system="ueg", n_electrons=54, n2_max=9, rs=1.0, truncation=2,
        tau=0.001, target_population=1e8, full_noncomposite=True, min_spawn_attempts=8,
        multispawn_threshold=1.0, noncomposite_threshold=1.0, precision="fp32", steps=200,
        extra=dict(bench_steps=10, bench_warmup=5)),
}


def serving_stream(n_requests: int = 64, rate: float = 2.0, seed: int = PHILOX_SEED):
    """Poisson arrival stream of UEG 14-electron solves for the serving benchmark:
    r_s in {0.5, 1, 2, 5}, M in {38, 66, 114}, CCSD or CCSDT, target population
    log-uniform in [1e4, 1e6]."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    out = []
    n2 = {38: 2, 66: 4, 114: 5}
    for r in range(n_requests):
        M = int(rng.choice([38, 66, 114]))
        trunc = int(rng.choice([2, 3]))
        out.append(dict(
            request_id=r, arrival=float(t[r]), rs=float(rng.choice([0.5, 1.0, 2.0, 5.0])),
            n2_max=n2[M], n_spin_orbitals=M, truncation=trunc,
            target_population=float(10 ** rng.uniform(4.0, 6.0)),
            tau=0.005 if trunc == 2 else 0.002,
            seed=int(rng.integers(1, 2**63 - 1))))
    return out


def state_amplitudes(levels, target: float, seed: int = PHILOX_SEED, decay: float = 2.0):
    """Seeded excitor amplitudes for a synthetic store: log-normal magnitudes whose median
    falls by exp(decay) per excitation level above 2, random signs, scaled so that
    sum |N_i| = target, and every |N_i| >= 1 (the default occupation threshold)."""
    rng = np.random.default_rng(seed)
    levels = np.asarray(levels)
    mag = np.exp(rng.normal(0.0, 1.0, size=len(levels)) - decay * np.maximum(levels - 2, 0))
    mag *= target / mag.sum()
    mag = np.maximum(mag, 1.0)
    sign = np.where(rng.random(len(levels)) < 0.5, -1.0, 1.0)
    return sign * mag


def ueg_ccsd_determinants(n_electrons: int = 14, n2_max: int = 8) -> np.ndarray:
    """The determinants of a closed-shell 3D UEG CCSD space as bitstrings [n][W]: the
    reference and every double excitation with total momentum and S_z conserved (momentum
    forbids singles).  Plane waves |n|^2 <= n2_max sorted by (|n|^2, n_x, n_y, n_z); spin
    orbital p = 2 * wave + spin; the reference fills spin orbitals 0 .. N-1; spin orbital p is
    bit p & 63 of word p >> 6.  For 14 electrons and n2_max = 8 (186 spin orbitals) these are
    the 3813 excitors of the co-distribution study (Sec. III.B).  The set is an input of that
    study, listed in key order."""
    r = int(np.floor(np.sqrt(n2_max)))
    waves = sorted((x * x + y * y + z * z, x, y, z) for x in range(-r, r + 1) for y in range(-r, r + 1)
                   for z in range(-r, r + 1) if x * x + y * y + z * z <= n2_max)
    k = np.array([w[1:] for w in waves], dtype=np.int64)
    M = 2 * len(waves)
    W = (M + 63) // 64
    occ = list(range(n_electrons))
    virt = list(range(n_electrons, M))
    index = {(tuple(k[p >> 1]), p & 1): p for p in range(M)}
    dets = [tuple(occ)]
    for ai, i in enumerate(occ):
        for j in occ[ai + 1:]:
            ktot = k[i >> 1] + k[j >> 1]
            stot = (i & 1) + (j & 1)
            for a in virt:
                sb = stot - (a & 1)
                if sb not in (0, 1):
                    continue
                b = index.get((tuple(ktot - k[a >> 1]), sb))
                if b is None or b <= a or b < n_electrons:
                    continue
                dets.append(tuple(sorted(set(occ) - {i, j} | {a, b})))
    out = np.zeros((len(dets), W), np.uint64)
    for n, d in enumerate(dets):
        for p in d:
            out[n, p >> 6] |= np.uint64(1 << (p & 63))
    order = sorted(range(len(dets)), key=lambda x: tuple(int(w) for w in out[x][::-1]))
    return out[order]
