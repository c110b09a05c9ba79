"""Helpers for the GPU-vs-oracle parity tests: paired runs and element-wise comparison.

Tolerances (FP64 mode): keys, record ids and every count bit-exact; spawn amplitudes to
1e-12 relative; death amounts -tau (K - S) A to 1e-12 relative plus the rounding of
K = H_DD - E_HF itself, |d| eps_K / |K - S| (the GPU forms K from the holes and particles
with a few table terms, the oracle from the full Slater-Condon diagonal minus E_HF, which
cancels terms as large as the diagonal's; where K - S nearly cancels that dominates).  eps_K
is eight times the random-walk rounding of the oracle's sums: 2^-53 sqrt(n) (A + A_HF) with
n = N + N^2 terms and A, A_HF bounds on the sums of their magnitudes (N max|h_pp| +
N^2/2 max|<pq||pq>|, and the same sum over the reference); annihilated
amplitudes to 1e-12 of the magnitude of what was summed (|N_old| + sum of each record's
magnitude and error bound), which bounds a sum whatever its cancellation; the
projected-energy numerator to 1e-11 relative (a tree reduction against a serial one).
"""
from __future__ import annotations

import math
from collections import defaultdict

import numpy as np

from oracle import binding as orc
from paper_1807_03749_amd import ccmc, inputs


def make_pair(system: str, n_el: int, l: int, opts: dict, n2_max: int = 0, rs: float = 1.0, n_spatial: int = 0,
              n_chol: int = 0, mol_seed: int = inputs.INTEGRAL_SEED, mol_kw: dict | None = None):
    if system == "ueg":
        S = orc.System.ueg(n_el, n2_max, rs)
        g = ccmc.State("ueg", n_el, l, n2_max=n2_max, rs=rs, keep_spawn_ids=1, **opts)
    else:
        h, B = inputs.molecule_like(n_spatial=n_spatial, n_electrons=n_el, n_chol=n_chol, seed=mol_seed,
                                    **(mol_kw or {}))
        S = orc.System.molecular(n_el, h, B)
        g = ccmc.State("mol", n_el, l, h=h, chol=B, keep_spawn_ids=1, **opts)
    oopts = {k: v for k, v in opts.items() if k in orc.RunOptions.__dataclass_fields__}
    R = orc.Run(S, l, orc.RunOptions(**oopts))
    return S, R, g


def evolve_oracle(R: orc.Run, steps: int, tau: float, first_nsel: int):
    st = R.step(tau, 0.0, first_nsel)
    for _ in range(steps - 1):
        st = R.step(tau, 0.0, int(round(st["n_total"])))
    return st


_EPS_K = {}


def diagonal_rounding(S: orc.System) -> float:
    """eps_K of the module docstring, once per system."""
    if id(S) not in _EPS_K:
        N, M = S.n_el, S.M
        hmax = max(abs(S.h1(p, p)) for p in range(M))
        vmax = max(abs(S.u2(p, q, p, q) - S.u2(p, q, q, p)) for p in range(M) for q in range(M) if p != q)
        a_hf = sum(abs(S.h1(p, p)) for p in range(N)) + 0.5 * sum(
            abs(S.u2(p, q, p, q) - S.u2(p, q, q, p)) for p in range(N) for q in range(N) if p != q)
        a_max = N * hmax + 0.5 * N * N * vmax
        _EPS_K[id(S)] = 8.0 * 2.0 ** -53 * math.sqrt(N + N * N) * (a_max + a_hf)
    return _EPS_K[id(S)]


def key_tuple(k):
    return tuple(int(x) for x in k)


def compare_step(S: orc.System, R: orc.Run, g: ccmc.State, tau: float, shift: float, n_sel: int,
                 amp_rtol: float = 1e-12):
    """Import the oracle's state into the GPU, run one step on both, compare everything."""
    keys, amps, n0, step = R.export_state()
    g.ccmc_import(keys, amps, n0, step)
    before = {key_tuple(k): abs(a) for k, a in zip(keys, amps)}
    hf = key_tuple(S.hf)
    before[hf] = abs(n0)
    os_ = R.step(tau, shift, n_sel)
    gs = g.ccmc_step(tau, shift, n_sel)
    for f in ("step", "n_selections", "n_discarded", "n_spawn_attempts", "n_spawns", "n_deaths", "n_excitors",
              "max_attempts_per_cluster"):
        assert gs[f] == os_[f], (f, gs[f], os_[f])
    # spawn and death records, in id order
    ok_, oa, oi = R.records()
    gk, ga, gi = g.ccmc_export_spawns()
    assert np.array_equal(gi, oi), "record ids differ"
    assert np.array_equal(gk, ok_), "record keys differ"
    ehf = S.ehf()
    eps_k = diagonal_rounding(S)
    death = (oi & np.uint64((1 << 30) - 1)) == 0
    bound = amp_rtol * np.abs(oa)
    dk_max = 0.0  # the largest difference of K the death amounts imply
    for r in np.nonzero(death)[0]:
        K = S.hamiltonian(ok_[r], ok_[r]) - ehf
        bound[r] += abs(oa[r]) * eps_k / max(abs(K - shift), 1e-300)
        if oa[r] != 0.0:
            dk_max = max(dk_max, abs(ga[r] - oa[r]) * abs(K - shift) / abs(oa[r]))
    print(f"[parity] death records: implied |dK| up to {dk_max:.2e}, allowance eps_K {eps_k:.2e}", flush=True)
    bad = np.abs(ga - oa) > bound
    assert not bad.any(), (int(bad.sum()), float(np.max(np.abs(ga - oa) - bound)))
    assert np.all(np.abs(ga[~death] - oa[~death]) <= amp_rtol * np.abs(oa[~death]))
    # store after annihilation, rounding and compaction
    scale = defaultdict(float, before)
    for k, a, b in zip(ok_, oa, bound):
        scale[key_tuple(k)] += abs(a) + b / amp_rtol
    k2, a2, r2, st2 = R.export_state()
    gk2, ga2, gr2, gst2 = g.ccmc_export()
    assert st2 == gst2
    assert np.array_equal(gk2, k2), "store keys differ"
    tol = np.array([amp_rtol * max(scale[key_tuple(k)], abs(a)) for k, a in zip(k2, a2)])
    assert np.all(np.abs(ga2 - a2) <= tol), float(np.max(np.abs(ga2 - a2) - tol))
    assert abs(gr2 - r2) <= amp_rtol * max(scale[hf], abs(r2))
    assert abs(gs["n_ref"] - os_["n_ref"]) <= amp_rtol * max(scale[hf], abs(os_["n_ref"]))
    assert gs["eproj_den"] == os_["eproj_den"]
    assert abs(gs["eproj_num"] - os_["eproj_num"]) <= 1e-11 * max(abs(os_["eproj_num"]), 1e-300)
    assert abs(gs["n_total"] - os_["n_total"]) <= 1e-12 * os_["n_total"]
    return gs, os_
