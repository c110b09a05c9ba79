"""Deterministic projective CCSD for systems whose CCSD space holds no singles (the UEG).

TEST INFRASTRUCTURE ONLY: a pin of the long-run CCMC energy, imported by the tests and by
the script that writes the stored long-run values.  The product package never imports it.

CCMC samples the coupled cluster wavefunction Psi = t_HF exp(T / t_HF) |D_HF> (Sec. II,
eq. 2) and propagates it with eq. 3; a stationary state of eq. 3 satisfies, for every
excitor i within the truncation,

    <D_i| (H - E_HF - E_c) |Psi> = 0,    E_c = sum_j <D_HF|H|D_j> <D_j|Psi> / t_HF   (eq. 7),

the projected coupled cluster equations.  This module solves them without sampling, for a
CCSD space of doubles only (momentum conservation forbids UEG singles): with t_HF = 1,
exp(T)|D_HF> projected onto determinants of level <= 4 (all that H can connect to a double)
is 1 + T + T^2/2.  Each product c_i c_j |D_HF> is collapsed by the oracle's own operator
algebra (``System.collapse``: c_i c_j = sigma c_Q), every matrix element is the oracle's
Slater-Condon ``System.hamiltonian``, and the amplitude equations are iterated with the
diagonal preconditioner t_i <- t_i - R_i / (H_ii - E_HF - E_c) until the residual vanishes.
Plain loops over Python dictionaries, FP64.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import binding as ob


def doubles_space(S: ob.System):
    """Every double excitation of the reference of a closed-shell UEG that conserves total
    momentum and S_z, as W-word bitstrings (levels by the oracle's own classification)."""
    nv = S.nvec()
    N, M = S.n_el, S.M
    hf = S.hf
    out = []
    for i, j in itertools.combinations(range(N), 2):
        for a, b in itertools.combinations(range(N, M), 2):
            if (i & 1) + (j & 1) != (a & 1) + (b & 1):
                continue
            if np.any(nv[i >> 1] + nv[j >> 1] != nv[a >> 1] + nv[b >> 1]):
                continue
            d = hf.copy()
            for p in (i, j, a, b):
                d[p >> 6] ^= np.uint64(1) << np.uint64(p & 63)
            assert S.level(d) == 2
            out.append(d)
    return out


def _key(d) -> tuple:
    return tuple(int(x) for x in d)


def ccsd_doubles(S: ob.System, tol: float = 1e-12, max_iter: int = 500):
    """Solve the projected CCSD equations of a doubles-only space.

    Returns (E_c, amplitudes {key: t_i}, iterations).  E_c is relative to E_HF."""
    dbl = doubles_space(S)
    keys = [_key(d) for d in dbl]
    hf = S.hf
    ehf = S.ehf()
    sd = {k: S.excitor_sign(d) for k, d in zip(keys, dbl)}
    h0 = {k: S.hamiltonian(hf, d) for k, d in zip(keys, dbl)}           # <D_HF|H|D_i>
    kdiag = {k: S.hamiltonian(d, d) - ehf for k, d in zip(keys, dbl)}   # K_i = H_ii - E_HF
    # products c_i c_j |D_HF> = sigma c_Q |D_HF> (i < j): the level-4 part of T^2 / 2
    pairs = []
    for x, y in itertools.combinations(range(len(dbl)), 2):
        q, sigma = S.collapse([dbl[x], dbl[y]])
        if q is not None:
            pairs.append((x, y, _key(q), sigma))
    quads = {}
    for _, _, q, _ in pairs:
        if q not in quads:
            quads[q] = np.array(q, dtype=np.uint64)
    sq_ = {q: S.excitor_sign(d) for q, d in quads.items()}
    # <D_i|H|D_J> for J among the doubles and quadruples that H connects to D_i: bitstrings
    # differing in at most four spin orbitals (the only candidates for a non-zero element)
    qkeys = list(quads)
    darr = np.array(keys, dtype=np.uint64).reshape(len(keys), S.W)
    qarr = np.array(qkeys, dtype=np.uint64).reshape(len(qkeys), S.W)

    def near(x, arr):
        return np.nonzero(np.bitwise_count(arr ^ darr[x]).sum(axis=1) <= 4)[0]

    row_dd, h_dq = {}, {}
    for x, kx in enumerate(keys):
        for y in near(x, darr):
            if y != x:
                v = S.hamiltonian(dbl[x], dbl[y])
                if v != 0.0:
                    row_dd.setdefault(kx, []).append((keys[y], v))
        for y in near(x, qarr):
            v = S.hamiltonian(dbl[x], quads[qkeys[y]])
            if v != 0.0:
                h_dq.setdefault(kx, []).append((qkeys[y], v))

    t = {k: 0.0 for k in keys}
    ec = 0.0
    for it in range(1, max_iter + 1):
        # excitor amplitudes of exp(T)|D_HF> up to level 4, then determinant coefficients
        psi_q = {}
        for x, y, q, sigma in pairs:
            psi_q[q] = psi_q.get(q, 0.0) + sigma * t[keys[x]] * t[keys[y]]
        ec = sum(h0[k] * sd[k] * t[k] for k in keys)
        res = {}
        for k in keys:
            r = h0[k]  # <D_i|H|D_HF> * 1 (H is real symmetric)
            r += (kdiag[k] - ec) * sd[k] * t[k]
            for ky, v in row_dd.get(k, ()):
                r += v * sd[ky] * t[ky]
            for q, v in h_dq.get(k, ()):
                r += v * sq_[q] * psi_q.get(q, 0.0)
            res[k] = r
        rmax = max(abs(r) for r in res.values())
        if rmax < tol:
            return ec, t, it
        for k in keys:
            # R_i is the determinant-basis residual; t_i carries the sign s_D(i)
            t[k] -= sd[k] * res[k] / (kdiag[k] - ec)
    raise RuntimeError(f"CCSD did not converge in {max_iter} iterations (residual {rmax:.3e})")
