"""Brute-force second quantisation on Python integers, used only to pin the oracle.

A determinant is a Python int whose bit p is the occupation of spin orbital p, standing
for c+_{d1} c+_{d2} ... c+_{dN} |0> with d1 < d2 < ... (Spencer et al., Sec. II).  The
textbook action c_p |n> = (-1)^{sum_{q<p} n_q} |n - e_p> defines every sign; nothing
here reuses the oracle's list-reordering or Slater-Condon code.
"""
from __future__ import annotations

import itertools
from collections import defaultdict


def popcount(x: int) -> int:
    return bin(x).count("1")


def annihilate(det: int, p: int):
    if not (det >> p) & 1:
        return None, 0
    return det ^ (1 << p), (-1) ** popcount(det & ((1 << p) - 1))


def create(det: int, p: int):
    if (det >> p) & 1:
        return None, 0
    return det | (1 << p), (-1) ** popcount(det & ((1 << p) - 1))


def apply_string(ops, det: int, coeff: float = 1.0):
    """Apply an operator string [(kind, p), ...] written left to right (rightmost acts
    first); kind 'c' = creator, 'a' = annihilator.  Returns (det, coeff) or (None, 0)."""
    for kind, p in reversed(ops):
        det, s = (create if kind == "c" else annihilate)(det, p)
        if det is None:
            return None, 0.0
        coeff *= s
    return det, coeff


def excitor_ops(det: int, hf: int):
    """c^{a1..aL}_{i1..iL} = c+_{a1} .. c+_{aL} c_{iL} .. c_{i1} for det relative to hf."""
    holes = sorted(p for p in range(hf.bit_length()) if (hf >> p) & 1 and not (det >> p) & 1)
    parts = sorted(p for p in range(det.bit_length()) if (det >> p) & 1 and not (hf >> p) & 1)
    return [("c", a) for a in parts] + [("a", i) for i in reversed(holes)]


def excitor_sign(det: int, hf: int) -> int:
    out, c = apply_string(excitor_ops(det, hf), hf)
    assert out == det
    return int(c)


def to_int(words) -> int:
    v = 0
    for w, x in enumerate(words):
        v |= int(x) << (64 * w)
    return v


def to_words(v: int, W: int):
    import numpy as np
    return np.array([(v >> (64 * w)) & 0xFFFFFFFFFFFFFFFF for w in range(W)], dtype=np.uint64)


def hamiltonian_apply(vec: dict, M: int, h1, u2, one_body_pairs=None, two_body_quads=None):
    """(H vec) with H = sum_pq h_pq c+_p c_q + 1/2 sum_pqrs <pq|rs> c+_p c+_q c_s c_r,
    integrals given as callables on spin orbitals.  The sums run over every index whose
    integral is non-zero (lists can be precomputed and passed in)."""
    if one_body_pairs is None:
        one_body_pairs = [(p, q, h1(p, q)) for p in range(M) for q in range(M) if h1(p, q) != 0.0]
    if two_body_quads is None:
        two_body_quads = [(p, q, r, s, u2(p, q, r, s)) for p, q, r, s in itertools.product(range(M), repeat=4)
                          if u2(p, q, r, s) != 0.0]
    out = defaultdict(float)
    for det, c in vec.items():
        if c == 0.0:
            continue
        for p, q, v in one_body_pairs:
            d, s = apply_string([("c", p), ("a", q)], det)
            if d is not None:
                out[d] += v * s * c
        for p, q, r, s_, v in two_body_quads:
            d, s = apply_string([("c", p), ("c", q), ("a", s_), ("a", r)], det)
            if d is not None:
                out[d] += 0.5 * v * s * c
    return dict(out)


def integral_lists(M: int, h1, u2):
    ob = [(p, q, h1(p, q)) for p in range(M) for q in range(M) if h1(p, q) != 0.0]
    tb = [(p, q, r, s, u2(p, q, r, s)) for p, q, r, s in itertools.product(range(M), repeat=4)
          if u2(p, q, r, s) != 0.0]
    return ob, tb


def cc_wavefunction(store: dict, n_ref: float, hf: int, max_order: int = 12) -> dict:
    """psi = t_HF exp(T / t_HF) |D_HF> with T = sum_i t_i c_i (Sec. II, eq. 2), expanded as
    the power series until it terminates."""
    psi = defaultdict(float)
    psi[hf] = n_ref
    term = {hf: n_ref}
    for k in range(1, max_order + 1):
        nxt = defaultdict(float)
        for det, c in term.items():
            for exc, t in store.items():
                d, s = apply_string(excitor_ops(exc, hf), det)
                if d is not None:
                    nxt[d] += s * c * t / n_ref / k
        term = {d: c for d, c in nxt.items() if c != 0.0}
        if not term:
            break
        for d, c in term.items():
            psi[d] += c
    return dict(psi)


def sz_determinants(M: int, n_el: int):
    """All determinants with n_el/2 alpha (even) and n_el/2 beta (odd) spin orbitals."""
    alpha = [p for p in range(M) if p % 2 == 0]
    beta = [p for p in range(M) if p % 2 == 1]
    out = []
    for A in itertools.combinations(alpha, n_el // 2):
        for B in itertools.combinations(beta, n_el // 2):
            v = 0
            for p in A + B:
                v |= 1 << p
            out.append(v)
    return sorted(out)
