"""Pins of the deterministic projective CCSD (oracle/ccsd.py) and, through it, of the
long-run CCMC energy of the oracle at the 14-electron / 38-spin-orbital UEG workload.

* Two electrons: CCSD is exact, so it must equal exact diagonalisation.
* Fourteen electrons: at the converged amplitudes, the residual <D_i|(H - E_HF - E_c)|Psi>
  recomputed by brute-force second quantisation (tests/sq.py: its own operator signs, its
  own Hamiltonian, exp(T) expanded term by term) vanishes, and so does the energy equation.
* The stored long-run oracle energy (tests/golden/ueg14_38_ccsd_longrun.txt, written by the
  committed script beside it from the oracle alone) agrees with the deterministic CCSD within
  two standard errors (eq. 3's stationary state is the CC solution).
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest
import sq

from oracle import binding as ob
from oracle import ccsd

HERE = os.path.dirname(os.path.abspath(__file__))


def test_doubles_space_size_is_the_printed_ccsd_space():
    """289 determinants: the reference and 288 momentum-conserving doubles."""
    S = ob.System.ueg(14, 2, 1.0)
    assert len(ccsd.doubles_space(S)) == 288


def test_two_electron_ccsd_equals_fci():
    S = ob.System.ueg(2, 2, 1.0)
    ec, t, it = ccsd.ccsd_doubles(S)
    # exact diagonalisation in the K = 0, S_z = 0 space (the reference and its doubles)
    hf = S.hf
    basis = [hf] + ccsd.doubles_space(S)
    H = np.array([[S.hamiltonian(a, b) for b in basis] for a in basis])
    w, v = np.linalg.eigh(H)
    k = int(np.argmax(np.abs(v[0, :]) > 0.3))
    e_fci = w[k] - S.ehf()
    assert ec < -1e-3
    assert ec == pytest.approx(e_fci, abs=1e-10)


def test_ccsd_residual_by_bruteforce_second_quantisation():
    S = ob.System.ueg(14, 2, 1.0)
    ec, t, it = ccsd.ccsd_doubles(S)
    hf = sq.to_int(S.hf)
    store = {sq.to_int(k): a for k, a in t.items()}
    psi = sq.cc_wavefunction(store, 1.0, hf, max_order=2)  # levels <= 4: all H reaches from a double
    ob_list, tb_list = sq.integral_lists(S.M, S.h1, S.u2)
    ehf = S.ehf()
    # the energy equation: E_c = <D_HF|H|Psi> - E_HF
    h_hf = sq.hamiltonian_apply({hf: 1.0}, S.M, None, None, ob_list, tb_list)
    assert sum(c * psi.get(d, 0.0) for d, c in h_hf.items()) - ehf == pytest.approx(ec, abs=1e-12)
    rng = np.random.default_rng(3)
    dets = sorted(store)
    for i in rng.choice(len(dets), 12, replace=False):
        d = dets[i]
        row = sq.hamiltonian_apply({d: 1.0}, S.M, None, None, ob_list, tb_list)  # H real symmetric
        r = sum(c * psi.get(x, 0.0) for x, c in row.items()) - (ehf + ec) * psi.get(d, 0.0)
        assert abs(r) < 1e-10, (d, r)


def _stored_long_run():
    path = os.path.join(HERE, "golden", "ueg14_38_ccsd_longrun.txt")
    rows, mean, sem, stored_ccsd = [], None, None, None
    with open(path) as f:
        for ln in f:
            if ln.startswith("# mean"):
                parts = ln.split()
                mean, sem = float(parts[2]), float(parts[4])
            elif ln.startswith("# deterministic_ccsd"):
                stored_ccsd = float(ln.split()[2])
            elif ln.strip() and not ln.startswith("#"):
                r, e, x = ln.split()
                rows.append((int(r), float(e), float(x)))
    return rows, mean, sem, stored_ccsd


def test_oracle_long_run_matches_deterministic_ccsd():
    rows, mean, sem, stored_ccsd = _stored_long_run()
    es = np.array([e for _, e, _ in rows])
    assert len(rows) >= 4 and mean == pytest.approx(es.mean(), abs=1e-9)
    assert sem == pytest.approx(es.std(ddof=1) / math.sqrt(len(es)), rel=1e-4)  # energies stored to 10 digits
    S = ob.System.ueg(14, 2, 1.0)
    ec, _, _ = ccsd.ccsd_doubles(S)
    assert stored_ccsd == pytest.approx(ec, abs=1e-11)  # the stored value is the solver's
    assert abs(mean - ec) <= 2 * sem, (mean, ec, sem)
