"""FP32 amplitudes on the GPU: statistically the same energy as FP64.

In FP32 mode the amplitudes, spawns and integrals are single precision while the
projected-energy terms and the population sum stay FP64.  Rounding differences change the
fixed-point selection weights and the stochastic rounding decisions, so an FP32 run is a
different Markov chain from the FP64 one: the comparison is between reblocked energies,
|E_32 - E_64| <= 4 sqrt(s_32^2 + s_64^2).
"""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

from paper_1807_03749_amd import ccmc, driver

pytestmark = pytest.mark.gpu


def _run(precision: str, steps: int, equil: int, target: float, seed: int):
    st = ccmc.State("ueg", 14, 2, n2_max=2, rs=1.0, precision=precision, init_pop=500.0, seed=seed)
    ctl = driver.ShiftControl(target=target, tau=0.005)
    nsel = 500
    num, den = [], []
    for i in range(equil + steps):
        s = st.ccmc_step(0.005, ctl.shift, nsel)
        ctl.update(s["n_total"])
        nsel = driver.selections(s["n_total"])
        if i >= equil:
            num.append(s["eproj_num"])
            den.append(s["eproj_den"])
    st.close()
    return driver.reblock_ratio(np.array(num), np.array(den))


def test_fp32_energy_matches_fp64():
    e64, s64, _ = _run("fp64", 6000, 3000, 2e4, 1234)
    e32, s32, _ = _run("fp32", 6000, 3000, 2e4, 1234)
    print(f"[fp32] E64 {e64:.6f}+-{s64:.6f}  E32 {e32:.6f}+-{s32:.6f}", flush=True)
    sys.stdout.flush()
    assert s64 > 0 and s32 > 0
    assert abs(e32 - e64) <= 4.0 * math.sqrt(s32 ** 2 + s64 ** 2)
    # a correlation energy of the right sign and size for 14 electrons at r_s = 1
    assert -1.0 < e64 < 0.0


def test_fp32_state_roundtrip_and_stats():
    """An FP32 state imports and exports through FP64 host arrays and keeps FP64 statistics."""
    st = ccmc.State("ueg", 14, 2, n2_max=2, precision="fp32", init_pop=200.0, seed=9)
    for _ in range(30):
        s = st.ccmc_step(0.005, 0.0, driver.selections(200.0))
    k, a, n0, step = st.ccmc_export()
    assert step == 30 and len(k) == s["n_excitors"]
    assert np.all(np.abs(a) > 0) and np.all(a.astype(np.float32).astype(np.float64) == a)
    assert abs(np.abs(a).sum() + abs(n0) - s["n_total"]) <= 1e-9 * s["n_total"]
    st.close()
