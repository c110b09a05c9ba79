"""Virtual processors on the GPU (Sec. III, eq. 9) against the CPU oracle.

Ranked steps compare exactly like the one-processor parity cases (records, ids and keys
bit-exact, amplitudes to 1e-12; see parity_util), at step indices where excitors move.  The
co-location sums of ccmc_codistribution are integers and compare exactly: against the
oracle's pair loop on small sets, and at full size (the 3813 excitors of 14e/186so) against
sums formed from the oracle's placements by counting.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import binding as orc
from paper_1807_03749_amd import ccmc, inputs
from parity_util import compare_step, evolve_oracle, make_pair

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    # name, system kwargs, truncation, options, tau, init steps, init selections
    ("ueg14_66_ccsdt_fnc_np24", dict(system="ueg", n_el=14, n2_max=4), 3,
     dict(full_noncomposite=True, init_pop=500.0, seed=21, n_ranks=24, move_shift=2, hash_seed=3), 0.002, 30, 500),
    ("ueg14_66_ccsdt_fnc_np240", dict(system="ueg", n_el=14, n2_max=4), 3,
     dict(full_noncomposite=True, init_pop=800.0, seed=22, n_ranks=240, move_shift=5), 0.002, 30, 800),
    ("ueg14_38_ccsd_original_np7", dict(system="ueg", n_el=14, n2_max=2), 2,
     dict(init_pop=400.0, seed=23, n_ranks=7, move_shift=1, hash_seed=99), 0.005, 30, 400),
    ("ueg14_114_ccsdt_fnc_ms4_np16", dict(system="ueg", n_el=14, n2_max=5), 3,
     dict(full_noncomposite=True, min_spawn_attempts=4, multispawn_threshold=1.0, init_pop=500.0, seed=24,
          n_ranks=16, move_shift=64), 0.002, 30, 500),
    ("mol4_12_ccsd_original_np3", dict(system="mol", n_el=4, n_spatial=6, n_chol=8, mol_seed=4), 2,
     dict(init_pop=300.0, p_single=0.3, seed=25, n_ranks=3, move_shift=0), 0.01, 30, 300),
]


@pytest.mark.parametrize("name,sysk,l,opts,tau,nsteps,nsel0", CASES, ids=[c[0] for c in CASES])
def test_ranked_step_matches_oracle(name, sysk, l, opts, tau, nsteps, nsel0):
    _say(f"[ranks] {name}: building")
    S, R, g = make_pair(l=l, opts=opts, **sysk)
    st = evolve_oracle(R, nsteps, tau, nsel0)
    _say(f"[ranks] {name}: state with {st['n_excitors']} excitors, N_tot {st['n_total']:.1f}")
    for rep in range(3):
        gs, os_ = compare_step(S, R, g, tau, [0.0, -0.05, 0.02][rep], int(round(st["n_total"])))
        st = os_
        _say(f"[ranks] {name}: step {rep} ok ({gs['n_discarded']} of {gs['n_selections']} selections discarded)")
    g.close()


def test_ranked_trajectory_matches_oracle():
    """Twelve consecutive steps with excitors moving every other step, each side from its own
    previous result."""
    S, R, g = make_pair("ueg", 14, 3, dict(full_noncomposite=True, init_pop=300.0, seed=31, n_ranks=5, move_shift=1),
                        n2_max=2)
    st = evolve_oracle(R, 10, 0.004, 300)
    keys, amps, n0, step = R.export_state()
    g.ccmc_import(keys, amps, n0, step)
    for t in range(12):
        nsel = int(round(st["n_total"]))
        st = R.step(0.004, -0.01 * t, nsel)
        gs = g.ccmc_step(0.004, -0.01 * t, nsel)
        for f in ("n_spawns", "n_deaths", "n_excitors", "n_spawn_attempts", "n_discarded"):
            assert gs[f] == st[f], (t, f)
        k2, a2, r2, _ = R.export_state()
        gk, ga, gr, _ = g.ccmc_export()
        assert np.array_equal(gk, k2)
        np.testing.assert_allclose(ga, a2, rtol=1e-11, atol=1e-12)
    g.close()
    _say("[ranks] trajectory ok")


def test_most_processors_empty_and_limits():
    """512 processors for a few dozen excitors: most selections find an empty processor and
    are discarded, identically on both sides; 513 processors are refused."""
    S, R, g = make_pair("ueg", 14, 2, dict(init_pop=60.0, seed=41, n_ranks=512, move_shift=3), n2_max=2)
    st = evolve_oracle(R, 8, 0.005, 60)
    gs, os_ = compare_step(S, R, g, 0.005, 0.0, int(round(st["n_total"])))
    assert gs["n_discarded"] > 0
    g.close()
    with pytest.raises(ccmc.CCMCError):
        ccmc.State("ueg", 14, 2, n2_max=2, n_ranks=513)
    _say("[ranks] limits ok")


def test_one_processor_options_change_nothing():
    """n_ranks = 1 ignores move_shift and hash_seed: the same step as the default options."""
    S, R, g1 = make_pair("ueg", 14, 2, dict(init_pop=200.0, seed=5), n2_max=2)
    st = evolve_oracle(R, 10, 0.005, 200)
    keys, amps, n0, step = R.export_state()
    g2 = ccmc.State("ueg", 14, 2, n2_max=2, init_pop=200.0, seed=5, keep_spawn_ids=1, n_ranks=1, move_shift=0,
                    hash_seed=77)
    for g in (g1, g2):
        g.ccmc_import(keys, amps, n0, step)
        g.ccmc_step(0.005, 0.0, int(round(st["n_total"])))
    a, b = g1.ccmc_export(), g2.ccmc_export()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    g1.close()
    g2.close()


@pytest.mark.parametrize("np_,nu,seed", [(2, 1, 0), (7, 3, 5), (32, 4, 9), (5, 64, 1)])
def test_codistribution_matches_oracle(np_, nu, seed):
    rng = np.random.default_rng(np_)
    dets = inputs.ueg_ccsd_determinants(14, 5)
    dets = dets[np.sort(rng.choice(len(dets), 70, replace=False))]
    cps = [0, 1, 3, 17, 64, 100]
    o1, o2 = orc.codistribution(dets, np_, nu, seed, cps)
    g1, g2 = ccmc.ccmc_codistribution(dets, np_, nu, seed, cps)
    assert np.array_equal(o1, g1) and np.array_equal(o2, g2)


def test_codistribution_full_size_3813():
    """All 3813 excitors of 14e/186so, N_p = 24, nu_move = 4, 64 iterations: both sums exact.
    sum c_ij = sum_t sum_r C(n_r(t), 2); sum c_ij^2 = sum_{t,t'} sum_{r,r'} C(n_{rr'}(t,t'), 2)
    with n_{rr'} the excitors on r at t and on r' at t'."""
    dets = inputs.ueg_ccsd_determinants(14, 8)
    np_, nu, seed, T = 24, 4, 2, 64
    _say("[ranks] placements of 3813 excitors from the oracle")
    pl = np.array([[orc.placement(d, t, np_, nu, seed) for d in dets] for t in range(T)], dtype=np.int64)
    c2 = lambda x: (x * (x - 1) // 2).sum()
    s1 = sum(int(c2(np.bincount(pl[t], minlength=np_))) for t in range(T))
    s2 = 0
    for t in range(T):
        for u in range(T):
            s2 += int(c2(np.bincount(pl[t] * np_ + pl[u], minlength=np_ * np_)))
    g1, g2 = ccmc.ccmc_codistribution(dets, np_, nu, seed, [T // 2, T])
    assert int(g1[1]) == s1 and int(g2[1]) == s2
    npairs = len(dets) * (len(dets) - 1) // 2
    assert abs(int(g1[1]) / (npairs * T) * np_ - 1.0) < 0.02
    _say("[ranks] co-distribution 3813 ok")
