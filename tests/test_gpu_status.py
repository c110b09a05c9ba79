"""Step statistics carry the call's wall time and each state's own outcome; the growth bound
(blow-up detector) rolls a step back and leaves the state exactly as it was; so does a step
refused for memory, wherever its planning ran out of budget; a batch reports every state's own
failure."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_1807_03749_amd import ccmc, driver

pytestmark = pytest.mark.gpu

TAU = 0.05  # a large time step: the population grows fast from the reference
EBLOWUP, ENOMEM = -5, -2


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _state(**kw):
    opts = dict(init_pop=50.0, seed=77)
    opts.update(kw)
    return ccmc.State("ueg", 14, 2, n2_max=2, rs=1.0, **opts)


def test_stats_carry_time_and_status():
    _say("[status] UEG 14e/38so CCSD, one step")
    s = _state()
    st = s.ccmc_step(TAU, 0.0, 50)
    assert st["status"] == 0 and st["ms"] > 0.0
    s.close()


def test_growth_bound_rolls_back_and_matches_an_unbounded_run():
    _say("[status] growth bound 1.3 against an unbounded twin")
    free = _state()
    bound = _state(blowup_factor=1.3)
    nsel, prev = 50, 50.0
    failed = False
    for it in range(300):
        ref = free.ccmc_step(TAU, 0.0, nsel)
        before = bound.ccmc_export()
        try:
            got = bound.ccmc_step(TAU, 0.0, nsel)
        except ccmc.CCMCError as e:
            assert e.status == EBLOWUP, e
            # the unbounded twin shows the growth that tripped the bound
            assert ref["n_total"] > 1.3 * prev
            after = bound.ccmc_export()
            assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
            assert before[2] == after[2] and before[3] == after[3]
            failed = True
            break
        for f in ("n_total", "n_ref", "n_excitors", "n_spawn_attempts", "eproj_num"):
            assert got[f] == ref[f], (it, f)
        assert ref["n_total"] <= 1.3 * prev
        prev = ref["n_total"]
        nsel = driver.selections(ref["n_total"])
    assert failed, "the population never grew by 30% in one step"
    free.close()
    bound.close()


def test_batch_reports_each_states_own_failure():
    _say("[status] batch: blow-up, out of budget, success")
    a = _state(blowup_factor=1.0001)  # any growth on the first step trips it
    b = _state()
    b.ccmc_set_budget(b.ccmc_memory() + 4096)  # no room for the step's buffers
    c = _state()
    ka = a.ccmc_export()
    res = ccmc.ccmc_step_batch([a, b, c], [TAU] * 3, [0.0] * 3, [50] * 3)
    assert isinstance(res[0], ccmc.CCMCError) and res[0].status == EBLOWUP, res[0]
    assert isinstance(res[1], ccmc.CCMCError) and res[1].status == ENOMEM, res[1]
    assert isinstance(res[2], dict) and res[2]["status"] == 0 and res[2]["step"] == 1
    kb = a.ccmc_export()
    assert kb[3] == ka[3] and len(kb[1]) == len(ka[1])
    for s in (a, b, c):
        s.close()


def test_budget_starved_twin_matches_after_every_retry():
    """A step refused for memory leaves the state unchanged, wherever in its planning the budget
    ran out: a twin whose budget is raised a little after each refusal (so that refusals fall
    between the growth of the store and of the arrays sized by it) takes the same steps as an
    unconstrained run.  Two key words per determinant (114 spin orbitals), so that a store laid
    out with a stale row pitch would show."""
    _say("[status] UEG 14e/114so CCSDT FP32: budget-starved twin against a free run")
    mk = lambda: ccmc.State("ueg", 14, 3, n2_max=5, rs=1.0, precision="fp32", init_pop=20.0, seed=4242,
                            full_noncomposite=1, min_spawn_attempts=4)
    free, starved = mk(), mk()
    assert free.n_words == 2
    budget = starved.ccmc_memory() + 4096
    starved.ccmc_set_budget(budget)
    nsel, refused = 20, 0
    for it in range(80):
        ref = free.ccmc_step(0.01, 0.0, nsel)
        # raise the twin's budget in steps of a sixth of the way to a little above what the free
        # run holds, so that refusals fall at several points of the twin's planning
        target = int(free.ccmc_memory() * 1.25) + (1 << 20)
        for _ in range(2000):
            try:
                got = starved.ccmc_step(0.01, 0.0, nsel)
                break
            except ccmc.CCMCError as e:
                assert e.status == ENOMEM, e
                refused += 1
                budget += max(65536, (target - budget) // 6)
                starved.ccmc_set_budget(budget)
        else:
            raise AssertionError("the budget never sufficed")
        for f in ("n_total", "n_ref", "n_excitors", "n_spawn_attempts", "eproj_num"):
            assert got[f] == ref[f], (it, f, got[f], ref[f])
        nsel = driver.selections(ref["n_total"])
    a, b = free.ccmc_export(), starved.ccmc_export()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    _say(f"[status] {refused} refusals, {len(a[1])} excitors, N_tot {ref['n_total']:.4g}")
    assert refused >= 10
    free.close()
    starved.close()


def test_import_refused_for_memory_leaves_the_store():
    """ccmc_import under a budget that is raised a little after each refusal: every refusal leaves
    the store, N_0 and the step index as they were (two key words, so that a stale row pitch
    would show), and the import that succeeds holds exactly the imported store."""
    _say("[status] UEG 14e/114so CCSDT FP64: import refused for memory")
    mk = lambda seed, pop: ccmc.State("ueg", 14, 3, n2_max=5, rs=1.0, init_pop=pop, seed=seed)
    big, small = mk(5, 2e4), mk(6, 20.0)
    nb, ns = 20000, 20
    for _ in range(40):
        ns = driver.selections(small.ccmc_step(0.01, 0.0, ns)["n_total"])
    for _ in range(60):
        nb = driver.selections(big.ccmc_step(0.01, 0.0, nb)["n_total"])
    kb, ab, n0b, stepb = big.ccmc_export()
    before = small.ccmc_export()
    # beyond the small state's store capacity (its excitors plus a step's records, >= 4096)
    assert len(ab) > 20000, (len(ab), len(before[1]))
    budget = small.ccmc_memory() + 4096
    small.ccmc_set_budget(budget)
    refused = 0
    for _ in range(2000):  # steps of 256 KiB: the import needs a few MB for ~3x10^4 excitors
        try:
            small.ccmc_import(kb, ab, n0b, stepb)
            break
        except ccmc.CCMCError as e:
            assert e.status == ENOMEM, e
            refused += 1
            now = small.ccmc_export()
            assert np.array_equal(now[0], before[0]) and np.array_equal(now[1], before[1])
            assert now[2] == before[2] and now[3] == before[3]
            budget += 1 << 18
            small.ccmc_set_budget(budget)
    else:
        raise AssertionError("the budget never sufficed")
    after = small.ccmc_export()
    assert np.array_equal(after[0], kb) and np.array_equal(after[1], ab) and after[2] == n0b and after[3] == stepb
    _say(f"[status] {refused} refusals before the import of {len(ab)} excitors")
    assert refused >= 5
    big.close()
    small.close()
