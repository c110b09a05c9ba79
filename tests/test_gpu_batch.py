"""ccmc_step_batch: several solves in shared launches give, state by state, exactly the
result of stepping each state alone (same stores, same Philox keys and step indices), also
when states of different sizes, truncations, selection modes and precisions are mixed and
join the batch at different times."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_1807_03749_amd import ccmc, driver

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


SOLVES = [
    dict(system="ueg", n_electrons=14, truncation=2, n2_max=2, rs=1.0, init_pop=300.0, seed=11),
    dict(system="ueg", n_electrons=14, truncation=3, n2_max=4, rs=0.5, init_pop=500.0, seed=12, full_noncomposite=1,
         min_spawn_attempts=4, multispawn_threshold=1.0),
    dict(system="ueg", n_electrons=14, truncation=3, n2_max=5, rs=2.0, init_pop=800.0, seed=13, full_noncomposite=1,
         min_spawn_attempts=2, multispawn_threshold=1.0),
    dict(system="ueg", n_electrons=14, truncation=2, n2_max=2, rs=5.0, init_pop=200.0, seed=14, precision="fp32"),
    dict(system="ueg", n_electrons=14, truncation=2, n2_max=4, rs=1.0, init_pop=400.0, seed=15, precision="fp32",
         full_noncomposite=1),
    # virtual processors (Sec. III) in the same batch
    dict(system="ueg", n_electrons=14, truncation=3, n2_max=4, rs=0.5, init_pop=500.0, seed=16, full_noncomposite=1,
         n_ranks=24, move_shift=2),
    dict(system="ueg", n_electrons=14, truncation=2, n2_max=2, rs=1.0, init_pop=300.0, seed=17, n_ranks=240,
         move_shift=0),
]
TAU = [0.005, 0.002, 0.002, 0.005, 0.005, 0.002, 0.005]


def _make(cfg):
    c = dict(cfg)
    return ccmc.State(c.pop("system"), c.pop("n_electrons"), c.pop("truncation"), **c)


def _drive(states, starts, steps, batched):
    """Step each state `steps` times from its start index (state i joins at starts[i]) with a
    shift held at 0 and n_sel = round(N_tot); return each state's exported store."""
    nsel = [driver.selections(s_.options.init_pop) for s_ in states]
    for t in range(max(starts) + steps):
        active = [i for i in range(len(states)) if starts[i] <= t < starts[i] + steps]
        if not active:
            continue
        if batched:
            res = ccmc.ccmc_step_batch([states[i] for i in active], [TAU[i] for i in active], [0.0] * len(active),
                                       [nsel[i] for i in active])
        else:
            res = [states[i].ccmc_step(TAU[i], 0.0, nsel[i]) for i in active]
        for i, r in zip(active, res):
            assert isinstance(r, dict), r
            nsel[i] = driver.selections(r["n_total"])
    return [s_.ccmc_export() for s_ in states]


def _no_time(stats: dict) -> dict:
    """Step statistics without the wall time of the call (which differs run to run)."""
    return {k: v for k, v in stats.items() if k != "ms"}


def test_batch_equals_alone():
    starts = [0, 3, 5, 1, 8, 2, 6]
    alone = _drive([_make(c) for c in SOLVES], starts, 25, batched=False)
    mixed = _drive([_make(c) for c in SOLVES], starts, 25, batched=True)
    for i, (a, b) in enumerate(zip(alone, mixed)):
        ka, aa, ra, sa = a
        kb, ab, rb, sb = b
        assert sa == sb == 25, (i, sa, sb)
        assert np.array_equal(ka, kb), i
        assert np.array_equal(aa, ab), i  # bit-identical: every sum has the same order
        assert ra == rb, i
        _say(f"[batch] solve {i}: {len(ka)} excitors, N_0 {ra:.3f} identical alone and batched")


def test_batch_rejects_bad_arguments():
    s1, s2 = _make(SOLVES[0]), _make(SOLVES[3])
    with pytest.raises(ccmc.CCMCError):
        ccmc.ccmc_step_batch([s1, s1], [0.005, 0.005], [0.0, 0.0], [10, 10])
    with pytest.raises(ccmc.CCMCError):
        ccmc.ccmc_step_batch([s1, s2], [0.005, -1.0], [0.0, 0.0], [10, 10])
    assert s1.ccmc_export()[3] == 0 and s2.ccmc_export()[3] == 0


def test_batch_failure_is_per_state():
    """One state overflows its attempt count (EOVERFLOW) and stays unchanged; the other steps."""
    good = _make(SOLVES[0])
    bad = ccmc.State("ueg", 14, 2, n2_max=2, full_noncomposite=1, noncomposite_threshold=1e-9, init_pop=10.0)
    before = bad.ccmc_export()
    res = ccmc.ccmc_step_batch([good, bad], [0.005, 0.005], [0.0, 0.0], [300, 10])
    assert isinstance(res[0], dict) and res[0]["step"] == 1
    assert isinstance(res[1], ccmc.CCMCError) and res[1].status == -3
    after = bad.ccmc_export()
    assert np.array_equal(before[0], after[0]) and before[2] == after[2] and before[3] == after[3]


def test_alternating_alone_and_batched_steps():
    """A solve stepped alone, then in batches, then alone again (each path clears its step
    area in its own way) follows, step by step, the same solve stepped alone throughout."""
    cfg, tau = SOLVES[1], TAU[1]
    a, b, partner = _make(cfg), _make(cfg), _make(SOLVES[0])
    na = nb = npart = driver.selections(cfg["init_pop"])
    plan = ["alone"] * 3 + ["batch"] * 3 + ["alone"] * 4 + ["batch"] * 2 + ["alone"] * 3
    for t, how in enumerate(plan):
        ra = b.ccmc_step(tau, 0.0, nb)
        if how == "alone":
            rb = a.ccmc_step(tau, 0.0, na)
        else:
            rb, rp = ccmc.ccmc_step_batch([a, partner], [tau, TAU[0]], [0.0, 0.0], [na, npart])
            assert isinstance(rp, dict), rp
            npart = driver.selections(rp["n_total"])
        assert isinstance(rb, dict), rb
        assert _no_time(ra) == _no_time(rb), (t, how, ra, rb)
        na, nb = driver.selections(rb["n_total"]), driver.selections(ra["n_total"])
    ka, aa, ra_, sa = a.ccmc_export()
    kb, ab, rb_, sb = b.ccmc_export()
    assert sa == sb == len(plan) and np.array_equal(ka, kb) and np.array_equal(aa, ab) and ra_ == rb_
    _say(f"[batch] alternating alone/batched: {len(ka)} excitors identical after {len(plan)} steps")
