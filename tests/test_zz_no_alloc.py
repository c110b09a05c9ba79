"""ccmc_step_noalloc: the allocation-free variant of ccmc_step (fixed per-GPU step area, no
buffer growth) gives exactly ccmc_step's results, on two calls in a row of which the second
has a smaller input, and refuses -- leaving the state unchanged -- a step that would need
more than the state holds."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import binding as orc
from paper_1807_03749_amd import ccmc

pytestmark = pytest.mark.gpu

OPTS = dict(full_noncomposite=1, min_spawn_attempts=2, multispawn_threshold=1.0, init_pop=400.0, seed=4321)
TAU = 0.002


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _grown_store(steps):
    """A store grown by the oracle (UEG 14e/114so CCSDT, full non-composite sampling)."""
    S = orc.System.ueg(14, 5, 1.0)
    R = orc.Run(S, 3, orc.RunOptions(**OPTS))
    st = R.step(TAU, 0.0, 400)
    for _ in range(steps - 1):
        st = R.step(TAU, 0.0, int(round(st["n_total"])))
    keys, amps, n0, step = R.export_state()
    return keys, amps, n0, step, int(round(st["n_total"]))


def _state():
    return ccmc.State("ueg", 14, 3, n2_max=5, rs=1.0, **OPTS)


def _no_time(d):
    return {k: v for k, v in d.items() if k != "ms"}


def _same(a, b):
    ka, aa, ra, sa = a.ccmc_export()
    kb, ab, rb, sb = b.ccmc_export()
    assert np.array_equal(ka, kb) and np.array_equal(aa, ab) and ra == rb and sa == sb


def test_noalloc_step_matches_ccmc_step():
    big = _grown_store(40)
    small = (big[0][::3].copy(), big[1][::3].copy(), big[2], big[3], max(1, big[4] // 3))
    _say(f"[noalloc] UEG 14e/114so CCSDT: {len(big[1])} then {len(small[1])} excitors")
    ref, na = _state(), _state()
    # the state of the allocation-free call reserves its buffers with the same two steps taken
    # the ordinary way first (a step of a grown population needs larger buffers)
    na.ccmc_import(*big[:4])
    r = na.ccmc_step(TAU, -0.1, big[4])
    na.ccmc_step(TAU, -0.1, int(round(r["n_total"])))
    for keys, amps, n0, step, nsel in (big, small):
        ref.ccmc_import(keys, amps, n0, step)
        na.ccmc_import(keys, amps, n0, step)
        mem = na.ccmc_memory()
        a = ref.ccmc_step(TAU, -0.1, nsel)
        b = na.ccmc_step_noalloc(TAU, -0.1, nsel)
        assert _no_time(a) == _no_time(b)
        assert na.ccmc_memory() == mem  # nothing allocated
        _same(ref, na)
        # a second step from there, again both ways
        a = ref.ccmc_step(TAU, -0.1, int(round(a["n_total"])))
        b = na.ccmc_step_noalloc(TAU, -0.1, int(round(b["n_total"])))
        assert _no_time(a) == _no_time(b)
        _same(ref, na)
        _say(f"[noalloc] {len(amps)} excitors: identical to ccmc_step over two steps")
    ref.close()
    na.close()


def test_noalloc_refuses_to_grow_and_leaves_the_state():
    keys, amps, n0, step, nsel = _grown_store(40)
    _say("[noalloc] unreserved state: the step needs buffers it does not hold")
    st = _state()
    st.ccmc_import(keys, amps, n0, step)
    before = st.ccmc_export()
    mem = st.ccmc_memory()
    with pytest.raises(ccmc.CCMCError) as e:
        st.ccmc_step_noalloc(TAU, 0.0, nsel)
    assert e.value.status == -2
    assert st.ccmc_memory() == mem
    after = st.ccmc_export()
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    assert before[2] == after[2] and before[3] == after[3]
    # after an ordinary step has reserved the buffers, the same call goes through
    st.ccmc_step(TAU, 0.0, nsel)
    st.ccmc_import(keys, amps, n0, step)
    r = st.ccmc_step_noalloc(TAU, 0.0, nsel)
    assert r["status"] == 0 and r["step"] == step + 1
    st.close()
