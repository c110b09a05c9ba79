"""ccmc_run: steps in the library's own loop under its population control give exactly the
statistics, shifts and stores of the same steps driven one at a time from Python with
driver.ShiftControl and driver.selections, also when the control starts during the run and
when runs are chained."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_1807_03749_amd import ccmc, driver

pytestmark = pytest.mark.gpu

CFG = dict(n2_max=4, rs=1.0, init_pop=300.0, seed=31, full_noncomposite=1, min_spawn_attempts=2,
           multispawn_threshold=1.0)
TAU, TARGET = 0.005, 1000.0


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _python_loop(st, n_steps, ctl, nsel):
    out = []
    for _ in range(n_steps):
        r = st.ccmc_step(TAU, ctl.shift, nsel)
        ctl.update(r["n_total"])
        nsel = driver.selections(r["n_total"])
        out.append(r)
    return out, nsel


@pytest.mark.parametrize("chunks", [[120], [7, 50, 63]], ids=["one-run", "chained"])
def test_run_matches_python_loop(chunks):
    _say(f"[run] UEG 14e CCSDT, tau {TAU}, target {TARGET}, chunks {chunks}")
    n = sum(chunks)
    a = ccmc.State("ueg", 14, 3, **CFG)
    b = ccmc.State("ueg", 14, 3, **CFG)
    nsel0 = driver.selections(CFG["init_pop"])
    py_ctl = driver.ShiftControl(target=TARGET, tau=TAU)
    ref, nsel_py = _python_loop(a, n, py_ctl, nsel0)
    assert py_ctl.varying, "the control should start during the run"
    c = ccmc.ccmc_shift_control.new(TARGET)
    got, nsel = [], nsel0
    for k in chunks:
        out, nsel = b.ccmc_run(k, TAU, c, nsel)
        got += [out[i].as_dict() for i in range(k)]
    for t, (x, y) in enumerate(zip(ref, got)):
        x, y = ({k: v for k, v in z.items() if k != "ms"} for z in (x, y))  # the call's wall time differs
        assert x == y, (t, x, y)
    assert nsel == nsel_py and c.shift == py_ctl.shift and bool(c.varying)
    ka, aa, na, sa = a.ccmc_export()
    kb, ab, nb, sb = b.ccmc_export()
    assert np.array_equal(ka, kb) and np.array_equal(aa, ab) and na == nb and sa == sb
    _say(f"[run] ok: {n} steps, N_tot {ref[-1]['n_total']:.1f}, shift {c.shift:.6f}")
    a.close()
    b.close()


def test_run_refuses_bad_control_and_stops_at_a_failing_step():
    st = ccmc.State("ueg", 14, 2, n2_max=2, init_pop=200.0, seed=3)
    bad = ccmc.ccmc_shift_control.new(1e9, period=0)
    with pytest.raises(ccmc.CCMCError):
        st.ccmc_run(3, 0.005, bad, 200)
    ok = ccmc.ccmc_shift_control.new(1e9)
    with pytest.raises(ccmc.CCMCError):  # a step with 2^32 selections is refused before it runs
        st.ccmc_run(3, 0.005, ok, 1 << 32)
    assert st.ccmc_export()[3] == 0  # no step was taken
    out, nsel = st.ccmc_run(2, 0.005, ok, 200)
    assert out[1].step == 2 and nsel == driver.selections(out[1].n_total)
    st.close()
