"""Checkpoint / resume on the CPU with the oracle: a run saved mid-trajectory (store, N_0,
step index, population control, selection count, energy series) and resumed into a fresh
calculation continues exactly as the uninterrupted run, step for step."""
from __future__ import annotations

import numpy as np

from oracle import binding as ob
from paper_1807_03749_amd import driver

TAU = 0.005


def _steps(run, ctl, nsel, n, series):
    out = []
    for _ in range(n):
        st = run.step(TAU, ctl.shift, nsel)
        ctl.update(st["n_total"])
        nsel = driver.selections(st["n_total"])
        series["num"].append(st["eproj_num"])
        series["den"].append(st["eproj_den"])
        out.append(st)
    return out, nsel


def _run():
    S = ob.System.ueg(14, 2, 1.0)
    return ob.Run(S, 2, ob.RunOptions(init_pop=200.0, seed=91, full_noncomposite=True, min_spawn_attempts=2,
                                      multispawn_threshold=1.0))


def test_resume_continues_the_trajectory_exactly(tmp_path):
    whole, nsel = _run(), driver.selections(200.0)
    ctl = driver.ShiftControl(target=600.0, tau=TAU)
    ref_series = {"num": [], "den": []}
    ref, _ = _steps(whole, ctl, nsel, 40, ref_series)
    assert ctl.varying  # the control started during the run, before the checkpoint below

    first = _run()
    ctl1 = driver.ShiftControl(target=600.0, tau=TAU)
    series = {"num": [], "den": []}
    _, nsel1 = _steps(first, ctl1, driver.selections(200.0), 25, series)
    path = str(tmp_path / "ckpt.npz")
    driver.save_checkpoint(path, first, ctl1, nsel1, series)
    del first

    again = _run()
    ctl2, nsel2, series2 = driver.resume(again, driver.load_checkpoint(path))
    assert isinstance(ctl2, driver.ShiftControl) and ctl2.to_dict() == ctl1.to_dict() and nsel2 == nsel1
    rest, _ = _steps(again, ctl2, nsel2, 15, series2)
    for a, b in zip(ref[25:], rest):
        assert a == b
    assert series2["num"] == ref_series["num"] and series2["den"] == ref_series["den"]
    ka, aa, ra, sa = whole.export_state()
    kb, ab, rb, sb = again.export_state()
    assert np.array_equal(ka, kb) and np.array_equal(aa, ab) and ra == rb and sa == sb == 40
