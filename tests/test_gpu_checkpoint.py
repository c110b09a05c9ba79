"""Checkpoint / resume through the C ABI: a GPU run exported mid-trajectory (ccmc_export),
saved with its native population control, and imported into a fresh state (ccmc_import)
continues bit for bit as the uninterrupted run -- the Philox counters are keyed by the
absolute step index, so nothing else needs saving."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_1807_03749_amd import ccmc, driver

pytestmark = pytest.mark.gpu

CFG = dict(n2_max=4, rs=1.0, init_pop=300.0, seed=53, full_noncomposite=1, min_spawn_attempts=4,
           multispawn_threshold=1.0)
TAU, TARGET = 0.005, 1500.0


def _no_time(d):
    return {k: v for k, v in d.items() if k != "ms"}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_resume_through_the_abi_is_exact(tmp_path, precision):
    print(f"[ckpt] UEG 14e/66so CCSDT {precision}: 60 steps against 35 + resume + 25", flush=True)
    sys.stdout.flush()
    whole = ccmc.State("ueg", 14, 3, precision=precision, **CFG)
    ctl = ccmc.ccmc_shift_control.new(TARGET)
    out, _ = whole.ccmc_run(60, TAU, ctl, driver.selections(CFG["init_pop"]))
    ref = [_no_time(out[i].as_dict()) for i in range(60)]

    first = ccmc.State("ueg", 14, 3, precision=precision, **CFG)
    c1 = ccmc.ccmc_shift_control.new(TARGET)
    out1, nsel1 = first.ccmc_run(35, TAU, c1, driver.selections(CFG["init_pop"]))
    series = dict(num=[out1[i].eproj_num for i in range(35)], den=[out1[i].eproj_den for i in range(35)])
    path = str(tmp_path / "ckpt.npz")
    driver.save_checkpoint(path, first, c1, nsel1, series)
    first.close()

    again = ccmc.State("ueg", 14, 3, precision=precision, **CFG)
    c2, nsel2, series2 = driver.resume(again, driver.load_checkpoint(path))
    assert nsel2 == nsel1 and c2.shift == c1.shift and c2.since == c1.since and c2.varying == c1.varying
    out2, _ = again.ccmc_run(25, TAU, c2, nsel2)
    for i in range(25):
        assert _no_time(out2[i].as_dict()) == ref[35 + i], i
    assert c2.shift == ctl.shift and series2["num"] == [r["eproj_num"] for r in ref[:35]]
    ka, aa, ra, sa = whole.ccmc_export()
    kb, ab, rb, sb = again.ccmc_export()
    assert np.array_equal(ka, kb) and np.array_equal(aa, ab) and ra == rb and sa == sb == 60
    whole.close()
    again.close()
