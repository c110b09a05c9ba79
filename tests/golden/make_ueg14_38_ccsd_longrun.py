"""Write ueg14_38_ccsd_longrun.txt: the oracle's own long-run CCMC energy of the 14-electron
UEG in 38 spin orbitals (r_s = 1, CCSD, original selection, one attempt per cluster,
tau = 0.005, target population 5e4), from independent replicas (distinct Philox keys), and
beside it the deterministic projective CCSD energy of the same system (oracle/ccsd.py).

Calls only oracle/ (the CPU oracle and numpy).  Each replica grows from N_0 = 1000 with the
shift held at zero until N_tot reaches the target, then varies the shift every 10 steps
(damping 0.05), equilibrates, and records the projected-energy terms (Sec. II, eq. 7).  Its
energy and standard error come from Flyvbjerg-Petersen blocking of the linearised ratio
series with the optimal block of Lee et al. (2011); the replicas' energies are combined by
their mean, with the standard error of that mean from their scatter.

Usage: python tests/golden/make_ueg14_38_ccsd_longrun.py [replicas] [equil] [steps]
"""
from __future__ import annotations

import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import binding as ob  # noqa: E402
from oracle import ccsd  # noqa: E402

TAU, TARGET, INIT, SEED0 = 0.005, 5e4, 1000.0, 1234


def blocked_error(x: np.ndarray) -> float:
    """Standard error of the mean of a correlated series at the optimal blocking level."""
    y = np.asarray(x, float)
    n0 = len(y)
    se = []
    while len(y) >= 2:
        se.append(y.std(ddof=1) / math.sqrt(len(y)))
        m = len(y) // 2 * 2
        y = 0.5 * (y[0:m:2] + y[1:m:2])
    for i, s in enumerate(se):
        if (2 ** i) ** 3 > 2 * n0 * (s / se[0]) ** 4:
            return float(s)
    return float(se[-1])


def replica(args):
    r, equil, steps = args
    S = ob.System.ueg(14, 2, 1.0)
    run = ob.Run(S, 2, ob.RunOptions(init_pop=INIT, seed=SEED0 + 1000 * (r + 1)))
    st = run.step(TAU, 0.0, int(INIT))
    shift, hist, varying = 0.0, [], False
    num, den = [], []
    t0 = time.time()
    for it in range(10 ** 7):
        ntot = st["n_total"]
        if not varying and ntot >= TARGET:
            varying, anchor = True, len(hist)
        hist.append(ntot)
        if varying and len(hist) - 1 > anchor and (len(hist) - 1 - anchor) % 10 == 0:
            shift -= 0.05 / (10 * TAU) * math.log(hist[-1] / hist[-11])
        st = run.step(TAU, shift, int(math.floor(ntot + 0.5)))
        if varying and len(hist) - anchor > equil:
            num.append(st["eproj_num"])
            den.append(st["eproj_den"])
            if len(num) == steps:
                break
    num, den = np.array(num), np.array(den)
    e = num.mean() / den.mean()
    err = blocked_error(num - e * den) / den.mean()
    print(f"replica {r}: E {e:.6f} +- {err:.6f} ({time.time() - t0:.0f} s)", flush=True)
    return e, err


def main():
    nrep = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    equil = int(sys.argv[2]) if len(sys.argv) > 2 else 2000
    steps = int(sys.argv[3]) if len(sys.argv) > 3 else 16000
    with mp.Pool(nrep) as pool:
        res = pool.map(replica, [(r, equil, steps) for r in range(nrep)])
    e_ccsd, _, _ = ccsd.ccsd_doubles(ob.System.ueg(14, 2, 1.0))
    es = np.array([e for e, _ in res])
    errs = np.array([x for _, x in res])
    mean = es.mean()
    sem = es.std(ddof=1) / math.sqrt(nrep)
    out = os.path.join(HERE, "ueg14_38_ccsd_longrun.txt")
    with open(out, "w") as f:
        f.write("# Long-run CCMC correlation energy of the CPU oracle (written by make_ueg14_38_ccsd_longrun.py)\n")
        f.write("# UEG 14 electrons, 38 spin orbitals (|n|^2 <= 2), r_s = 1, CCSD, original selection,\n")
        f.write(f"# tau = {TAU}, target N_tot = {TARGET:g}, N_0 from {INIT:g}, shift damping 0.05 every 10 steps,\n")
        f.write(f"# {equil} equilibration steps then {steps} recorded steps per replica; Philox keys "
                f"{SEED0} + 1000 (r + 1)\n")
        f.write("# columns: replica  E_corr  blocked_error\n")
        for r, (e, x) in enumerate(res):
            f.write(f"{r} {e:.10f} {x:.10f}\n")
        f.write(f"# mean {mean:.10f} standard_error_of_mean {sem:.10f}\n")
        f.write(f"# deterministic_ccsd {e_ccsd:.12f}\n")
    print(f"mean {mean:.6f} +- {sem:.6f} over {nrep} replicas -> {out}")


if __name__ == "__main__":
    main()
