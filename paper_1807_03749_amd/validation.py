"""Scale validation: the CCSDTQ correlation energy of the 14-electron 3D UEG in 358 spin
orbitals at r_s = 1 bohr (Sec. III.B prints -0.51856(7), -0.51866(7) and -0.51875(7) Eh from three
calculations; its CISDTQ space holds 2.6(1)x10^8 determinants).

The solve grows the population at zero shift from the reference, varies the shift to hold it at
the target, skips an equilibration window, and records the projected-energy terms, which are
reblocked (and reweighted for population control) at the end.  The paper used even selection,
which it does not define; this run uses full non-composite sampling with the p_size
distribution of the rest of the library.  Progress goes to stderr.  With --checkpoint the
whole calculation (store, N_0, step index, population control, series) is saved every
`save_every` recorded steps, and --resume continues such a checkpoint exactly (the Philox
counters are keyed by the absolute step index), so a run can span several sessions.

``python -m paper_1807_03749_amd.validation --target 3e7 --tau 0.003 --equil 4000 --samples 30000``
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import ccmc, driver

PRINTED = {"OpenMP (Neufeld 2017)": (-0.51856, 0.00007), "8 MPI x 12 OpenMP": (-0.51866, 0.00007),
           "96 MPI": (-0.51875, 0.00007)}


def _log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def run(target: float = 3e7, tau: float = 0.003, equil: int = 4000, samples: int = 30000, seed: int = 358,
        tau_grow: float = 0.005, save: str | None = None, save_every: int = 2000, report_every: int = 100,
        checkpoint: str | None = None, resume: str | None = None, seconds_budget: float = 0.0):
    st = ccmc.State("ueg", 14, 4, n2_max=12, rs=1.0, full_noncomposite=1, min_spawn_attempts=1,
                    multispawn_threshold=1.0, init_pop=target / 300.0, seed=seed)
    t0 = time.perf_counter()
    num, den, shf, ref, nexc = [], [], [], [], []
    start = 0
    if resume:
        ck = driver.load_checkpoint(resume)
        ctl, nsel, series = driver.resume(st, ck)
        num, den, shf = list(series["num"]), list(series["den"]), list(series["shift"])
        ref, nexc = list(series["ref"]), list(series["nexc"])
        start = int(series["done"][0])
        _log(f"[358] resumed at step {start} of the run ({len(num)} samples), step index {ck['step']}")
    else:
        nsel = driver.selections(target / 300.0)
        steps = 0
        s = None
        while True:  # growth at S = 0
            s = st.ccmc_step(tau_grow, 0.0, nsel)
            nsel = driver.selections(s["n_total"])
            steps += 1
            if s["n_total"] >= target or steps > 20000:
                break
        _log(f"[358] grown in {steps} steps: N {s['n_total']:.3e}, {s['n_excitors']} excitors, "
             f"{time.perf_counter() - t0:.1f} s")
        ctl = driver.ShiftControl(target=target, tau=tau)
    attempts = 0
    t1 = time.perf_counter()
    stopped = False
    for it in range(start, equil + samples):
        used = ctl.shift
        s = st.ccmc_step(tau, used, nsel)
        ctl.update(s["n_total"])
        nsel = driver.selections(s["n_total"])
        attempts += s["n_spawn_attempts"]
        if it >= equil:
            num.append(s["eproj_num"])
            den.append(s["eproj_den"])
            shf.append(used)
            ref.append(s["n_ref"] / s["n_total"])
            nexc.append(s["n_excitors"])
        if (it + 1) % report_every == 0:
            msg = (f"[358] step {it + 1}: N {s['n_total']:.3e}, {s['n_excitors']} excitors, S {ctl.shift:.5f}, "
                   f"{1e3 * (time.perf_counter() - t1) / (it + 1 - start):.1f} ms/step")
            if len(num) >= 64:
                e, err, _ = driver.reblock_ratio(np.array(num), np.array(den))
                msg += f", E {e:.6f} +- {err:.6f} ({len(num)} samples)"
            _log(msg)
        if save and len(num) and len(num) % save_every == 0:
            np.savez(save, num=np.array(num), den=np.array(den), shift=np.array(shf), tau=tau)
        last = it + 1 == equil + samples
        out_of_time = seconds_budget > 0 and time.perf_counter() - t0 > seconds_budget
        if checkpoint and ((len(num) and len(num) % save_every == 0) or last or out_of_time):
            driver.save_checkpoint(checkpoint, st, ctl, nsel, dict(num=num, den=den, shift=shf, ref=ref, nexc=nexc,
                                                                   done=[it + 1]))
        if out_of_time and not last:
            _log(f"[358] time budget reached after step {it + 1}; checkpoint written")
            stopped = True
            break
    seconds = time.perf_counter() - t1
    num, den = np.array(num), np.array(den)
    e, err, lvl = driver.reblock_ratio(num, den)
    rw = driver.reweight(num, den, np.array(shf), tau, memories=(0, 100, 1000, 4000))
    if save:
        np.savez(save, num=num, den=den, shift=np.array(shf), tau=tau)
    res = dict(system="ueg", electrons=14, spin_orbitals=358, truncation=4, rs=1.0, target=target, tau=tau,
               equil=equil, samples=len(num), complete=not stopped, energy=e, error=err, block_level=lvl,
               reweighted=[dict(memory=k, energy=x, error=y) for k, x, y in rw],
               reference_fraction=float(np.mean(ref)), excitors=float(np.mean(nexc)),
               seconds=seconds, attempts_per_s=attempts / seconds,
               printed={k: dict(energy=v[0], error=v[1], sigmas=(e - v[0]) / float(np.hypot(err, v[1])))
                        for k, v in PRINTED.items()})
    st.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--target", type=float, default=3e7)
    ap.add_argument("--tau", type=float, default=0.003)
    ap.add_argument("--equil", type=int, default=4000)
    ap.add_argument("--samples", type=int, default=30000)
    ap.add_argument("--seed", type=int, default=358)
    ap.add_argument("--save", help="write the recorded series to this .npz")
    ap.add_argument("--checkpoint", help="save the whole calculation here every 2000 samples and at the end")
    ap.add_argument("--resume", help="continue the calculation saved in this checkpoint")
    ap.add_argument("--seconds", type=float, default=0.0, help="stop (with a checkpoint) after this wall time")
    ap.add_argument("--out", help="also write the result JSON here")
    args = ap.parse_args()
    res = run(args.target, args.tau, args.equil, args.samples, args.seed, save=args.save, checkpoint=args.checkpoint,
              resume=args.resume, seconds_budget=args.seconds)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
