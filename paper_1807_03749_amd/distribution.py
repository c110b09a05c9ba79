"""The distributed algorithm's placement of excitors, and its bias, studied on one GPU
(Sec. III: the placement of eq. 9; Sec. III.B: its co-distribution figure and bias study).

Two studies, both run through the C ABI:

* co-location: the 3813 excitors of the 14e/186so UEG CCSD space are placed by eq. 9
  for iterations 0 .. T-1; for each N_p and nu_move the mean and the standard deviation over
  all pairs of p_ij(T), the fraction of those iterations in which excitors i and j shared a
  processor, rescaled as in the co-distribution figure: mean * N_p (1 is exact), standard
  deviation * N_p * sqrt(T / (N_p - 1)) for the N_p scan and * N_p * sqrt(T / 2^nu_move) for
  the nu_move scan (``ccmc_codistribution``).
* bias: the CCSDT projected energy of the 14e/66so UEG (r_s = 0.5 and 5 bohr, full
  non-composite sampling) with N_p virtual processors, against N_p, the time step and
  nu_move, each compared with the one-processor run of the same r_s and time step.  Every
  configuration is a separate solve; all of them step together in shared launches
  (``ccmc_step_batch``), each with its own shift control.

``python -m paper_1807_03749_amd.distribution --codist`` / ``--bias`` prints one JSON line per
configuration and progress on stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import ccmc, driver, inputs


def _log(msg: str):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------- co-location

def codistribution(n_ranks: int, move_shift: int, checkpoints, hash_seed: int = 0, dets=None) -> dict:
    """Mean and standard deviation over pairs of p_ij(T) at each checkpoint T."""
    dets = inputs.ueg_ccsd_determinants(14, 8) if dets is None else dets
    n = len(dets)
    npairs = n * (n - 1) // 2
    cps = [int(t) for t in checkpoints]
    s1, s2 = ccmc.ccmc_codistribution(dets, n_ranks, move_shift, hash_seed, cps)
    rows = []
    for T, a, b in zip(cps, s1, s2):
        mean = float(a) / (npairs * T)
        var = float(b) / (npairs * T * T) - mean * mean
        std = math.sqrt(max(var, 0.0))
        rows.append(dict(T=T, mean=mean, std=std, mean_scaled=mean * n_ranks,
                         std_scaled_np=std * n_ranks * math.sqrt(T / max(n_ranks - 1, 1)),
                         std_scaled_nu=std * n_ranks * math.sqrt(T / 2.0 ** min(move_shift, 60))))
    return dict(n_excitors=n, n_ranks=n_ranks, move_shift=move_shift, hash_seed=hash_seed, rows=rows)


def codistribution_study(ranks=(2, 4, 8, 16, 32, 64, 128, 240), nu_fixed: int = 4, np_fixed: int = 32,
                         nus=(0, 2, 4, 6, 8), t_max: int = 1 << 14):
    cps = [1 << k for k in range(4, int(math.log2(t_max)) + 1)]
    dets = inputs.ueg_ccsd_determinants(14, 8)
    out = []
    for np_ in ranks:
        t0 = time.perf_counter()
        out.append(dict(scan="n_ranks", **codistribution(np_, nu_fixed, cps, dets=dets)))
        _log(f"[codist] N_p {np_} nu {nu_fixed}: {time.perf_counter() - t0:.2f} s")
    for nu in nus:
        t0 = time.perf_counter()
        out.append(dict(scan="move_shift", **codistribution(np_fixed, nu, cps, dets=dets)))
        _log(f"[codist] N_p {np_fixed} nu {nu}: {time.perf_counter() - t0:.2f} s")
    return out


# ----------------------------------------------------------------------------- bias

def bias_configs(rs_values=(0.5, 5.0), ranks=(1, 4, 16, 60, 120, 240), tau: float = 0.001, move_shift: int = 5,
                 taus=(0.0005, 0.002, 0.004), nus=(1, 3, 7), scan_ranks: int = 240):
    """The N_p scan at (tau, nu_move), then at N_p = scan_ranks the time-step scan (with the
    one-processor runs it is compared with) and the nu_move scan."""
    cfg = []
    for rs in rs_values:
        for np_ in ranks:
            cfg.append(dict(scan="n_ranks", rs=rs, n_ranks=np_, tau=tau, move_shift=move_shift))
        for t in taus:
            cfg.append(dict(scan="tau", rs=rs, n_ranks=1, tau=t, move_shift=move_shift))
            cfg.append(dict(scan="tau", rs=rs, n_ranks=scan_ranks, tau=t, move_shift=move_shift))
        for nu in nus:
            cfg.append(dict(scan="move_shift", rs=rs, n_ranks=scan_ranks, tau=tau, move_shift=nu))
    return cfg


def bias_study(configs, target: float = 2e5, equil: int = 4000, samples: int = 30000, grow_max: int = 20000,
               seed: int = 2018, report_every: int = 2000):
    """Run every configuration to `samples` recorded steps after growth and `equil` steps of
    shift control; returns one dict per configuration (energy, reblocked error, reference
    fraction, steps)."""
    states, ctls, nsel, since, num, den, ref, shf = [], [], [], [], [], [], [], []
    for i, c in enumerate(configs):
        st = ccmc.State("ueg", 14, 3, n2_max=4, rs=c["rs"], full_noncomposite=1, init_pop=target / 10.0,
                        seed=seed + 7919 * i, n_ranks=c["n_ranks"], move_shift=c["move_shift"], hash_seed=seed)
        states.append(st)
        ctls.append(driver.ShiftControl(target=target, tau=c["tau"]))
        nsel.append(driver.selections(target / 10.0))
        since.append(-1)
        num.append([])
        den.append([])
        ref.append([])
        shf.append([])
    n = len(configs)
    done = [False] * n
    t0 = time.perf_counter()
    it = 0
    while not all(done):
        active = [i for i in range(n) if not done[i]]
        used = [ctls[i].shift for i in active]
        res = ccmc.ccmc_step_batch([states[i] for i in active], [configs[i]["tau"] for i in active], used,
                                   [nsel[i] for i in active])
        for i, r, s_used in zip(active, res, used):
            if isinstance(r, Exception):
                raise r
            was = ctls[i].varying
            ctls[i].update(r["n_total"])
            if ctls[i].varying and not was:
                since[i] = it
            nsel[i] = driver.selections(r["n_total"])
            if since[i] >= 0 and it - since[i] > equil:
                num[i].append(r["eproj_num"])
                den[i].append(r["eproj_den"])
                shf[i].append(s_used)
                ref[i].append(abs(r["n_ref"]) / r["n_total"])
                done[i] = len(num[i]) >= samples
            elif since[i] < 0 and it >= grow_max:
                raise RuntimeError(f"configuration {configs[i]} did not reach the target in {grow_max} steps")
        it += 1
        if it % report_every == 0:
            left = sum(1 for d in done if not d)
            _log(f"[bias] step {it}: {left} of {n} running, {time.perf_counter() - t0:.1f} s")
    out = []
    for i, c in enumerate(configs):
        e, err, lvl = driver.reblock_ratio(np.array(num[i]), np.array(den[i]))
        rw = driver.reweight(np.array(num[i]), np.array(den[i]), np.array(shf[i]), c["tau"],
                             memories=(0, 100, 1000, 5000))
        out.append(dict(c, energy=e, error=err, block_level=lvl, samples=len(num[i]),
                        reference_fraction=float(np.mean(ref[i])), shift=ctls[i].shift,
                        reweighted=[dict(memory=k, energy=x, error=y) for k, x, y in rw]))
        states[i].close()
    # each processor count against the one-processor run of the same r_s and time step
    for o in out:
        base = [b for b in out if b["rs"] == o["rs"] and b["tau"] == o["tau"] and b["n_ranks"] == 1]
        if base:
            b = base[0]
            o["bias"] = o["energy"] - b["energy"]
            o["bias_error"] = math.hypot(o["error"], b["error"])
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--codist", action="store_true", help="co-location statistics of the placement")
    ap.add_argument("--bias", action="store_true", help="energy bias against N_p, the time step and nu_move")
    ap.add_argument("--t-max", type=int, default=1 << 14)
    ap.add_argument("--target", type=float, default=2e5)
    ap.add_argument("--equil", type=int, default=4000)
    ap.add_argument("--samples", type=int, default=30000)
    args = ap.parse_args()
    if args.codist:
        for row in codistribution_study(t_max=args.t_max):
            print(json.dumps(row), flush=True)
    if args.bias:
        for row in bias_study(bias_configs(), target=args.target, equil=args.equil, samples=args.samples):
            print(json.dumps(row), flush=True)


if __name__ == "__main__":
    main()
