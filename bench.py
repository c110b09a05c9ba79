#!/usr/bin/env python3
"""CCMC step throughput on one MI355X: cluster spawn attempts per second.

Workload (default): 3D uniform electron gas, 14 electrons in 114 spin orbitals (57 plane
waves, |n|^2 <= 5, two 64-bit bitstring words), r_s = 1, CCSDT, full non-composite
sampling, at least 4 spawning attempts per cluster (multi-spawn threshold 1), tau = 0.002,
target population 1e6.  Synthetic and analytic: there is no dataset.

Procedure: grow the population from the reference at a larger time step with the shift held
at zero until it reaches the target, switch to tau = 0.002 with population control, run the
warm-up steps, then time exactly `--steps` steps (each a full ccmc_step: selection,
spawning, death and annihilation).  Inputs stay resident on the GPU throughout.  Kernel
times come from HIP events recorded by the library on its own stream over the timed steps.

Prints one JSON line.  --gpus N > 1 is not supported (one GPU only).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1807_03749_amd import ccmc, driver, inputs  # noqa: E402

METRIC = "cluster spawn attempts/s on 1 MI355X; FP32 vs FP64 at equal E_proj error"
HBM_PEAK_GBS = 8000.0
# Plain 32-bit vector ALU lane operations: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
ALU_PEAK_GOPS = 256 * 4 * 16 * 2.4
# Algorithmic lane operations of one spawning attempt: Philox4x32-10 blocks (10 rounds of two
# 32x32 multiplies (4 ops), 4 xors and 2 key adds = 100 ops per block) -- 2 blocks for the UEG
# generator's three 64-bit draws, 3 for the molecular generator's five -- plus about 100
# (UEG) / 150 (molecular) for the excitation, the Slater-Condon element, the signs, the
# amplitude and the cutoff rounding.
OPS_PER_ATTEMPT = {"ueg": 300.0, "mol": 450.0}
# Algorithmic lane operations of one item of the items kernel (a sampled cluster or a
# non-composite item): about two Philox blocks for the size and the excitor draws (E[blocks]
# = 2.2 for CCSDT composites, s in [2, 5]) = 220, plus about 80 for the prefix searches, the
# collapse with its sign, the level and the amplitude.
OPS_PER_ITEM = 300.0
ALU_KERNELS = {"generate": ("attempt", lambda w: OPS_PER_ATTEMPT[w.system]), "items": ("item", lambda w: OPS_PER_ITEM)}


class _Roctx:
    """roctxProfilerResume/Pause around the timed steps, so that a profiler started with
    --selected-regions sees exactly the timed region (no-op without a profiler)."""

    def __init__(self, enabled: bool):
        self.lib = None
        if enabled:
            import ctypes
            for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so", "libroctx64.so"):
                try:
                    self.lib = ctypes.CDLL(name)
                    break
                except OSError:
                    continue

    def resume(self):
        if self.lib is not None:
            self.lib.roctxProfilerResume(0)

    def pause(self):
        if self.lib is not None:
            self.lib.roctxProfilerPause(0)


ROCTX = _Roctx(False)


def calibrate_copy(gib: float = 1.0, reps: int = 5):
    """A plain device-to-device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = int(gib * (1 << 30)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    ROCTX.resume()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    ROCTX.pause()
    print(json.dumps({"calibrate_copy_bytes": n * 4, "reps": reps}))


VIRTUAL = dict(n_ranks=1, move_shift=5)  # virtual processors of every state (--n-ranks, --move-shift)


def make_state(w: inputs.Workload, precision: str, init_pop: float):
    kw = dict(precision=precision, full_noncomposite=int(w.full_noncomposite),
              min_spawn_attempts=w.min_spawn_attempts, multispawn_threshold=w.multispawn_threshold,
              noncomposite_threshold=w.noncomposite_threshold, init_pop=init_pop, seed=w.seed, **VIRTUAL)
    if w.system == "ueg":
        return ccmc.State("ueg", w.n_electrons, w.truncation, n2_max=w.n2_max, rs=w.rs, **kw)
    h, B = inputs.molecule_like(n_spatial=w.n_spatial, n_electrons=w.n_electrons, n_chol=w.n_chol)
    return ccmc.State("mol", w.n_electrons, w.truncation, h=h, chol=B, **kw)


def grow(state, w: inputs.Workload, log, max_steps: int = 20000, tau_grow_factor: float = 5.0):
    """Shift held at zero (E_HF) until N_tot reaches the target."""
    tau = w.tau * tau_grow_factor
    nsel = driver.selections(state.options.init_pop)
    st = None
    for it in range(max_steps):
        st = state.ccmc_step(tau, 0.0, nsel)
        nsel = driver.selections(st["n_total"])
        if it % 200 == 0:
            log(f"grow step {it}: N_tot {st['n_total']:.3e} excitors {st['n_excitors']}")
        if st["n_total"] >= w.target_population:
            return st, it + 1
    return st, max_steps


def run_leg(w: inputs.Workload, precision: str, steps: int, warmup: int, log, profile: bool = True,
            load_state: str | None = None, save_state: str | None = None, breakdown_steps: int = 20):
    state = make_state(w, precision, init_pop=max(100.0, w.target_population / 50))
    if load_state:
        z = np.load(load_state)
        state.ccmc_import(z["keys"], z["amps"], float(z["n_ref"]), int(z["step"]))
        st = {"n_total": float(np.abs(z["amps"]).sum() + abs(float(z["n_ref"])))}
        ngrow = 0
        shift0 = float(z["shift"])
    else:
        st, ngrow = grow(state, w, log)
        shift0 = 0.0
    # population control from here on in the library's own step loop (ccmc_run): the shift
    # varies from the first step, as driver.ShiftControl would once started at this N_tot
    ctl = ccmc.ccmc_shift_control.new(w.target_population, shift=shift0, started_at=st["n_total"])
    nsel = driver.selections(st["n_total"])

    def run(k):
        nonlocal st, nsel
        out, nsel = state.ccmc_run(k, w.tau, ctl, nsel)
        if k:
            st = out[k - 1].as_dict()
        return out

    def totals(out, k):
        return (sum(out[i].n_spawn_attempts for i in range(k)), sum(out[i].n_selections for i in range(k)),
                sum(out[i].n_spawns for i in range(k)))

    run(warmup)
    if save_state:
        keys, amps, n0, step = state.ccmc_export()
        np.savez(save_state, keys=keys, amps=amps, n_ref=n0, step=step, shift=ctl.shift)

    # per-kernel breakdown: every launch timed with events (not the timed region)
    breakdown = {}
    dominant = None
    if profile:
        state.ccmc_profile("*")
        run(min(steps, breakdown_steps))
        breakdown = state.ccmc_profile_read()
        state.ccmc_profile(None)
        dominant = max(breakdown.items(), key=lambda kv: kv[1]["ms"])[0]
    # the timed region: only the dominant kernel carries events
    if dominant:
        state.ccmc_profile(dominant)
        state.ccmc_profile_read()
    ROCTX.resume()
    t0 = time.perf_counter()
    out = run(steps)
    elapsed = time.perf_counter() - t0
    attempts, selections, spawns = totals(out, steps)
    ROCTX.pause()
    timed = state.ccmc_profile_read() if dominant else {}
    state.ccmc_profile(None)
    keys, amps, n0, step = state.ccmc_export()
    out = dict(attempts=attempts, selections=selections, spawns=spawns, seconds=elapsed, grow_steps=ngrow,
               n_total=st["n_total"], n_ref=st["n_ref"], excitors=st["n_excitors"], shift=ctl.shift,
               profile=breakdown, timed=timed, memory=state.ccmc_memory())
    state.close()
    return out


def source_hash() -> str:
    """SHA-256 of the HIP sources and the C ABI header: counter figures taken on other
    sources do not describe the kernels that run now."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1807_03749_amd", "csrc")
    for f in sorted(os.listdir(csrc)) + ["../../include/ccmc.h"]:
        path = os.path.normpath(os.path.join(csrc, f))
        if path.endswith((".h", ".hip")):
            with open(path, "rb") as fh:
                h.update(os.path.basename(path).encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/<kernel>_<workload>_traffic.txt: FETCH_SIZE and WRITE_SIZE per dispatch,
    scaled by the same counters on a copy of known size), or None when the summary is
    missing or was taken on other sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for ln in f:
            if "=" in ln and not ln.lstrip().startswith("#"):
                k, v = ln.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def roofline(timed: dict, w: inputs.Workload):
    """Roofline entry for the dominant kernel, from its HIP-event durations in the timed
    region.  generate and items are bound by the vector ALUs: their algorithmic work is the
    integer and FP operations of one spawning attempt (OPS_PER_ATTEMPT) or one item
    (OPS_PER_ITEM); every other kernel is priced by its algorithmic HBM bytes against the
    8 TB/s peak."""
    if not timed:
        return None
    name, p = max(timed.items(), key=lambda kv: kv[1]["ms"])
    avg_s = p["ms"] / p["launches"] / 1e3
    if name in ALU_KERNELS:
        unit, ops_of = ALU_KERNELS[name]
        ops = ops_of(w)
        achieved = p["items"] / p["launches"] * ops / avg_s / 1e9
        r = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_GOPS, "unit": "Gop/s",
             f"ops_per_{unit}": ops, f"{unit}s_per_launch": p["items"] / p["launches"]}
    else:
        achieved = p["bytes"] / p["launches"] / avg_s / 1e9
        r = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s")
    r.update(frac=r["achieved"] / r["peak"], traffic=measured_traffic(name, w.name), kernel=name,
             launches=p["launches"], avg_ms=p["ms"] / p["launches"],
             algorithmic_bytes_per_launch=p["bytes"] / p["launches"])
    return r


ANNIHILATION = ("gather", "radix_ghist", "radix_onesweep", "seg_fold", "seg_close", "merge")


def annihilation_roofline(prof: dict):
    """Algorithmic HBM bandwidth of the annihilation kernels (sort, fold, merge, rounding,
    compaction) taken together, from the per-kernel breakdown."""
    names = [n for n in ANNIHILATION if n in prof]
    ms = sum(prof[n]["ms"] for n in names)
    by = sum(prof[n]["bytes"] for n in names)
    if ms <= 0:
        return None
    return dict(kernels=names, ms=ms, bytes=by, achieved=by / (ms / 1e3) / 1e9, peak=HBM_PEAK_GBS,
                unit="GB/s", frac=by / (ms / 1e3) / 1e9 / HBM_PEAK_GBS)


def precision_study(w: inputs.Workload, steps: int, equil: int, log):
    """FP64 against FP32 amplitudes at equal E_proj error: each precision grows its own
    population, equilibrates for `equil` steps under shift control, then records the E_proj
    terms of `steps` steps.  Reblocked E_proj and its standard error give the FP32 shift in
    units of the combined error, and -- since the error falls as 1/sqrt(time) -- the time each
    precision needs to reach the larger of the two errors."""
    res = {}
    for prec in ("fp64", "fp32"):
        state = make_state(w, prec, init_pop=max(100.0, w.target_population / 50))
        st, ngrow = grow(state, w, log)
        ctl = driver.ShiftControl(target=w.target_population, tau=w.tau)
        ctl.update(st["n_total"])
        nsel = driver.selections(st["n_total"])
        for _ in range(equil):
            st = state.ccmc_step(w.tau, ctl.shift, nsel)
            ctl.update(st["n_total"])
            nsel = driver.selections(st["n_total"])
        num = np.empty(steps)
        den = np.empty(steps)
        shifts = np.empty(steps)
        attempts = 0
        t0 = time.perf_counter()
        for i in range(steps):
            shifts[i] = ctl.shift
            st = state.ccmc_step(w.tau, ctl.shift, nsel)
            ctl.update(st["n_total"])
            nsel = driver.selections(st["n_total"])
            num[i] = st["eproj_num"]
            den[i] = st["eproj_den"]
            attempts += st["n_spawn_attempts"]
        el = time.perf_counter() - t0
        e, err, lv = driver.reblock_ratio(num, den)
        # population-control check: E(K) reweighted over the last K steps
        rw = driver.reweight(num, den, shifts, w.tau, memories=(0, 50, 200, 1000, 4000))
        res[prec] = dict(e_proj=e, error=err, block_level=lv, steps=steps, seconds=el,
                         attempts_per_s=attempts / el, ms_per_step=1e3 * el / steps, shift=ctl.shift,
                         n_total=st["n_total"], excitors=st["n_excitors"],
                         reweighted=[dict(memory=k, e_proj=x, error=y) for k, x, y in rw])
        log(f"precision {prec}: E_proj {e:.6f} +- {err:.6f} ({steps} steps, {1e3 * el / steps:.3f} ms/step)")
        state.close()
    a, b = res["fp64"], res["fp32"]
    comb = math.sqrt(a["error"] ** 2 + b["error"] ** 2)
    target = max(a["error"], b["error"])
    t = {p: res[p]["seconds"] * (res[p]["error"] / target) ** 2 for p in res}
    return dict(workload=w.name, equilibration_steps=equil, fp64=a, fp32=b,
                fp32_shift_in_sigma=(b["e_proj"] - a["e_proj"]) / comb if comb > 0 else None,
                equal_error=target, seconds_to_equal_error=t,
                fp32_speedup_at_equal_error=t["fp64"] / t["fp32"] if t["fp32"] > 0 else None)


def serving_benchmark(n_requests: int, max_steps: int, tol: float, budget: float, slots: int, log):
    """The served stream: Poisson arrivals (mean 2/s) of UEG 14-electron solves with FP32
    amplitudes and FP64 energy reductions, admitted by HBM budget and stepped together in
    shared launches until each one's reblocked E_proj error is below `tol` (or `max_steps`)."""
    from paper_1807_03749_amd import serve
    reqs = serve.requests_from_stream(inputs.serving_stream(n_requests), precision="fp32")
    srv = serve.Server(hbm_budget=budget, max_active=slots, tol=tol, max_steps=max_steps, log=log)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    wall = time.perf_counter() - t0
    out = serve.summary(res, wall)
    out.update(batch_steps=srv.batch_steps, state_steps=srv.state_steps, max_steps=max_steps, tol=tol,
               hbm_budget=budget, slots=slots,
               per_request=[dict(id=r.request_id, arrival=round(r.arrival, 3), tte=round(r.time_to_energy, 3),
                                 steps=r.steps, e=r.energy, err=r.error, ok=r.converged,
                                 **({"failed": r.failed} if r.failed else {}),
                                 **({"grown": r.grown} if r.grown else {})) for r in res])
    return out


def cpu_baseline(w: inputs.Workload, seconds: float, log):
    """The CPU oracle, timed on this host on a bounded sample of the same workload: the
    whole truncated space occupied with seeded amplitudes (N_tot = target), stepped until
    `seconds` of CPU time have passed."""
    from oracle import binding as orc  # CPU baseline leg only
    import itertools

    if w.system != "ueg":
        return None
    S = orc.System.ueg(w.n_electrons, w.n2_max, w.rs)
    nv = S.nvec()
    N, M = S.n_el, S.M
    dets = []
    for L in range(1, w.truncation + 1):
        table = {}
        for parts in itertools.combinations(range(N, M), L):
            key = (tuple(int(x) for x in sum(nv[p >> 1] for p in parts)), sum(1 for p in parts if p % 2 == 0))
            table.setdefault(key, []).append(parts)
        for holes in itertools.combinations(range(N), L):
            key = (tuple(int(x) for x in sum(nv[p >> 1] for p in holes)), sum(1 for p in holes if p % 2 == 0))
            for parts in table.get(key, []):
                v = (1 << N) - 1
                for i in holes:
                    v ^= 1 << i
                for a in parts:
                    v |= 1 << a
                dets.append(v)
    dets.sort()
    levels = np.array([bin(d >> N).count("1") for d in dets])
    n0 = 0.2 * w.target_population
    amps = inputs.state_amplitudes(levels, target=0.8 * w.target_population, seed=1)
    keys = np.array([[(d >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(S.W)] for d in dets], dtype=np.uint64)
    R = orc.Run(S, w.truncation, orc.RunOptions(full_noncomposite=w.full_noncomposite,
                                                 min_spawn_attempts=w.min_spawn_attempts,
                                                 multispawn_threshold=w.multispawn_threshold,
                                                 noncomposite_threshold=w.noncomposite_threshold, seed=w.seed))
    R.import_state(keys, amps, n0, 0)
    nsel = driver.selections(np.abs(amps).sum() + n0)
    attempts, steps = 0, 0
    t0 = time.process_time()
    while time.process_time() - t0 < seconds:
        st = R.step(w.tau, 0.0, nsel)
        attempts += st["n_spawn_attempts"]
        nsel = driver.selections(st["n_total"])
        steps += 1
    el = time.process_time() - t0
    log(f"cpu oracle: {steps} steps, {attempts} attempts in {el:.1f} s")
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    cpu = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(value=attempts / el, unit="attempts/s", cores=1, kind="oracle",
                sample=f"{steps} serial FP64 oracle steps of {w.name} from a store holding the whole truncated "
                       f"space ({len(keys)} excitors, N_tot {w.target_population:.0e}) on {cpu}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="ueg14_114_ccsdt_fnc", choices=sorted(inputs.WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--roctx-region", action="store_true",
                    help="mark the timed steps for a profiler run with --selected-regions")
    ap.add_argument("--no-kernel-timing", action="store_true", help="no HIP-event timing in the timed region")
    ap.add_argument("--calibrate-copy", action="store_true", help="only run a 1 GiB device copy (counter scaling)")
    ap.add_argument("--save-state", help="write the equilibrated store (after warm-up) to this .npz")
    ap.add_argument("--load-state", help="start from a store written by --save-state instead of growing one")
    ap.add_argument("--study-steps", type=int, default=50000,
                    help="steps per precision of the FP64 / FP32 equal-error study (0: skip)")
    ap.add_argument("--study-equil", type=int, default=4000, help="equilibration steps before the study")
    ap.add_argument("--serve", action="store_true", help="also run the served stream (continuous batching)")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-max-steps", type=int, default=20000)
    ap.add_argument("--serve-tol", type=float, default=1e-4)
    ap.add_argument("--serve-budget", type=float, default=64e9, help="HBM budget of the server (bytes)")
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--serve-only", action="store_true", help="only the served stream")
    ap.add_argument("--n-ranks", type=int, default=1,
                    help="virtual processors of eq. 9 (selection restricted to one processor's excitors)")
    ap.add_argument("--move-shift", type=int, default=5, help="nu_move of the virtual processors")
    args = ap.parse_args()
    global ROCTX
    ROCTX = _Roctx(args.roctx_region)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: the library steps a population on one GPU "
              f"(sharding over several GPUs is designed but not implemented)", file=sys.stderr)
        sys.exit(2)
    log = (lambda m: None) if args.quiet else (lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
    VIRTUAL.update(n_ranks=args.n_ranks, move_shift=args.move_shift)
    if args.serve_only:
        sv = serving_benchmark(args.serve_requests, args.serve_max_steps, args.serve_tol, args.serve_budget,
                               args.serve_slots, log)
        print(json.dumps({"metric": "served CCMC solves: time to energy", "serving": sv}))
        return
    w = inputs.WORKLOADS[args.workload]
    log(f"workload {w.name} precision {args.precision}: growing to {w.target_population:.0e}")
    main_leg = run_leg(w, args.precision, args.steps, args.warmup, log, profile=not args.no_kernel_timing,
                       load_state=args.load_state, save_state=args.save_state)
    value = main_leg["attempts"] / main_leg["seconds"]
    log(f"{args.precision}: {value:.4e} attempts/s, {1e3 * main_leg['seconds'] / args.steps:.3f} ms/step")
    prof = main_leg["profile"]
    for k, p in sorted(prof.items(), key=lambda kv: -kv[1]["ms"]):
        log(f"  {k:16s} {p['ms'] / max(p['launches'], 1):8.4f} ms avg  x{p['launches']}")
    nb = max(1, prof.get("gather", {}).get("launches", 0))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * main_leg["seconds"] / args.steps,
        "selections_per_s": main_leg["selections"] / main_leg["seconds"],
        "spawns_per_s": main_leg["spawns"] / main_leg["seconds"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic (analytic UEG; population grown from the reference on the GPU)",
        "config": {"workload": w.name, "system": w.system, "electrons": w.n_electrons,
                   "spin_orbitals": w.n_spin_orbitals, "truncation": w.truncation, "tau": w.tau,
                   "target_population": w.target_population, "full_noncomposite": w.full_noncomposite,
                   "min_spawn_attempts": w.min_spawn_attempts, "excitors": main_leg["excitors"],
                   "n_total": main_leg["n_total"], "selections_per_step": main_leg["selections"] / args.steps,
                   "spawns_per_step": main_leg["spawns"] / args.steps,
                   "records_per_step": prof.get("gather", {}).get("items", 0) / nb, "parallelism": "1 GPU",
                   **({"virtual_processors": args.n_ranks, "move_shift": args.move_shift} if args.n_ranks > 1 else {})},
        "roofline": roofline(main_leg["timed"], w),
        "annihilation_roofline": annihilation_roofline(prof),
        "kernels": {k: dict(avg_ms=p["ms"] / max(p["launches"], 1), launches=p["launches"],
                            items_per_launch=p["items"] / max(p["launches"], 1),
                            bytes_per_launch=p["bytes"] / max(p["launches"], 1),
                            share=p["ms"] / max(1e-9, sum(q["ms"] for q in prof.values())))
                    for k, p in prof.items()},
        "breakdown_note": "per-kernel figures from a separate pass with every launch timed by HIP events; "
                          "the timed region carries events on the dominant kernel only",
        "device_memory_bytes": main_leg["memory"],
    }
    if not args.no_fp32 and args.precision == "fp64":
        log("fp32 leg")
        f32 = run_leg(w, "fp32", args.steps, args.warmup, log, profile=False)
        out["fp32"] = dict(value=f32["attempts"] / f32["seconds"], ms_per_step=1e3 * f32["seconds"] / args.steps,
                           excitors=f32["excitors"], n_total=f32["n_total"])
    if args.study_steps > 0 and args.precision == "fp64" and not args.no_fp32:
        log("precision study")
        out["precision_study"] = precision_study(w, args.study_steps, args.study_equil, log)
    if args.serve:
        log("served stream")
        out["serving"] = serving_benchmark(args.serve_requests, args.serve_max_steps, args.serve_tol,
                                           args.serve_budget, args.serve_slots, log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, log)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
