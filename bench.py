#!/usr/bin/env python3
"""CCMC step throughput on one MI355X: cluster spawn attempts per second.

Workload of the headline value: 3D uniform electron gas, 14 electrons in 114 spin orbitals
(57 plane waves, |n|^2 <= 5, two 64-bit bitstring words), r_s = 1, CCSDT, full non-composite
sampling, at least 4 spawning attempts per cluster (multi-spawn threshold 1), tau = 0.002,
target population 1e6, FP64.  Synthetic and analytic: there is no dataset.

Procedure of every leg: grow the population from the reference with the shift held at zero
until it reaches the target, hand over to population control, run the warm-up steps, then
time exactly the leg's steps (each a full ccmc_step: selection, spawning, death and
annihilation).  Inputs stay resident on the GPU throughout.  Kernel times come from HIP
events recorded by the library on its own stream.

Beside the headline leg the JSON line carries the FP32 leg of the same workload, the other
single-GPU workloads as `legs` (14e/38so CCSD FP64; the 16e/92so molecule-like CCSDTQ FP32;
54e/246so CCSD FP32 at 1e8), the FP32-against-FP64 study over independent replicas, the
14e/38so check against the oracle's stored long run and deterministic CCSD, the served
stream, and the CPU oracle's rate.

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
# 32-bit vector ALU lane operations: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78.6 T lane-ops/s,
# the published FP32 vector rate (157.3 TFLOP/s) with an FMA counted as one operation.  The
# counters show the kernels here issuing more than 16 lane operations per SIMD and cycle (the
# molecule-like generator: 41.6 T lane-ops/s executed), so a 16-lane peak would be exceeded.
ALU_PEAK_GOPS = 256 * 4 * 32 * 2.4
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


def make_state(w: inputs.Workload, precision: str, init_pop: float, seed: int | None = None):
    kw = dict(precision=precision, full_noncomposite=int(w.full_noncomposite),
              min_spawn_attempts=w.min_spawn_attempts, multispawn_threshold=w.multispawn_threshold,
              noncomposite_threshold=w.noncomposite_threshold, init_pop=init_pop,
              seed=w.seed if seed is None else seed, **VIRTUAL)
    if w.system == "ueg":
        return ccmc.State("ueg", w.n_electrons, w.truncation, n2_max=w.n2_max, rs=w.rs, **kw)
    h, B = inputs.molecule_like(n_spatial=w.n_spatial, n_electrons=w.n_electrons, n_chol=w.n_chol)
    return ccmc.State("mol", w.n_electrons, w.truncation, h=h, chol=B, **kw)


def grow(state, w: inputs.Workload, log, max_steps: int = 20000, tau_grow_factor: float | None = None):
    """Shift held at zero (E_HF) until N_tot reaches the target.  Returns the last step's
    statistics, the number of growth steps, the N_tot series and the growth time step."""
    f = tau_grow_factor if tau_grow_factor is not None else float(w.extra.get("grow_factor", 5.0))
    tau = w.tau * f
    nsel = driver.selections(state.options.init_pop)
    st, hist = None, []
    for it in range(max_steps):
        st = state.ccmc_step(tau, 0.0, nsel)
        hist.append(st["n_total"])
        nsel = driver.selections(st["n_total"])
        if it % 200 == 0:
            log(f"grow step {it}: N_tot {st['n_total']:.3e} excitors {st['n_excitors']}")
        if st["n_total"] >= w.target_population:
            return st, it + 1, hist, tau
    return st, max_steps, hist, tau


def start_shift(w: inputs.Workload, hist: list, tau_grow: float) -> float:
    """The shift that population control starts from.  0 (E_HF) by default; for a workload
    whose growth rate at the target is far from zero (shift_from_growth), the growth rate of
    the last growth steps at the shift 0, -ln(N_t / N_{t-k}) / (k tau), so that the control
    does not have to catch up with the whole of it."""
    if not w.extra.get("shift_from_growth"):
        return 0.0
    k = min(5, len(hist) - 1)
    return -math.log(hist[-1] / hist[-1 - k]) / (k * tau_grow) if k > 0 else 0.0


def run_leg(w: inputs.Workload, precision: str, steps: int, warmup: int, log, profile: bool = True,
            load_state: str | None = None, save_state: str | None = None, breakdown_steps: int = 20):
    """Grow, hand over to population control, warm up, then time `steps` steps.

    Population control is the library's log-growth update (damping 0.05 every 10 steps),
    started at the step that reached the target from start_shift().  A workload below its
    shoulder (control_damping) keeps a damping of 0.5 throughout: its reference population
    decays while its growth rate drifts, and the weak default control would let the total
    population run away from the target (Sec. IV.A)."""
    state = make_state(w, precision, init_pop=max(100.0, w.target_population / 50))
    shoulder = driver.Shoulder()
    if load_state:
        ck = driver.load_checkpoint(load_state)
        ctl, nsel, _ = driver.resume(state, ck)
        st = {"n_total": float(np.abs(ck["amps"]).sum() + abs(ck["n_ref"])), "n_ref": ck["n_ref"]}
        ngrow, shift0 = 0, float(ctl.shift)
    else:
        st, ngrow, hist, tau_g = grow(state, w, log)
        shift0 = start_shift(w, hist, tau_g)
        ctl = ccmc.ccmc_shift_control.new(w.target_population, shift=shift0, started_at=st["n_total"])
        nsel = driver.selections(st["n_total"])
    shoulder.update(st["n_total"], st["n_ref"])
    ctl.damping = float(w.extra.get("control_damping", ctl.damping))

    def run(k):
        nonlocal st, nsel
        out, nsel = state.ccmc_run(k, w.tau, ctl, nsel)
        for i in range(k):
            shoulder.update(out[i].n_total, out[i].n_ref)
        if k:
            st = out[k - 1].as_dict()
        return out

    def totals(out, k):
        return (sum(out[i].n_spawn_attempts for i in range(k)), sum(out[i].n_selections for i in range(k)),
                sum(out[i].n_spawns for i in range(k)))

    run(warmup)
    if save_state:
        driver.save_checkpoint(save_state, state, ctl, nsel)

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
    n_start = st["n_total"]
    ROCTX.resume()
    t0 = time.perf_counter()
    out = run(steps)
    elapsed = time.perf_counter() - t0
    attempts, selections, spawns = totals(out, steps)
    ROCTX.pause()
    timed = state.ccmc_profile_read() if dominant else {}
    state.ccmc_profile(None)
    res = dict(attempts=attempts, selections=selections, spawns=spawns, seconds=elapsed, grow_steps=ngrow,
               control_damping=ctl.damping, start_shift=shift0, n_total=st["n_total"], n_total_at_start=n_start,
               n_ref=st["n_ref"], excitors=st["n_excitors"], shift=ctl.shift, shoulder=shoulder.as_dict(),
               profile=breakdown, timed=timed, memory=state.ccmc_memory())
    state.close()
    return res


def leg_record(w: inputs.Workload, precision: str, res: dict, steps: int, warmup: int) -> dict:
    """One leg's figures: throughput, population and the rooflines of its kernels."""
    prof = res["profile"]
    nb = max(1, prof.get("gather", {}).get("launches", 0))
    return dict(
        value=res["attempts"] / res["seconds"], unit="attempts/s", steps=steps, warmup=warmup,
        ms_per_step=1e3 * res["seconds"] / steps, selections_per_s=res["selections"] / res["seconds"],
        spawns_per_s=res["spawns"] / res["seconds"], dtype="f64" if precision == "fp64" else "f32",
        config={"workload": w.name, "system": w.system, "electrons": w.n_electrons,
                "spin_orbitals": w.n_spin_orbitals, "truncation": w.truncation, "tau": w.tau,
                "target_population": w.target_population, "full_noncomposite": w.full_noncomposite,
                "min_spawn_attempts": w.min_spawn_attempts, "precision": precision},
        population=dict(n_total=res["n_total"], n_total_at_start=res["n_total_at_start"], n_ref=res["n_ref"],
                        excitors=res["excitors"], shift=res["shift"], start_shift=res["start_shift"],
                        grow_steps=res["grow_steps"], control_damping=res["control_damping"],
                        within_20pct_of_target=bool(abs(res["n_total"] / w.target_population - 1) <= 0.2),
                        shoulder=res["shoulder"]),
        attempts_per_step=res["attempts"] / steps, records_per_step=prof.get("gather", {}).get("items", 0) / nb,
        roofline=roofline(res["timed"], w), annihilation_roofline=annihilation_roofline(prof, w),
        kernels={k: dict(avg_ms=p["ms"] / max(p["launches"], 1), launches=p["launches"],
                         items_per_launch=p["items"] / max(p["launches"], 1),
                         bytes_per_launch=p["bytes"] / max(p["launches"], 1)) for k, p in prof.items()},
        device_memory_bytes=res["memory"])


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


def measured_traffic(kernel: str, workload: str, key: str = "hbm_bytes_per_launch"):
    """HBM bytes per launch of `kernel` (or per step of a kernel group such as
    "annihilation", key hbm_bytes_per_step) from the committed counter summary
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
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def measured_valu(kernel: str, workload: str):
    """Vector-ALU counters of `kernel` on `workload` from the committed summary
    (profiles/valu_<workload>.txt: SQ_WAVES and SQ_INSTS_VALU per dispatch over the timed
    steps), or None when the summary is missing or was taken on other sources."""
    path = os.path.join(ROOT, "profiles", f"valu_{workload}.txt")
    if not os.path.exists(path):
        return None
    rows, src = {}, None
    with open(path) as f:
        for ln in f:
            if ln.startswith("source_hash"):
                src = ln.split("=", 1)[1].strip()
            elif ln.startswith("  k_"):
                parts = ln.split()
                rows[parts[0].rstrip("<")] = dict(waves=float(parts[2]), insts=float(parts[3]),
                                                  busy=float(parts[4].rstrip("%")) / 100.0)
    if src != source_hash():
        return None
    return rows.get(f"k_{kernel}")


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
        m = measured_valu(name, w.name)
        if m:  # the executed VALU instructions (64 lane operations each) over the same duration
            lane_ops = m["waves"] * m["insts"] * 64.0
            r["measured_valu"] = dict(waves_per_launch=m["waves"], valu_insts_per_wave=m["insts"],
                                      lane_ops_per_launch=lane_ops, achieved=lane_ops / avg_s / 1e9,
                                      frac=lane_ops / avg_s / 1e9 / ALU_PEAK_GOPS, valu_busy=m["busy"])
    else:
        achieved = p["bytes"] / p["launches"] / avg_s / 1e9
        r = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s")
    r.update(frac=r["achieved"] / r["peak"], traffic=measured_traffic(name, w.name), kernel=name,
             launches=p["launches"], avg_ms=p["ms"] / p["launches"],
             algorithmic_bytes_per_launch=p["bytes"] / p["launches"])
    return r


ANNIHILATION = ("gather", "radix_ghist", "radix_onesweep", "seg_fold", "seg_close", "merge")


def annihilation_roofline(prof: dict, w: inputs.Workload | None = None):
    """Algorithmic HBM bandwidth of the annihilation kernels (sort, fold, merge, rounding,
    compaction) taken together, from the per-kernel breakdown; with the committed counter
    summary of the workload (profiles/annihilation_<workload>_traffic.txt, per step), also
    the measured HBM bytes per step and the bandwidth they give over the same kernel time."""
    names = [n for n in ANNIHILATION if n in prof]
    ms = sum(prof[n]["ms"] for n in names)
    by = sum(prof[n]["bytes"] for n in names)
    if ms <= 0:
        return None
    steps = max(1, prof.get("gather", {}).get("launches", 1))
    out = dict(kernels=names, ms_per_step=ms / steps, bytes_per_step=by / steps, achieved=by / (ms / 1e3) / 1e9,
               peak=HBM_PEAK_GBS, unit="GB/s", frac=by / (ms / 1e3) / 1e9 / HBM_PEAK_GBS)
    t = measured_traffic("annihilation", w.name, "hbm_bytes_per_step") if w is not None else None
    out["traffic_per_step"] = t
    if t is not None:
        gbs = t / (ms / steps / 1e3) / 1e9
        out.update(measured_gbs=gbs, measured_frac=gbs / HBM_PEAK_GBS)
    return out


def replica_runs(w: inputs.Workload, precision: str, replicas: int, steps: int, equil: int, log):
    """`replicas` independent solves (Philox keys seed + 7919 (r + 1)) of workload w stepped
    together in shared launches (ccmc_step_batch): each grows at 5 tau with the shift at 0 to
    the target, then runs under its own population control (damping 0.05 every 10 steps) for
    `equil` steps and records the projected-energy terms of `steps` steps.  Returns each
    replica's reblocked E_proj and error, and the series' shifts for the reweighting."""
    init = max(100.0, w.target_population / 50)
    states = [make_state(w, precision, init_pop=init, seed=w.seed + 7919 * (r + 1)) for r in range(replicas)]
    R = len(states)
    nsel = [driver.selections(init)] * R
    ctl = [driver.ShiftControl(target=w.target_population, tau=w.tau) for _ in range(R)]
    phase = [0] * R  # 0 growing, then the number of steps under control
    num = [[] for _ in range(R)]
    den = [[] for _ in range(R)]
    shifts = [[] for _ in range(R)]
    attempts = 0
    t0 = time.perf_counter()
    for it in range(200000):
        live = [r for r in range(R) if phase[r] < equil + steps]
        if not live:
            break
        taus = [w.tau * (5.0 if phase[r] == 0 else 1.0) for r in live]
        res = ccmc.ccmc_step_batch([states[r] for r in live], taus, [ctl[r].shift if phase[r] else 0.0 for r in live],
                                   [nsel[r] for r in live])
        for r, st in zip(live, res):
            if isinstance(st, Exception):
                raise st
            attempts += st["n_spawn_attempts"]
            nsel[r] = driver.selections(st["n_total"])
            if phase[r] == 0:
                if st["n_total"] >= w.target_population:
                    ctl[r].update(st["n_total"])
                    phase[r] = 1
                continue
            if phase[r] > equil:
                num[r].append(st["eproj_num"])
                den[r].append(st["eproj_den"])
                shifts[r].append(ctl[r].shift)
            ctl[r].update(st["n_total"])
            phase[r] += 1
    el = time.perf_counter() - t0
    out = []
    for r in range(R):
        e, err, lv = driver.reblock_ratio(np.array(num[r]), np.array(den[r]))
        out.append(dict(e_proj=e, error=err, block_level=lv))
        states[r].close()
    log(f"{w.name} {precision}: {R} replicas x {steps} steps in {el:.1f} s")
    return out, dict(seconds=el, attempts=attempts, shifts=shifts, num=num, den=den)


def combine_replicas(reps: list) -> dict:
    """Mean E_proj of independent replicas, its standard error from their scatter, and the
    mean of their own (reblocked) squared errors."""
    es = np.array([r["e_proj"] for r in reps])
    ers = np.array([r["error"] for r in reps])
    return dict(e_proj=float(es.mean()), sem=float(es.std(ddof=1) / math.sqrt(len(es))),
                mean_reblocked_error=float(ers.mean()), mean_reblocked_var=float((ers ** 2).mean()),
                replicas=[dict(e_proj=float(e), error=float(x)) for e, x in zip(es, ers)])


def precision_study(w: inputs.Workload, replicas: int, steps: int, equil: int, ms_per_step: dict, log):
    """FP32 against FP64 amplitudes over independent replicas of each (every replica its own
    Philox key and population): the FP32 shift of E_proj in units of the combined standard
    error (from the replicas' scatter), and the time each precision needs to reach an equal
    error.  One solve's time to an error eps is ms_per_step x var_1 / eps^2, with var_1 the
    variance one step contributes (R steps x error^2 of a replica); the ratio of the two times
    is the ratio of the single-solve step times (from the timed legs) times the ratio of the
    replicas' squared errors.  Its 95% interval comes from the F distribution of the ratio of
    the replicas' sample variances, and from a bootstrap over the replicas' reblocked errors."""
    from scipy import stats as sps

    res, raw = {}, {}
    for prec in ("fp64", "fp32"):
        reps, raw[prec] = replica_runs(w, prec, replicas, steps, equil, log)
        res[prec] = combine_replicas(reps)
        res[prec]["steps_per_replica"] = steps
        res[prec]["seconds"] = raw[prec]["seconds"]
        # population-control check on the pooled series: E(K) reweighted over the last K steps
        rw = [driver.reweight(np.array(raw[prec]["num"][r]), np.array(raw[prec]["den"][r]),
                              np.array(raw[prec]["shifts"][r]), w.tau, memories=(0, 200, 1000))
              for r in range(replicas)]
        res[prec]["reweighted_mean"] = [dict(memory=rw[0][i][0], e_proj=float(np.mean([x[i][1] for x in rw])))
                                        for i in range(len(rw[0]))]
        log(f"precision {prec}: E_proj {res[prec]['e_proj']:.6f} +- {res[prec]['sem']:.6f} (replica scatter), "
            f"mean reblocked error {res[prec]['mean_reblocked_error']:.2e}")
    a, b = res["fp64"], res["fp32"]
    comb = math.sqrt(a["sem"] ** 2 + b["sem"] ** 2)
    shift_sigma = (b["e_proj"] - a["e_proj"]) / comb if comb > 0 else None
    t_ratio = ms_per_step["fp64"] / ms_per_step["fp32"]
    var_ratio = a["sem"] ** 2 / b["sem"] ** 2  # replica scatter: F(R-1, R-1)
    d = replicas - 1
    f_lo, f_hi = sps.f.ppf(0.025, d, d), sps.f.ppf(0.975, d, d)
    ea = np.array([r["error"] for r in a["replicas"]]) ** 2
    eb = np.array([r["error"] for r in b["replicas"]]) ** 2
    rng = np.random.default_rng(5)
    boot = [ea[rng.integers(0, replicas, replicas)].mean() / eb[rng.integers(0, replicas, replicas)].mean()
            for _ in range(4000)]
    speed = dict(
        step_time_ratio_fp64_over_fp32=t_ratio,
        from_replica_scatter=dict(ratio=t_ratio * var_ratio, ci95=[t_ratio * var_ratio / f_hi, t_ratio * var_ratio / f_lo]),
        from_reblocked_errors=dict(ratio=t_ratio * ea.mean() / eb.mean(),
                                   ci95=[float(t_ratio * np.percentile(boot, 2.5)), float(t_ratio * np.percentile(boot, 97.5))]))
    lo, hi = speed["from_reblocked_errors"]["ci95"]
    verdict = ("FP32 reaches an equal error faster" if lo > 1 else
               "FP64 reaches an equal error faster" if hi < 1 else "no difference in time to equal error resolved")
    return dict(workload=w.name, replicas=replicas, steps_per_replica=steps, equilibration_steps=equil,
                fp64=a, fp32=b, fp32_shift_in_sigma=shift_sigma, within_one_sigma=bool(abs(shift_sigma) <= 1.0),
                ms_per_step=ms_per_step, fp64_over_fp32_time_to_equal_error=speed, conclusion=verdict)


def stored_long_run(path: str = os.path.join(ROOT, "tests", "golden", "ueg14_38_ccsd_longrun.txt")):
    """The oracle's long-run energy of 14e/38so CCSD and the deterministic CCSD energy, as
    stored by the script beside the file (a text file: nothing of the oracle runs here)."""
    if not os.path.exists(path):
        return None
    mean = sem = e_ccsd = None
    with open(path) as f:
        for ln in f:
            if ln.startswith("# mean"):
                parts = ln.split()
                mean, sem = float(parts[2]), float(parts[4])
            elif ln.startswith("# deterministic_ccsd"):
                e_ccsd = float(ln.split()[2])
    return dict(oracle_mean=mean, oracle_sem=sem, deterministic_ccsd=e_ccsd)


def oracle_energy_check(replicas: int, steps: int, equil: int, log):
    """14e/38so CCSD (the 289-determinant space): FP64 and FP32 replicas on the GPU against the
    oracle's own stored long run and the deterministic projective CCSD energy."""
    w = inputs.WORKLOADS["ueg14_38_ccsd_fp64"]
    ref = stored_long_run()
    out = dict(workload=w.name, replicas=replicas, steps_per_replica=steps, reference=ref)
    for prec in ("fp64", "fp32"):
        reps, raw = replica_runs(w, prec, replicas, steps, equil, log)
        c = combine_replicas(reps)
        c["seconds"] = raw["seconds"]
        if ref and ref["deterministic_ccsd"] is not None:
            c["minus_ccsd_in_sigma"] = (c["e_proj"] - ref["deterministic_ccsd"]) / c["sem"]
        if ref and ref["oracle_mean"] is not None:
            c["minus_oracle_in_sigma"] = (c["e_proj"] - ref["oracle_mean"]) / math.hypot(c["sem"], ref["oracle_sem"])
        out[prec] = c
        log(f"c1 check {prec}: E {c['e_proj']:.6f} +- {c['sem']:.6f}; "
            f"CCSD {ref['deterministic_ccsd'] if ref else None}")
    return out


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
    est = sorted(r.steps * (r.error / tol) ** 2 for r in res if r.outcome == "capped" and r.error == r.error)
    out["capped_steps_to_tol_median"] = float(np.median(est)) if est else None
    out.update(batch_steps=srv.batch_steps, state_steps=srv.state_steps, max_steps=max_steps, tol=tol,
               hbm_budget=budget, slots=slots,
               per_request=[dict(id=r.request_id, arrival=round(r.arrival, 3), tte=round(r.time_to_energy, 3),
                                 steps=r.steps, e=r.energy, err=r.error, outcome=r.outcome,
                                 shoulder=round(r.shoulder, 2),
                                 # a capped solve's error falls as 1/sqrt(steps): the steps it would need
                                 **({"steps_to_tol_estimate": round(r.steps * (r.error / tol) ** 2)}
                                    if r.outcome == "capped" and r.error == r.error else {}),
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


LEGS = ("ueg14_38_ccsd_fp64", "mol16_92_ccsdtq_fp32", "ueg54_246_ccsd_fp32")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="ueg14_114_ccsdt_fnc", choices=sorted(inputs.WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 leg and the precision study")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated other workloads measured beside the headline one ('' for none)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--roctx-region", action="store_true",
                    help="mark the timed steps for a profiler run with --selected-regions")
    ap.add_argument("--no-kernel-timing", action="store_true", help="no HIP-event timing in the timed region")
    ap.add_argument("--calibrate-copy", action="store_true", help="only run a 1 GiB device copy (counter scaling)")
    ap.add_argument("--save-state", help="write a checkpoint after the warm-up to this .npz")
    ap.add_argument("--load-state", help="start from a checkpoint written by --save-state instead of growing")
    ap.add_argument("--study-replicas", type=int, default=8, help="replicas per precision of the FP32/FP64 study")
    ap.add_argument("--study-steps", type=int, default=10000,
                    help="recorded steps per replica of the FP32/FP64 study (0: skip)")
    ap.add_argument("--study-equil", type=int, default=2000, help="equilibration steps before the study")
    ap.add_argument("--check-steps", type=int, default=12000,
                    help="recorded steps per replica of the 14e/38so check against the oracle (0: skip)")
    ap.add_argument("--no-serve", action="store_true", help="skip the served stream")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-max-steps", type=int, default=20000)
    ap.add_argument("--serve-tol", type=float, default=1e-4)
    ap.add_argument("--serve-budget", type=float, default=64e9, help="HBM budget of the server (bytes)")
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--serve-only", action="store_true", help="only the served stream")
    ap.add_argument("--legs-only", action="store_true", help="only the legs named by --legs (profiling runs)")
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
    legs = [x for x in args.legs.split(",") if x]
    if args.legs_only:
        out = {}
        for name in legs:
            lw = inputs.WORKLOADS[name]
            k, wu = int(lw.extra.get("bench_steps", args.steps)), int(lw.extra.get("bench_warmup", args.warmup))
            log(f"leg {name}")
            out[name] = leg_record(lw, lw.precision, run_leg(lw, lw.precision, k, wu, log), k, wu)
        print(json.dumps({"legs": out}))
        return
    w = inputs.WORKLOADS[args.workload]
    log(f"workload {w.name} precision {args.precision}: growing to {w.target_population:.0e}")
    main_leg = run_leg(w, args.precision, args.steps, args.warmup, log, profile=not args.no_kernel_timing,
                       load_state=args.load_state, save_state=args.save_state)
    rec = leg_record(w, args.precision, main_leg, args.steps, args.warmup)
    value = rec["value"]
    log(f"{args.precision}: {value:.4e} attempts/s, {rec['ms_per_step']:.3f} ms/step")
    prof = main_leg["profile"]
    for k, p in sorted(prof.items(), key=lambda kv: -kv[1]["ms"]):
        log(f"  {k:16s} {p['ms'] / max(p['launches'], 1):8.4f} ms avg  x{p['launches']}")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "selections_per_s": rec["selections_per_s"],
        "spawns_per_s": rec["spawns_per_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": rec["dtype"],
        "data": "synthetic (analytic UEG and seeded molecule-like integrals; populations grown on the GPU)",
        "config": dict(rec["config"], excitors=main_leg["excitors"], n_total=main_leg["n_total"],
                       selections_per_step=main_leg["selections"] / args.steps,
                       spawns_per_step=main_leg["spawns"] / args.steps, records_per_step=rec["records_per_step"],
                       parallelism="1 GPU",
                       **({"virtual_processors": args.n_ranks, "move_shift": args.move_shift}
                          if args.n_ranks > 1 else {})),
        "roofline": rec["roofline"],
        "annihilation_roofline": rec["annihilation_roofline"],
        "kernels": {k: dict(v, share=prof[k]["ms"] / max(1e-9, sum(q["ms"] for q in prof.values())))
                    for k, v in rec["kernels"].items()},
        "breakdown_note": "per-kernel figures from a separate pass with every launch timed by HIP events; "
                          "the timed region carries events on the dominant kernel only",
        "population": rec["population"],
        "device_memory_bytes": main_leg["memory"],
    }
    ms = {args.precision: rec["ms_per_step"]}
    if not args.no_fp32 and args.precision == "fp64":
        log("fp32 leg")
        f32 = run_leg(w, "fp32", args.steps, args.warmup, log, profile=False)
        out["fp32"] = dict(value=f32["attempts"] / f32["seconds"], ms_per_step=1e3 * f32["seconds"] / args.steps,
                           excitors=f32["excitors"], n_total=f32["n_total"])
        ms["fp32"] = out["fp32"]["ms_per_step"]
    if legs:
        out["legs"] = {}
        for name in legs:
            lw = inputs.WORKLOADS[name]
            k, wu = int(lw.extra.get("bench_steps", args.steps)), int(lw.extra.get("bench_warmup", args.warmup))
            log(f"leg {name} ({lw.precision}): {k} timed steps after {wu} warm-up")
            r = leg_record(lw, lw.precision, run_leg(lw, lw.precision, k, wu, log), k, wu)
            log(f"  {r['value']:.4e} attempts/s, {r['ms_per_step']:.3f} ms/step, N_tot {r['population']['n_total']:.3e}")
            out["legs"][name] = r
    if args.study_steps > 0 and args.precision == "fp64" and not args.no_fp32:
        log("precision study")
        out["precision_study"] = precision_study(w, args.study_replicas, args.study_steps, args.study_equil, ms, log)
    if args.check_steps > 0:
        log("14e/38so CCSD against the oracle's long run and the deterministic CCSD")
        out["oracle_energy_check"] = oracle_energy_check(args.study_replicas, args.check_steps, args.study_equil, log)
    if not args.no_serve:
        log("served stream")
        out["serving"] = serving_benchmark(args.serve_requests, args.serve_max_steps, args.serve_tol,
                                           args.serve_budget, args.serve_slots, log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, log)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
