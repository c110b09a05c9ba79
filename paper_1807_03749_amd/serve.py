"""Continuous-batching server of CCMC solves on one GPU.

Requests arrive over time.  Each one is a full CCMC calculation: grow the population with the
shift held at zero until it reaches the target, vary the shift to hold it there (Sec. II),
skip an equilibration window, then accumulate the projected-energy terms until their
reblocked standard error falls below a tolerance (Computational Methods).  The server keeps
every admitted solve's excitor store resident on the device between steps, and every
iteration steps all active solves together in shared launches (``ccmc_step_batch``).

Admission is by device memory: a request is admitted when a slot is free and its estimated
footprint fits the remaining HBM budget; its state is created with that estimate (times a
safety factor) as its own budget.  A solve that outgrows it (a step that fails with ENOMEM and
leaves the state unchanged) gets its reservation doubled and steps again, up to `max_grow`
times and as long as the server's budget has room; otherwise it fails alone.  So does a solve
whose population runs away beyond what one step can select (2^32 selections).
Finished solves free their memory at once, so waiting requests join the running batch
between two steps -- continuous batching, not a queue of whole runs.

A solve whose population keeps growing after the shift has started to vary, to `runaway`
times its target, is ended as diverged: its target lies below the population at which the
walk stabilises (the shoulder of Sec. IV.A, whose height the solve's largest N_tot / N_0
tracks), and stepping it further would only hold memory.  Results are reported as converged
(time to energy), capped (the step cap reached first: a right-censored time) or failed.

Each solve's result does not depend on what else is in the batch: its steps use its own
store and its own Philox key, and the shift and selection count come from its own
statistics, so a solve served in a mix returns exactly the energy it returns alone.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import ccmc, driver


@dataclass
class Request:
    request_id: int
    arrival: float          # seconds after the start of the stream
    system: dict            # ccmc.State keyword arguments (system, n_electrons, truncation, ...)
    target: float           # target population
    tau: float
    seed: int
    precision: str = "fp32"


@dataclass
class Solve:
    req: Request
    state: object
    est_bytes: int
    ctl: driver.ShiftControl
    nsel: int
    admitted: float
    steps: int = 0
    varying_since: int = -1
    grown: int = 0          # times its memory reservation was doubled
    num: list = field(default_factory=list)
    den: list = field(default_factory=list)
    attempts: int = 0
    shoulder: float = 0.0   # largest N_tot / N_0 so far (Sec. IV.A)
    shoulder_at: float = 0.0  # the N_tot where it was seen


@dataclass
class Result:
    request_id: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    energy: float
    error: float
    converged: bool
    attempts: int
    failed: str = ""
    grown: int = 0          # times the solve's memory reservation was doubled
    shoulder: float = 0.0   # largest N_tot / N_0 of the solve, and the N_tot where it was seen
    shoulder_at: float = 0.0

    @property
    def time_to_energy(self) -> float:
        return self.finished - self.arrival

    @property
    def outcome(self) -> str:
        return "converged" if self.converged else ("failed" if self.failed else "capped")


def estimate_bytes(req: Request) -> int:
    """Device memory of a solve at its target population: a fixed part plus about 300 bytes
    per unit of population (store, items, record regions and sort buffers; measured at
    N = 1e6 for 14 electrons in 114 spin orbitals), doubled for the FP64 amplitudes."""
    per = 300.0 * (2.0 if req.precision == "fp64" else 1.0)
    return int(32e6 + per * req.target)


class Server:
    def __init__(self, hbm_budget: float = 64e9, max_active: int = 32, tol: float = 1e-4, equil: int = 500,
                 min_samples: int = 512, check_every: int = 256, max_steps: int = 20000, safety: float = 4.0,
                 max_grow: int = 3, runaway: float = 20.0, clock=time.perf_counter, sleep=time.sleep, log=None):
        self.hbm_budget = hbm_budget
        self.max_active = max_active
        self.tol = tol
        self.equil = equil
        self.min_samples = min_samples
        self.check_every = check_every
        self.max_steps = max_steps
        self.safety = safety
        self.max_grow = max_grow
        self.runaway = runaway
        self.clock = clock
        self.sleep = sleep
        self.log = log or (lambda m: None)
        self.batch_steps = 0
        self.state_steps = 0

    # ------------------------------------------------------------------------ one solve
    def _start(self, req: Request, now: float) -> Solve:
        est = estimate_bytes(req)
        kw = dict(req.system)
        system, nel, trunc = kw.pop("system"), kw.pop("n_electrons"), kw.pop("truncation")
        init_pop = max(10.0, req.target / 5.0)  # the walk starts on the reference (Sec. II)
        st = ccmc.State(system, nel, trunc, precision=req.precision, seed=req.seed, init_pop=init_pop,
                        hbm_budget_bytes=int(self.safety * est), **kw)
        ctl = driver.ShiftControl(target=req.target, tau=req.tau)
        return Solve(req=req, state=st, est_bytes=est, ctl=ctl, nsel=driver.selections(init_pop), admitted=now)

    def _advance(self, s: Solve, stats: dict) -> bool:
        """Book one step's statistics; True when the solve is finished."""
        s.steps += 1
        s.attempts += stats["n_spawn_attempts"]
        if stats["n_ref"] != 0.0:
            r = stats["n_total"] / abs(stats["n_ref"])
            if r > s.shoulder:
                s.shoulder, s.shoulder_at = r, stats["n_total"]
        was = s.ctl.varying
        s.ctl.update(stats["n_total"])
        if s.ctl.varying and not was:
            s.varying_since = s.steps
        s.nsel = driver.selections(stats["n_total"])
        if s.varying_since >= 0 and s.steps - s.varying_since > self.equil:
            s.num.append(stats["eproj_num"])
            s.den.append(stats["eproj_den"])
            if len(s.num) >= self.min_samples and len(s.num) % self.check_every == 0:
                _, err, _ = driver.reblock_ratio(np.array(s.num), np.array(s.den))
                if err < self.tol:
                    return True
        return s.steps >= self.max_steps

    def _runaway(self, s: Solve, stats: dict) -> bool:
        """The population grew to `runaway` times its target after the shift started to vary."""
        return s.varying_since >= 0 and self.runaway > 0 and stats["n_total"] > self.runaway * s.req.target

    def _finish(self, s: Solve, now: float, failed: str = "") -> Result:
        e = err = float("nan")
        if len(s.num) >= 16:
            e, err, _ = driver.reblock_ratio(np.array(s.num), np.array(s.den))
        s.state.close()
        return Result(s.req.request_id, s.req.arrival, s.admitted, now, s.steps, e, err,
                      bool(err < self.tol) and not failed, s.attempts, failed, s.grown, s.shoulder, s.shoulder_at)

    # ------------------------------------------------------------------------ the loop
    def run(self, requests: list[Request]) -> list[Result]:
        """Serve `requests` (arrival times relative to the call) to completion."""
        pending = sorted(requests, key=lambda r: r.arrival)
        waiting: list[Request] = []
        active: list[Solve] = []
        results: list[Result] = []
        t0 = self.clock()
        used = 0
        while pending or waiting or active:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.pop(0))
            # admission: in arrival order, while memory and slots allow
            for req in list(waiting):
                est = estimate_bytes(req)
                if len(active) < self.max_active and used + est <= self.hbm_budget:
                    waiting.remove(req)
                    active.append(self._start(req, now))
                    used += est
                    self.log(f"admit {req.request_id} at {now:.2f}s ({len(active)} active)")
            if not active:
                if pending:
                    self.sleep(max(0.0, pending[0].arrival - (self.clock() - t0)))
                continue
            # a population beyond one step's selection range (or a shift gone non-finite) ends
            # that solve alone, before it could invalidate the batch's arguments
            for s in [s for s in active if not (s.nsel < (1 << 32) and math.isfinite(s.ctl.shift))]:
                active.remove(s)
                results.append(self._finish(s, now, failed="population beyond 2^32 selections per step"))
                used -= s.est_bytes
            if not active:
                continue
            res = ccmc.ccmc_step_batch([s.state for s in active], [s.req.tau for s in active],
                                       [s.ctl.shift for s in active], [s.nsel for s in active])
            self.batch_steps += 1
            self.state_steps += len(active)
            now = self.clock() - t0
            keep = []
            for s, r in zip(active, res):
                if isinstance(r, Exception):
                    if (getattr(r, "status", None) == ccmc.CCMC_ENOMEM_STATUS and s.grown < self.max_grow
                            and used + s.est_bytes <= self.hbm_budget):
                        # the step was rolled back: double the reservation and step again
                        used += s.est_bytes
                        s.est_bytes *= 2
                        s.grown += 1
                        s.state.ccmc_set_budget(int(self.safety * s.est_bytes))
                        keep.append(s)
                        self.log(f"grow {s.req.request_id} to {s.est_bytes / 1e6:.0f} MB at {now:.2f}s")
                        continue
                    results.append(self._finish(s, now, failed=str(r)))
                    used -= s.est_bytes
                elif self._advance(s, r):
                    results.append(self._finish(s, now))
                    used -= s.est_bytes
                    self.log(f"done {s.req.request_id} at {now:.2f}s after {s.steps} steps")
                elif self._runaway(s, r):
                    results.append(self._finish(
                        s, now, failed=f"diverged: N_tot {r['n_total']:.3g} is {r['n_total'] / s.req.target:.0f}x the "
                                       f"target under shift control, N_tot/N_0 up to {s.shoulder:.0f} (target below "
                                       f"the shoulder)"))
                    used -= s.est_bytes
                    self.log(f"diverged {s.req.request_id} at {now:.2f}s after {s.steps} steps")
                else:
                    keep.append(s)
            active = keep
        return sorted(results, key=lambda r: r.request_id)


def requests_from_stream(stream: list[dict], precision: str = "fp32") -> list[Request]:
    """Requests from ``inputs.serving_stream`` records (UEG, 14 electrons)."""
    out = []
    for d in stream:
        system = dict(system="ueg", n_electrons=14, truncation=d["truncation"], n2_max=d["n2_max"], rs=d["rs"])
        out.append(Request(d["request_id"], d["arrival"], system, d["target_population"], d["tau"], d["seed"],
                           precision))
    return out


def summary(results: list[Result], wall: float) -> dict:
    """Time-to-energy percentiles over the converged solves only; capped solves (the step cap
    reached before the error fell below the tolerance) are right-censored times, listed apart;
    failed solves are counted by kind."""
    conv = [r for r in results if r.outcome == "converged"]
    capped = [r for r in results if r.outcome == "capped"]
    failed = [r for r in results if r.outcome == "failed"]
    tte = np.array([r.time_to_energy for r in conv])
    kinds: dict = {}
    for r in failed:
        k = r.failed.split(":")[0].strip()[:60]
        kinds[k] = kinds.get(k, 0) + 1
    return dict(requests=len(results), converged=len(conv), capped=len(capped), failed=len(failed),
                failures=kinds, reservations_grown=sum(r.grown for r in results),
                p50_time_to_energy_s=float(np.percentile(tte, 50)) if len(tte) else None,
                p99_time_to_energy_s=float(np.percentile(tte, 99)) if len(tte) else None,
                capped_after_s=sorted(round(r.time_to_energy, 2) for r in capped),
                attempts_per_s=sum(r.attempts for r in results) / wall if wall > 0 else None,
                wall_s=wall, mean_steps=float(np.mean([r.steps for r in results])) if results else None)
