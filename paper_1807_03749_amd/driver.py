"""Host-side driver of a CCMC calculation: shift update, number of selections, projected
energy with Flyvbjerg-Petersen reblocking, and a run loop over ``ccmc_step``.

Paper: Spencer et al., arXiv:1807.03749, Sec. II (the shift is held until the population
reaches its target, then varied to keep it stable; projected energy, eq. 7) and the
Computational Methods section (reblocking analysis of the stochastic error).
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ShiftControl:
    """Log-growth population control (the standard form used by FCIQMC / DMC; the paper
    cites it without giving the formula): every `period` steps once the population has
    reached `target`, S <- S - damping / (period tau) * ln(N(t) / N(t - period))."""
    target: float
    tau: float
    damping: float = 0.05
    period: int = 10
    shift: float = 0.0
    varying: bool = False
    history: list = field(default_factory=list)

    def update(self, n_total: float) -> float:
        self.history.append(n_total)
        if not self.varying and n_total >= self.target:
            self.varying = True
            self._anchor = len(self.history) - 1
        if self.varying and (len(self.history) - 1 - self._anchor) % self.period == 0 and \
                len(self.history) - 1 > self._anchor:
            prev = self.history[-1 - self.period]
            self.shift -= self.damping / (self.period * self.tau) * math.log(n_total / prev)
        return self.shift


    def to_dict(self) -> dict:
        d = dict(target=self.target, tau=self.tau, damping=self.damping, period=self.period, shift=self.shift,
                 varying=self.varying, history=list(self.history))
        if self.varying:
            d["anchor"] = self._anchor
        return d

    @classmethod
    def from_dict(cls, d: dict) -> "ShiftControl":
        c = cls(target=d["target"], tau=d["tau"], damping=d["damping"], period=d["period"], shift=d["shift"],
                varying=d["varying"], history=list(d["history"]))
        if c.varying:
            c._anchor = d["anchor"]
        return c


@dataclass
class Shoulder:
    """The shoulder statistic of Sec. IV.A: the largest N_tot / N_0 of a run and the total
    population where it occurred.  A run that has passed its shoulder shows a maximum that
    stays put while N_tot grows; a run still below it (whose population control is unstable)
    shows a ratio that keeps rising."""
    ratio: float = 0.0
    at: float = 0.0
    last: float = 0.0

    def update(self, n_total: float, n_ref: float) -> None:
        if n_ref != 0.0:
            self.last = n_total / abs(n_ref)
            if self.last > self.ratio:
                self.ratio, self.at = self.last, n_total

    def as_dict(self) -> dict:
        return dict(max_ntot_over_n0=self.ratio, at_ntot=self.at, last_ntot_over_n0=self.last,
                    passed=bool(self.last < 0.9 * self.ratio))


def selections(n_total: float) -> int:
    """Cluster selections per step: the total amplitude, rounded half up (Sec. IV.B)."""
    return int(math.floor(n_total + 0.5))


# ------------------------------------------------------------------------ reblocking

def _blocks(x: np.ndarray):
    """Successive pairwise block averages of the rows of x (shape [n, k])."""
    out = []
    y = np.asarray(x, dtype=np.float64)
    while len(y) >= 2:
        out.append(y)
        n = len(y) // 2 * 2
        y = 0.5 * (y[0:n:2] + y[1:n:2])
    return out


def reblock_mean(x: np.ndarray):
    """Flyvbjerg-Petersen blocking of a 1D series.  Returns (mean, standard error at the
    optimal block, optimal level, per-level standard errors).  The optimal level is the
    smallest with B^3 > 2 n (SE_B / SE_0)^4 (Lee, Kent, Foulkes & Needs 2011)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    levels = _blocks(x)
    se = np.array([y.std(ddof=1) / math.sqrt(len(y)) for y in levels])
    opt = len(se) - 1
    for i in range(len(se)):
        if (2 ** i) ** 3 > 2 * n * (se[i] / se[0]) ** 4:
            opt = i
            break
    return float(x.mean()), float(se[opt]), opt, se


def reblock_ratio(num: np.ndarray, den: np.ndarray):
    """Ratio of means E = <num>/<den> with its standard error: the linearised series
    x_t = num_t - E den_t is blocked and the error of its mean, divided by <den>, is the error
    of E (first-order propagation; blocking x rather than num and den separately picks the
    block length from the ratio's own correlation time, not from the slower fluctuations of
    the population that num and den share).  Returns (E, error, optimal level)."""
    num = np.asarray(num, dtype=np.float64)
    den = np.asarray(den, dtype=np.float64)
    mn, md = num.mean(), den.mean()
    e = mn / md
    _, se, lv, _ = reblock_mean(num - e * den)
    return float(e), float(abs(se / md)), lv


def reweight(num: np.ndarray, den: np.ndarray, shift: np.ndarray, tau: float, memories=(0, 10, 20, 50, 100, 200)):
    """Population-control reweighting of the projected energy (the analysis the paper uses to
    check its energies, after Umrigar, Nightingale & Runge 1993 and Vigor et al. 2015).

    With the shift S(t) in force at step t, the population of step t was multiplied by
    prod exp(delta_tau (S(t') - S_bar)) over the earlier steps relative to a run held at the
    mean shift S_bar.  Undoing that over the last K steps gives the weights
    W_t(K) = exp(-delta_tau sum_{j=1..K} (S(t-j) - S_bar)), and the estimate
    E(K) = sum_t W_t num_t / sum_t W_t den_t over the steps t >= K of the series (reblocked as a
    ratio).  K = 0 is the plain estimate; an E(K) flat in K within its error shows no
    population-control bias.  Returns [(K, E, error)]."""
    num = np.asarray(num, dtype=np.float64)
    den = np.asarray(den, dtype=np.float64)
    shift = np.asarray(shift, dtype=np.float64)
    if not (len(num) == len(den) == len(shift)):
        raise ValueError("num, den and shift must have one entry per step")
    dev = shift - shift.mean()
    c = np.concatenate([[0.0], np.cumsum(dev)])  # c[t] = sum of dev over steps < t
    out = []
    for K in memories:
        if K >= len(num) - 16:
            continue
        t = np.arange(K, len(num))
        logw = -tau * (c[t] - c[t - K])
        w = np.exp(logw - logw.max())
        e, err, _ = reblock_ratio(w * num[t], w * den[t])
        out.append((int(K), e, err))
    return out


# ------------------------------------------------------------------ checkpoint / resume

def _ctl_to_dict(ctl) -> dict:
    if isinstance(ctl, ShiftControl):
        return dict(kind="python", **ctl.to_dict())
    # the library's native control (ccmc.ccmc_shift_control): its fields, ring included
    return dict(kind="native", target=ctl.target, damping=ctl.damping, period=ctl.period, varying=ctl.varying,
                shift=ctl.shift, since=ctl.since, n_hist=[float(x) for x in ctl.n_hist])


def _ctl_from_dict(d: dict):
    if d["kind"] == "python":
        return ShiftControl.from_dict({k: v for k, v in d.items() if k != "kind"})
    from . import ccmc
    c = ccmc.ccmc_shift_control(target=d["target"], damping=d["damping"], period=d["period"], varying=d["varying"],
                                shift=d["shift"], since=d["since"])
    for i, x in enumerate(d["n_hist"]):
        c.n_hist[i] = x
    return c


def save_checkpoint(path: str, state, ctl, nsel: int, series: dict | None = None) -> None:
    """Everything a run needs to continue exactly (the paper restarts runs from checkpoints,
    Sec. III.A): the excitor store (keys and amplitudes as FP64), N_0, the step index (which
    keys every Philox counter of the next step), the population control's whole state, the
    next step's selection count and the energy series recorded so far.  `state` is anything
    with export_state() -> (keys, amps, n_ref, step)."""
    keys, amps, n_ref, step = state.export_state()
    arrays = {f"series_{k}": np.asarray(v) for k, v in (series or {}).items()}
    np.savez(path, keys=keys, amps=amps, n_ref=np.float64(n_ref), step=np.uint64(step), nsel=np.uint64(nsel),
             ctl=np.array(json.dumps(_ctl_to_dict(ctl))), **arrays)


def load_checkpoint(path: str) -> dict:
    with np.load(path, allow_pickle=False) as z:
        out = dict(keys=z["keys"], amps=z["amps"], n_ref=float(z["n_ref"]), step=int(z["step"]), nsel=int(z["nsel"]),
                   ctl=_ctl_from_dict(json.loads(str(z["ctl"]))),
                   series={k[len("series_"):]: z[k] for k in z.files if k.startswith("series_")})
    return out


def resume(state, ckpt: dict):
    """Load a checkpoint into `state` (import_state); returns (control, next selections,
    series)."""
    state.import_state(ckpt["keys"], ckpt["amps"], ckpt["n_ref"], ckpt["step"])
    return ckpt["ctl"], ckpt["nsel"], {k: list(v) for k, v in ckpt["series"].items()}


# -------------------------------------------------------------------------- run loop

@dataclass
class RunResult:
    steps: int
    energy: float = float("nan")
    error: float = float("nan")
    shift: float = 0.0
    n_total: list = field(default_factory=list)
    n_ref: list = field(default_factory=list)
    num: list = field(default_factory=list)
    den: list = field(default_factory=list)
    attempts: int = 0
    seconds: float = 0.0


def run(state, tau: float, steps: int, target: float, equilibrate: int = 0, shift: ShiftControl | None = None,
        first_selections: int | None = None, callback=None, jsonl=None) -> RunResult:
    """Propagate `state` (a ccmc.State) for `steps` steps with population control; the
    projected-energy terms after `equilibrate` steps enter the reblocked estimate.  With
    `jsonl` (a writable text file), every step's statistics and shift go to it as one JSON
    line."""
    import time

    ctl = shift or ShiftControl(target=target, tau=tau)
    res = RunResult(steps=steps)
    nsel = first_selections if first_selections is not None else selections(state.options.init_pop)
    t0 = time.perf_counter()
    for it in range(steps):
        st = state.ccmc_step(tau, ctl.shift, nsel)
        res.attempts += st["n_spawn_attempts"]
        res.n_total.append(st["n_total"])
        res.n_ref.append(st["n_ref"])
        if it >= equilibrate:
            res.num.append(st["eproj_num"])
            res.den.append(st["eproj_den"])
        ctl.update(st["n_total"])
        nsel = selections(st["n_total"])
        if jsonl is not None:
            jsonl.write(json.dumps(dict(st, shift=ctl.shift)) + "\n")
        if callback:
            callback(it, st, ctl)
    res.seconds = time.perf_counter() - t0
    res.shift = ctl.shift
    if len(res.num) >= 16:
        res.energy, res.error, _ = reblock_ratio(np.array(res.num), np.array(res.den))
    return res
