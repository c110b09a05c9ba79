"""The serving loop's host logic (no GPU): the library's state and batched step are replaced by
scripted fakes, so that memory growth, its cap and a runaway population can be forced."""
from __future__ import annotations

import pytest

from paper_1807_03749_amd import ccmc, serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeState:
    """Population grows by `growth` per step; steps fail with ENOMEM while the budget is
    below `needs` bytes."""

    def __init__(self, kind, n_el, trunc, *, seed, init_pop, hbm_budget_bytes, **kw):
        self.seed, self.n, self.budget = seed, float(init_pop), hbm_budget_bytes
        self.growth, self.needs = FakeState.script[seed]
        self.closed = False

    def ccmc_set_budget(self, b):
        self.budget = b

    def close(self):
        self.closed = True


def fake_batch(states, tau, shift, nsel):
    out = []
    for st, n in zip(states, nsel):
        assert n < (1 << 32)  # the server must never pass an out-of-range count
        if st.budget < st.needs:
            out.append(ccmc.CCMCError(ccmc.CCMC_ENOMEM_STATUS, "CCMC_ENOMEM: HBM budget exceeded"))
            continue
        st.n *= st.growth
        out.append(dict(n_total=st.n, n_ref=0.1 * st.n, eproj_num=-0.05 * st.n, eproj_den=0.1 * st.n,
                        n_spawn_attempts=int(st.n), n_excitors=10))
    return out


@pytest.fixture
def fakes(monkeypatch):
    monkeypatch.setattr(ccmc, "State", FakeState)
    monkeypatch.setattr(ccmc, "ccmc_step_batch", fake_batch)


def _req(i, seed, target=1e4):
    return serve.Request(i, 0.0, dict(system="ueg", n_electrons=14, truncation=2, n2_max=2), target, 0.005, seed)


def _run(reqs, **kw):
    c = FakeClock()
    args = dict(hbm_budget=1e12, max_active=8, tol=1e-9, equil=5, min_samples=16, check_every=16, max_steps=60)
    args.update(kw)
    return serve.Server(clock=c, sleep=c.sleep, **args).run(reqs)


def test_reservation_grows_then_the_solve_runs(fakes):
    est = serve.estimate_bytes(_req(0, 1))
    FakeState.script = {1: (1.0, 4.0 * est * 3.5)}  # needs a bit under 4x the initial budget
    r = _run([_req(0, 1)])[0]
    assert not r.failed and r.grown == 2 and r.steps == 60


def test_growth_is_capped(fakes):
    est = serve.estimate_bytes(_req(0, 1))
    FakeState.script = {1: (1.0, 4.0 * est * 100)}
    r = _run([_req(0, 1)], max_grow=3)[0]
    assert r.failed.startswith("CCMC_ENOMEM") and r.grown == 3 and r.steps == 0


def test_growth_needs_room_in_the_server_budget(fakes):
    est = serve.estimate_bytes(_req(0, 1))
    FakeState.script = {1: (1.0, 4.0 * est * 3.5)}
    r = _run([_req(0, 1)], hbm_budget=2.5 * est)[0]  # room for one doubling only
    assert r.failed.startswith("CCMC_ENOMEM") and r.grown == 1


def test_runaway_population_ends_alone(fakes):
    FakeState.script = {1: (1.0, 0.0), 2: (4.0, 0.0)}  # solve 2 quadruples every step
    res = _run([_req(0, 1), _req(1, 2)], runaway=0)  # no divergence rule: the 2^32 guard ends it
    assert not res[0].failed and res[0].steps == 60
    assert res[1].failed == "population beyond 2^32 selections per step" and res[1].steps < 60


def test_population_runaway_under_shift_control_is_diverged(fakes):
    """A solve that passes 20 times its target after the shift started to vary ends as
    diverged, early, with its N_tot / N_0 record; the other solve runs on."""
    FakeState.script = {1: (1.0, 0.0), 2: (4.0, 0.0)}
    res = _run([_req(0, 1), _req(1, 2)])
    assert not res[0].failed and res[0].steps == 60
    assert res[1].failed.startswith("diverged") and res[1].steps == 4 and res[1].shoulder == pytest.approx(10.0)


def _result(i, arrival, finished, converged, failed=""):
    return serve.Result(i, arrival, arrival, finished, 100, -0.1, 1e-5, converged, 1000, failed)


def test_summary_percentiles_over_converged_only():
    res = [_result(0, 0.0, 10.0, True), _result(1, 1.0, 21.0, True), _result(2, 2.0, 92.0, False),
           _result(3, 3.0, 5.0, False, failed="CCMC_ENOMEM: budget"), _result(4, 4.0, 7.0, False, failed="diverged: x")]
    s = serve.summary(res, wall=100.0)
    assert (s["requests"], s["converged"], s["capped"], s["failed"]) == (5, 2, 1, 2)
    assert s["p50_time_to_energy_s"] == pytest.approx(15.0) and s["p99_time_to_energy_s"] == pytest.approx(19.9)
    assert s["capped_after_s"] == [90.0]
    assert s["failures"] == {"CCMC_ENOMEM": 1, "diverged": 1}
    assert s["attempts_per_s"] == pytest.approx(50.0)
