"""The continuous-batching server: a request served in a mix of others (joining and leaving
at different steps) returns exactly the result it returns when served alone."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_1807_03749_amd import serve

pytestmark = pytest.mark.gpu


class FakeClock:
    """Advances 1 ms per reading, so that arrivals are admitted between batch steps."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


def _requests():
    ueg = lambda trunc, n2, rs: dict(system="ueg", n_electrons=14, truncation=trunc, n2_max=n2, rs=rs)
    return [serve.Request(0, 0.0, ueg(2, 2, 1.0), 1e3, 0.005, 101, "fp32"),
            serve.Request(1, 0.02, ueg(2, 2, 0.5), 1.5e3, 0.005, 102, "fp64"),
            serve.Request(2, 0.05, ueg(3, 4, 1.0), 2e3, 0.005, 103, "fp32"),
            serve.Request(3, 0.08, ueg(2, 4, 0.5), 1e3, 0.005, 104, "fp32"),
            # two-word determinants: a group of their own, queued beside the one-word groups
            serve.Request(4, 0.09, ueg(2, 5, 1.0), 1e3, 0.005, 105, "fp32")]


def _server(clock):
    return serve.Server(hbm_budget=8e9, max_active=3, tol=1e-9, equil=50, min_samples=64, check_every=64,
                        max_steps=1500, clock=clock, sleep=clock.sleep)


def test_results_same_alone_and_in_the_mix():
    c = FakeClock()
    mixed = _server(c).run(_requests())
    assert [r.request_id for r in mixed] == [0, 1, 2, 3, 4]
    # with three slots, request 3 waits for a free one: admitted after it arrived
    assert mixed[3].admitted > mixed[3].arrival
    for req in _requests():
        c1 = FakeClock()
        alone = _server(c1).run([serve.Request(req.request_id, 0.0, req.system, req.target, req.tau, req.seed,
                                               req.precision)])[0]
        m = mixed[req.request_id]
        assert not m.failed and not alone.failed
        assert (m.steps, m.attempts) == (alone.steps, alone.attempts)
        assert np.isfinite(m.energy) and np.isfinite(m.error), m
        assert m.energy == alone.energy and m.error == alone.error, (req.request_id, m, alone)
        print(f"[serve] request {req.request_id}: E {m.energy:.6f} +- {m.error:.6f} in {m.steps} steps, "
              f"identical alone and in the mix", flush=True)
        sys.stdout.flush()


def test_admission_respects_memory_budget():
    """A budget that fits one request at a time serialises them (no overlap of residency)."""
    c = FakeClock()
    reqs = _requests()[:3]
    one = max(serve.estimate_bytes(r) for r in reqs)
    res = serve.Server(hbm_budget=one * 1.5, max_active=8, tol=1e-9, equil=50, min_samples=64, check_every=64,
                       max_steps=120, clock=c, sleep=c.sleep).run(reqs)
    spans = sorted((r.admitted, r.finished) for r in res)
    for (a0, f0), (a1, f1) in zip(spans, spans[1:]):
        assert a1 >= f0


def test_outgrown_reservation_is_doubled_and_the_result_unchanged():
    """A per-solve budget far below what the solve needs: each step that fails with ENOMEM leaves
    the state unchanged, the server doubles the reservation and steps again, and the solve ends
    with exactly the result it gets with room to spare."""
    req = _requests()[0]
    kw = dict(hbm_budget=8e9, max_active=3, tol=1e-9, equil=50, min_samples=64, check_every=64, max_steps=300)
    c1, c2 = FakeClock(), FakeClock()
    roomy = serve.Server(clock=c1, sleep=c1.sleep, **kw).run([req])[0]
    tight = serve.Server(clock=c2, sleep=c2.sleep, safety=0.1, max_grow=20, **kw).run([req])[0]
    assert not roomy.failed and not tight.failed, tight.failed
    assert tight.grown >= 1 and roomy.grown == 0
    assert (tight.steps, tight.attempts, tight.energy, tight.error) == (roomy.steps, roomy.attempts, roomy.energy,
                                                                        roomy.error)
    print(f"[serve] reservation doubled {tight.grown} times, same result", flush=True)
    sys.stdout.flush()
