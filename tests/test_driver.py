"""Host-side analysis of the driver (no GPU): reblocking and population-control reweighting.

Pins: the blocked standard error of an AR(1) series against its closed form; the reweighted
estimate against the ratio it must reproduce when the population-control factors are
planted exactly (the weights then cancel them), and against the plain estimate when the
shift is constant.
"""
from __future__ import annotations

import math

import numpy as np

from paper_1807_03749_amd import driver


def test_reblocking_ar1_error():
    """x_t = phi x_{t-1} + e_t: the standard error of the mean is
    sigma_e / (1 - phi) / sqrt(n) for large n."""
    rng = np.random.default_rng(1)
    phi, n = 0.9, 1 << 17
    e = rng.normal(0.0, 1.0, n)
    x = np.empty(n)
    x[0] = e[0] / math.sqrt(1 - phi * phi)
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    _, err, _, _ = driver.reblock_mean(x)
    want = 1.0 / (1 - phi) / math.sqrt(n)
    assert abs(err / want - 1.0) < 0.15


def test_reweighting_removes_planted_population_control():
    rng = np.random.default_rng(2)
    n, tau, K0 = 200000, 0.02, 40
    # a shift that wanders (an AR(1) process around -0.3)
    S = np.empty(n)
    S[0] = -0.3
    for t in range(1, n):
        S[t] = -0.3 + 0.95 * (S[t - 1] + 0.3) + rng.normal(0.0, 0.05)
    dev = S - S.mean()
    c = np.concatenate([[0.0], np.cumsum(dev)])
    f = np.ones(n)
    t = np.arange(K0, n)
    f[t] = np.exp(tau * (c[t] - c[t - K0]))  # the factor population control put on step t
    b = 1000.0 + rng.normal(0.0, 20.0, n)
    a = (-0.5 + 2.0 * np.log(f)) * b + rng.normal(0.0, 2.0, n)  # estimator correlated with the factor
    num, den = f * a, f * b
    res = dict((k, (e, err)) for k, e, err in driver.reweight(num, den, S, tau, memories=(0, K0)))
    truth = a[K0:].sum() / b[K0:].sum()
    assert abs(res[K0][0] - truth) <= 1e-12 * abs(truth)
    assert abs(res[0][0] - truth) > 4 * res[0][1]  # the plain estimate is biased


def test_reweighting_constant_shift_is_plain_ratio():
    rng = np.random.default_rng(3)
    n = 4000
    den = 500.0 + rng.normal(0.0, 5.0, n)
    num = -0.25 * den + rng.normal(0.0, 1.0, n)
    for k, e, _ in driver.reweight(num, den, np.full(n, -0.1), 0.005, memories=(0, 7, 100)):
        assert abs(e - num[k:].sum() / den[k:].sum()) <= 1e-12


def test_ratio_error_independent_samples():
    """Independent samples: the error of <num>/<den> is sigma / (sqrt(n) <den>) when
    num = E den + noise of deviation sigma."""
    rng = np.random.default_rng(4)
    n, sigma = 1 << 16, 3.0
    den = 200.0 + rng.normal(0.0, 4.0, n)
    num = -0.4 * den + rng.normal(0.0, sigma, n)
    e, err, _ = driver.reblock_ratio(num, den)
    assert abs(err / (sigma / math.sqrt(n) / 200.0) - 1.0) < 0.15
    assert abs(e + 0.4) < 5 * err
