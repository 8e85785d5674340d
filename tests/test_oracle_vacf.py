"""Pins of the oracle's velocity autocorrelation sums and of lambda from the
VACF: the sums against explicit loops over particles and time origins; the
reading lambda = dt_cg / tau against processes whose collision statistics
are known: velocities redrawn at Poisson times of rate 1/tau (the expected
number of redraws in dt_cg is dt_cg / tau), an exponential C(t) sampled
exactly, and ballistic motion (no decay)."""
import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import md as omd


def test_sums_equal_explicit_loops():
    rng = np.random.default_rng(2)
    P, n = 7, 9
    vel = rng.normal(size=(P, n, 2))
    offsets = [0, 4, 4, 9]
    lags = [0, 1, 3, 6]
    got = omd.vacf_sums(offsets, vel, lags)
    for r in range(3):
        for s, lag in enumerate(lags):
            acc = 0.0
            for j in range(offsets[r], offsets[r + 1]):
                for p in range(P - lag):
                    acc += vel[p, j, 0] * vel[p + lag, j, 0] + vel[p, j, 1] * vel[p + lag, j, 1]
            assert got[r, s] == pytest.approx(acc, rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("tau", [0.2, 0.7])
def test_poisson_redraws_give_the_collision_count(tau):
    rng = np.random.default_rng(7)
    n, h, P, kT = 20000, 0.01, 800, 20.0
    v = rng.normal(0.0, math.sqrt(kT), (n, 2))
    vs = [v.copy()]
    q = 1.0 - math.exp(-h / tau)            # a redraw in a step of h: Poisson process of rate 1/tau
    for _ in range(P - 1):
        hit = rng.uniform(size=n) < q
        v[hit] = rng.normal(0.0, math.sqrt(kT), (int(hit.sum()), 2))
        vs.append(v.copy())
    vel = np.stack(vs)
    lags = list(range(0, 601, 8))
    s = omd.vacf_sums([0, n], vel, lags)[0]
    c = s / np.array([n * (P - l) for l in lags])
    t = np.array(lags) * h
    for dt_cg in (0.3911, 1.1261):
        tau_est, lam = cf.lambda_vacf(t, c, dt_cg)
        # the reading integrates to the 1% level: tau (1 - 0.01) for an exact exponential
        assert tau_est == pytest.approx(0.99 * tau, rel=0.04)
        assert lam == pytest.approx(dt_cg / tau / 0.99, rel=0.04)


def test_exact_exponential_and_ballistic():
    tau, h = 0.5, 0.005
    t = np.arange(0, 2000) * h
    c = 40.0 * np.exp(-t / tau)
    tau_est, lam = cf.lambda_vacf(t, c, 1.0)
    # trapezoid to the first sample at or below 1%, exactly
    k = int(np.argmax(c <= 0.01 * c[0]))
    want = np.sum((t[1:k + 1] - t[:k]) * (c[1:k + 1] + c[:k]) / 2) / c[0]
    assert tau_est == pytest.approx(want, rel=1e-12)
    assert tau_est == pytest.approx(tau * (1 - c[k] / c[0]), rel=1e-4)
    tau_b, lam_b = cf.lambda_vacf(t, np.full_like(t, 3.0), 2.0)
    assert tau_b == pytest.approx(t[-1], rel=1e-12) and lam_b == pytest.approx(2.0 / t[-1], rel=1e-12)
