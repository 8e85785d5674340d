"""Pins of the oracle's equilibria and lambda against the mathematics.

f^eq,G (Eq.(feq_gaussian)) and f^eq,WSG (Eq.(f_eq_wsg)) are closed forms of
Eq.(theory_feq): with the start position uniform in a lattice cell, the
probability of a lattice displacement v along one axis is E[tri(d - v)], the
expected hat function tri(t) = max(0, 1 - |t|) of the displacement d in
lattice units.  These tests evaluate that expectation by quadrature, by
Monte Carlo and through exact identities, none of which reuse the erf/exp
expressions being tested.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import closed_forms as cf
from oracle import lattice


def hat_expectation(w, var):
    """E[max(0, 1 - |Z - w|)], Z ~ N(0, var), by adaptive quadrature."""
    s = math.sqrt(var)

    def f(z):
        return max(0.0, 1.0 - abs(z - w)) * math.exp(-z * z / (2 * var)) / (s * math.sqrt(2 * math.pi))

    lo, hi = w - 1.0, w + 1.0
    val, err = integrate.quad(f, lo, hi, points=[w], epsabs=1e-15, epsrel=1e-13, limit=200)
    return val


@pytest.mark.parametrize("a2", [1e-4, 0.05, 0.1611, 1 / 6, 0.5])
@pytest.mark.parametrize("u", [0.0, 0.13, -0.4])
def test_gauss_1d_equals_hat_quadrature(a2, u):
    for v in range(-3, 4):
        ref = hat_expectation(v - u, a2)
        got = float(cf.f1d_gauss(v - u, a2))
        assert got == pytest.approx(ref, abs=2e-14, rel=1e-11)


def test_gauss_exact_identities():
    t = lattice.d2q49()
    for a2, u in [(1e-4, (0.0, 0.0)), (0.1611, (0.0, 0.0)), (0.1611, (0.13, -0.07)), (0.08, (0.2, 0.1))]:
        g = cf.feq_gauss(a2, u)
        assert g.sum() == pytest.approx(1.0, abs=1e-13)
        assert (t[:, 0] * g).sum() == pytest.approx(u[0], abs=1e-13)
        assert (t[:, 1] * g).sum() == pytest.approx(u[1], abs=1e-13)
        assert np.all(g >= 0)
    # u = 0: symmetric under the 8 lattice symmetries; a2 -> 0 puts all weight on v = 0
    g = cf.feq_gauss(0.1611)
    for idx in lattice.shells():
        assert np.ptp(g[idx]) < 1e-16
    # per axis g(0) = 1 - 2 E[(Z - 1)_+ ... ] -> 1 - 2 s / sqrt(2 pi) up to exp(-1/(2 s^2)) terms
    assert cf.feq_gauss(1e-8)[0] == pytest.approx((1.0 - 2 * math.sqrt(1e-8 / (2 * math.pi))) ** 2, rel=1e-14)


def test_gauss_monte_carlo():
    # sample start offsets y ~ U[0,1) and displacements d ~ N(u, a2); the lattice
    # velocity is floor(y + d) per axis
    rng = np.random.default_rng(0)
    a2, u = 0.1611, (0.21, -0.1)
    m = 2_000_000
    y = rng.uniform(0, 1, (m, 2))
    d = rng.normal(0, math.sqrt(a2), (m, 2)) + np.array(u)
    v = np.floor(y + d).astype(int)
    t = lattice.d2q49()
    g = cf.feq_gauss(a2, u)
    for i in range(25):
        p = np.mean((v[:, 0] == t[i, 0]) & (v[:, 1] == t[i, 1]))
        se = math.sqrt(max(g[i] * (1 - g[i]), 1e-300) / m)
        assert abs(p - g[i]) < 4.5 * se + 1e-7


def test_wsg_term_is_gaussian_with_scaled_variance():
    # Eq.(f_eq_wsg) with N_c = sqrt(2 a2 (c+1)/(lam+1)) is Eq.(feq_gaussian)
    # at variance a2 (c+1)/(lam+1): two printed formulas, checked term by term
    for a2, lam, c in [(0.1611, 0.7, 0), (0.1611, 0.7, 3), (0.02, 5.0, 9), (0.3, 2.0, 1)]:
        for w in [-2.3, -1.0, 0.0, 0.4, 2.0]:
            a = float(cf.f1d_wsg_c(w, a2, lam, c))
            b = float(cf.f1d_gauss(w, a2 * (c + 1) / (lam + 1)))
            assert a == pytest.approx(b, rel=1e-14, abs=1e-30)


def test_wsg_limits():
    g0 = cf.feq_gauss(0.1611)
    assert np.array_equal(cf.feq_wsg(0.1611, 0.0), g0)  # lam = 0: one Gaussian
    # lam -> inf: (c+1)/(lam+1) -> 1 with variance 1/(lam+1), so WSG -> G as 1/lam
    d25 = np.max(np.abs(cf.feq_wsg(0.1611, 25.0) - g0))
    d100 = np.max(np.abs(cf.feq_wsg(0.1611, 100.0) - g0))
    assert d100 < 1.2e-3
    assert 3.0 < d25 / d100 < 5.0


def test_wsg_exact_identities_and_monte_carlo():
    t = lattice.d2q49()
    a2, lam, u = 0.1611, 1.3, (0.1, 0.0)
    g = cf.feq_wsg(a2, lam, u)
    # the heavy-tailed terms leave ~4e-8 of the mass beyond |v_a| = 3
    assert 1.0 - 1e-7 < g.sum() <= 1.0 + 1e-15
    assert (t[:, 0] * g).sum() == pytest.approx(u[0], abs=1e-6)
    rng = np.random.default_rng(1)
    m = 2_000_000
    c = rng.poisson(lam, m)
    sd = np.sqrt(a2 * (c + 1) / (lam + 1))
    d = rng.normal(0, 1, (m, 2)) * sd[:, None] + np.array(u)
    v = np.floor(rng.uniform(0, 1, (m, 2)) + d).astype(int)
    for i in range(25):
        p = np.mean((v[:, 0] == t[i, 0]) & (v[:, 1] == t[i, 1]))
        se = math.sqrt(max(g[i] * (1 - g[i]), 1e-300) / m)
        assert abs(p - g[i]) < 4.5 * se + 1e-7


def wsg_pdf_moment(k, mu2, lam):
    """k-th moment of the continuous Poisson-WSG PDF (Eq.(poisson_v2) with
    Eq.(p_wsg_one), u = 0), by quadrature of each Gaussian term."""
    lo, hi = cf.poisson_window(lam)
    tot = 0.0
    for c in range(lo, hi + 1):
        w = stats.poisson.pmf(c, lam)
        var = (c + 1) * mu2 / (lam + 1)
        sd = math.sqrt(var)
        m, _ = integrate.quad(lambda x: x ** k * math.exp(-x * x / (2 * var)) / (sd * math.sqrt(2 * math.pi)),
                              -40 * sd, 40 * sd, epsabs=0, epsrel=1e-13, limit=400)
        tot += w * m
    return tot


@pytest.mark.parametrize("lam", [0.0, 0.3, 1.0, 4.0])
def test_fourth_moment_formula(lam):
    mu2 = 2.7
    assert wsg_pdf_moment(2, mu2, lam) == pytest.approx(mu2, rel=1e-10)
    assert wsg_pdf_moment(4, mu2, lam) == pytest.approx(cf.wsg_mu4(mu2, lam), rel=1e-10)


def test_lambda_roots():
    # (lam = 1 is the double root, where the roots are only sqrt(ulp)-conditioned)
    for lam in [0.05, 0.4, 0.9, 2.5, 17.0]:
        mu2 = 1.9
        mu4 = cf.wsg_mu4(mu2, lam)
        l1, l2 = cf.lambda_roots(mu2, mu4)
        assert l1 * l2 == pytest.approx(1.0, rel=1e-12)
        assert min(l1, l2) == pytest.approx(min(lam, 1 / lam), rel=1e-10)
        assert l2 >= l1  # the printed "-" root is the larger one
        # each root solves Eq.(lambda_eq)
        for r_ in (l1, l2):
            assert 3 * mu2 ** 2 / (r_ + 1) ** 2 * (r_ ** 2 + 3 * r_ + 1) - mu4 == pytest.approx(0, abs=1e-11)
        lam2, r = cf.lambda_from_moments(mu2, mu4, branch=2)
        assert r == pytest.approx(1 + lam / (1 + lam) ** 2, rel=1e-13)
        assert lam2 == pytest.approx(max(lam, 1 / lam), rel=1e-10)
        # round trip mu2, mu4 -> lambda -> mu4
        assert cf.wsg_mu4(mu2, lam2) == pytest.approx(mu4, rel=1e-12)


def test_lambda_edge_cases():
    l1, l2 = cf.lambda_roots(1.9, cf.wsg_mu4(1.9, 1.0))
    assert l1 == pytest.approx(1.0, abs=1e-6) and l2 == pytest.approx(1.0, abs=1e-6)
    assert cf.lambda_from_moments(1.0, 3.0) == (0.0, 1.0)      # Gaussian kurtosis
    assert cf.lambda_from_moments(1.0, 2.5)[0] == 0.0          # lighter tails than Gaussian
    assert cf.lambda_from_moments(1.0, 3.75)[0] == 1.0         # r = 5/4, double root
    assert cf.lambda_from_moments(1.0, 5.0)[0] == 1.0          # beyond the model's reach


@pytest.mark.parametrize("lam", [0.2, 1.0, 3.0])
def test_wsg_vs_gauss_sign_pattern(lam):
    # Results section: relative to the single Gaussian, WSG has more particles at
    # node 0, a depression at nodes 1-8 and larger second-layer values 9-24
    a2 = 0.1611
    r = cf.feq_wsg(a2, lam) / cf.feq_gauss(a2)
    assert r[0] > 1
    assert np.all(r[1:9] < 1)
    assert np.all(r[9:25] > 1)


def test_measured_and_symmetrize():
    counts = np.arange(50, dtype=np.int64)
    g, ovf = cf.feq_measured(counts, 10, 7)
    assert g[5] == 5 / 70 and ovf == 49 / 70
    s = cf.symmetrize(g)
    assert s[1] == pytest.approx(np.mean(g[1:5]))
    assert s[13] == pytest.approx(np.mean(g[13:21]))
    assert s.sum() == pytest.approx(g.sum())


def test_kl_divergence():
    r = np.array([0.5, 0.5, 0.0])
    q = np.array([0.25, 0.5, 0.25])
    assert cf.kl_divergence(r, q) == pytest.approx(0.5 * math.log(2))
    assert cf.kl_divergence(q, q) == 0.0
