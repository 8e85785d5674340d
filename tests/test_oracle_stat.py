"""Statistical pins of the oracle chain: coarse-graining -> measured f_eq ->
moments -> lambda, on sources whose displacement law is known exactly.

* ballistic limit: free particles (eps = 0) move by v dt_cg with Maxwellian v,
  so the displacement is Gaussian and the measured f_eq is f^eq,G;
* diffusive limit: the displacement of an Ornstein-Uhlenbeck velocity process
  is exactly Gaussian at any dt_cg (kurtosis ratio r = 1, lambda = 0);
* Poisson-WSG source: the measured f_eq is f^eq,WSG and the moment-matched
  lambda recovers the source's lambda (as lambda or 1/lambda, the two roots).

Tolerances: |measured - model| within 4.5 standard errors of a multinomial
count per node (a Bonferroni-style margin over the 25 inner nodes).
"""
import math

import numpy as np

import mdlg_inputs as mi
from oracle import closed_forms as cf
from oracle import md
from tests import _sources as src


def _zmax(g_meas, g_model, m, nodes=25):
    se = np.sqrt(np.maximum(g_model * (1 - g_model), 1e-300) / m)
    return float(np.max(np.abs(g_meas[:nodes] - g_model[:nodes]) / (se[:nodes] + 1e-12)))


def test_ballistic_limit_free_particles():
    n, kT, lx = 50_000, 20.0, 211
    pos, vel, L = mi.initial_state(n, 0.0784, kT, 21, positions="uniform")
    dxl = L / lx
    dt, s_cg = 2e-3, 150  # dt_cg = 0.3, dx = 3.35: a2 = kT dt_cg^2 / dx^2 ~ 0.16
    acc = md.CGAccum(lx)
    md.md_run(pos, vel, np.zeros((n, 2), np.int64), L, s_cg, dt=dt, eps=0.0, cg=acc, s_cg=s_cg)
    assert acc.events == 1
    mu2 = acc.moments[1] / acc.moments[0]
    # displacement = v dt_cg exactly, and sum v^2 = 2 (N-1) kT by construction
    assert mu2 == pytest_approx(kT * (n - 1) / n * (dt * s_cg) ** 2, 1e-10)
    a2 = mu2 / dxl ** 2
    assert 0.1 < a2 < 0.25
    g, ovf = cf.feq_measured(acc.counts, n, 1)
    assert _zmax(g, cf.feq_gauss(a2), n) < 4.5
    r = (acc.moments[2] / acc.moments[0]) / (3 * mu2 ** 2)
    assert abs(r - 1.0) < 0.05


def test_diffusive_limit_ou_source():
    rng = np.random.default_rng(5)
    kT, gamma, t = 20.0, 4.0, 3.0  # many velocity relaxation times in one coarse step
    var = 2 * (kT / gamma) * (t - (1 - math.exp(-gamma * t)) / gamma)
    lx, n = 64, 400_000
    L = lx * math.sqrt(var / 0.1611)  # choose dx so that a2 = 0.1611, the paper's value
    x0, x1, i0, i1 = src.gaussian_step(rng, n, L, var)
    counts, _, mom = md.coarse_grain(lx, L, x0, x1, i0, i1)
    mu2 = mom[1] / mom[0]
    a2 = mu2 / (L / lx) ** 2
    assert abs(a2 - 0.1611) < 0.002
    g, _ = cf.feq_measured(counts, n, 1)
    assert _zmax(g, cf.feq_gauss(a2), n) < 4.5
    lam, r = cf.lambda_from_moments(mu2, mom[2] / mom[0])
    assert abs(r - 1.0) < 0.01
    # with r ~ 1 the model is (nearly) the single Gaussian whichever root is taken
    assert np.max(np.abs(cf.feq_wsg(a2, min(lam, 1 / lam) if lam > 0 else 0.0) - cf.feq_gauss(a2))) < 2e-3


def test_wsg_source_recovers_model_and_lambda():
    rng = np.random.default_rng(6)
    lam_true, lx, n = 0.3, 64, 400_000
    dxl = 2.0
    mu2_true = 0.1611 * dxl ** 2
    L = lx * dxl
    x0, x1, i0, i1 = src.wsg_step(rng, n, L, mu2_true, lam_true)
    counts, _, mom = md.coarse_grain(lx, L, x0, x1, i0, i1)
    mu2 = mom[1] / mom[0]
    mu4 = mom[2] / mom[0]
    lam2, r = cf.lambda_from_moments(mu2, mu4, branch=2)
    lam1, _ = cf.lambda_from_moments(mu2, mu4, branch=1)
    assert lam1 * lam2 == pytest_approx(1.0, 1e-9)
    assert abs(lam1 - lam_true) < 0.1
    a2 = mu2 / dxl ** 2
    g, _ = cf.feq_measured(counts, n, 1)
    # the source's own law is matched; the single Gaussian of the same a2 is not
    assert _zmax(g, cf.feq_wsg(a2, lam_true), n) < 4.5
    assert _zmax(g, cf.feq_gauss(a2), n) > 10.0


def pytest_approx(x, rel):
    import pytest
    return pytest.approx(x, rel=rel)
