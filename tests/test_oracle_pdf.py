"""Pins of the oracle's displacement-PDF pieces (the comparison of Fig. 2).

* The histogram of box-frame displacements is checked against numpy's own
  histogram on dyadic bins (where the bin rule is exact), exact edge values,
  a boundary crossing, mirror symmetry and ballistic trajectories whose
  displacement over every lag is known in closed form.
* The bin masses of P^G (Eq.(gaussian_df)) are checked against scipy's normal
  law; those of P^WSG (Eq.(poisson_v2), Eq.(p_wsg_one)) through their
  moments: on fine bins the grouped moments equal those of the law plus
  Sheppard's corrections (exact up to exponentially small terms for
  Gaussian mixtures), and the law's second and fourth moments are the msd and
  Eq.(fourth_order), from which Eq.(lambda_eq) recovers lambda.  Samples
  drawn as the model describes them (c ~ Poisson(lambda), then a normal law
  of variance msd (c + 1) / (lambda + 1)) pass a chi-square test against the
  masses, and a single Gaussian's samples fail it.
* The KL divergence (Eq.(k_Xi), Eq.(kullback_leibler)) is checked against the
  closed form between two normal laws, Gibbs' inequality and D(R||R) = 0.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import closed_forms as cf
from oracle import md as omd


def _pair(delta, L, rng):
    """Snapshot pair whose box-frame displacement is exactly `delta` [n, 2]
    when every value is dyadic: start inside the box, wrap the end point."""
    n = delta.shape[0]
    x0 = np.floor(rng.uniform(0, L, (n, 2)) * 64) / 64
    x1 = x0 + delta
    img1 = np.floor(x1 / L).astype(np.int64)
    x1w = x1 - L * img1
    img0 = rng.integers(-3, 4, (n, 2))
    return x0, img0, x1w, img1 + img0


def test_hist_matches_numpy_on_dyadic_bins():
    rng = np.random.default_rng(11)
    L, h, n_bin, n = 64.0, 0.25, 64, 20000
    xp = rng.uniform(0, L, (n, 2))
    xc = rng.uniform(0, L, (n, 2))
    ip = rng.integers(-2, 3, (n, 2))
    ic = ip + rng.integers(-1, 2, (n, 2))
    # keep most displacements inside the range
    xc = np.where(rng.uniform(size=(n, 2)) < 0.9, np.mod(xp + rng.normal(0, 3, (n, 2)), L), xc)
    ic = np.where(np.abs(xc - xp) < 10, ip, ic)
    hist = omd.displacement_hist(L, h, n_bin, xp, xc, ip, ic)
    edges = (np.arange(n_bin + 1) - n_bin / 2) * h
    for a in range(2):
        d = (xc[:, a] - xp[:, a]) + L * (ic[:, a] - ip[:, a]).astype(np.float64)
        ref, _ = np.histogram(d, bins=edges)
        assert np.array_equal(hist[a, :n_bin], ref)
        assert hist[a, n_bin] == int((d < edges[0]).sum())
        assert hist[a, n_bin + 1] == int((d >= edges[-1]).sum())
        assert hist[a].sum() == n


def test_hist_exact_edges_and_boundary_crossing():
    rng = np.random.default_rng(3)
    L, h, n_bin = 32.0, 0.5, 10
    ks = np.arange(-7, 8)
    delta = np.stack([ks * h, -ks * h], axis=1)
    x0, i0, x1, i1 = _pair(delta, L, rng)
    hist = omd.displacement_hist(L, h, n_bin, x0, x1, i0, i1)
    want = np.zeros((2, n_bin + 2), dtype=np.int64)
    for k in ks:
        for a, kk in ((0, k), (1, -k)):
            b = kk + n_bin // 2          # an edge value opens its bin [k h, (k+1) h)
            if b < 0:
                want[a, n_bin] += 1
            elif b >= n_bin:
                want[a, n_bin + 1] += 1
            else:
                want[a, b] += 1
    assert np.array_equal(hist, want)
    # across the periodic boundary: L - 1/8 -> 1/8 with one more image is +1/4
    hist = omd.displacement_hist(L, 0.25, 4, np.array([[L - 0.125, 1.0]]), np.array([[0.125, 1.0]]),
                                 np.array([[0, 0]]), np.array([[1, 0]]))
    assert hist[0, 3] == 1 and hist[1, 2] == 1


def test_hist_mirror_symmetry_odd_bins():
    rng = np.random.default_rng(5)
    L, n = 50.0, 5000
    xp = rng.uniform(0, L, (n, 2))
    d = rng.normal(0, 2.0, (n, 2))
    xc = xp + d
    ic = np.floor(xc / L).astype(np.int64)
    xc -= L * ic
    ip = np.zeros((n, 2), dtype=np.int64)
    fwd = omd.displacement_hist(L, 0.3, 31, xp, xc, ip, ic)
    bwd = omd.displacement_hist(L, 0.3, 31, xc, xp, ic, ip)
    assert np.array_equal(fwd[:, :31], bwd[:, 30::-1])
    assert np.array_equal(fwd[:, 31], bwd[:, 32]) and np.array_equal(fwd[:, 32], bwd[:, 31])


def test_series_ballistic_lags():
    """x(p) = x0 + v p (dyadic v): the displacement over lag l is exactly v l."""
    rng = np.random.default_rng(8)
    L, n, P = 16.0, 40, 9
    v = rng.integers(-12, 13, (n, 2)) / 8.0
    x0 = np.floor(rng.uniform(0, L, (n, 2)) * 8) / 8
    xs = np.stack([x0 + v * p for p in range(P)])
    img = np.floor(xs / L).astype(np.int64)
    pos = xs - L * img
    lags, h, n_bin = [1, 3, 8], [0.125, 0.25, 1.0], 40
    offsets = [0, 25, 25, 40]
    out = omd.displacement_hist_series(offsets, [L] * 3, pos, img, lags, h, n_bin)
    for r in range(3):
        a, b = offsets[r], offsets[r + 1]
        for s, lag in enumerate(lags):
            want = np.zeros((2, n_bin + 2), dtype=np.int64)
            for ax in range(2):
                k = np.floor(v[a:b, ax] * lag / h[s] + n_bin / 2).astype(np.int64)
                k = np.where(k < 0, n_bin, np.where(k >= n_bin, n_bin + 1, k))
                np.add.at(want[ax], k, P - lag)
            assert np.array_equal(out[r, s], want)


# ------------------------------------------------------------ bin masses ---

@pytest.mark.parametrize("msd,mean,h,n_bin", [(1.0, 0.0, 0.25, 41), (0.37, 0.21, 0.1, 60), (5.0, -1.3, 1.5, 9)])
def test_gauss_bins_equal_scipy_normal(msd, mean, h, n_bin):
    pg, pw = cf.pdf_bins(msd, 0.0, mean, h, n_bin)
    edges = (np.arange(n_bin + 1) - n_bin / 2) * h
    law = stats.norm(loc=mean, scale=math.sqrt(msd))
    ref = np.diff(law.cdf(edges))
    assert np.allclose(pg[:n_bin], ref, rtol=1e-12, atol=2e-16)
    assert pg[n_bin] == pytest.approx(law.cdf(edges[0]), rel=1e-12, abs=1e-300)
    assert pg[n_bin + 1] == pytest.approx(law.sf(edges[-1]), rel=1e-12, abs=1e-300)
    # lambda = 0 is the single Gaussian (the c = 0 term with weight 1)
    assert np.array_equal(pw, pg)


@pytest.mark.parametrize("lam", [0.0, 0.4, 3.0])
def test_wsg_bins_sheppard_moments_and_lambda(lam):
    msd, mean = 2.0, 0.37
    sd = math.sqrt(msd)
    h = sd / 8
    n_bin = 2 * int(math.ceil(32 * sd / h)) + 1  # wide enough for the c >> lam components
    pg, pw = cf.pdf_bins(msd, lam, mean, h, n_bin)
    assert sum(pw) == pytest.approx(1.0, abs=1e-15)
    assert sum(pg) == pytest.approx(1.0, abs=1e-15)
    assert pw[n_bin] + pw[n_bin + 1] < 1e-12
    mid = (np.arange(n_bin) - n_bin / 2 + 0.5) * h
    p = pw[:n_bin]
    m1 = float(np.dot(p, mid))
    c = mid - mean
    m2 = float(np.dot(p, c ** 2))
    m4 = float(np.dot(p, c ** 4))
    mu4 = cf.wsg_mu4(msd, lam)  # Eq.(fourth_order)
    assert m1 == pytest.approx(mean, abs=1e-12)
    assert m2 == pytest.approx(msd + h * h / 12, rel=1e-12)
    assert m4 == pytest.approx(mu4 + msd * h * h / 2 + h ** 4 / 80, rel=1e-11)
    if lam > 1:
        assert cf.lambda_from_moments(msd, mu4, branch=2)[0] == pytest.approx(lam, rel=1e-9)


def test_samples_of_the_model_pass_chi_square():
    rng = np.random.default_rng(21)
    msd, lam, h, n_bin, n = 1.0, 2.0, 0.25, 41, 400000
    c = rng.poisson(lam, n)
    d_wsg = rng.normal(0.0, np.sqrt(msd * (c + 1) / (lam + 1)))
    d_g = rng.normal(0.0, math.sqrt(msd), n)
    pg, pw = cf.pdf_bins(msd, lam, 0.0, h, n_bin)

    def hist_of(d):
        L = 64.0
        z = np.zeros((n, 2))
        x0 = np.full((n, 2), 32.0)
        dd = np.stack([d, np.zeros(n)], axis=1)
        return omd.displacement_hist(L, h, n_bin, x0, x0 + dd, z.astype(np.int64), z.astype(np.int64))[0]

    def pvalue(counts, p):
        e = n * p
        keep = e > 20
        chi = float((((counts - e) ** 2 / e)[keep]).sum())
        return stats.chi2.sf(chi, int(keep.sum()) - 1)

    assert pvalue(hist_of(d_wsg), pw) > 1e-4
    assert pvalue(hist_of(d_g), pg) > 1e-4
    # the test can tell the two models apart at this sample size
    assert pvalue(hist_of(d_g), pw) < 1e-12
    assert pvalue(hist_of(d_wsg), pg) < 1e-12


def test_pdf_measured_pools_axes():
    hist = np.array([[[1, 2, 3, 0, 4]], [[0, 2, 1, 1, 0]]], dtype=np.int64)
    p = cf.pdf_measured(hist)
    assert np.allclose(p, np.array([1, 4, 4, 1, 4]) / 14.0)


# -------------------------------------------------------------------- KL ---

def test_kl_of_normal_laws_on_fine_bins():
    """D(N(m1, s1^2) || N(m2, s2^2)) = ln(s2/s1) + (s1^2 + (m1 - m2)^2) / (2 s2^2) - 1/2;
    binning can only lower it (data processing), by O(h^2)."""
    s1, s2, m1, m2 = 1.0, 1.3, 0.2, -0.1
    h, n_bin = 0.02, 1601
    r, _ = cf.pdf_bins(s1 * s1, 0.0, m1, h, n_bin)
    q, _ = cf.pdf_bins(s2 * s2, 0.0, m2, h, n_bin)
    exact = math.log(s2 / s1) + (s1 * s1 + (m1 - m2) ** 2) / (2 * s2 * s2) - 0.5
    d = cf.kl_divergence(r, q)
    assert d <= exact + 1e-15
    assert d == pytest.approx(exact, rel=1e-4)
    K = cf.kl_elementwise(r, q)
    assert (K < 0).any()          # element-wise terms take both signs
    assert float(np.sum(K)) == pytest.approx(d, rel=1e-12)


def test_kl_gibbs_and_identity():
    rng = np.random.default_rng(4)
    for _ in range(20):
        r = rng.dirichlet(np.ones(12))
        q = rng.dirichlet(np.ones(12))
        r[rng.integers(12)] = 0.0
        r /= r.sum()
        assert cf.kl_divergence(r, q) >= 0.0
        assert cf.kl_divergence(r, r) == 0.0
    # R_i > 0 where Q_i = 0: infinite; R_i = 0 terms vanish
    assert math.isinf(cf.kl_divergence([0.5, 0.5], [1.0, 0.0]))
    assert cf.kl_elementwise([0.0, 1.0], [0.5, 0.5])[0] == 0.0
