"""Equilibria of the MDLG method, oracle side (test infrastructure only).

Everything is evaluated with mpmath at 50 significant digits and returned as
float64, so the paper's formulas can be written out exactly as printed (the
erf differences in them cancel badly in double precision at small a^2).

Follows
  * Eq.(theory_feq): f_i^eq is the average of n_i over the domain and all
    coarse steps; divided by the density rho = N / lx^2 it is the fraction of
    particle-events with lattice displacement v_i.
  * Eq.(feq_prod), Eq.(feq_gaussian), Eq.(a2_n_ua): single-Gaussian f^eq,G as
    a product over the two axes of the printed exp/erf expression with
    N = a / sqrt(2 pi) and u_{i,a} = v_{i,a} - u_a.
  * Eq.(poisson_v2), Eq.(f_eq_wsg) and the N_c definition below it:
    Poisson-WSG f^eq as sum_c e^-lam lam^c / c! prod_a f^{c,eq}_{i,a}.
  * Eq.(fourth_order), Eq.(lambda_eq) and the printed roots lambda_{1,2}.
  * Eq.(gaussian_df) and Eq.(poisson_v2) with Eq.(p_wsg_one): the
    one-axis displacement PDFs, integrated over the bins X_k of a histogram
    (the comparison of Fig. 2).
  * Eq.(k_Xi) and Eq.(kullback_leibler): element-wise and summed KL divergence.
  * lambda from the velocity autocorrelation function, the alternative the
    text names beside the moment matching of Eq.(lambda_eq) (no formula is
    given; the reading is in lambda_vacf).
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np

from . import lattice

mp.mp.dps = 50

NQ = 49


# ------------------------------------------------------------ measured ---

def feq_measured(counts, n_particles: int, n_events: int):
    """g_i = f_i^eq / rho from the summed counts (Eq.(theory_feq)).

    counts[0:49] are the summed n_i over every cell and coarse step and
    counts[49] the particle-events whose displacement left the D2Q49 set.
    Returns (g [49], overflow fraction)."""
    counts = np.asarray(counts, dtype=np.float64)
    denom = float(n_particles) * float(n_events)
    if denom <= 0:
        raise ValueError("need n_particles * n_events > 0")
    return counts[:NQ] / denom, counts[NQ] / denom


def symmetrize(g):
    """Average g over each |v|^2 shell (the Results section averages each of
    the D2Q25 sets to a symmetric distribution; valid for zero mean velocity)."""
    g = np.asarray(g, dtype=np.float64).copy()
    for idx in lattice.shells():
        g[idx] = g[idx].mean()
    return g


# ------------------------------------------------------ single Gaussian ---

def f1d_gauss(ui, a2):
    """Eq.(feq_gaussian) for one axis, as printed: u_i = v_i - u, a^2 > 0."""
    ui = mp.mpf(ui)
    a2 = mp.mpf(a2)
    a = mp.sqrt(a2)
    N = a / mp.sqrt(2 * mp.pi)
    s = a * mp.sqrt(2)
    return (N * (mp.exp(-(ui - 1) ** 2 / (2 * a2)) - 2 * mp.exp(-ui ** 2 / (2 * a2))
                 + mp.exp(-(ui + 1) ** 2 / (2 * a2)))
            + (ui - 1) / 2 * (mp.erf((ui - 1) / s) - mp.erf(ui / s))
            + (ui + 1) / 2 * (mp.erf((ui + 1) / s) - mp.erf(ui / s)))


def f1d_wsg_c(ui, a2, lam, c):
    """Eq.(f_eq_wsg) for one axis and one collision count c, as printed,
    with N_c = sqrt(2 a^2 (c + 1) / (lam + 1))."""
    ui = mp.mpf(ui)
    Nc = mp.sqrt(2 * mp.mpf(a2) * (c + 1) / (mp.mpf(lam) + 1))
    return (Nc / (2 * mp.sqrt(mp.pi)) * (mp.exp(-(ui - 1) ** 2 / Nc ** 2) - 2 * mp.exp(-ui ** 2 / Nc ** 2)
                                         + mp.exp(-(ui + 1) ** 2 / Nc ** 2))
            + (ui - 1) / 2 * (mp.erf((ui - 1) / Nc) - mp.erf(ui / Nc))
            + (ui + 1) / 2 * (mp.erf((ui + 1) / Nc) - mp.erf(ui / Nc)))


def feq_gauss(a2, u=(0.0, 0.0)):
    """g^G_i = f^eq,G_i / rho for the 49 velocities (Eq.(feq_prod))."""
    t = lattice.d2q49()
    fx = {v: f1d_gauss(v - mp.mpf(u[0]), a2) for v in range(-3, 4)}
    fy = {v: f1d_gauss(v - mp.mpf(u[1]), a2) for v in range(-3, 4)}
    return np.array([float(fx[int(vx)] * fy[int(vy)]) for vx, vy in t])


def poisson_window(lam):
    """Collision counts c kept in the Poisson sum: the weight outside
    [c_lo, c_hi] is below 1e-20 (the infinite sum is truncated there)."""
    lam = float(lam)
    if lam <= 0.0:
        return 0, 0
    lo = max(0, int(math.floor(lam - 12.0 * math.sqrt(lam) - 10.0)))
    hi = int(math.ceil(lam + 12.0 * math.sqrt(lam) + 40.0))
    return lo, hi


def feq_wsg(a2, lam, u=(0.0, 0.0)):
    """g^WSG_i: Poisson-weighted sum over c of the product over axes of
    Eq.(f_eq_wsg).  The collision count c is shared by both axes."""
    t = lattice.d2q49()
    lam_m = mp.mpf(lam)
    lo, hi = poisson_window(lam)
    acc = [mp.mpf(0)] * NQ
    for c in range(lo, hi + 1):
        w = mp.exp(-lam_m) * (lam_m ** c if c > 0 else mp.mpf(1)) / mp.factorial(c)
        fx = {v: f1d_wsg_c(v - mp.mpf(u[0]), a2, lam_m, c) for v in range(-3, 4)}
        fy = {v: f1d_wsg_c(v - mp.mpf(u[1]), a2, lam_m, c) for v in range(-3, 4)}
        for i, (vx, vy) in enumerate(t):
            acc[i] += w * fx[int(vx)] * fy[int(vy)]
    return np.array([float(a) for a in acc])


# ------------------------------------------------------------- lambda ---

def wsg_mu4(mu2, lam):
    """Fourth moment of the Poisson-WSG displacement PDF, Eq.(fourth_order)."""
    mu2 = mp.mpf(mu2)
    lam = mp.mpf(lam)
    return float(3 * mu2 ** 2 / (lam + 1) ** 2 * (lam ** 2 + 3 * lam + 1))


def lambda_roots(mu2, mu4):
    """The printed roots of Eq.(lambda_eq): (lambda_1, lambda_2) for the +
    and - sign of the square root.  Returns None when the discriminant is
    negative or the denominator vanishes."""
    mu2 = mp.mpf(mu2)
    mu4 = mp.mpf(mu4)
    disc = 3 * (15 * mu2 ** 4 - 4 * mu2 ** 2 * mu4)
    den = 2 * (3 * mu2 ** 2 - mu4)
    if disc < 0 or den == 0:
        return None
    sq = mp.sqrt(disc)
    l1 = (-9 * mu2 ** 2 + sq + 2 * mu4) / den
    l2 = (-9 * mu2 ** 2 - sq + 2 * mu4) / den
    return float(l1), float(l2)


def lambda_from_moments(mu2, mu4, branch: int = 2):
    """lambda for the WSG model from measured moments, with r = mu4 / (3 mu2^2).

    Readings where the paper is silent: r <= 1 (no positive root; the data
    are at most Gaussian-tailed) gives lambda = 0, the single Gaussian;
    r >= 5/4 (the largest r the model reaches, at the double root lambda = 1)
    gives lambda = 1.  Otherwise branch 1 / 2 take the printed + / - root;
    the paper uses lambda_2.  Returns (lambda, r)."""
    r = float(mp.mpf(mu4) / (3 * mp.mpf(mu2) ** 2))
    if r <= 1.0:
        return 0.0, r
    if r >= 1.25:
        return 1.0, r
    roots = lambda_roots(mu2, mu4)
    return (roots[0] if branch == 1 else roots[1]), r


# ---------------------------------------------------- displacement PDF ---

def bin_edges(h, n_bin):
    """Edges of the histogram intervals X_k = [(k - n_bin/2) h, (k + 1 - n_bin/2) h)."""
    return [(mp.mpf(k) - mp.mpf(n_bin) / 2) * mp.mpf(h) for k in range(n_bin + 1)]


def _normal_masses(edges, mean, var):
    """Masses of a normal law (mean, var) on the bins between consecutive edges,
    then below the first edge and at or above the last: [n_bin + 2]."""
    s = mp.sqrt(2 * mp.mpf(var))
    E = [mp.erf((e - mp.mpf(mean)) / s) for e in edges]
    inner = [(E[k + 1] - E[k]) / 2 for k in range(len(edges) - 1)]
    return inner + [(1 + E[0]) / 2, (1 - E[-1]) / 2]


def pdf_bins(msd, lam, mean, h, n_bin):
    """Probability of each bin X_k under the single Gaussian P^G and under the
    Poisson WSG P^WSG of one axis (Eq.(gaussian_df); Eq.(poisson_v2) with
    P^c of Eq.(p_wsg_one), whose variance is msd (c + 1) / (lam + 1)).
    msd is <(delta x)^2> about the mean displacement `mean` (u dt).
    Entries [n_bin] and [n_bin + 1] are the masses below and above the range.
    lam = 0 gives P^WSG = P^G.  Returns (pG, pW) float64 [n_bin + 2]."""
    edges = bin_edges(h, n_bin)
    pg = _normal_masses(edges, mean, msd)
    lam_m = mp.mpf(lam)
    lo, hi = poisson_window(lam)
    pw = [mp.mpf(0)] * (n_bin + 2)
    for c in range(lo, hi + 1):
        w = mp.exp(-lam_m) * (lam_m ** c if c > 0 else mp.mpf(1)) / mp.factorial(c)
        pc = _normal_masses(edges, mean, mp.mpf(msd) * (c + 1) / (lam_m + 1))
        pw = [a + w * b for a, b in zip(pw, pc)]
    return np.array([float(x) for x in pg]), np.array([float(x) for x in pw])


def pdf_measured(hist):
    """P^MD(X_k): the counts of one or more histograms [..., n_bin + 2] pooled
    (summed over the leading axes) and divided by their total."""
    h = np.asarray(hist, dtype=np.int64).reshape(-1, np.shape(hist)[-1]).sum(axis=0)
    tot = int(h.sum())
    if tot <= 0:
        raise ValueError("empty histogram")
    return h.astype(np.float64) / float(tot)


# ----------------------------------------------------------------- KL ---

def kl_elementwise(R, Q):
    """K(X_i) = R(X_i) log(R(X_i) / Q(X_i)), Eq.(k_Xi), at 50 digits.  A term
    with R_i = 0 is 0 (the limit of r log r); R_i > 0 with Q_i = 0 is +inf."""
    out = []
    for r, q in zip(np.asarray(R, dtype=np.float64), np.asarray(Q, dtype=np.float64)):
        if r == 0.0:
            out.append(0.0)
        elif q == 0.0:
            out.append(math.inf)
        else:
            out.append(float(mp.mpf(r) * mp.log(mp.mpf(r) / mp.mpf(q))))
    return np.array(out)


def kl_divergence(R, Q):
    """D_KL(R || Q) = sum_i K(X_i), Eq.(kullback_leibler), summed at 50 digits."""
    K = kl_elementwise(R, Q)
    if np.isinf(K).any():
        return math.inf
    R = np.asarray(R, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    acc = mp.mpf(0)
    for r, q in zip(R, Q):
        if r > 0:
            acc += mp.mpf(r) * mp.log(mp.mpf(r) / mp.mpf(q))
    return float(acc)


# ------------------------------------------------------- lambda from VACF ---

def lambda_vacf(t, c, dt_cg, cut=0.01):
    """Average number of collisions in a coarse step from the velocity
    autocorrelation C(t) (t ascending, t[0] = 0).  Reading: if collisions
    arrive as a Poisson process of rate 1/tau and each one forgets the
    velocity, C(t) = C(0) exp(-t / tau) and the expected count in dt_cg is
    lambda = dt_cg / tau.  tau is taken as the integral of C(t) / C(0)
    (trapezoid rule) up to the first sample with C <= cut C(0), or over all
    samples if none is.  Returns (tau, lambda)."""
    t = [mp.mpf(float(x)) for x in t]
    c = [mp.mpf(float(x)) for x in c]
    if len(t) < 2 or c[0] <= 0:
        raise ValueError("need >= 2 samples and C(0) > 0")
    tau = mp.mpf(0)
    for k in range(1, len(t)):
        tau += (t[k] - t[k - 1]) * (c[k] + c[k - 1]) / (2 * c[0])
        if c[k] <= cut * c[0]:
            break
    return float(tau), float(mp.mpf(float(dt_cg)) / tau)
