"""Synthetic trajectory sources for coarse-graining tests (no MD involved).

Each source returns one coarse step: (pos_prev, pos_cur, img_prev, img_cur)
with positions wrapped into [0, L) and image counts carrying the wraps, so
that pos + L * img is the unwrapped trajectory.  Start positions are uniform
in the box, displacements are drawn from a stated distribution.
"""
from __future__ import annotations

import numpy as np


def _place(x0, d, L):
    x1 = x0 + d
    img = np.floor(x1 / L).astype(np.int64)
    x1 = x1 - L * img
    x1[x1 >= L] = 0.0  # a value within an ulp below 0 that rounded up to L
    return x1, img


def gaussian_step(rng, n, L, var, mean=(0.0, 0.0)):
    """Displacements N(mean, var) per axis, independent axes.  This is also the
    exact displacement law of an Ornstein-Uhlenbeck velocity process started
    in equilibrium, with var = 2 (kT/g) [t - (1 - exp(-g t)) / g]."""
    x0 = rng.uniform(0.0, L, (n, 2))
    d = rng.normal(0.0, np.sqrt(var), (n, 2)) + np.asarray(mean)[None, :]
    x1, img = _place(x0, d, L)
    return x0, x1, np.zeros((n, 2), np.int64), img


def wsg_step(rng, n, L, mu2, lam, mean=(0.0, 0.0)):
    """Poisson weighted sum of Gaussians: one collision count c ~ Poisson(lam)
    per particle, shared by both axes; then N(mean, mu2 (c+1)/(lam+1)) per axis."""
    x0 = rng.uniform(0.0, L, (n, 2))
    c = rng.poisson(lam, n).astype(np.float64)
    sd = np.sqrt(mu2 * (c + 1.0) / (lam + 1.0))
    d = rng.normal(0.0, 1.0, (n, 2)) * sd[:, None] + np.asarray(mean)[None, :]
    x1, img = _place(x0, d, L)
    return x0, x1, np.zeros((n, 2), np.int64), img


def integer_step(rng, n, lx, L, vmax=4):
    """Particles at random points of random cells, displaced by whole numbers
    of cells in [-vmax, vmax] per axis (the in-cell offset is kept), so each
    particle's lattice velocity is known exactly.  Returns the four arrays
    and the integer displacements [n, 2]."""
    dxl = L / lx
    cells = rng.integers(0, lx, (n, 2))
    frac = rng.uniform(0.05, 0.95, (n, 2))
    x0 = (cells + frac) * dxl
    v = rng.integers(-vmax, vmax + 1, (n, 2))
    x1, img = _place(x0, v * dxl, L)
    return x0, x1, np.zeros((n, 2), np.int64), img, v
