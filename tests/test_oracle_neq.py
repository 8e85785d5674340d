"""Pins of the oracle's non-equilibrium MDLG sums: ensemble occupation numbers
and the lattice gas collision operator Xi_i = n_i(x + v_i, t + dt) - n_i(x, t)
of Eq.(mdlg_evolution).

* Free streaming on the lattice (every particle moves the same whole number of
  cells each coarse step, a lattice gas without collisions) gives Xi = 0.
* A velocity reversal gives Xi_i = -1 for the old and +1 for the new
  direction at its cell, and nothing elsewhere.
* Mass and momentum per cell: sum_i Xi_i(x, t) and sum_i v_i Xi_i(x, t) equal
  what the particles in cell x at t carry in and out, computed particle by
  particle from the unwrapped cell trajectories.
* The occupation sums equal the literal Eq.(n_i) loop; the ensemble sums
  equal the sums of single-replica calls.
"""
import numpy as np
import pytest

from oracle import lattice
from oracle import md as omd


def _wrap(xs, L):
    img = np.floor(xs / L).astype(np.int64)
    pos = xs - L * img
    img[pos >= L] += 1
    pos[pos >= L] = 0.0
    return pos, img


def _walk(n, L, P, step, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, L, (n, 2))
    xs = [x]
    for _ in range(P - 1):
        x = x + rng.normal(0.0, step, (n, 2))
        xs.append(x)
    return _wrap(np.stack(xs), L)


def _cells(pos, img, lx, L):
    """Unwrapped lattice cells [P, n, 2] of wrapped positions with image counts."""
    return np.floor(pos * (lx / L)).astype(np.int64) + lx * img


def test_free_streaming_has_no_collisions():
    rng = np.random.default_rng(1)
    lx, n, P = 12, 300, 6
    L = float(lx)                         # dx = 1: exact cell arithmetic
    vt = lattice.d2q49()
    w = vt[rng.integers(0, 49, n)].astype(np.float64)
    w[:7] = [4, 0]                        # these leave D2Q49 every step
    x0 = rng.integers(0, lx, (n, 2)) + rng.uniform(0.1, 0.9, (n, 2))
    pos, img = _wrap(np.stack([x0 + w * p for p in range(P)]), L)
    f, ovf, xi = omd.neq_mdlg(lx, L, [0, n], pos, img)
    assert not xi.any()
    assert (ovf == 7).all()
    assert (f.reshape(P - 1, -1).sum(axis=1) == n - 7).all()


def test_velocity_reversal():
    lx, L = 10, 10.0
    # one particle: cell 4 -> 5 -> 4 along x (v = +1, then -1), at y-cell 2
    xs = np.array([[[4.5, 2.5]], [[5.5, 2.5]], [[4.5, 2.5]]])
    img = np.zeros((3, 1, 2), dtype=np.int64)
    f, ovf, xi = omd.neq_mdlg(lx, L, [0, 1], xs, img)
    vt = lattice.d2q49()
    ip = int(np.where((vt == [1, 0]).all(axis=1))[0][0])
    im = int(np.where((vt == [-1, 0]).all(axis=1))[0][0])
    want = np.zeros((1, 49, lx, lx), dtype=np.int32)
    want[0, ip, 2, 5] = -1      # arrived at x = 5 with +1, does not continue with +1
    want[0, im, 2, 5] = 1       # leaves x = 5 with -1
    assert np.array_equal(xi, want)
    assert f[0, ip, 2, 5] == 1 and f[1, im, 2, 4] == 1 and f.sum() == 2 and not ovf.any()


@pytest.mark.parametrize("lx,step", [(9, 0.5), (16, 1.2), (7, 2.5), (16, 4.0)])
def test_mass_and_momentum_per_cell(lx, step):
    L, n, P = 40.0, 400, 7
    pos, img = _walk(n, L, P, step, seed=lx)
    f, ovf, xi = omd.neq_mdlg(lx, L, [0, n], pos, img)
    C = _cells(pos, img, lx, L)
    vt = lattice.d2q49().astype(np.int64)
    for p in range(1, P - 1):
        d_prev = C[p] - C[p - 1]
        d_next = C[p + 1] - C[p]
        in_prev = (np.abs(d_prev) <= 3).all(axis=1)
        in_next = (np.abs(d_next) <= 3).all(axis=1)
        cx, cy = np.mod(C[p, :, 0], lx), np.mod(C[p, :, 1], lx)
        mass = np.zeros((lx, lx), dtype=np.int64)
        mom = np.zeros((lx, lx, 2), dtype=np.int64)
        np.add.at(mass, (cy, cx), in_next.astype(np.int64) - in_prev.astype(np.int64))
        np.add.at(mom, (cy, cx), d_next * in_next[:, None] - d_prev * in_prev[:, None])
        x = xi[p - 1].astype(np.int64)
        assert np.array_equal(x.sum(axis=0), mass)
        assert np.array_equal(np.einsum("iyx,ia->yxa", x, vt), mom)
        assert ovf[p - 1] == int((~in_prev).sum())
    if step == 4.0:
        assert ovf.sum() > 0          # the overflow terms are exercised


def test_occupation_sums_equal_the_literal_definition():
    lx, L, P = 8, 16.0, 4
    parts = [_walk(n, L, P, 1.3, seed=20 + n) for n in (30, 0, 17)]
    pos = np.concatenate([p[0] for p in parts], axis=1)
    img = np.concatenate([p[1] for p in parts], axis=1)
    offsets = [0, 30, 30, 47]
    f, ovf, xi = omd.neq_mdlg(lx, L, offsets, pos, img)
    for p in range(1, P):
        lit = np.zeros((49, lx, lx), dtype=np.int64)
        for r in range(3):
            a, b = offsets[r], offsets[r + 1]
            if b > a:
                # the literal loop takes wrapped positions: exact while every displacement is < L/2
                _, ne = omd.coarse_grain_literal(lx, L, pos[p - 1, a:b], pos[p, a:b])
                lit += ne
        assert np.array_equal(f[p - 1], lit)
    # ensemble sums are the sums of the single-replica calls
    tot_f = np.zeros_like(f)
    tot_x = np.zeros_like(xi)
    for r in range(3):
        a, b = offsets[r], offsets[r + 1]
        fr, _, xr = omd.neq_mdlg(lx, L, [0, b - a], pos[:, a:b], img[:, a:b])
        tot_f += fr
        tot_x += xr
    assert np.array_equal(tot_f, f) and np.array_equal(tot_x, xi)


def test_two_snapshots_have_no_collision_term():
    pos, img = _walk(20, 10.0, 2, 0.5, seed=3)
    f, ovf, xi = omd.neq_mdlg(5, 10.0, [0, 20], pos, img)
    assert f.shape == (1, 49, 5, 5) and xi.shape == (0, 49, 5, 5)
    assert f.sum() + ovf.sum() == 20
