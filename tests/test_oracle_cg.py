"""Pins of the oracle's coarse-graining (Eq.(n_i)) and of its D2Q49 numbering."""
import os

import numpy as np
import pytest

from oracle import lattice, md
from tests import _sources as src

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_d2q49_table_shape_and_sets():
    t = lattice.d2q49()
    assert t.shape == (49, 2)
    assert len({(int(a), int(b)) for a, b in t}) == 49
    assert np.all(np.abs(t) <= 3)
    assert tuple(t[0]) == (0, 0)
    # the six D2Q25 sets of the Results section, one |v| per set, in the
    # printed index ranges, and nothing of |v_a| = 3 among indices 0..24
    rows = [tuple(map(int, ln.split())) for ln in open(os.path.join(GOLDEN, "d2q25_sets.txt"))
            if ln.strip() and not ln.startswith("#")]
    r2 = t[:, 0] ** 2 + t[:, 1] ** 2
    seen = set()
    for lo, hi in rows:
        vals = set(r2[lo:hi + 1].tolist())
        assert len(vals) == 1
        seen |= vals
    assert len(seen) == 6
    assert np.all(np.abs(t[:25]) <= 2)
    # 1..4 are the axis neighbours, 5..8 the diagonals (D2Q9 part)
    assert set(map(tuple, t[1:5].tolist())) == {(1, 0), (0, 1), (-1, 0), (0, -1)}
    assert set(map(tuple, t[5:9].tolist())) == {(1, 1), (-1, 1), (-1, -1), (1, -1)}


@pytest.mark.parametrize("lx,n,seed,u", [(8, 60, 0, (0.0, 0.0)), (9, 120, 1, (0.0, 0.0)),
                                         (10, 100, 2, (0.37, -0.21)), (7, 50, 3, (0.0, 0.0))])
def test_binned_equals_literal_definition(lx, n, seed, u):
    rng = np.random.default_rng(seed)
    L = lx * 2.3
    # displacements of up to ~2.5 cells per axis: some land outside D2Q49? no:
    # the literal form needs |v| < lx/2, so keep them inside +-3 cells
    x0, x1, i0, i1 = src.gaussian_step(rng, n, L, var=(1.1 * 2.3) ** 2)
    d = (x1 + L * i1) - x0
    keep = np.all(np.abs(d) < 2.4 * 2.3, axis=1)
    x0, x1, i0, i1 = x0[keep], x1[keep], i0[keep], i1[keep]
    k0, k1 = 3, 4
    cb, nb, _ = md.coarse_grain(lx, L, x0, x1, i0, i1, k0, k1, u=u, dense=True)
    cl, nl = md.coarse_grain_literal(lx, L, x0, x1, k0, k1, u=u)
    assert np.array_equal(cb, cl)
    assert np.array_equal(nb, nl)
    assert cb.sum() == len(x0)


def test_integer_displacements_give_known_counts():
    rng = np.random.default_rng(7)
    lx, L, n = 16, 40.0, 5000
    x0, x1, i0, i1, v = src.integer_step(rng, n, lx, L, vmax=4)
    counts, n_event, mom = md.coarse_grain(lx, L, x0, x1, i0, i1, dense=True)
    t = lattice.d2q49()
    expect = np.zeros(50, np.int64)
    for vx, vy in v:
        hit = np.nonzero((t[:, 0] == vx) & (t[:, 1] == vy))[0]
        expect[hit[0] if len(hit) else 49] += 1
    assert np.array_equal(counts, expect)
    # dense field: each particle sits at its destination cell
    dest = np.floor(x1 * (lx / L)).astype(int) % lx
    assert n_event.sum() == n - expect[49]
    for i in [0, 3, 17, 48]:
        sel = (v[:, 0] == t[i, 0]) & (v[:, 1] == t[i, 1])
        field = np.zeros((lx, lx), np.int64)
        np.add.at(field, (dest[sel, 1], dest[sel, 0]), 1)
        assert np.array_equal(n_event[i], field)
    # the displacement moments of whole-cell moves are exact multiples of dx
    dxl = L / lx
    d = v * dxl
    assert mom[0] == 2 * n
    assert mom[1] == pytest.approx(np.sum(d ** 2), rel=1e-12)
    assert mom[2] == pytest.approx(np.sum(d ** 4), rel=1e-12)
    assert mom[3] == pytest.approx(d[:, 0].sum(), abs=1e-9)


def test_sums_occupancy_and_momentum():
    rng = np.random.default_rng(9)
    lx, L, n = 24, 50.0, 20000
    x0, x1, i0, i1 = src.gaussian_step(rng, n, L, var=(0.9 * L / lx) ** 2)
    counts, n_event, _ = md.coarse_grain(lx, L, x0, x1, i0, i1, dense=True)
    inv = lx / L
    q0 = np.floor(x0 * inv).astype(np.int64)
    q1 = np.floor(x1 * inv).astype(np.int64)
    C0, C1 = q0, q1 + lx * i1
    dv = C1 - C0
    inside = np.all(np.abs(dv) <= 3, axis=1)
    # sum_i n_i(x, t) + overflow(x) = occupancy of cell x at time t
    occ = np.zeros((lx, lx), np.int64)
    np.add.at(occ, (q1[inside, 1] % lx, q1[inside, 0] % lx), 1)
    assert np.array_equal(n_event.sum(axis=0), occ)
    assert counts.sum() == n
    assert counts[49] == np.count_nonzero(~inside)
    # sum_x sum_i v_i n_i = sum_j (C_j(t) - C_j(t - dt_cg)) over D2Q49 particles
    t = lattice.d2q49()
    mom = (t[:, :, None, None] * n_event[:, None, :, :]).sum(axis=(0, 2, 3))
    assert np.array_equal(mom, dv[inside].sum(axis=0))


def test_permutation_invariance():
    rng = np.random.default_rng(10)
    lx, L, n = 20, 40.0, 3000
    x0, x1, i0, i1 = src.wsg_step(rng, n, L, mu2=(0.8 * L / lx) ** 2, lam=1.5)
    a = md.coarse_grain(lx, L, x0, x1, i0, i1, dense=True)
    p = rng.permutation(n)
    b = md.coarse_grain(lx, L, x0[p], x1[p], i0[p], i1[p], dense=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2][1] == pytest.approx(b[2][1], rel=1e-14)


def test_frame_shift_is_a_galilean_boost():
    # particles displaced by exactly one cell in x in the lab frame; a frame
    # drifting by u = (-1, 0) cells per coarse step sees them at rest
    rng = np.random.default_rng(12)
    lx, L, n = 16, 32.0, 2000
    dxl = L / lx
    cells = rng.integers(0, lx, (n, 2))
    x0 = (cells + rng.uniform(0.1, 0.9, (n, 2))) * dxl
    x1 = x0.copy()
    x1[:, 0] += dxl
    img = np.floor(x1 / L).astype(np.int64)
    x1 -= L * img
    c_lab, _, m_lab = md.coarse_grain(lx, L, x0, x1, None, img, 5, 6)
    c_mov, _, m_mov = md.coarse_grain(lx, L, x0, x1, None, img, 5, 6, u=(-1.0, 0.0))
    assert c_lab[1] == n and c_mov[0] == n
    assert m_lab[3] == pytest.approx(n * dxl, rel=1e-12)
    # moments about the drift: the boost leaves them at the box-frame displacement
    assert m_mov[3] == pytest.approx(n * dxl, rel=1e-12)
    assert m_mov[1] == m_lab[1]
    # a half-cell drift: the boosted count equals the count of the shifted positions
    c_half, _, _ = md.coarse_grain(lx, L, x0, x1, None, img, 0, 1, u=(0.5, 0.0))
    xs0 = x0.copy()
    xs1 = x1.copy()
    xs1[:, 0] += 0.5 * dxl
    ref, _, _ = md.coarse_grain(lx, L, xs0, xs1, None, img, 0, 1)
    assert np.array_equal(c_half, ref)


def _offset_grid(M, lx):
    """Particles at every in-cell offset (i/M, j/M) of every cell (dx = 1): exact binary fractions."""
    o = np.arange(M) / M
    c = np.arange(lx)
    x = (c[:, None] + o[None, :]).ravel()
    X, Y = np.meshgrid(x, x, indexing="ij")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


@pytest.mark.parametrize("s", [(0.0, 0.0), (0.125, 0.0), (0.625, 0.375), (3.5, 1.875)])
def test_translated_lattice_counts_crossing_fraction(s):
    # rigid displacement (3/8, 0) cells: exactly 3/8 of uniformly spread particles
    # cross one cell boundary, whatever the lattice origin
    lx, M = 6, 8
    p0 = _offset_grid(M, lx)
    p1 = p0 + np.array([3 / 8, 0.0])
    img1 = np.zeros(p1.shape, dtype=np.int64)
    img1[p1[:, 0] >= lx, 0] = 1
    p1[p1[:, 0] >= lx, 0] -= lx
    c, _ = md.coarse_grain_shift(lx, float(lx), p0, p1, np.zeros_like(img1), img1, s, s)
    n = p0.shape[0]
    v = lattice.d2q49()
    i10 = int(np.flatnonzero((v[:, 0] == 1) & (v[:, 1] == 0))[0])
    assert c[i10] * 8 == 3 * n
    assert c[0] * 8 == 5 * n
    assert c.sum() == n


def test_shift_difference_acts_as_drift():
    # a later lattice shifted by u dx = (1/4, -1/8) relative to the earlier one,
    # particles at rest: the fractions 1/4 and 1/8 see velocities +1 in x and -1 in y
    lx, M = 5, 8
    p = _offset_grid(M, lx)
    z = np.zeros(p.shape, dtype=np.int64)
    c, _ = md.coarse_grain_shift(lx, float(lx), p, p, z, z, (0.5, 0.25), (0.75, 0.125))
    n = p.shape[0]
    v = lattice.d2q49()
    idx = {tuple(v[i]): i for i in range(49)}
    assert c[idx[(1, 0)]] * 32 == n * (1 * 7)    # x crosses (1/4), y does not (7/8)
    assert c[idx[(0, -1)]] * 32 == n * (3 * 1)   # x stays (3/4), y crosses (1/8)
    assert c[idx[(1, -1)]] * 32 == n * (1 * 1)
    assert c[idx[(0, 0)]] * 32 == n * (3 * 7)
