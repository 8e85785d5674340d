"""Pins of the oracle's molecular dynamics against what the physics fixes.

The oracle implements the 6-12 Lennard-Jones potential and velocity-Verlet
NVE integration of the "Simulations setup" section.  Nothing here compares
the oracle with itself: each test checks a closed form, an invariant, a
special case with a known answer, or a brute-force evaluation.
"""
import math

import numpy as np
import pytest

import mdlg_inputs as mi
from oracle import md

RC = 2.5


def lj_force_closed(r):
    """-dV/dr of V = 4 (r^-12 - r^-6), differentiated by hand."""
    return 48.0 * r ** -13 - 24.0 * r ** -7


def test_pair_force_closed_form():
    L = 20.0
    for r in [0.9, 1.0, 2.0 ** (1 / 6), 1.5, 2.2, 2.499]:
        pos = np.array([[5.0, 7.0], [5.0 + r, 7.0]])
        f, pe = md.forces(pos, L, shift=False, method="brute")
        # particle 0 sits at smaller x: a repulsive force pushes it to -x
        assert f[0, 0] == pytest.approx(-lj_force_closed(r), rel=1e-13, abs=1e-13)
        assert f[1, 0] == pytest.approx(lj_force_closed(r), rel=1e-13, abs=1e-13)
        assert f[0, 1] == 0.0 and f[1, 1] == 0.0
        assert pe == pytest.approx(4 * (r ** -12 - r ** -6), rel=1e-13)
    # at the minimum of the potential the force vanishes
    pos = np.array([[1.0, 1.0], [1.0 + 2.0 ** (1 / 6), 1.0]])
    f, _ = md.forces(pos, L, method="brute")
    assert abs(f[0, 0]) < 1e-12


def test_cutoff_and_energy_shift():
    L = 20.0
    vrc = 4 * (RC ** -12 - RC ** -6)
    assert vrc == pytest.approx(-0.0163169, abs=1e-7)
    pos = np.array([[1.0, 1.0], [1.0 + RC + 1e-9, 1.0]])
    f, pe = md.forces(pos, L, shift=True, method="brute")
    assert np.all(f == 0.0) and pe == 0.0
    r = 1.3
    pos = np.array([[1.0, 1.0], [1.0, 1.0 + r]])
    _, pe = md.forces(pos, L, shift=True, method="brute")
    assert pe == pytest.approx(4 * (r ** -12 - r ** -6) - vrc, rel=1e-13)


def test_minimum_image_across_boundary():
    L = 10.0
    r = 1.2
    pos = np.array([[0.2, 5.0], [L - (r - 0.2), 5.0]])
    f, _ = md.forces(pos, L, method="brute")
    assert f[0, 0] == pytest.approx(lj_force_closed(r), rel=1e-12)


def _dense_config(n, phi, seed):
    pos, vel, L = mi.initial_state(n, phi, 20.0, seed)
    return pos, vel, L


@pytest.mark.parametrize("n,phi", [(400, 0.4), (1000, 0.2), (4096, 0.0784)])
def test_cells_equal_brute_force(n, phi):
    pos, vel, L = _dense_config(n, phi, 3)
    # advance a little so that particles interact (the grid start has gaps)
    pos, vel, img, _ = md.md_run(pos, vel, np.zeros((n, 2), np.int64), L, 300, cells=True)
    fb, peb = md.forces(pos, L, method="brute")
    fc, pec = md.forces(pos, L, method="cells")
    scale = np.abs(fb).max()
    assert scale > 0
    assert np.max(np.abs(fb - fc)) <= 1e-13 * scale
    assert pec == pytest.approx(peb, rel=1e-13)


def test_newton_third_law():
    pos, vel, L = _dense_config(1000, 0.4, 5)
    pos, vel, img, _ = md.md_run(pos, vel, np.zeros((1000, 2), np.int64), L, 200)
    f, _ = md.forces(pos, L)
    assert np.linalg.norm(f.sum(axis=0)) <= 1e-12 * np.abs(f).sum()


def test_grid_start_has_no_potential_energy():
    # phi = 0.0784, N = 512: a 23 x 23 grid of spacing L/23 = 3.114 sigma; the
    # jitter of +-0.25 sigma per axis keeps every pair beyond 2.61 sigma > rc.
    pos, vel, L = mi.initial_state(512, 0.0784, 20.0, 0)
    assert L == pytest.approx(71.618, abs=1e-3)
    e = md.energy(pos, vel, L)
    assert e[1] == 0.0
    assert e[0] == pytest.approx(511 * 20.0, rel=1e-13)
    assert abs(e[2]) < 1e-10 and abs(e[3]) < 1e-10


def test_conservation_dense_gas():
    n = 512
    pos, vel, L = mi.initial_state(n, 0.4, 20.0, 11)
    img = np.zeros((n, 2), np.int64)
    pos, vel, img, et = md.md_run(pos, vel, img, L, 2000, energy_every=100)
    ke0 = et[0, 0]
    e_tot = et[:, 0] + et[:, 1]
    assert np.max(np.abs(et[:, 1])) > 1.0  # collisions happened
    assert np.max(np.abs(e_tot - e_tot[0])) / ke0 <= 1e-6
    vth = math.sqrt(20.0)
    assert np.max(np.abs(et[:, 2:] - et[0, 2:])) <= 1e-10 * math.sqrt(n) * vth


def test_time_reversal():
    n = 400
    pos0, vel0, L = mi.initial_state(n, 0.3, 20.0, 2)
    img0 = np.zeros((n, 2), np.int64)
    pos, vel, img, _ = md.md_run(pos0.copy(), vel0.copy(), img0.copy(), L, 500)
    vel = -vel
    pos, vel, img, _ = md.md_run(pos, vel, img, L, 500)
    unwrapped = pos + L * img
    assert np.max(np.abs(unwrapped - pos0)) < 1e-8
    assert np.max(np.abs(-vel - vel0)) < 1e-8


def test_free_particles_stream():
    # eps = 0 switches the interaction off: x(t) = x0 + v t exactly, up to rounding
    n = 300
    pos0, vel0, L = mi.initial_state(n, 0.2, 20.0, 4, positions="uniform")
    steps, dt = 1000, 1e-4
    pos, vel, img, _ = md.md_run(pos0.copy(), vel0.copy(), np.zeros((n, 2), np.int64), L, steps,
                                 dt=dt, eps=0.0)
    assert np.array_equal(vel, vel0)
    expect = pos0 + vel0 * (steps * dt)
    assert np.max(np.abs((pos + L * img) - expect)) < 1e-10


def test_head_on_collision_is_symmetric():
    L = 30.0
    pos = np.array([[10.0, 15.0], [14.0, 15.0]])
    vel = np.array([[5.0, 0.0], [-5.0, 0.0]])
    img = np.zeros((2, 2), np.int64)
    pos, vel, img, et = md.md_run(pos, vel, img, L, 20000, energy_every=1000)
    # elastic bounce: velocities reversed, centre of mass fixed, y untouched
    assert vel[0, 0] == pytest.approx(-5.0, rel=1e-6)
    assert vel[1, 0] == pytest.approx(5.0, rel=1e-6)
    assert (pos[0, 0] + pos[1, 0]) / 2 == pytest.approx(12.0, abs=1e-10)
    assert np.all(pos[:, 1] == 15.0)
    e = et[:, 0] + et[:, 1]
    # the force jumps at rc (energy-shifted, force unshifted): O(dt) energy kick per crossing
    assert np.max(np.abs(e - e[0])) / e[0] < 1e-6
