"""Seeded synthetic inputs for the 2D Lennard-Jones MDLG workloads.

This module only draws random numbers and lays out arrays.  It holds none of
the method's arithmetic (no forces, no integration, no coarse-graining, no
closed forms), so both the CPU oracle and the GPU path may take their inputs
from it.

Recipe (the paper's workload, Section "Simulations setup": a dilute hot 2D
LJ gas at area fraction phi with homogeneous initial positions and kinetic
energy at temperature kT, zero mean velocity):

* box side  L = sqrt(N * pi * sigma^2 / (4 phi))   (area fraction definition)
* positions: jittered square grid, nx = ceil(sqrt(N)), ny = ceil(N / nx);
  site (i, j) at ((i + 1/2) L/nx, (j + 1/2) L/ny), filled row-major, each
  coordinate jittered by U(-0.25, 0.25) sigma, then wrapped into [0, L).
  `positions="uniform"` draws U[0, L) instead (used where the shared
  in-cell offset of the grid would bias early-time lattice statistics).
* velocities: N(0, kT) per axis, mean removed, rescaled so that the kinetic
  energy equals (N - 1) kT (2N - 2 degrees of freedom in 2D).
* random numbers: numpy PCG64(seed); draws are made as four blocks of N:
  jitter_x, jitter_y, v_x, v_y (uniform positions: x, y, v_x, v_y).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "box_length",
    "initial_state",
    "uniform_positions",
    "jittered_grid",
    "maxwell_velocities",
    "ReplicaSpec",
    "replica_sweep",
    "surrogate_sweep",
    "mlp_init",
    "shear_wave_state",
]


def box_length(n: int, phi: float) -> float:
    """Side of the square box holding n discs of diameter 1 at area fraction phi."""
    return math.sqrt(n * math.pi / (4.0 * phi))


def _wrap(a: np.ndarray, L: float) -> np.ndarray:
    a = np.mod(a, L)
    a[a >= L] = 0.0
    return a


def jittered_grid(n: int, L: float, rng: np.random.Generator, jitter: float = 0.25) -> np.ndarray:
    nx = int(math.ceil(math.sqrt(n)))
    ny = int(math.ceil(n / nx))
    k = np.arange(n)
    i = k % nx
    j = k // nx
    jx = rng.uniform(-jitter, jitter, n)
    jy = rng.uniform(-jitter, jitter, n)
    x = (i + 0.5) * (L / nx) + jx
    y = (j + 0.5) * (L / ny) + jy
    return np.ascontiguousarray(np.stack([_wrap(x, L), _wrap(y, L)], axis=1))


def uniform_positions(n: int, L: float, rng: np.random.Generator) -> np.ndarray:
    x = rng.uniform(0.0, L, n)
    y = rng.uniform(0.0, L, n)
    return np.ascontiguousarray(np.stack([_wrap(x, L), _wrap(y, L)], axis=1))


def maxwell_velocities(n: int, kT: float, rng: np.random.Generator) -> np.ndarray:
    v = np.stack([rng.normal(0.0, math.sqrt(kT), n), rng.normal(0.0, math.sqrt(kT), n)], axis=1)
    if n > 1:
        v -= v.mean(axis=0, keepdims=True)
        ke = 0.5 * float(np.sum(v * v))
        target = (n - 1) * kT
        if ke > 0.0:
            v *= math.sqrt(target / ke)
    return np.ascontiguousarray(v)


def initial_state(n: int, phi: float, kT: float, seed: int, positions: str = "grid"):
    """Return (pos [n,2] f64 in [0,L), vel [n,2] f64, L)."""
    L = box_length(n, phi)
    rng = np.random.Generator(np.random.PCG64(seed))
    if positions == "grid":
        pos = jittered_grid(n, L, rng)
    elif positions == "uniform":
        pos = uniform_positions(n, L, rng)
    else:
        raise ValueError(f"unknown positions kind {positions!r}")
    vel = maxwell_velocities(n, kT, rng)
    return pos, vel, L


@dataclass(frozen=True)
class ReplicaSpec:
    n: int
    phi: float
    kT: float
    seed: int
    L: float
    lx: int


def replica_sweep(n_rep: int = 256, n_min: int = 4096, n_max: int = 262144,
                  phis=(0.0784, 0.2, 0.4), kTs=(1.0, 5.0, 20.0), cell=2.0):
    """Replica table of the batched workload.

    Replica r takes grid entry m = r mod 9: phi = phis[m // 3], kT = kTs[m % 3];
    its size is round(exp(U(ln n_min, ln n_max))) drawn from PCG64(seed=r);
    its particle seed is r; its lattice has lx = max(4, round(L / cell)) cells.
    """
    out = []
    for r in range(n_rep):
        m = r % (len(phis) * len(kTs))
        phi = phis[m // len(kTs)]
        kT = kTs[m % len(kTs)]
        rng = np.random.Generator(np.random.PCG64(r))
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        L = box_length(n, phi)
        lx = max(4, int(round(L / cell)))
        out.append(ReplicaSpec(n=n, phi=phi, kT=kT, seed=r, L=L, lx=lx))
    return out


def surrogate_sweep(n_rep: int, seed: int = 12345, n: int = 16384,
                    phi_range=(0.05, 0.4), kT_range=(1.0, 20.0), cell=2.0):
    """Replica table for surrogate training data: phi ~ U(phi_range), kT ~ U(kT_range)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for r in range(n_rep):
        phi = float(rng.uniform(*phi_range))
        kT = float(rng.uniform(*kT_range))
        L = box_length(n, phi)
        lx = max(4, int(round(L / cell)))
        out.append(ReplicaSpec(n=n, phi=phi, kT=kT, seed=seed * 1000 + r, L=L, lx=lx))
    return out


def shear_wave_state(n: int, L: float, kT: float, amp: float, seed: int, modes: int = 1):
    """A flowing (non-equilibrium) start for the ensemble workload: jittered-grid
    positions in a box of side L and Maxwellian velocities at kT (as
    initial_state, same draws), plus a transverse wave
    v_x += amp * sin(2 pi modes y / L).  Returns (pos, vel)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = jittered_grid(n, L, rng)
    vel = maxwell_velocities(n, kT, rng)
    vel[:, 0] += amp * np.sin(2.0 * math.pi * modes * pos[:, 1] / L)
    return pos, np.ascontiguousarray(vel)


MLP_DIMS = (6, 256, 256, 256, 49)


def mlp_init(seed: int) -> np.ndarray:
    """Initial parameters of the f_eq surrogate network, one flat float64 vector
    in the order W1 [6,256], b1, W2 [256,256], b2, W3, b3, W4 [256,49], b4:
    weights U(-a, a) with a = sqrt(6 / (fan_in + fan_out)), biases zero,
    drawn from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fi, fo in zip(MLP_DIMS[:-1], MLP_DIMS[1:]):
        a = math.sqrt(6.0 / (fi + fo))
        parts.append(rng.uniform(-a, a, fi * fo))
        parts.append(np.zeros(fo))
    return np.concatenate(parts)
