"""GPU parity of the standalone coarse-graining (mdlg_coarse_grain) with the
oracle: integer outputs bit-exact, moments within 1e-12 relative."""
import math

import numpy as np
import pytest

from oracle import md as omd
from tests import _sources as src

pytestmark = pytest.mark.gpu


def _cuda(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def run_gpu(lx, L, x0, x1, i0, i1, k0=0, k1=1, u=(0.0, 0.0), dense=True, acc=True):
    import torch

    import paper_2101_01160_amd as m
    n = x0.shape[0]
    counts = torch.zeros(50, dtype=torch.int64, device="cuda")
    moments = torch.zeros(5, dtype=torch.float64, device="cuda")
    n_event = torch.full((49, lx, lx), 7, dtype=torch.int32, device="cuda") if dense else None
    cell_acc = torch.zeros((49, lx, lx), dtype=torch.int32, device="cuda") if acc else None
    ip = None if i0 is None else _cuda(i0, torch.int32)
    ic = None if i1 is None else _cuda(i1, torch.int32)
    m.mdlg_coarse_grain(lx, L, _cuda(x0), _cuda(x1), counts, moments, ip, ic, k0, k1, u, n_event, cell_acc)
    torch.cuda.synchronize()
    return (counts.cpu().numpy(), None if n_event is None else n_event.cpu().numpy(), moments.cpu().numpy(),
            None if cell_acc is None else cell_acc.cpu().numpy())


def compare(lx, L, x0, x1, i0, i1, k0=0, k1=1, u=(0.0, 0.0)):
    print(f"coarse_grain n={x0.shape[0]} lx={lx} L={L:.3f} k=({k0},{k1}) u={u}", flush=True)
    cg, ng, mg, ag = run_gpu(lx, L, x0, x1, i0, i1, k0, k1, u)
    co, no, mo = omd.coarse_grain(lx, L, x0, x1, i0, i1, k0, k1, u=u, dense=True)
    assert np.array_equal(cg, co)
    assert np.array_equal(ng, no)
    assert np.array_equal(ag, no)
    assert mg[0] == mo[0]
    for j in range(1, 5):
        assert mg[j] == pytest.approx(mo[j], rel=1e-12, abs=1e-12 * math.sqrt(max(mo[1], 1e-300)))
    return cg


@pytest.mark.parametrize("n", [1, 63, 256, 1000, 4097, 100_003])
def test_gaussian_steps_ragged_sizes(n):
    rng = np.random.default_rng(n)
    lx, L = 32, 71.618
    x0, x1, i0, i1 = src.gaussian_step(rng, n, L, var=(1.2 * L / lx) ** 2)
    compare(lx, L, x0, x1, i0, i1)


def test_integer_displacements_and_overflow():
    rng = np.random.default_rng(1)
    lx, L, n = 64, 140.0, 200_000
    x0, x1, i0, i1, v = src.integer_step(rng, n, lx, L, vmax=5)
    c = compare(lx, L, x0, x1, i0, i1)
    assert c[49] > 0 and c.sum() == n


def test_images_and_frame_shift():
    rng = np.random.default_rng(2)
    lx, L, n = 50, 100.0, 50_000
    x0, x1, i0, i1 = src.wsg_step(rng, n, L, mu2=(0.7 * L / lx) ** 2, lam=1.2)
    # both snapshots carry image counts
    i0 = rng.integers(-3, 4, (n, 2)).astype(np.int64)
    i1 = i1 + i0
    compare(lx, L, x0, x1, i0, i1, k0=17, k1=18, u=(0.13, -0.19))
    compare(lx, L, x0, x1, i0, i1, k0=1000, k1=1001, u=(-0.2, 0.05))


def test_null_images_and_empty_input():
    import torch

    import paper_2101_01160_amd as m
    rng = np.random.default_rng(3)
    lx, L, n = 16, 30.0, 3000
    x0 = rng.uniform(0, L, (n, 2))
    x1 = np.mod(x0 + rng.normal(0, 0.5, (n, 2)), L)
    compare(lx, L, x0, x1, None, None)
    counts = torch.zeros(50, dtype=torch.int64, device="cuda")
    e = torch.empty((0, 2), dtype=torch.float64, device="cuda")
    m.mdlg_coarse_grain(lx, L, e, e, counts)
    torch.cuda.synchronize()
    assert int(counts.sum()) == 0


def test_counts_accumulate_and_cell_boundaries():
    # positions exactly on cell edges: the floor rule puts them in the upper cell
    lx, L = 10, 25.0
    dxl = L / lx
    g = np.arange(lx) * dxl
    x0 = np.stack(np.meshgrid(g, g), axis=-1).reshape(-1, 2)
    x1 = x0.copy()
    x1[:, 0] = np.mod(x1[:, 0] + dxl, L)
    i1 = np.zeros_like(x0, dtype=np.int64)
    i1[:, 0] = (x0[:, 0] + dxl >= L).astype(np.int64)
    c = compare(lx, L, x0, x1, np.zeros_like(i1), i1)
    assert c[1] == lx * lx


def test_large_lattice_one_million():
    rng = np.random.default_rng(4)
    lx, L, n = 1024, 3241.058, 1 << 20
    x0, x1, i0, i1 = src.gaussian_step(rng, n, L, var=0.02)
    compare(lx, L, x0, x1, i0, i1)


def test_invalid_arguments_are_rejected():
    import torch

    import paper_2101_01160_amd as m
    x = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    counts = torch.zeros(50, dtype=torch.int64, device="cuda")
    with pytest.raises(m.MDLGError):
        m.mdlg_coarse_grain(0, 10.0, x, x, counts)
    with pytest.raises(m.MDLGError):
        m.mdlg_coarse_grain(8, -1.0, x, x, counts)
    with pytest.raises(ValueError):
        m.mdlg_coarse_grain(8, 10.0, x.float(), x, counts)
