"""GPU parity of the trajectory coarse-graining for many lags and drifts
(mdlg_coarse_grain_series) with the oracle's single-event coarse-graining on
the translated lattice of each pair, summed over every snapshot pair: counts
bit-exact, moments within 1e-12."""
import math

import numpy as np
import pytest

from oracle import md as omd

pytestmark = pytest.mark.gpu


def walk(n, L, P, step, seed):
    """Random-walk snapshots wrapped into [0, L) with image counts (inputs only)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(0.0, L, (n, 2))
    img = np.zeros((n, 2), dtype=np.int32)
    xs, imgs = [x.copy()], [img.copy()]
    for _ in range(P - 1):
        y = x + rng.normal(0.0, step, (n, 2))
        k = np.floor(y / L)
        x = y - k * L
        k[x >= L] += 1
        x[x >= L] = 0.0
        img = img + k.astype(np.int32)
        xs.append(x.copy())
        imgs.append(img.copy())
    return np.stack(xs), np.stack(imgs)


def reference(specs, xs, imgs, lags, us, offs=None):
    """Sum of oracle events over all pairs (p - l, p): lattice shifted by o dx
    and (o + u) dx, o = offs[p - l]."""
    P = xs.shape[0]
    off = 0
    counts = np.zeros((len(specs), len(lags), len(us), 50), dtype=np.int64)
    moments = np.zeros((len(specs), len(lags), 5))
    for r, (n, L, lx, _) in enumerate(specs):
        sl = slice(off, off + n)
        off += n
        if n == 0:
            continue
        for s, l in enumerate(lags):
            for t, u in enumerate(us):
                m = np.zeros(5)
                dxl = L / lx
                for p in range(l, P):
                    o = np.zeros(2) if offs is None else np.asarray(offs[p - l], dtype=np.float64)
                    uu = np.asarray(u, dtype=np.float64)
                    omd.coarse_grain_shift(lx, L, xs[p - l, sl], xs[p, sl], imgs[p - l, sl], imgs[p, sl],
                                           o * dxl, (o + uu) * dxl, counts=counts[r, s, t], moments=m)
                if t == 0:
                    moments[r, s] = m
    return counts, moments


def run(specs, lags, us, P, seed=0, repeat=1, offs=None):
    import torch

    import paper_2101_01160_amd as m
    xs, imgs = [], []
    for r, (n, L, lx, step) in enumerate(specs):
        x, i = walk(n, L, P, step, seed + r)
        xs.append(x)
        imgs.append(i)
    xs = np.concatenate(xs, axis=1)
    imgs = np.concatenate(imgs, axis=1)
    offsets = np.concatenate([[0], np.cumsum([s[0] for s in specs])])
    counts = torch.zeros((len(specs), len(lags), len(us), 50), dtype=torch.int64, device="cuda")
    moments = torch.zeros((len(specs), len(lags), 5), dtype=torch.float64, device="cuda")
    pos = torch.from_numpy(np.ascontiguousarray(xs)).cuda()
    img = torch.from_numpy(np.ascontiguousarray(imgs)).cuda()
    for _ in range(repeat):
        m.mdlg_coarse_grain_series(offsets, [s[1] for s in specs], [s[2] for s in specs], pos, img, lags, us,
                                   counts, moments, lattice_offset=offs)
    torch.cuda.synchronize()
    return xs, imgs, counts.cpu().numpy(), moments.cpu().numpy()


def check(specs, lags, us, P, seed=0, offs=None):
    print(f"cg_series specs={specs} lags={lags} n_u={len(us)} P={P} offsets={offs is not None}", flush=True)
    xs, imgs, c, mo = run(specs, lags, us, P, seed, offs=offs)
    rc, rm = reference(specs, xs, imgs, lags, us, offs)
    assert np.array_equal(c, rc)
    scale = np.maximum(1.0, np.abs(rm).max())
    assert np.allclose(mo, rm, rtol=1e-12, atol=1e-12 * scale)
    return c


@pytest.mark.parametrize("with_offsets", [False, True])
def test_series_matches_summed_events(with_offsets):
    specs = [(300, 30.0, 15, 0.4), (129, 20.0, 10, 0.9), (0, 10.0, 5, 0.1), (200, 17.3, 5, 3.0)]
    lags = [1, 2, 5, 7]
    us = [(0.0, 0.0), (0.13, -0.07), (-0.2, 0.19)]
    offs = np.random.default_rng(9).uniform(0.0, 1.0, (9, 2)) if with_offsets else None
    c = check(specs, lags, us, P=9, offs=offs)
    # the large steps of the last replica reach the overflow bin
    assert c[3, :, :, 49].sum() > 0
    # every particle lands in one bin per pair
    for r, (n, *_rest) in enumerate(specs):
        for s, l in enumerate(lags):
            assert np.all(c[r, s].sum(axis=-1) == n * (9 - l))


def test_series_largest_configuration():
    # 32 lags x 8 drifts = 256 jobs with a 32-deep ring: the full LDS budget
    specs = [(257, 40.0, 20, 0.3), (64, 12.0, 6, 0.5)]
    lags = list(range(1, 33))
    rng = np.random.default_rng(1)
    us = [tuple(v) for v in rng.uniform(-0.2, 0.2, (8, 2))]
    check(specs, lags, us, P=34, seed=5, offs=rng.uniform(-2.0, 2.0, (34, 2)))


def test_series_accumulates():
    specs = [(100, 15.0, 7, 0.5)]
    lags, us = [1, 3], [(0.1, 0.0)]
    _, _, c1, m1 = run(specs, lags, us, P=6)
    _, _, c2, m2 = run(specs, lags, us, P=6, repeat=2)
    assert np.array_equal(c2, 2 * c1)
    assert np.allclose(m2, 2 * m1, rtol=1e-14)


def test_series_invalid_arguments():
    import torch

    import paper_2101_01160_amd as m
    pos = torch.zeros((4, 10, 2), dtype=torch.float64, device="cuda")
    img = torch.zeros((4, 10, 2), dtype=torch.int32, device="cuda")
    off = [0, 10]

    def call(lags, us):
        counts = torch.zeros((1, len(lags), len(us), 50), dtype=torch.int64, device="cuda")
        m.mdlg_coarse_grain_series(off, [5.0], [3], pos, img, lags, us, counts)

    call([1, 3], [(0.0, 0.0)])
    for lags, us in (([4], [(0.0, 0.0)]), ([0], [(0.0, 0.0)]), ([1], [(0.0, 0.0)] * 17),
                     ([1], [(math.nan, 0.0)])):
        with pytest.raises(m.MDLGError, match="EINVAL"):
            call(lags, us)
