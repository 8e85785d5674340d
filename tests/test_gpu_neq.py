"""GPU parity of the non-equilibrium MDLG sums (mdlg_neq_mdlg) with the
oracle, which builds every replica's n_i and Xi_i from the definitions before
summing: ensemble occupation sums, overflow counts and collision-operator
sums bit-exact, on random-walk ensembles (several lattices, with and without
displacements beyond D2Q49, 2 and 3 snapshots, many snapshots per block
chunk), on positions exactly on cell edges and just below the box side, and on
an ensemble of the GPU MD started as a shear wave."""
import numpy as np
import pytest

from oracle import md as omd

pytestmark = pytest.mark.gpu


def walk(n, L, P, step, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(0.0, L, (n, 2))
    xs = [x]
    for _ in range(P - 1):
        x = x + rng.normal(0.0, step, (n, 2))
        xs.append(x)
    xs = np.stack(xs)
    img = np.floor(xs / L).astype(np.int64)
    pos = xs - L * img
    img[pos >= L] += 1
    pos[pos >= L] = 0.0
    return pos, img.astype(np.int32)


def gpu(L, lx, pos, img, xi=True):
    import torch

    import paper_2101_01160_amd as m
    P, n = pos.shape[0], pos.shape[1]
    tp = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
    ti = torch.from_numpy(np.ascontiguousarray(img, dtype=np.int32)).cuda()
    f = torch.full((P - 1, 49, lx, lx), 7, dtype=torch.int32, device="cuda")   # overwritten
    o = torch.full((P - 1,), 7, dtype=torch.int64, device="cuda")
    x = torch.full((max(P - 2, 0), 49, lx, lx), 7, dtype=torch.int32, device="cuda") if xi else None
    m.mdlg_neq_mdlg(L, lx, tp, ti, f, o, x)
    torch.cuda.synchronize()
    return f.cpu().numpy(), o.cpu().numpy(), (x.cpu().numpy() if xi else None)


@pytest.mark.parametrize("n,L,lx,P,step", [(3000, 40.0, 16, 9, 1.2), (257, 30.0, 7, 40, 3.0),
                                           (5000, 64.0, 33, 3, 0.8), (100, 20.0, 10, 2, 1.0),
                                           (20000, 100.0, 25, 6, 2.5)])
def test_random_walk_ensemble_matches_oracle(n, L, lx, P, step):
    print("neq walk", n, L, lx, P, step, flush=True)
    pos, img = walk(n, L, P, step, seed=n + lx)
    f, o, x = gpu(L, lx, pos, img)
    rf, ro, rx = omd.neq_mdlg(lx, L, [0, n], pos, img)
    assert np.array_equal(f, rf) and np.array_equal(o, ro)
    assert np.array_equal(x, rx)
    fo, oo, _ = gpu(L, lx, pos, img, xi=False)
    assert np.array_equal(fo, rf) and np.array_equal(oo, ro)


def test_cell_edges_and_box_side():
    L, lx, n, P = 25.0, 7, 512, 4
    rng = np.random.default_rng(4)
    k = rng.integers(0, 7, (P, n, 2))
    pos = k * (L / lx)                                 # on (the rounded) cell edges
    pos[:, :16] = np.nextafter(L, 0.0)                 # here x lx / L rounds up to lx
    assert np.floor(np.nextafter(L, 0.0) * (lx / L)) == lx
    img = rng.integers(-2, 3, (P, n, 2)).astype(np.int32)
    f, o, x = gpu(L, lx, pos, img)
    rf, ro, rx = omd.neq_mdlg(lx, L, [0, n], pos, img)
    assert np.array_equal(f, rf) and np.array_equal(o, ro) and np.array_equal(x, rx)
    assert o.sum() > 0


def test_shear_wave_md_ensemble_matches_oracle():
    import torch

    import mdlg_inputs as mi
    import paper_2101_01160_amd as m
    R, n, L, lx, s_cg, P = 6, 998, 100.0, 25, 400, 7
    states = [mi.shear_wave_state(n, L, 20.0, 4.0, seed=100 + r) for r in range(R)]
    pos0 = np.concatenate([s[0] for s in states])
    vel0 = np.concatenate([s[1] for s in states])
    sysm = m.LJSystem(torch.from_numpy(pos0).cuda(), torch.from_numpy(vel0).cuda(),
                      params=[m.lj_params(n, L) for _ in range(R)])
    sp = torch.empty((P, R * n, 2), dtype=torch.float64, device="cuda")
    si = torch.empty((P, R * n, 2), dtype=torch.int32, device="cuda")
    for p in range(P):
        if p:
            sysm.step(s_cg)
        m.lj_md_get_state(sysm.handle, sp[p], None, si[p])
    torch.cuda.synchronize()
    sysm.check()
    sysm.close()
    pos, img = sp.cpu().numpy(), si.cpu().numpy()
    f, o, x = gpu(L, lx, pos, img)
    rf, ro, rx = omd.neq_mdlg(lx, L, [0, R * n], pos, img)
    assert np.array_equal(f, rf) and np.array_equal(o, ro) and np.array_equal(x, rx)
    # the flow is visible: more +x than -x lattice moves in the rows where sin > 0
    assert f[0, 1, 2:10].sum() > f[0, 3, 2:10].sum()


def test_invalid_arguments_raise():
    import torch

    import paper_2101_01160_amd as m
    pos, img = walk(10, 10.0, 3, 0.5, seed=1)
    tp, ti = torch.from_numpy(pos).cuda(), torch.from_numpy(img).cuda()
    for L, lx in ((10.0, 6), (0.0, 8), (float("inf"), 8)):
        f = torch.zeros((2, 49, lx, lx), dtype=torch.int32, device="cuda")
        o = torch.zeros(2, dtype=torch.int64, device="cuda")
        with pytest.raises(m.MDLGError):
            m.mdlg_neq_mdlg(L, lx, tp, ti, f, o)
