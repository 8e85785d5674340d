"""GPU parity of the velocity autocorrelation sums (mdlg_vacf) with the
oracle's sums over particles and origins (FP64, within 1e-12 relative), on
ragged replica batches with an empty replica, lags 0 .. n_snap - 1, repeated
accumulation, and velocity snapshots of the GPU MD; lambda from the MD's VACF
through the library against the oracle's reading."""
import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import md as omd

pytestmark = pytest.mark.gpu


def run(offsets, vel, lags, repeat=1):
    import torch

    import paper_2101_01160_amd as m
    tv = torch.from_numpy(np.ascontiguousarray(vel)).cuda()
    c = torch.zeros((len(offsets) - 1, len(lags)), dtype=torch.float64, device="cuda")
    for _ in range(repeat):
        m.mdlg_vacf(offsets, tv, lags, c)
    torch.cuda.synchronize()
    return c.cpu().numpy()


def test_ragged_batch_matches_oracle():
    rng = np.random.default_rng(12)
    sizes = [700, 0, 1, 300, 4097]
    P = 33
    vel = rng.normal(0.0, 4.0, (P, sum(sizes), 2))
    offsets = np.concatenate([[0], np.cumsum(sizes)])
    lags = [0, 1, 2, 5, 16, 31, 32]
    got = run(offsets, vel, lags, repeat=2)
    ref = omd.vacf_sums(offsets, vel, lags)
    assert np.allclose(got, 2 * ref, rtol=1e-12, atol=1e-9)
    assert (got[1] == 0).all()


def test_md_velocities_and_lambda():
    import torch

    import mdlg_inputs as mi
    import paper_2101_01160_amd as m
    n, P, stride = 4096, 120, 20
    pos0, vel0, L = mi.initial_state(n, 0.0784, 20.0, seed=3)
    sysm = m.LJSystem(torch.from_numpy(pos0).cuda(), torch.from_numpy(vel0).cuda(), box_l=L)
    sysm.step(2000)
    vs = torch.empty((P, n, 2), dtype=torch.float64, device="cuda")
    for p in range(P):
        if p:
            sysm.step(stride)
        m.lj_md_get_state(sysm.handle, None, vs[p], None)
    torch.cuda.synchronize()
    sysm.check()
    sysm.close()
    vel = vs.cpu().numpy()
    lags = list(range(0, P - 20))
    got = run([0, n], vel, lags)[0]
    ref = omd.vacf_sums([0, n], vel, lags)[0]
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-9)
    c = got / np.array([n * (P - l) for l in lags])
    t = np.array(lags) * stride * 1e-4
    tau, lam = m.mdlg_lambda_vacf(t, c, 0.3911, 0.01)
    rtau, rlam = cf.lambda_vacf(t, ref / np.array([n * (P - l) for l in lags]), 0.3911, 0.01)
    assert tau == pytest.approx(rtau, rel=1e-9) and lam == pytest.approx(rlam, rel=1e-9)
    print(f"VACF: C(0) = {c[0]:.3f} (2 kT = 40), tau = {tau:.3f}, lambda(0.3911) = {lam:.3f}", flush=True)
    assert 30.0 < c[0] < 50.0 and 0.05 < tau < 20.0


def test_invalid_arguments_raise():
    import torch

    import paper_2101_01160_amd as m
    vel = torch.zeros((4, 10, 2), dtype=torch.float64, device="cuda")
    c = torch.zeros((1, 1), dtype=torch.float64, device="cuda")
    for lags in ([4], [-1]):
        with pytest.raises(m.MDLGError):
            m.mdlg_vacf([0, 10], vel, lags, c)
    with pytest.raises(m.MDLGError):
        m.mdlg_vacf([0, 10], vel, list(range(4)) * 300, torch.zeros((1, 1200), dtype=torch.float64, device="cuda"))
