"""What the trained surrogate gains over the method without it.

A small version of the surrogate pipeline runs end to end on the GPU: batched
MD generates trajectories, the trajectory coarse-graining measures g_i for
10 coarse-graining times x 16 drifts per replica, the network trains on the
GPU, and replicas it never saw test it.  Without the network, f_eq at a new
(phi, kT, dt_cg/dx, u) needs a molecular dynamics run (the closed forms need
the measured displacement moments too); with it, one batched inference.
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pipeline():
    import torch

    from paper_2101_01160_amd import surrogate as S
    print("surrogate pipeline: 2 groups x 16 replicas x 16384 particles", flush=True)
    data = S.generate(n_groups=2, reps_per_group=16, n=16384, n_snap=201, equil=2000, log=print)
    tr, va, te = S.split_by_replica(data)
    net, hist = S.train(data, tr, steps=8000, batch=1024, val_idx=va, val_every=2000, log=print)
    torch.cuda.synchronize()
    return S, data, tr, te, net, hist


def test_heldout_accuracy_and_guard(pipeline):
    S, data, tr, te, net, _ = pipeline
    res = S.evaluate(net, data, te, with_guard=True)
    print(res, flush=True)
    # the trained network against measurements on unseen replicas
    assert res["mean_err"] < 3e-3
    # a model that needs no MD either: every particle stays in its cell
    naive = np.abs(np.eye(49)[0][None, :] - data.G[te]).max(axis=1).mean()
    assert res["mean_err"] < 0.05 * naive
    # the guard keeps every answer within tol of WSG, hence within tol plus
    # the WSG error of the measurement
    assert res["guarded_max_err"] <= 1e-3 + res["wsg_max_err"] + 1e-12
    # the closed form, given the measured moments, is within the sampling noise
    assert res["wsg_max_err"] < 2e-3


def test_guard_entry_point_matches_batched_rule(pipeline):
    import paper_2101_01160_amd as m
    S, data, _, te, net, _ = pipeline
    g_net = S.predict(net, data.X[te[:32]])
    for k, i in enumerate(te[:32]):
        g, fb, err = net.feq(data.X[i], data.a2[i], data.lam[i], tol=1e-3)
        w = m.mdlg_feq_wsg(data.a2[i], data.lam[i], data.u[i])
        assert err == pytest.approx(np.abs(g_net[k] - w).max(), rel=1e-6, abs=1e-9)
        assert fb == (err > 1e-3)
        assert np.array_equal(g, w) if fb else np.allclose(g, g_net[k], rtol=0, atol=1e-7)


def test_inference_is_cheaper_than_md(pipeline):
    import torch

    import paper_2101_01160_amd as m
    S, data, _, te, net, _ = pipeline
    B = 16384
    big = m.SurrogateMLP(net.params(), B)
    x = torch.from_numpy(np.resize(data.X[te], (B, 6)).astype(np.float32)).cuda()
    out = torch.empty((B, 49), dtype=torch.float32, device="cuda")
    m.mdlg_mlp_forward(big.handle, x, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        m.mdlg_mlp_forward(big.handle, x, out)
    torch.cuda.synchronize()
    sec_nn = (time.perf_counter() - t0) / (10 * B)
    sec_md = (data.timing["md_s"] + data.timing["cg_s"]) / len(data)
    print(f"seconds per f_eq: MD + coarse-graining {sec_md:.3e}, surrogate {sec_nn:.3e}, "
          f"ratio {sec_md / sec_nn:.0f}", flush=True)
    assert sec_md / sec_nn > 1000
