"""What the trained surrogate gains over the method without it.

A small version of the surrogate pipeline runs end to end on the GPU: batched
MD generates trajectories, the trajectory coarse-graining measures g_i for
10 coarse-graining times x 16 drifts per replica, the network trains on the
GPU, and replicas it never saw test it.  Without the network, f_eq at a new
(phi, kT, dt_cg/dx, u) needs a molecular dynamics run (the closed forms need
the measured displacement moments too); with it, one batched inference, and
its Poisson-WSG guard takes a^2 and lambda from the moment table fitted to
the training replicas, so no trajectory is needed either.
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pipeline():
    import torch

    from paper_2101_01160_amd import surrogate as S
    print("surrogate pipeline: 2 groups x 16 replicas x 32768 particles", flush=True)
    data = S.generate(n_groups=2, reps_per_group=16, n=32768, n_snap=201, equil=2000, log=print)
    tr, va, te = S.split_by_replica(data)
    # 100,000 Adam steps of 2048 samples; the network returned is the mean of
    # the parameters over the last 30% of the steps
    net, hist = S.train(data, tr, steps=100000, batch=2048, val_idx=va, val_every=25000, log=print,
                        average_tail=0.3)
    # the guard's moments at points without a trajectory: fitted to the
    # training replicas only, over the design's parameter box
    table = S.moment_table(data, tr, box=S.parameter_box(data))
    torch.cuda.synchronize()
    return S, data, tr, te, net, hist, table


def test_heldout_accuracy_and_guard(pipeline):
    S, data, tr, te, net, _, table = pipeline
    res = S.evaluate(net, data, te, with_guard=True, table=table)
    print(res, flush=True)
    # the trained network against measurements on unseen replicas: every one
    # of the 49 values of every sample within 1e-3
    assert res["max_err"] <= 1e-3
    # a model that needs no MD either: every particle stays in its cell
    naive = np.abs(np.eye(49)[0][None, :] - data.G[te]).max(axis=1).mean()
    assert res["mean_err"] < 0.02 * naive
    # the guard without a trajectory (moments from the table) keeps the
    # answer within 1e-3 of the measurement
    assert res["table_guarded_max_err"] <= 1e-3
    # the closed form, given the measured moments, is within the sampling noise
    assert res["wsg_max_err"] < 2e-3
    # and with the table's moments it stays close to the measurement as well
    assert res["table_wsg_max_err"] < 3e-3


def test_moment_table_tracks_the_measured_moments(pipeline):
    S, data, tr, te, net, _, table = pipeline
    got = np.array([table(data.X[i, :3]) for i in te])
    rel_a2 = np.abs(got[:, 0] / data.a2[te] - 1.0)
    print(f"held-out a2 relative error: max {rel_a2.max():.3e} mean {rel_a2.mean():.3e}; "
          f"r error max {np.abs(got[:, 2] - data.r[te]).max():.3e}", flush=True)
    assert rel_a2.max() < 0.1
    assert np.abs(got[:, 2] - data.r[te]).max() < 0.05


def test_guard_entry_point_matches_batched_rule(pipeline):
    import paper_2101_01160_amd as m
    S, data, _, te, net, _, table = pipeline
    g_net = S.predict(net, data.X[te[:32]])
    for k, i in enumerate(te[:32]):
        g, fb, err = net.feq(data.X[i], data.a2[i], data.lam[i], tol=1e-3)
        w = m.mdlg_feq_wsg(data.a2[i], data.lam[i], data.u[i])
        assert err == pytest.approx(np.abs(g_net[k] - w).max(), rel=1e-6, abs=1e-9)
        assert fb == (err > 1e-3)
        assert np.array_equal(g, w) if fb else np.allclose(g, g_net[k], rtol=0, atol=1e-7)
        # the same rule with the table's moments, through the C entry point
        gt, fbt, errt, a2t, lamt = net.feq_table(data.X[i], table, tol=1e-3)
        assert (a2t, lamt) == table(data.X[i, :3])[:2]
        g2, fb2, err2 = net.feq(data.X[i], a2t, lamt, tol=1e-3)
        assert np.array_equal(gt, g2) and fbt == fb2 and errt == err2


def test_inference_is_cheaper_than_md(pipeline):
    import torch

    import paper_2101_01160_amd as m
    S, data, _, te, net, _, _ = pipeline
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
