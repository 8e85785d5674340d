"""GPU parity of the f_eq surrogate network (BF16 matrix-core products, FP32
accumulation) with its FP64 reference:

* forward: within 2e-3 relative of the reference evaluated with the same
  bf16 roundings (weights, encoded inputs, hidden activations), and within
  the bf16 error budget (3e-2 relative) of the exact FP64 network;
* gradient: per parameter block cosine >= 0.999 and relative L2 <= 3e-2
  against the exact FP64 backpropagation;
* Adam: the first update moves each parameter by lr * sign(g);
* training on a fixed batch lowers the loss like the reference does;
* the WSG guard returns the closed form exactly when it falls back.
"""
import numpy as np
import pytest

import mdlg_inputs as mi
from oracle import mlp as om

pytestmark = pytest.mark.gpu

BLOCKS = [("W1", 0, 1536), ("b1", 1536, 1792), ("W2", 1792, 67328), ("b2", 67328, 67584),
          ("W3", 67584, 133120), ("b3", 133120, 133376), ("W4", 133376, 145920), ("b4", 145920, 145969)]


def inputs(seed, B):
    rng = np.random.default_rng(seed)
    th = rng.uniform(0, 2 * np.pi, B)
    return np.stack([rng.uniform(0.05, 0.4, B), rng.uniform(1, 20, B), rng.uniform(5e-4, 1e-2, B),
                     rng.uniform(0, 0.2, B), np.cos(th), np.sin(th)], axis=1)


def targets(seed, B):
    return np.random.default_rng(seed + 1000).dirichlet(np.ones(49) * 0.3, B)


def params(seed=0):
    return mi.mlp_init(seed).astype(np.float32).astype(np.float64)


def forward_bf16(theta, X):
    """The reference forward pass with the kernel's bf16 roundings applied."""
    W1, b1, W2, b2, W3, b3, W4, b4 = om.unpack(theta)
    h = om.to_bf16(om.encode(np.asarray(X, np.float32), dtype=np.float32).astype(np.float64))
    for W, b in ((W1, b1), (W2, b2), (W3, b3)):
        z = h @ om.to_bf16(W) + b
        h = om.to_bf16(om.silu(z))
    return om.softmax(h @ om.to_bf16(W4) + b4)


def _t(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def make(theta, max_batch):
    import paper_2101_01160_amd as m
    return m.SurrogateMLP(theta.astype(np.float32), max_batch)


@pytest.mark.parametrize("B", [1, 63, 77, 256])
def test_forward_matches_reference(B):
    print(f"mlp forward B={B}", flush=True)
    theta = params(0)
    X = inputs(B, B)
    net = make(theta, 256)
    g = net.forward(_t(X)).cpu().numpy().astype(np.float64)
    ref = forward_bf16(theta, X)
    assert np.allclose(g.sum(axis=1), 1.0, atol=1e-5)
    assert np.max(np.abs(g - ref) / ref) < 2e-3
    exact, _ = om.forward(theta, X)
    assert np.max(np.abs(g - exact) / exact) < 3e-2


def test_forward_full_batch_sampled_rows():
    B = 16384
    print(f"mlp forward B={B}", flush=True)
    theta = params(1)
    X = inputs(7, B)
    net = make(theta, B)
    g = net.forward(_t(X)).cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(3).choice(B, 64, replace=False)
    ref = forward_bf16(theta, X[rows])
    assert np.max(np.abs(g[rows] - ref) / ref) < 2e-3
    g2 = net.forward(_t(X)).cpu().numpy().astype(np.float64)
    assert np.array_equal(g, g2)  # deterministic


@pytest.mark.parametrize("B", [64, 200])
def test_gradient_matches_reference(B):
    print(f"mlp gradient B={B}", flush=True)
    theta = params(2)
    X, R = inputs(11, B), targets(11, B)
    net = make(theta, B)
    loss, grad = net.gradient(_t(X), _t(R))
    loss = float(loss.cpu().numpy()[0])
    grad = grad.cpu().numpy().astype(np.float64)
    assert loss == pytest.approx(om.loss(theta, X, R), rel=1e-2)
    ref = om.grad(theta, X, R)
    for name, a, b in BLOCKS:
        g, r = grad[a:b], ref[a:b]
        cos = g @ r / (np.linalg.norm(g) * np.linalg.norm(r))
        rel = np.linalg.norm(g - r) / np.linalg.norm(r)
        print(f"  {name}: cos={cos:.6f} rel={rel:.3e}", flush=True)
        assert cos >= 0.999, name
        assert rel <= 3e-2, name


def test_first_adam_step_is_lr_times_sign():
    import torch
    B, lr = 128, 1e-3
    theta = params(3)
    X, R = inputs(5, B), targets(5, B)
    net = make(theta, B)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.train_step(_t(X), _t(R), lr, loss)
    step = net.params().astype(np.float64) - theta
    g = om.grad(theta, X, R)
    big = np.abs(g) > 1e-3 * np.abs(g).max()  # far from the sign change of g, and from eps
    assert big.sum() > 1000
    assert np.mean(np.abs(step[big] + lr * np.sign(g[big])) < 1e-2 * lr) > 0.99
    assert float(loss.cpu()[0]) == pytest.approx(om.loss(theta, X, R), rel=1e-2)


def test_training_lowers_the_loss():
    import torch
    B = 256
    theta = params(4)
    X = inputs(9, B)
    # targets that depend smoothly on the inputs, so that the batch can be fitted
    M = np.random.default_rng(4).normal(size=(6, 49))
    R = om.softmax(2.0 * om.encode(X) @ M)
    net = make(theta, B)
    x, r = _t(X), _t(R)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for _ in range(60):
        net.train_step(x, r, 1e-3, loss)
        hist.append(float(loss.cpu()[0]))
    l_final = om.loss(net.params().astype(np.float64), X, R)
    assert l_final < 0.2 * hist[0]
    # the reference on the same batch and schedule reaches a similar loss
    th, mm, vv = theta.copy(), np.zeros_like(theta), np.zeros_like(theta)
    for t in range(1, 61):
        th, mm, vv = om.adam(th, mm, vv, om.grad(th, X, R), t, lr=1e-3)
    l_ref = om.loss(th, X, R)
    print(f"loss0={hist[0]:.4f} gpu={l_final:.4f} ref={l_ref:.4f}", flush=True)
    assert abs(l_final - l_ref) < 0.15 * l_ref


def test_surrogate_guard():
    import paper_2101_01160_amd as m
    theta = params(5)
    net = make(theta, 4)
    x = np.array([0.0784, 20.0, 5e-3, 0.1, 0.6, 0.8])
    a2, lam = 2e-3, 0.3
    wsg = m.mdlg_feq_wsg(a2, lam, (x[3] * x[4], x[3] * x[5]))
    # the untrained network is far from the closed form: the guard falls back
    g, fb, err = net.feq(x, a2, lam, tol=1e-3)
    assert fb and err > 1e-3
    assert np.array_equal(g, wsg)
    # with a loose tolerance it returns the network's own values
    g2, fb2, err2 = net.feq(x, a2, lam, tol=10.0)
    assert not fb2 and err2 == pytest.approx(err)
    net_g = net.forward(_t(x[None, :])).cpu().numpy()[0].astype(np.float64)
    assert np.array_equal(g2, net_g)
    assert np.max(np.abs(g2 - wsg)) == pytest.approx(err, rel=1e-12)


def test_invalid_arguments():
    import torch

    import paper_2101_01160_amd as m
    theta = params(0).astype(np.float32)
    bad = theta.copy()
    bad[7] = np.nan
    with pytest.raises(m.MDLGError, match="EINVAL"):
        m.SurrogateMLP(bad, 8)
    with pytest.raises(m.MDLGError, match="EINVAL"):
        m.SurrogateMLP(theta, 0)
    net = m.SurrogateMLP(theta, 8)
    x9 = torch.zeros((9, 6), dtype=torch.float32, device="cuda")
    with pytest.raises(m.MDLGError, match="EINVAL"):
        net.forward(x9)
    x = torch.zeros((4, 6), dtype=torch.float32, device="cuda")
    r = torch.full((4, 49), 1 / 49, dtype=torch.float32, device="cuda")
    with pytest.raises(m.MDLGError, match="EINVAL"):
        net.train_step(x, r, 0.0)
    with pytest.raises(m.MDLGError, match="EINVAL"):
        net.forward(x[:0])
