"""Pins of the surrogate network's FP64 reference: central finite differences
for the analytic gradient, softmax normalisation, the softmax-KL gradient
identity, Adam against its textbook update, bf16 rounding, and that training
on a fixed batch lowers the loss."""
import numpy as np
import pytest

import mdlg_inputs as mi
from oracle import mlp


def small_problem(seed=0, B=16):
    rng = np.random.default_rng(seed)
    theta = mi.mlp_init(seed)
    X = np.stack([rng.uniform(0.05, 0.4, B), rng.uniform(1, 20, B), rng.uniform(5e-4, 1e-2, B),
                  rng.uniform(0, 0.2, B), np.cos(rng.uniform(0, 6.28, B)), np.sin(rng.uniform(0, 6.28, B))], axis=1)
    R = rng.dirichlet(np.ones(49) * 0.3, B)
    return theta, X, R


def test_parameter_count():
    assert mlp.n_params() == 145969
    assert mi.mlp_init(0).shape == (145969,)


def test_softmax_rows_sum_to_one():
    theta, X, _ = small_problem()
    Q, _ = mlp.forward(theta, X)
    assert np.allclose(Q.sum(axis=1), 1.0, atol=1e-14)
    assert np.all(Q > 0)


def test_gradient_matches_central_differences():
    theta, X, R = small_problem(1, B=8)
    g = mlp.grad(theta, X, R)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(1536, 8, replace=False), 1536 + rng.choice(256, 4, replace=False),
                          1792 + rng.choice(65536, 8, replace=False), 133632 + rng.choice(12544, 8, replace=False),
                          145920 + np.arange(4)])
    h = 1e-4  # truncation error ~h^2, rounding ~eps * loss / h: both below 1e-11 here
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, R) - mlp.loss(tm, X, R)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-7, abs=1e-11)


def test_logit_gradient_identity():
    # d/dz sum R log(R / softmax(z)) = softmax(z) - R for rows of R summing to one
    rng = np.random.default_rng(2)
    z = rng.normal(size=(3, 49))
    R = rng.dirichlet(np.ones(49), 3)
    q = mlp.softmax(z)
    h = 1e-6
    for b in range(3):
        for i in (0, 7, 48):
            zp, zm = z.copy(), z.copy()
            zp[b, i] += h
            zm[b, i] -= h
            fd = (mlp.kl(R[b:b + 1], mlp.softmax(zp[b:b + 1]))[0] - mlp.kl(R[b:b + 1], mlp.softmax(zm[b:b + 1]))[0]) / (2 * h)
            assert fd == pytest.approx(q[b, i] - R[b, i], rel=1e-6, abs=1e-10)


def test_adam_first_step_moves_by_lr_times_sign():
    theta = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 0.0, 3.0])
    t1, m, v = mlp.adam(theta, np.zeros(5), np.zeros(5), g, 1, lr=1e-3)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> step = lr * g / (|g| + eps)
    assert np.allclose(t1, -1e-3 * g / (np.abs(g) + 1e-8))


def test_bf16_rounding():
    a = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.1415926])
    r = mlp.to_bf16(a)
    assert r[0] == 1.0
    assert r[1] == 1.0 + 2 ** -7 or r[1] == 1.0  # exactly half way: ties to even -> 1.0
    assert r[1] == 1.0
    assert r[2] == 1.0 + 2 ** -7
    assert r[3] == -2.5
    assert abs(r[4] - 3.1415926) < 2 ** -7 * 2


def test_training_lowers_the_loss():
    theta, X, R = small_problem(3, B=32)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss(theta, X, R)
    for t in range(1, 31):
        theta, m, v = mlp.adam(theta, m, v, mlp.grad(theta, X, R), t, lr=1e-3)
    assert mlp.loss(theta, X, R) < 0.85 * l0
