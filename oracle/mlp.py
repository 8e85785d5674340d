"""FP64 reference of the f_eq surrogate network (test infrastructure only).

The network maps six inputs of an equilibrium LJ gas and its lattice —
area fraction phi, temperature kT, coarse time step over lattice spacing
dt_cg/dx (tau/sigma), the drift |u| (cells per coarse step) and the drift
direction (cos, sin) — to the 49 D2Q49 equilibrium values g_i = f_i^eq / rho:

    x' = encode(x)                      (fixed input map, below)
    h1 = silu(x' W1 + b1)               6 -> 256
    h2 = silu(h1 W2 + b2)               256 -> 256
    h3 = silu(h2 W3 + b3)               256 -> 256
    q  = softmax(h3 W4 + b4)            256 -> 49

and is trained on measured f_eq with the Kullback-Leibler divergence
sum_i R_i log(R_i / Q_i) of Eq.(kullback_leibler) as the loss (mean over the
batch).  Parameters are one flat vector: W1 [6,256] (input-major), b1, W2,
b2, W3, b3, W4 [256,49], b4.
"""
from __future__ import annotations

import numpy as np

DIMS = (6, 256, 256, 256, 49)
LN20 = float(np.log(20.0))


def encode(X, dtype=np.float64):
    """The network's fixed input map of x = (phi, kT, dt_cg/dx, |u|, cos, sin):
    (phi / 0.4, ln kT / ln 20, (ln(dt_cg/dx) + 6) / 1.5, 5 |u| cos, 5 |u| sin,
    5 |u|): logarithms for the two scale variables (in the ballistic limit
    a^2 = kT (dt_cg/dx)^2, linear in them), the drift as a vector.  dtype
    float32 evaluates it the way the device does, operation by operation."""
    X = np.asarray(X, dtype=dtype)
    f = lambda v: np.asarray(v, dtype=dtype)
    out = np.empty(X.shape, dtype=dtype)
    tiny = f(1e-30)
    out[:, 0] = X[:, 0] * f(2.5)
    out[:, 1] = np.log(np.maximum(X[:, 1], tiny)) * f(1.0 / LN20)
    out[:, 2] = (np.log(np.maximum(X[:, 2], tiny)) + f(6.0)) * f(1.0 / 1.5)
    out[:, 3] = (X[:, 3] * X[:, 4]) * f(5.0)
    out[:, 4] = (X[:, 3] * X[:, 5]) * f(5.0)
    out[:, 5] = X[:, 3] * f(5.0)
    return out


def shapes():
    out = []
    for a, b in zip(DIMS[:-1], DIMS[1:]):
        out += [(a, b), (b,)]
    return out


def n_params():
    return int(sum(np.prod(s) for s in shapes()))


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for s in shapes():
        k = int(np.prod(s))
        out.append(theta[o:o + k].reshape(s))
        o += k
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def forward(theta, X):
    """Returns (Q [B,49], cache) for inputs X [B,6] (unscaled)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    x = encode(X)
    z1 = x @ W1 + b1
    h1 = silu(z1)
    z2 = h1 @ W2 + b2
    h2 = silu(z2)
    z3 = h2 @ W3 + b3
    h3 = silu(z3)
    z4 = h3 @ W4 + b4
    q = softmax(z4)
    return q, (x, z1, h1, z2, h2, z3, h3, z4)


def kl(R, Q):
    """Per-sample sum_i R_i log(R_i / Q_i); terms with R_i = 0 vanish."""
    R = np.asarray(R, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(R > 0, R * (np.log(np.where(R > 0, R, 1.0)) - np.log(Q)), 0.0)
    return t.sum(axis=1)


def loss(theta, X, R):
    Q, _ = forward(theta, X)
    return float(np.mean(kl(R, Q)))


def grad(theta, X, R):
    """Analytic gradient of `loss` (backpropagation).  R rows sum to one."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    Q, (x, z1, h1, z2, h2, z3, h3, z4) = forward(theta, X)
    B = x.shape[0]
    R = np.asarray(R, dtype=np.float64)
    # d/dz4 of mean_b sum_i R log(R/Q) with Q = softmax(z4): (Q * sum_i R - R) / B
    g4 = (Q * R.sum(axis=1, keepdims=True) - R) / B
    dW4 = h3.T @ g4
    db4 = g4.sum(axis=0)
    g3 = (g4 @ W4.T) * dsilu(z3)
    dW3 = h2.T @ g3
    db3 = g3.sum(axis=0)
    g2 = (g3 @ W3.T) * dsilu(z2)
    dW2 = h1.T @ g2
    db2 = g2.sum(axis=0)
    g1 = (g2 @ W2.T) * dsilu(z1)
    dW1 = x.T @ g1
    db1 = g1.sum(axis=0)
    return np.concatenate([a.ravel() for a in (dW1, db1, dW2, db2, dW3, db3, dW4, db4)])


def adam(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1).  Returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def to_bf16(a):
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))
