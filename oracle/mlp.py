"""Oracle for the learned correction of the mean spatial solve (test
infrastructure only; see oracle/__init__.py).

The correction is a three-layer perceptron acting on one spatial field x
(length n):  h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3,
with W1 (w x n), W2 (w x w), W3 (n x w).  In the preconditioner the field is a
mean-solve right-hand side r scaled to unit norm, and the target is the part
of the exact mean solve F_avg^-1 r (eq. 5.23) that a Jacobi step D^-1 r misses,
scaled the same way.  Training minimizes the mean over a batch of relative
squared errors ||y_s - t_s||^2 / ||t_s||^2.

Weights are held in FP16 on the device; the oracle takes the same FP16-rounded
values and computes in FP64.  Gradients are derived by hand (backpropagation)
and pinned in tests by central finite differences of the forward pass.
"""
from __future__ import annotations

import numpy as np


def init_params(n: int, width: int, seed: int):
    """He-scaled normal weights, zero biases, rounded to FP16 values."""
    g = np.random.default_rng(seed)
    W1 = g.standard_normal((width, n)) * np.sqrt(2.0 / n)
    W2 = g.standard_normal((width, width)) * np.sqrt(2.0 / width)
    W3 = g.standard_normal((n, width)) * np.sqrt(1.0 / width)
    p = dict(W1=W1, b1=np.zeros(width), W2=W2, b2=np.zeros(width), W3=W3, b3=np.zeros(n))
    return {k: v.astype(np.float16).astype(np.float64) for k, v in p.items()}


def forward(p, X):
    """X: (n, B) columns of inputs -> (Y, cache)."""
    z1 = p["W1"] @ X + p["b1"][:, None]
    h1 = np.maximum(z1, 0.0)
    z2 = p["W2"] @ h1 + p["b2"][:, None]
    h2 = np.maximum(z2, 0.0)
    Y = p["W3"] @ h2 + p["b3"][:, None]
    return Y, (X, z1, h1, z2, h2)


def _to_f16(a):
    # round as the device does: its FP32 value to the nearest FP16
    return a.astype(np.float32).astype(np.float16).astype(np.float64)


def forward_f16(p, X):
    """The forward with FP16 operands: the input and each hidden activation
    rounded to FP16 before the product that consumes it (weights are FP16
    already), products and sums otherwise exact (FP64 here; the device
    accumulates in FP32)."""
    h0 = _to_f16(X)
    h1 = np.maximum(p["W1"] @ h0 + p["b1"][:, None], 0.0)
    h2 = np.maximum(p["W2"] @ _to_f16(h1) + p["b2"][:, None], 0.0)
    return p["W3"] @ _to_f16(h2) + p["b3"][:, None]


def loss(p, X, T):
    """Mean relative squared error over the batch columns."""
    Y, _ = forward(p, X)
    return float(np.mean(np.sum((Y - T) ** 2, axis=0) / np.sum(T * T, axis=0)))


def grads(p, X, T):
    """Backpropagation of loss(): returns (loss, {name: dloss/dname})."""
    Y, (X, z1, h1, z2, h2) = forward(p, X)
    B = X.shape[1]
    tn = np.sum(T * T, axis=0)
    L = float(np.mean(np.sum((Y - T) ** 2, axis=0) / tn))
    dY = 2.0 * (Y - T) / tn[None, :] / B
    g = {"W3": dY @ h2.T, "b3": dY.sum(axis=1)}
    dh2 = p["W3"].T @ dY
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2 @ h1.T
    g["b2"] = dz2.sum(axis=1)
    dh1 = p["W2"].T @ dz2
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1 @ X.T
    g["b1"] = dz1.sum(axis=1)
    return L, g


def adam_step(master, grad, state, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, ICLR 2015) of an FP32-like master copy;
    returns the new master and its FP16-rounded working copy."""
    m, v = state
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    new = master - lr * mh / (np.sqrt(vh) + eps)
    state[0], state[1] = m, v
    return new, new.astype(np.float16).astype(np.float64)
