"""Pins of the learned-correction oracle: the hand-derived gradients agree
with central finite differences of the forward pass, and the loss is zero
exactly when the network reproduces the targets."""
import numpy as np

from oracle import mlp


def _setup(seed=0, n=40, w=16, B=7):
    p = mlp.init_params(n, w, seed)
    g = np.random.default_rng(seed + 1)
    p["b1"] = 0.1 * g.standard_normal(w)
    p["b2"] = 0.1 * g.standard_normal(w)
    X = g.standard_normal((n, B))
    T = g.standard_normal((n, B))
    return p, X, T


def test_gradients_match_central_differences():
    p, X, T = _setup()
    L, g = mlp.grads(p, X, T)
    assert abs(L - mlp.loss(p, X, T)) <= 1e-14 * L
    rng = np.random.default_rng(5)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        P = p[name]
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in P.shape)
            old = P[idx]
            P[idx] = old + h
            Lp = mlp.loss(p, X, T)
            P[idx] = old - h
            Lm = mlp.loss(p, X, T)
            P[idx] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, g[name][idx])


def test_loss_zero_on_own_outputs_and_weights_fp16():
    p, X, _ = _setup(3)
    Y, _ = mlp.forward(p, X)
    assert mlp.loss(p, X, Y) == 0.0
    for k in ("W1", "W2", "W3"):
        assert np.array_equal(p[k], p[k].astype(np.float16).astype(np.float64))


def test_adam_first_step_is_sign_times_lr():
    # with zero state, the bias-corrected first Adam step is lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3])
    state = [np.zeros(3), np.zeros(3)]
    new, _ = mlp.adam_step(np.zeros(3), g, state, 0.01, 1)
    assert np.allclose(new, -0.01 * g / (np.abs(g) + 1e-8))


def test_forward_f16_rounds_only_the_operands():
    # with inputs, weights and every activation exact in FP16 (small dyadic
    # numbers) the FP16-operand forward is the exact forward; with general
    # inputs it differs by the FP16 rounding of the three operands only
    g = np.random.default_rng(4)
    n, w, B = 12, 8, 5
    p = {"W1": g.integers(-3, 4, (w, n)) / 8.0, "b1": g.integers(-2, 3, w) / 4.0,
         "W2": g.integers(-3, 4, (w, w)) / 8.0, "b2": g.integers(-2, 3, w) / 4.0,
         "W3": g.integers(-3, 4, (n, w)) / 8.0, "b3": g.integers(-2, 3, n) / 4.0}
    X = g.integers(-4, 5, (n, B)) / 4.0
    Y, _ = mlp.forward(p, X)
    assert np.array_equal(mlp.forward_f16(p, X), Y)
    p = mlp.init_params(40, 16, 2)
    X = g.standard_normal((40, 9)) / np.sqrt(40)
    Y, _ = mlp.forward(p, X)
    d = np.linalg.norm(mlp.forward_f16(p, X) - Y) / np.linalg.norm(Y)
    assert 1e-6 < d < 3 * 2.0 ** -11 * 10
