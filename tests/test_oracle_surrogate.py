"""Pins for the surrogate oracle: gradients against float64 central finite
differences of the loss, Adam's behaviour under a constant gradient, and the
feature/target maps."""

import numpy as np
import pytest

from oracle import surrogate as sg
from workloads import he_normal_mlp


def _params(seed=0):
    m = he_normal_mlp([4, 16, 16, 16, 2], seed=seed)
    return [W.astype(np.float64) for W in m.Ws], [b.astype(np.float64) for b in m.bs]


def test_gradients_match_finite_differences():
    Ws, bs = _params()
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (12, 4))
    T = rng.normal(0, 1, (12, 2))
    out, acts = sg.forward(Ws, bs, X)
    dWs, dbs = sg.backward(Ws, acts, out, T)
    h = 1e-6
    for li in range(len(Ws)):
        for arr, grad in ((Ws[li], dWs[li]), (bs[li], dbs[li])):
            flat = arr.reshape(-1)
            idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
            for i in idx:
                old = flat[i]
                flat[i] = old + h
                lp = sg.loss(sg.forward(Ws, bs, X)[0], T)
                flat[i] = old - h
                lm = sg.loss(sg.forward(Ws, bs, X)[0], T)
                flat[i] = old
                fd = (lp - lm) / (2 * h)
                assert grad.reshape(-1)[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_adam_constant_gradient_moves_by_lr_per_step():
    # with a constant gradient g the bias-corrected moments are exactly g and
    # g^2, so every step moves each parameter by lr * g / (|g| + eps)
    p = [np.array([1.0, -2.0, 0.5])]
    g = [np.array([0.3, -4.0, 1e-3])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    lr = 1e-2
    for t in range(1, 6):
        before = p[0].copy()
        sg.adam_step(p, g, m, v, t, lr)
        np.testing.assert_allclose(before - p[0], lr * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-9)


def test_features_and_targets():
    c = np.array([[0.25, -0.5, 0.75]])
    h = np.array([[2.0 ** -6] * 3])  # cell size 2^-5 -> log2 = -5
    X = sg.features(c, h, a=0.25, b=1.0)
    np.testing.assert_array_equal(X, [[0.25, -0.5, 0.75, -0.25]])
    T = sg.targets([1.5], [np.e], mu_bar=0.5, scale=2.0)
    np.testing.assert_allclose(T, [[0.5, 1.0]])


def test_training_reduces_loss_on_a_smooth_target():
    Ws, bs = _params(3)
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, (256, 4))
    T = np.stack([np.sin(2 * X[:, 0]) * X[:, 3], 0.5 * X[:, 1] - X[:, 3]], 1)
    params = Ws + bs
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    l0 = sg.loss(sg.forward(Ws, bs, X)[0], T)
    for t in range(1, 301):
        out, acts = sg.forward(Ws, bs, X)
        dWs, dbs = sg.backward(Ws, acts, out, T)
        sg.adam_step(params, dWs + dbs, m, v, t, 3e-3)
    l1 = sg.loss(sg.forward(Ws, bs, X)[0], T)
    assert l1 < 0.2 * l0


def test_base_targets_invert_base_prediction():
    rng = np.random.default_rng(9)
    f = rng.normal(0, 1, 50)
    s = np.exp(rng.normal(-3, 1, 50))
    s[:5] = 0.0  # below the floor
    mu = f + s * rng.normal(0, 0.1, 50)
    sigma = np.maximum(s, 1e-6) * np.exp(rng.normal(0, 0.05, 50))
    T = sg.base_targets(mu, sigma, f, s, 1e-6)
    back = sg.base_prediction(T, f, s, 1e-6)
    np.testing.assert_allclose(back[:, 0], mu, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(back[:, 1], sigma, rtol=1e-12)
    # a perfect linearisation gives zero targets
    Z = sg.base_targets(f[5:], s[5:], f[5:], s[5:], 1e-6)
    np.testing.assert_allclose(Z, 0.0, atol=1e-12)
