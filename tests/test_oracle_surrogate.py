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


def test_partition_hand_cases():
    """Band partition, worked by hand.  t = 3, err_mu = 0.1, err_ls = 0.2,
    z = 2, z_acc = 1, isos (0, 5), unit 1:
      prune band: t sigma e^{0.4} = 3 sigma * 1.4918..., mu margin 0.2
      accept band: t sigma e^{-0.2} = 3 sigma * 0.8187..., mu margin 0.1"""
    from oracle.surrogate import partition

    isos = [0.0, 5.0]
    pred = np.array([
        [2.0, 0.1],    # iso 0: d 2, 2-0.2 > 0.4476 -> outside; iso 5: d 3 -> outside => pruned
        [0.05, 1.0],   # iso 0: d 0.05+0.1 < 2.456 -> inside; iso 5: 4.95-0.2=4.75 > 4.4755 -> outside
        [1.0, 0.3],    # iso 0: 1-0.2 = 0.8 <= 1.343 (not outside), 1.1 >= 0.737 (not inside) -> unsure
        [0.05, 1.0],   # as row 1, but the parent carries only iso 5 -> outside => pruned
        [np.nan, 1.0], # non-finite prediction -> fallback
        [4.0, 1.0],    # iso 0: outside? 3.8 <= 4.4755 no; inside? 4.1 < 2.456 no -> unsure
    ])
    pm = np.array([3, 3, 3, 2, 3, 1], dtype=np.uint32)
    mask, fb, slack = partition(pred, None, 3.0, isos, pm, 0.1, 0.2, 2.0, 1.0, leaf=False, accept_leaves=False)
    np.testing.assert_array_equal(mask, [0, 1, 0, 0, 0, 0])
    np.testing.assert_array_equal(fb, [False, False, True, False, True, True])
    # at the leaf level an accepted bit falls back unless leaves may be accepted
    mask, fb, _ = partition(pred, None, 3.0, isos, pm, 0.1, 0.2, 2.0, 1.0, leaf=True, accept_leaves=False)
    np.testing.assert_array_equal(fb, [False, True, True, False, True, True])
    np.testing.assert_array_equal(mask, [0, 0, 0, 0, 0, 0])
    mask, fb, _ = partition(pred, None, 3.0, isos, pm, 0.1, 0.2, 2.0, 1.0, leaf=True, accept_leaves=True)
    np.testing.assert_array_equal(mask, [0, 1, 0, 0, 0, 0])
    # the per-cell unit scales only the mu margin: unit 10 on row 0 makes
    # iso 0 unsure (2 - 2 = 0 <= 0.4476)
    mask, fb, _ = partition(pred[:1], np.array([10.0]), 3.0, isos, pm[:1], 0.1, 0.2, 2.0, 1.0, False, False)
    assert fb[0] and mask[0] == 0
    # a cell exactly on a threshold is within slack 0
    p2 = np.array([[0.2 + 3.0 * np.exp(0.4), 1.0]])
    _, _, s2 = partition(p2, None, 3.0, [0.0], np.array([1], np.uint32), 0.1, 0.2, 2.0, 1.0, False, False)
    assert s2[0] < 1e-15


def test_partition_is_the_plain_test_with_zero_bands():
    """With zero error and zero bands the rule is the soft-bound test itself
    (strict on both sides, so a bound touching c is unsure): outside iff
    |mu - c| > t sigma, inside iff |mu - c| < t sigma."""
    from oracle.surrogate import partition

    rng = np.random.default_rng(0)
    pred = np.stack([rng.normal(0, 1, 500), np.abs(rng.normal(0, 0.5, 500))], 1)
    isos = [-0.5, 0.4]
    pm = np.full(500, 3, np.uint32)
    mask, fb, _ = partition(pred, None, 3.0, isos, pm, 0.0, 0.0, 0.0, 0.0, False, False)
    want = np.zeros(500, np.uint32)
    for j, c in enumerate(isos):
        want |= (np.abs(pred[:, 0] - c) < 3.0 * pred[:, 1]).astype(np.uint32) << np.uint32(j)
    assert not fb.any()
    np.testing.assert_array_equal(mask, want)
