"""Float64 reference for the surrogate MLP: features, forward, loss, backward
and one Adam step.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The surrogate maps a cell (centre c, per-axis half-width h) to a predicted
(mean, sigma) of the INR output over the cell, either directly or as a
correction to a base (f, s) per cell (the centre linearisation).  Features: x = (c_x, c_y, c_z,
a * log2(2 h_x) + b) (cell size normalised by a fixed affine map); a ReLU MLP
4 -> 128 -> 128 -> 128 -> 2 outputs standardised targets
t = ((mu - mu_bar) / S, ln sigma).  Loss: half the sum of the two mean squared
errors over the batch.  Optimiser: Adam (Kingma & Ba, 2015) with bias
correction.
"""

from __future__ import annotations

import numpy as np


def features(centres, halves, a, b):
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    halves = np.asarray(halves, dtype=np.float64).reshape(-1, 3)
    return np.concatenate([centres, (a * np.log2(2.0 * halves[:, :1]) + b)], axis=1)


def targets(mu, sigma, mu_bar, scale):
    return np.stack([(np.asarray(mu, np.float64) - mu_bar) / scale, np.log(np.asarray(sigma, np.float64))], axis=1)


def base_targets(mu, sigma, f, s, s_floor):
    """Targets relative to a base (f, s) per cell, the centre linearisation:
    ((mu - f) / s_b, ln(sigma / s_b)) with s_b = max(s, s_floor)."""
    sb = np.maximum(np.asarray(s, np.float64), s_floor)
    return np.stack([(np.asarray(mu, np.float64) - np.asarray(f, np.float64)) / sb,
                     np.log(np.asarray(sigma, np.float64) / sb)], axis=1)


def base_prediction(out, f, s, s_floor):
    """(mu_hat, sigma_hat) from the network outputs and the base."""
    sb = np.maximum(np.asarray(s, np.float64), s_floor)
    return np.stack([np.asarray(f, np.float64) + sb * out[:, 0], sb * np.exp(out[:, 1])], axis=1)


def forward(Ws, bs, X):
    """Returns (output [B, 2], activations [X, H1, H2, H3])."""
    acts = [np.asarray(X, dtype=np.float64)]
    h = acts[0]
    for li, (W, b) in enumerate(zip(Ws, bs)):
        h = h @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
        if li + 1 < len(Ws):
            h = np.maximum(h, 0.0)
            acts.append(h)
    return h, acts


def loss(out, T):
    d = out - T
    return 0.5 * np.mean(d[:, 0] ** 2) + 0.5 * np.mean(d[:, 1] ** 2)


def backward(Ws, acts, out, T):
    """Gradients (dWs, dbs) of ``loss`` with respect to the weights."""
    B = out.shape[0]
    dy = (out - T) / B  # d loss / d out
    dWs = [None] * len(Ws)
    dbs = [None] * len(Ws)
    for li in range(len(Ws) - 1, -1, -1):
        h_in = acts[li]
        dWs[li] = dy.T @ h_in
        dbs[li] = dy.sum(axis=0)
        if li > 0:
            dy = (dy @ np.asarray(Ws[li], np.float64)) * (acts[li] > 0.0)
    return dWs, dbs


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step count t >= 1) of lists of arrays, in place."""
    for p, g, mi, vi in zip(params, grads, m, v):
        mi *= beta1
        mi += (1.0 - beta1) * g
        vi *= beta2
        vi += (1.0 - beta2) * g * g
        mhat = mi / (1.0 - beta1 ** t)
        vhat = vi / (1.0 - beta2 ** t)
        p -= lr * mhat / (np.sqrt(vhat) + eps)
