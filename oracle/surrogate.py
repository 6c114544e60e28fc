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


def partition(pred, unit, k, isos, parent_mask, err_mu, err_ls, z, z_acc, leaf, accept_leaves):
    """Band partition of cells by the surrogate's prediction (the learned
    part's safety band around the soft-bound test of Alg. 1), float64.

    pred [n, 2] = (mu_hat, sigma_hat); unit [n] scales err_mu per cell (None =
    1, field units); err_mu / err_ls are the standard deviations of the
    surrogate's error in mu (times unit) and in ln sigma; z / z_acc the prune
    and accept bands in those units.  For every iso-value c_j the cell
    carries (bit j of parent_mask), with d = |mu_hat - c_j|:
      outside  if d - z err_mu unit > t sigma_hat e^{+z err_ls}      (bit dropped)
      inside   if d + z_acc err_mu unit < t sigma_hat e^{-z_acc err_ls}  (bit kept)
      unsure   otherwise.
    A cell with no unsure iso-value is decided without propagation (its mask
    is the set of inside bits); one with an unsure iso-value, a non-finite
    prediction, or -- at the leaf level unless accept_leaves -- any inside
    bit, falls back to propagation (mask 0, fallback 1).

    Returns (mask uint32 [n], fallback bool [n], slack [n]): slack is the
    smallest distance of a decision quantity to its threshold, relative to the
    larger side, over the carried iso-values (a cell whose slack is within
    float32 rounding may be decided either way in float32 arithmetic)."""
    pred = np.asarray(pred, np.float64)
    n = pred.shape[0]
    mu, sg = pred[:, 0], pred[:, 1]
    u = np.ones(n) if unit is None else np.asarray(unit, np.float64)
    pm = np.asarray(parent_mask, np.uint32)
    hi_s = k * sg * np.exp(z * err_ls)
    lo_s = k * sg * np.exp(-z_acc * err_ls)
    e, ea = z * err_mu * u, z_acc * err_mu * u
    inside = np.zeros(n, np.uint32)
    unsure = np.zeros(n, bool)
    slack = np.full(n, np.inf)
    for j, c in enumerate(isos):
        carried = ((pm >> np.uint32(j)) & np.uint32(1)).astype(bool)
        d = np.abs(mu - np.float64(c))
        out_q, in_q = d - e, d + ea
        is_out = out_q > hi_s
        is_in = (~is_out) & (in_q < lo_s)
        inside |= np.where(carried & is_in, np.uint32(1) << np.uint32(j), np.uint32(0))
        unsure |= carried & ~is_out & ~is_in
        rel = np.minimum(np.abs(out_q - hi_s) / np.maximum(np.maximum(np.abs(out_q), hi_s), 1e-300),
                         np.abs(in_q - lo_s) / np.maximum(np.maximum(np.abs(in_q), lo_s), 1e-300))
        slack = np.where(carried, np.minimum(slack, rel), slack)
    unsure |= ~np.isfinite(mu) | ~np.isfinite(sg)
    fallback = unsure | (bool(leaf) and not accept_leaves) & (inside != 0)
    mask = np.where(fallback, np.uint32(0), inside)
    return mask.astype(np.uint32), fallback, slack
