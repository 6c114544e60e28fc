"""Centre linearisation of a box, float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A ReLU MLP is piecewise linear.  Around the centre c of a box, where no
pre-activation is exactly zero, it coincides with its tangent
f(c) + J(c) (x - c), J(c) the product of the layer matrices with the rows of
inactive neurons removed.  Pushing the uncertainty propagation's input form
(x = c + diag(h / sqrt 3) Z, Sec. IV-C) through that tangent gives the normal
law N(f(c), s^2) with s = |J(c) diag(h)| / sqrt 3 (Eq. 6-8 with every
activation linear).  This is the limit of the propagation for boxes that no
ReLU kink crosses, and the base that the learned surrogate corrects.

The derivative of ReLU at exactly 0 is taken as 0.
"""

from __future__ import annotations

import numpy as np

from .mlp import as_f64_layers


def linearize(layers, centres, halves, return_margin: bool = False):
    """(f(c), s) per box as two float64 arrays [N]; with ``return_margin``
    also the smallest |pre-activation| at the centre over all hidden neurons
    (how far the centre is from the nearest ReLU kink, in output-free units)."""
    layers = as_f64_layers(layers)
    c = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    h = np.asarray(halves, dtype=np.float64).reshape(-1, 3)
    x = c.copy()
    # tangent directions, one row per input symbol: T[i, a, :] = d x / d Z_a
    T = np.zeros((c.shape[0], 3, 3))
    for a in range(3):
        T[:, a, a] = h[:, a] / np.sqrt(3.0)
    margin = np.full(c.shape[0], np.inf)
    last = len(layers) - 1
    for li, (W, b) in enumerate(layers):
        pre = x @ W.T + b
        T = T @ W.T
        if li == last:
            x = pre
            break
        on = pre > 0.0
        margin = np.minimum(margin, np.abs(pre).min(axis=1))
        x = np.where(on, pre, 0.0)
        T = T * on[:, None, :]
    f = x[:, 0]
    s = np.sqrt(np.sum(T[:, :, 0] ** 2, axis=1))
    if return_margin:
        return f, s, margin
    return f, s
