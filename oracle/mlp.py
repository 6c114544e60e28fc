"""Plain coordinate-MLP evaluation in float64 (Sec. III-B: a chain of linear
layers, each but the last followed by the activation: ReLU, or sine / ELU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""

from __future__ import annotations

import numpy as np


def as_f64_layers(layers):
    """[(W, b), ...] -> float64 copies.  Accepts an object with ``layers()``."""
    if hasattr(layers, "layers"):
        layers = layers.layers()
    return [(np.asarray(W, dtype=np.float64), np.asarray(b, dtype=np.float64)) for W, b in layers]


def mlp_forward(layers, x, chunk: int = 1 << 16, act: str = "relu") -> np.ndarray:
    """f(x) for points ``x [N, 3]``; returns ``[N]`` float64."""
    from .rules import activation

    layers = as_f64_layers(layers)
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(x.shape[0], dtype=np.float64)
    for s in range(0, x.shape[0], chunk):
        h = x[s : s + chunk]
        for li, (W, b) in enumerate(layers):
            h = h @ W.T + b
            if li + 1 < len(layers):
                h = activation(act, h)
        out[s : s + chunk] = h[:, 0]
    return out
