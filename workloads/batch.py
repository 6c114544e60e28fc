"""The batched workload: 64 independent ReLU INRs of uneven shape.

INR i (i = 0..63) draws, from ``numpy.random.default_rng(3 + i)`` in this
order, its hidden width uniformly from {64, 128, 256, 512}, its number of
hidden layers uniformly from 3..8, and four quantile levels
sort(U(0.1, 0.9)).  Its weights and biases are He-normal from
``default_rng(3 + i)`` in a generator of their own (``he_normal_mlp``).  Its
iso-values are the MLP's output quantiles at those levels over 10^4 uniform
points (the iso-value protocol of the other workloads; stored by
``workloads.make_isovalues`` in ``isovalues.json`` under "batch64").
Octree depth 8 (256^3), t = 3, BF16 propagation.
"""

from __future__ import annotations

import numpy as np

from .weights import he_normal_mlp

N_INRS = 64
DEPTH = 8
WIDTHS = (64, 128, 256, 512)


def batch_shapes(n: int = N_INRS):
    """[(widths list, quantile levels [4])] of the n INRs."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(3 + i)
        w = int(rng.choice(WIDTHS))
        d = int(rng.integers(3, 9))
        q = np.sort(rng.uniform(0.1, 0.9, 4))
        out.append(([3] + [w] * d + [1], q))
    return out


def batch_mlps(n: int = N_INRS):
    return [he_normal_mlp(widths, 3 + i) for i, (widths, _) in enumerate(batch_shapes(n))]
