"""Random axis-aligned boxes and sample points (seeded)."""

from __future__ import annotations

import numpy as np


def random_boxes(n: int, levels, seed: int, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0)):
    """``n`` random cubes of a dyadic grid over [lo, hi]^3.

    Each box draws a level L uniformly from ``levels`` and integer grid
    coordinates in [0, 2^L)^3; its centre is lo + (2i+1)(hi-lo)/2^(L+1) and its
    half-width (hi-lo)/2^(L+1) per axis.  On the default [-1, 1]^3 domain both
    are exact in float32.  Returns float32 ``centres [n,3]``, ``halves [n,3]``
    and int ``levels [n]``.
    """
    rng = np.random.default_rng(seed)
    levels = np.asarray(list(levels), dtype=np.int64)
    L = rng.choice(levels, size=n)
    ijk = np.floor(rng.random((n, 3)) * (2.0 ** L)[:, None]).astype(np.int64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    scale = (hi - lo)[None, :] / (2.0 ** (L + 1))[:, None]
    centres = lo[None, :] + (2 * ijk + 1) * scale
    halves = np.broadcast_to(scale, (n, 3)).copy()
    return centres.astype(np.float32), halves.astype(np.float32), L


def uniform_points(n: int, seed: int, lo=-1.0, hi=1.0) -> np.ndarray:
    """``n`` points uniform in [lo, hi]^3 from ``default_rng(seed)`` (float64)."""
    return np.random.default_rng(seed).uniform(lo, hi, (n, 3))
