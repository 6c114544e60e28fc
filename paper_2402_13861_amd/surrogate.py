"""Training of the learned surrogate: argument marshalling around the
library's one-call ``isx_surrogate_fit`` (sampling of the training cells,
their propagation, the forward/backward passes and Adam steps, and the
calibration of the safety bands all run in the library).

The surrogate is a ReLU MLP 4 -> 128 -> 128 -> 128 -> 2 that maps a cell
(centre, log2 size) to the propagation's predicted (mean, sigma).  It is
trained on (cell, propagated mean/sigma) pairs produced by the method itself:
about half are cells a plain extraction visited, the rest uniform random
cells at octree levels 3..D.  Its two outputs are either standardised targets
((mu - mu_bar)/S, ln sigma), or, with ``base=True``, corrections to the
centre linearisation (f(c), s) of the INR: ((mu - f)/s_b, ln(sigma/s_b)).
Its error is calibrated per octree level on held-out pairs; during
extraction a cell is decided by the surrogate only when every iso-value it
carries lies outside (or inside) the predicted soft bound by more than z
standard deviations of that error, and is propagated otherwise.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class SurrogateInfo:
    sid: int
    n_pairs: int
    steps: int
    train_seconds: float
    final_loss: float
    err_mu: List[float] = field(default_factory=list)
    err_logsig: List[float] = field(default_factory=list)
    losses: Optional[np.ndarray] = None
    z: float = 2.0
    z_accept: float = 2.0
    z_levels: List[float] = field(default_factory=list)
    z_accept_levels: List[float] = field(default_factory=list)
    holdout_miss: float = 0.0
    holdout_false_accept: float = 0.0


def train_surrogate(ctx, mlp_id: int, depth: int, mu_bar: float, scale: float, visited=None,
                    n_pairs: int = 5_000_000, steps: int = 2000, batch: int = 4096, lr: float = 1e-3,
                    seed: int = 0, holdout: int = 200_000, k: float = 3.0, miss_target: float = 1e-4,
                    accept_target: float = 1e-3, accept_leaves: bool = False, base: bool = False,
                    min_level_kept: int = 20000, log=None) -> SurrogateInfo:
    """Train a surrogate for ``mlp_id`` (whose iso-values must be set) and
    attach it for extraction.

    visited: optional Mesh of a plain extraction made with KEEP_LEVELS; about
    half of the training and held-out cells are drawn from the cells it
    examined.  The prune band per level is the smallest ladder value whose
    held-out miss rate (cells the plain test keeps for an iso-value the rule
    would drop) is at most ``miss_target``; the accept band likewise for the
    false-accept rate and ``accept_target`` (levels with fewer than
    ``min_level_kept`` kept held-out cells use the bands chosen over all
    levels)."""
    log = log or (lambda *a: None)
    t0 = time.perf_counter()
    sid, cal, losses = ctx.surrogate_fit(mlp_id, visited, n_pairs=n_pairs, n_holdout=holdout, steps=steps,
                                         batch=batch, lr=lr, seed=seed, depth=depth, mu_bar=mu_bar, scale=scale, k=k,
                                         use_base=base, accept_leaves=accept_leaves, miss_target=miss_target,
                                         accept_target=accept_target, min_level_kept=min_level_kept)
    total_s = time.perf_counter() - t0
    log(f"surrogate: {n_pairs} pairs, {steps} steps of batch {batch} in {total_s:.2f} s (sampling, propagation, "
        f"training and calibration), loss {losses[0]:.4f} -> {losses[-20:].mean():.4f}")
    log("surrogate: per-level error (mu, log sigma): " +
        ", ".join(f"L{L} {a:.3g}/{b:.3g}" for L, (a, b) in enumerate(zip(cal["err_mu"], cal["err_logsig"]))))
    log("surrogate: per-level bands (prune/accept): " +
        ", ".join(f"L{L} {a}/{b}" for L, (a, b) in enumerate(zip(cal["z"], cal["z_accept"]))) +
        f"; held-out miss {cal['holdout_miss']:.2e}, false accept {cal['holdout_false_accept']:.2e}")
    info = SurrogateInfo(sid, n_pairs, steps, total_s, float(losses[-20:].mean()), cal["err_mu"], cal["err_logsig"],
                         losses)
    info.z = cal["z_global"]
    info.z_accept = cal["z_accept_global"]
    info.z_levels = cal["z"]
    info.z_accept_levels = cal["z_accept"]
    info.holdout_miss = cal["holdout_miss"]
    info.holdout_false_accept = cal["holdout_false_accept"]
    return info
