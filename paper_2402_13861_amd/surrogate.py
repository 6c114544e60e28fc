"""Training pipeline of the learned surrogate (orchestration only; every
propagation, forward/backward pass and optimiser step runs in the library's
HIP kernels).

The surrogate is a ReLU MLP 4 -> 128 -> 128 -> 128 -> 2 that maps a cell
(centre, log2 size) to the propagation's predicted (mean, sigma).  It is
trained on (cell, propagated mean/sigma) pairs produced by the method itself:
half are uniform random cells at octree levels 3..D, half are cells visited
by a plain extraction.  Its two outputs are either standardised targets
((mu - mu_bar)/S, ln sigma), or, with ``base=True``, corrections to the
centre linearisation (f(c), s) of the INR, which the library computes
alongside: ((mu - f)/s_b, ln(sigma/s_b)).  Its error is calibrated per octree
level on held-out pairs; during extraction a cell is decided by the
surrogate only when every iso-value it carries lies outside (or inside) the
predicted soft bound by more than z standard deviations of that error, and
is propagated otherwise.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import _lib

SIZE_A = 0.25  # size feature: a * log2(cell size) + b (maps levels 0..10 into [-1.5, 1])
SIZE_B = 1.0


def _morton_decode(ids):
    ids = np.asarray(ids, dtype=np.uint64)
    out = []
    for axis in range(3):
        v = np.zeros(ids.shape, dtype=np.int64)
        for t in range(11):
            v |= (((ids >> np.uint64(3 * t + axis)) & np.uint64(1)).astype(np.int64)) << t
        out.append(v)
    return np.stack(out, axis=1)


def level_boxes(level: int, ids, lo=(-1.0,) * 3, hi=(1.0,) * 3):
    """Centres and half-widths (float32) of Morton cells at a level."""
    ijk = _morton_decode(ids).astype(np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    step = (hi - lo) / (2.0 ** (level + 1))
    c = lo[None, :] + (2 * ijk + 1) * step[None, :]
    h = np.broadcast_to(step, c.shape)
    return c.astype(np.float32), np.ascontiguousarray(h, dtype=np.float32)


def random_level_cells(n: int, levels, rng, lo=(-1.0,) * 3, hi=(1.0,) * 3):
    L = rng.choice(np.asarray(list(levels)), size=n)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    ijk = np.floor(rng.random((n, 3)) * (2.0 ** L)[:, None])
    step = (hi - lo)[None, :] / (2.0 ** (L + 1))[:, None]
    c = lo[None, :] + (2 * ijk + 1) * step
    return c.astype(np.float32), step.astype(np.float32), L


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


def miss_rate(pred, true, levels, err_mu, err_ls, isos, k, z, unit=None):
    """Fraction of held-out cells that the plain test keeps for some iso-value
    but the surrogate rule at band z would drop for that iso-value (err_mu in
    units of ``unit`` per cell when given)."""
    mu_h, sg_h = pred[:, 0], pred[:, 1]
    mu, sg = true[:, 0], true[:, 1]
    em = np.asarray(err_mu)[levels] * (1.0 if unit is None else unit)
    el = np.asarray(err_ls)[levels]
    hi_s = k * sg_h * np.exp(z * el)
    miss = np.zeros(len(mu), dtype=bool)
    kept = np.zeros(len(mu), dtype=bool)
    for c in isos:
        plain_keep = np.abs(mu - c) <= k * sg
        drop = np.abs(mu_h - c) - z * em > hi_s
        kept |= plain_keep
        miss |= plain_keep & drop
    return miss.sum() / max(kept.sum(), 1)


def false_accept_rate(pred, true, levels, err_mu, err_ls, isos, k, z, unit=None):
    """Held-out cells that the surrogate rule at accept band z would accept
    for an iso-value the plain test rejects, per cell the plain test keeps."""
    mu_h, sg_h = pred[:, 0], pred[:, 1]
    mu, sg = true[:, 0], true[:, 1]
    em = np.asarray(err_mu)[levels] * (1.0 if unit is None else unit)
    el = np.asarray(err_ls)[levels]
    lo_s = k * sg_h * np.exp(-z * el)
    bad = np.zeros(len(mu), dtype=bool)
    kept = np.zeros(len(mu), dtype=bool)
    for c in isos:
        plain_keep = np.abs(mu - c) <= k * sg
        accept = np.abs(mu_h - c) + z * em < lo_s
        kept |= plain_keep
        bad |= accept & ~plain_keep
    return bad.sum() / max(kept.sum(), 1)


Z_LADDER = (0.0, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0, 5.0, 6.0, 8.0, 12.0)


def train_surrogate(ctx, mlp_id: int, depth: int, mu_bar: float, scale: float, visited=None,
                    n_pairs: int = 5_000_000, steps: int = 2000, batch: int = 4096, lr: float = 1e-3,
                    hidden=(128, 128, 128), seed: int = 0, holdout: int = 200_000, z: Optional[float] = None,
                    isos=None, k: float = 3.0, miss_target: float = 1e-4, accept_target: float = 1e-3,
                    z_accept: Optional[float] = None, accept_leaves: bool = False, base: bool = False,
                    per_level: bool = True, min_level_kept: int = 20000,
                    lo=(-1.0,) * 3, hi=(1.0,) * 3, log=None) -> SurrogateInfo:
    """Train a surrogate for ``mlp_id`` and attach it for extraction.

    visited: optional list, per octree level, of Morton ids of cells a plain
    extraction propagated; half of the training pairs are drawn from them.
    Targets are the float32 uncertainty propagation of each training cell;
    with ``base`` the network learns corrections to the INR's centre
    linearisation (s_b floored at 1e-6 S) and err_mu is in units of s_b.
    The safety band is z standard deviations of the surrogate's per-level
    error; with z None it is the smallest of a ladder of values whose miss
    rate on the held-out cells (against the iso-values ``isos`` and the
    bound multiplier k) is at most ``miss_target``.  A wrong accept only
    costs work, so the accept band z_accept is calibrated on its own: with
    None, the smallest ladder value whose held-out false-accept rate is at
    most ``accept_target``.  With ``per_level``, each octree level whose
    held-out set has at least ``min_level_kept`` cells that the plain test
    keeps gets its own bands by the same rules (the others use the global
    ones).
    """
    import torch

    log = log or (lambda *a: None)
    rng = np.random.default_rng(seed)
    n_train = n_pairs
    n_total = n_train + holdout
    # --- training cells: half random levels 3..depth, half visited cells
    n_vis = n_total // 2 if visited else 0
    parts_c, parts_h, parts_L = [], [], []
    if n_vis:
        sizes = np.array([len(v) for v in visited], dtype=np.float64)
        p = sizes / sizes.sum()
        counts = rng.multinomial(n_vis, p)
        for L, (ids, cnt) in enumerate(zip(visited, counts)):
            if cnt == 0 or len(ids) == 0:
                continue
            pick = np.asarray(ids)[rng.integers(0, len(ids), cnt)]
            c, h = level_boxes(L, pick, lo, hi)
            parts_c.append(c)
            parts_h.append(h)
            parts_L.append(np.full(cnt, L))
    c, h, L = random_level_cells(n_total - n_vis, range(min(3, depth), depth + 1), rng, lo, hi)
    parts_c.append(c)
    parts_h.append(h)
    parts_L.append(L)
    centres = np.concatenate(parts_c)
    halves = np.concatenate(parts_h)
    levels = np.concatenate(parts_L)
    perm = rng.permutation(n_total)
    centres, halves, levels = centres[perm], halves[perm], levels[perm]

    dev = torch.device("cuda", ctx.device)
    C = torch.from_numpy(np.ascontiguousarray(centres)).to(dev)
    H = torch.from_numpy(np.ascontiguousarray(halves)).to(dev)
    T = torch.empty((n_total, 2), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    ctx.propagate(mlp_id, _lib.UP, _lib.FP32, C, H, T)
    torch.cuda.synchronize(dev)
    log(f"surrogate: {n_total} training cells propagated in {time.perf_counter() - t0:.1f} s")

    # --- model: He-normal weights N(0, 2/fan_in), small random biases
    widths = [4, *hidden, 2]
    Ws, bs = [], []
    for fi, fo in zip(widths[:-1], widths[1:]):
        std = np.sqrt(2.0 / fi)
        Ws.append((rng.standard_normal((fo, fi)) * std).astype(np.float32))
        bs.append((rng.standard_normal(fo) * std * 0.1).astype(np.float32))
    sid = ctx.surrogate_load(Ws, bs)
    ctx.surrogate_set_norm(sid, mu_bar, scale, SIZE_A, SIZE_B)
    s_floor = 1e-6 * scale
    if base:
        ctx.surrogate_set_base(sid, mlp_id, s_floor)

    Ct, Ht, Tt = C[:n_train], H[:n_train], T[:n_train]
    losses = torch.empty(steps, dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    ctx.surrogate_train(sid, Ct, Ht, Tt, steps=steps, batch=batch, lr=lr, loss=losses)
    torch.cuda.synchronize(dev)
    train_s = time.perf_counter() - t0
    losses = losses.cpu().numpy()
    log(f"surrogate: {steps} steps of batch {batch} in {train_s:.2f} s, loss {losses[0]:.4f} -> "
        f"{losses[-20:].mean():.4f}")

    # --- calibration on held-out cells: error std per level
    Cv, Hv, Tv = C[n_train:], H[n_train:], T[n_train:]
    P = torch.empty((holdout, 2), dtype=torch.float32, device=dev)
    ctx.surrogate_predict(sid, Cv, Hv, P)
    torch.cuda.synchronize(dev)
    p = P.cpu().numpy().astype(np.float64)
    tv = Tv.cpu().numpy().astype(np.float64)
    lv = levels[n_train:]
    unit = None
    if base:
        Bv = torch.empty((holdout, 2), dtype=torch.float32, device=dev)
        ctx.linearize(mlp_id, Cv, Hv, Bv)
        torch.cuda.synchronize(dev)
        unit = np.maximum(Bv.cpu().numpy()[:, 1].astype(np.float64), s_floor)
    err_mu, err_ls = [], []
    for L in range(depth + 1):
        sel = lv == L
        if sel.sum() < 50:
            err_mu.append(err_mu[-1] if err_mu else scale)
            err_ls.append(err_ls[-1] if err_ls else 1.0)
            continue
        dmu = p[sel, 0] - tv[sel, 0]
        if unit is not None:
            dmu = dmu / unit[sel]
        dls = np.log(np.maximum(p[sel, 1], 1e-30)) - np.log(np.maximum(tv[sel, 1], 1e-30))
        err_mu.append(float(np.sqrt(np.mean(dmu ** 2))))
        err_ls.append(float(np.sqrt(np.mean(dls ** 2))))
    log("surrogate: per-level error (mu, log sigma): " +
        ", ".join(f"L{L} {a:.3g}/{b:.3g}" for L, (a, b) in enumerate(zip(err_mu, err_ls))))
    if (z is None or z_accept is None) and isos is None:
        raise ValueError("calibrating a band needs the iso-values")
    if z is None:
        rates = {}
        for zc in Z_LADDER[4:]:
            rates[zc] = miss_rate(p, tv, lv, err_mu, err_ls, isos, k, zc, unit)
            if rates[zc] <= miss_target:
                break
        z = zc
        log("surrogate: held-out miss rate by prune band: " + ", ".join(f"z={a}: {b:.2e}" for a, b in rates.items()))
    if z_accept is None:
        rates = {}
        for zc in Z_LADDER:
            rates[zc] = false_accept_rate(p, tv, lv, err_mu, err_ls, isos, k, zc, unit)
            if rates[zc] <= accept_target:
                break
        z_accept = zc
        log("surrogate: held-out false-accept rate by accept band: " +
            ", ".join(f"z={a}: {b:.2e}" for a, b in rates.items()))
    z_lv = [float(z)] * (depth + 1)
    za_lv = [float(z_accept)] * (depth + 1)
    if per_level and isos is not None:
        for L in range(depth + 1):
            sel = lv == L
            if not sel.any():
                continue
            mu_t, sg_t = tv[sel, 0], tv[sel, 1]
            kept = np.zeros(sel.sum(), dtype=bool)
            for c in isos:
                kept |= np.abs(mu_t - c) <= k * sg_t
            if kept.sum() < min_level_kept:
                continue
            u = None if unit is None else unit[sel]
            args = (p[sel], tv[sel], lv[sel], err_mu, err_ls, isos, k)
            z_lv[L] = next((zc for zc in Z_LADDER[4:] if miss_rate(*args, zc, u) <= miss_target), Z_LADDER[-1])
            za_lv[L] = next((zc for zc in Z_LADDER if false_accept_rate(*args, zc, u) <= accept_target),
                            Z_LADDER[-1])
        log("surrogate: per-level bands (prune/accept): " +
            ", ".join(f"L{L} {a}/{b}" for L, (a, b) in enumerate(zip(z_lv, za_lv))))
    ctx.surrogate_attach(mlp_id, sid, err_mu, err_ls, z=z_lv, accept_leaves=accept_leaves, z_accept=za_lv)
    info = SurrogateInfo(sid, n_train, steps, train_s, float(losses[-20:].mean()), err_mu, err_ls, losses)
    info.z = z
    info.z_accept = z_accept
    info.z_levels = z_lv
    info.z_accept_levels = za_lv
    if isos is not None:
        zl, zal = np.asarray(z_lv)[lv], np.asarray(za_lv)[lv]
        info.holdout_miss = float(miss_rate(p, tv, lv, err_mu, err_ls, isos, k, zl, unit))
        info.holdout_false_accept = float(false_accept_rate(p, tv, lv, err_mu, err_ls, isos, k, zal, unit))
    return info
