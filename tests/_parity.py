"""Shared helpers for the GPU parity tests (comparison against the oracle)."""

from __future__ import annotations

import numpy as np

from oracle.mlp import mlp_forward
from oracle.metrics import margin
from oracle.octree import bound_k, morton_decode
from workloads import uniform_points


def output_scale(mlp, seed=1, n=10_000):
    """S: std of the float64 MLP output over uniform points (scale for
    relative errors and borderline bands)."""
    return float(np.std(mlp_forward(mlp, uniform_points(n, seed))))


def assert_pair_close(got, ref, S, rtol, label="", k=3.0, spread_rtol=None):
    """Bounds parity: centre and both bound endpoints centre -/+ k*spread
    within rtol * max(|o|, S) (S = output scale); the spread itself within
    spread_rtol * max(o, 1e-3 S) (default 10 * rtol: a sum of squares of
    coefficients that each carry the cancellation error of their own dot
    products, so it is less well conditioned than the bounds)."""
    got = np.asarray(got, dtype=np.float64)
    spread_rtol = 10 * rtol if spread_rtol is None else spread_rtol
    oc, os_ = np.asarray(ref[0]), np.asarray(ref[1])
    gc, gs = got[:, 0], got[:, 1]
    errs = {}
    errs["centre"] = np.abs(gc - oc) / np.maximum(np.abs(oc), S)
    for name, sgn in (("lo", -1.0), ("hi", 1.0)):
        o = oc + sgn * k * os_
        g = gc + sgn * k * gs
        errs[name] = np.abs(g - o) / np.maximum(np.abs(o), S)
    s_err = np.abs(gs - os_) / np.maximum(os_, 1e-3 * S)
    worst = {n: float(e.max()) if e.size else 0.0 for n, e in errs.items()}
    worst_s = float(s_err.max()) if s_err.size else 0.0
    print(f"[{label}] max rel err centre {worst['centre']:.3e} lo {worst['lo']:.3e} hi {worst['hi']:.3e} "
          f"(tol {rtol:.0e}); spread {worst_s:.3e} (tol {spread_rtol:.0e}); n={got.shape[0]}", flush=True)
    for n, w in worst.items():
        assert w <= rtol, f"{label}: {n} rel err {w:.3e}"
    assert worst_s <= spread_rtol, f"{label}: spread rel err {worst_s:.3e}"
    return worst, worst_s


def close_sets(oracle_levels, method, k, isos, S, band_rel=1e-4):
    """Per level, ids of oracle-evaluated cells whose bound endpoint lies
    within band_rel*S of an iso-value (borderline cells)."""
    kk = bound_k(method, k)
    out = []
    for lv in oracle_levels:
        m = margin(lv["centre"], lv["spread"], kk, isos)
        out.append(set(lv["ids"][m <= band_rel * S].tolist()))
    return out


def is_excused(cell, level, close):
    """A difference in `cell` is excused iff it or an ancestor is borderline."""
    for L in range(level, -1, -1):
        if (int(cell) >> (3 * (level - L))) in close[L]:
            return True
    return False


def unexcused_level_diffs(gpu_levels, oracle_levels, close):
    """[(level, n_diff, sample of unexcused ids)] for levels whose active sets
    differ outside the borderline exemption."""
    bad = []
    for L, (g, o) in enumerate(zip(gpu_levels, oracle_levels)):
        g_ids, _, g_mask = g
        g_act = set(g_ids[g_mask != 0].tolist())
        o_act = set(o["ids"][o["mask"] != 0].tolist())
        diff = g_act ^ o_act
        unexcused = [c for c in diff if not is_excused(c, L, close)]
        if unexcused:
            bad.append((L, len(diff), sorted(unexcused)[:5]))
    return bad


def leaf_ijk(ids):
    i, j, k = morton_decode(np.asarray(ids, dtype=np.uint64))
    return np.stack([i, j, k], axis=1)


def unexplained_unshared_edges(gmap, omap, depth, f, iso, S, diff_leaves, band_rel=1e-4):
    """Grid edges that carry a vertex in only one of the two meshes and are
    explained by neither of the two allowed causes: a containing cell that is
    an active leaf in one run only (``diff_leaves``, Morton ids, each already
    excused by the active-set check), or an endpoint whose value lies within
    band_rel * S of the iso-value (the case bits may differ there).  Keys are
    (grid point linear index) * 3 + axis on the (2^D + 1)^3 grid."""
    from oracle.octree import morton_encode

    R = (1 << depth) + 1
    n = 1 << depth
    bad = []
    for key in set(gmap) ^ set(omap):
        p, axis = divmod(int(key), 3)
        i, j, kk = p % R, (p // R) % R, p // (R * R)
        ijk = [i, j, kk]
        end = list(ijk)
        end[axis] += 1
        step = 2.0 / n
        pts = np.array([[-1.0 + step * q for q in ijk], [-1.0 + step * q for q in end]])
        v = f(pts)
        if np.abs(v - iso).min() <= band_rel * S:
            continue
        cells = []
        others = [a for a in range(3) if a != axis]
        for d0 in (-1, 0):
            for d1 in (-1, 0):
                c = list(ijk)
                c[others[0]] += d0
                c[others[1]] += d1
                if all(0 <= c[a] < n for a in range(3)):
                    cells.append(int(morton_encode(c[0], c[1], c[2])))
        if not any(c in diff_leaves for c in cells):
            bad.append(int(key))
    return bad
