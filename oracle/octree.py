"""Hierarchical active-cell search, octree form of Alg. 1, float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Alg. 1 recurses top-down from the domain box: a node is propagated, its
soft bound [mu - t sigma, mu + t sigma] (or the AA hard range) is tested
against the iso-value, a node whose bound misses the iso-value is dropped
(the test is strict, so a bound touching c keeps the node), and surviving
nodes are split until the maximum depth, where they are the active cells.
Here every split is the 8-way octree split (three widest-axis k-d splits of
a cube at once), the nodes of one level are handled together (each node's
decision depends only on its own box, so the result equals the depth-first
recursion), and several iso-values are tracked with a bit mask per cell: bit
j survives while iso j stays inside the bound of the cell and all of its
ancestors.

Cell (L, i, j, k) covers lo + [i, i+1] * s_L (per axis, s_L = (hi-lo)/2^L);
its id is the Morton code with the x bit lowest, so the 8 children of id p
are 8p + (dz<<2 | dy<<1 | dx) and child lists stay in Morton order.
"""

from __future__ import annotations

import numpy as np

from .propagate import AA, UP, RAUA, propagate


def morton_encode(i, j, k):
    i = np.asarray(i, dtype=np.uint64)
    j = np.asarray(j, dtype=np.uint64)
    k = np.asarray(k, dtype=np.uint64)
    code = np.zeros(np.broadcast(i, j, k).shape, dtype=np.uint64)
    for t in range(21):
        one = np.uint64(1)
        code |= ((i >> np.uint64(t)) & one) << np.uint64(3 * t)
        code |= ((j >> np.uint64(t)) & one) << np.uint64(3 * t + 1)
        code |= ((k >> np.uint64(t)) & one) << np.uint64(3 * t + 2)
    return code


def morton_decode(code):
    code = np.asarray(code, dtype=np.uint64)
    i = np.zeros(code.shape, dtype=np.int64)
    j = np.zeros(code.shape, dtype=np.int64)
    k = np.zeros(code.shape, dtype=np.int64)
    for t in range(21):
        one = np.uint64(1)
        i |= (((code >> np.uint64(3 * t)) & one).astype(np.int64)) << t
        j |= (((code >> np.uint64(3 * t + 1)) & one).astype(np.int64)) << t
        k |= (((code >> np.uint64(3 * t + 2)) & one).astype(np.int64)) << t
    return i, j, k


def cell_boxes(level, ids, lo=(-1.0,) * 3, hi=(1.0,) * 3):
    """Centres and half-widths [C, 3] of the level-L cells with Morton ``ids``
    (Alg. 1: centre = (x_l + x_u)/2, axes = (x_u - x_c))."""
    i, j, k = morton_decode(ids)
    ijk = np.stack([i, j, k], axis=1).astype(np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    size = (hi - lo) / (2.0 ** level)
    centres = lo[None, :] + (ijk + 0.5) * size[None, :]
    halves = np.broadcast_to(size / 2.0, centres.shape).copy()
    return centres, halves


def classify(centre, spread, k, isos, parent_mask):
    """Per-iso soft-bound test (Alg. 1): bit j is kept iff
    centre - k spread <= c_j <= centre + k spread and the parent has bit j."""
    isos = np.asarray(isos, dtype=np.float64)
    lo = centre - k * spread
    hi = centre + k * spread
    inside = (lo[:, None] <= isos[None, :]) & (isos[None, :] <= hi[:, None])
    bits = (inside.astype(np.uint32) << np.arange(isos.size, dtype=np.uint32)[None, :]).sum(axis=1)
    return (bits.astype(np.uint32) & np.asarray(parent_mask, dtype=np.uint32)).astype(np.uint32)


def bound_k(method, k):
    return 1.0 if method == AA else float(k)


def extract_active(layers, method, isos, depth, k=3.0, lo=(-1.0,) * 3, hi=(1.0,) * 3,
                   max_cells=None, act="relu"):
    """Octree search of Alg. 1 from the root to ``depth``.

    Returns a list, one dict per level 0..depth, with the evaluated cells
    ``ids`` (uint64 Morton), their ``centre``/``spread`` read-off and ``mask``
    (uint32 iso bits after the test; 0 = dropped).  The active leaves are the
    entries of the last level with mask != 0.
    """
    isos = np.atleast_1d(np.asarray(isos, dtype=np.float64))
    full = np.uint32((1 << isos.size) - 1)
    kk = bound_k(method, k)
    ids = np.zeros(1, dtype=np.uint64)
    pmask = np.array([full], dtype=np.uint32)
    levels = []
    for L in range(depth + 1):
        if L > 0:
            keep = levels[-1]["mask"] != 0
            par = levels[-1]["ids"][keep]
            pm = levels[-1]["mask"][keep]
            ids = (par[:, None] * np.uint64(8) + np.arange(8, dtype=np.uint64)[None, :]).ravel()
            pmask = np.repeat(pm, 8)
        if max_cells is not None and ids.size > max_cells:
            raise MemoryError(f"level {L}: {ids.size} cells exceed max_cells={max_cells}")
        c, h = cell_boxes(L, ids, lo, hi)
        centre, spread = propagate(layers, c, h, method, act=act)
        mask = classify(centre, spread, kk, isos, pmask)
        levels.append(dict(level=L, ids=ids, centre=centre, spread=spread, mask=mask))
    return levels


# ---------------------------------------------------------------- k-d tree
def widest_axis(half):
    """Split axis of Alg. 1: the widest dimension of the box, ties broken
    towards the lower axis index (x, then y, then z)."""
    half = np.asarray(half, dtype=np.float64)
    return int(np.argmax(half))  # argmax returns the first of equal maxima


def kd_split(centre, half, axis):
    """The two halves of a box split at its centre along ``axis``: (lower,
    upper), each as (centre, half-widths)."""
    c0, c1 = np.array(centre, dtype=np.float64), np.array(centre, dtype=np.float64)
    h = np.array(half, dtype=np.float64)
    h[axis] *= 0.5
    c0[axis] -= h[axis]
    c1[axis] += h[axis]
    return (c0, h), (c1, h.copy())


def extract_active_kd(layers, method, isos, depth, k=3.0, lo=(-1.0,) * 3, hi=(1.0,) * 3, act="relu"):
    """Alg. 1 with its binary k-d tree: every node is split along its widest
    dimension (ties x, y, z) until depth ``depth`` (the paper takes a multiple
    of 3, so that a cube domain ends in cubes), nodes of one depth handled
    together (each node's decision depends only on its box).  Node ids:
    the root is 0 and the children of node p are 2p (lower half) and 2p + 1
    (upper half).  Returns one dict per depth 0..depth with ``ids``,
    ``centre``, ``half`` (per-axis half-widths), ``spread`` and ``mask`` as in
    ``extract_active``."""
    isos = np.atleast_1d(np.asarray(isos, dtype=np.float64))
    full = np.uint32((1 << isos.size) - 1)
    kk = bound_k(method, k)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    ids = np.zeros(1, dtype=np.uint64)
    cen = ((lo + hi) / 2.0)[None, :]
    hal = ((hi - lo) / 2.0)[None, :]
    pmask = np.array([full], dtype=np.uint32)
    levels = []
    for d in range(depth + 1):
        if d > 0:
            prev = levels[-1]
            keep = prev["mask"] != 0
            par_ids, par_c, par_h, par_m = prev["ids"][keep], prev["centre_box"][keep], prev["half"][keep], prev["mask"][keep]
            n = par_ids.size
            ids = np.empty(2 * n, dtype=np.uint64)
            cen = np.empty((2 * n, 3))
            hal = np.empty((2 * n, 3))
            for i in range(n):
                lower, upper = kd_split(par_c[i], par_h[i], widest_axis(par_h[i]))
                ids[2 * i], ids[2 * i + 1] = 2 * par_ids[i], 2 * par_ids[i] + np.uint64(1)
                cen[2 * i], hal[2 * i] = lower
                cen[2 * i + 1], hal[2 * i + 1] = upper
            pmask = np.repeat(par_m, 2)
        centre, spread = propagate(layers, cen, hal, method, act=act) if ids.size else (np.zeros(0), np.zeros(0))
        mask = classify(centre, spread, kk, isos, pmask)
        levels.append(dict(level=d, ids=ids, centre_box=cen, half=hal, centre=centre, spread=spread, mask=mask))
    return levels


def kd_to_morton(ids, depth3):
    """Octree Morton id (x bit lowest) of the k-d node ``ids`` at depth
    3 * depth3 of a cube domain, whose splits cycle x, y, z: each triple of
    id bits, read from the top, is the (x, y, z) side of one octree level."""
    ids = np.asarray(ids, dtype=np.uint64)
    out = np.zeros(ids.shape, dtype=np.uint64)
    for q in range(depth3):
        t = (ids >> np.uint64(3 * (depth3 - 1 - q))) & np.uint64(7)
        bx, by, bz = (t >> np.uint64(2)) & np.uint64(1), (t >> np.uint64(1)) & np.uint64(1), t & np.uint64(1)
        out |= (bx | (by << np.uint64(1)) | (bz << np.uint64(2))) << np.uint64(3 * (depth3 - 1 - q))
    return out
