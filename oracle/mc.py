"""Marching cubes on leaf cells and on the dense grid, float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper reconstructs the INR at the corners of the active leaves and runs
marching cubes there (Sec. IV-D, end; Sec. V-A-4); the dense baseline runs it
on the whole grid (Sec. IV-D, start).  It does not fix a case table, so the
table is generated here from a rule (this is the oracle's own generator; the
HIP library generates its table independently):

* a corner is "inside" iff its value is < c (a value equal to c is outside);
* on each face, walking the corners counter-clockwise as seen from outside
  the cube, an edge is an *entry* edge if the walk goes outside -> inside
  across it and an *exit* edge if inside -> outside; each entry edge is joined
  to the next exit edge.  On a face with two diagonal inside corners this
  separates the inside corners (face-consistent: both cubes sharing the face
  see the same segments, so the surface has no cracks);
* segments are directed entry -> exit; every crossed edge is the exit of one
  face segment and the entry of the other face's, so they chain into closed
  cycles.  Each cycle starts at its smallest edge number, cycles are ordered
  by that number, and each is fanned from its first vertex.  With this
  direction the triangles' right-hand normals point toward the outside
  (larger values).

Corner numbering: 0 (0,0,0), 1 (1,0,0), 2 (1,1,0), 3 (0,1,0), 4 (0,0,1),
5 (1,0,1), 6 (1,1,1), 7 (0,1,1).  Edge e joins corners EDGES[e] = (lower,
upper) along axis EDGE_AXIS[e]; a vertex on an edge is interpolated from the
lower corner p to the upper corner q as p + (c - v_p)/(v_q - v_p) (q - p).
"""

from __future__ import annotations

import numpy as np

CORNERS = np.array(
    [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)],
    dtype=np.int64,
)
EDGES = [(0, 1), (1, 2), (3, 2), (0, 3), (4, 5), (5, 6), (7, 6), (4, 7), (0, 4), (1, 5), (2, 6), (3, 7)]
EDGE_AXIS = [0, 1, 0, 1, 0, 1, 0, 1, 2, 2, 2, 2]


def _faces_ccw():
    """The six faces, corners ordered counter-clockwise about the outward normal."""
    faces = []
    for axis in range(3):
        for side in (0, 1):
            idx = [c for c in range(8) if CORNERS[c][axis] == side]
            normal = np.zeros(3)
            normal[axis] = 1.0 if side == 1 else -1.0
            centre = CORNERS[idx].mean(axis=0)
            # order by angle around the outward normal
            u = np.zeros(3)
            u[(axis + 1) % 3] = 1.0
            v = np.cross(normal, u)
            ang = [np.arctan2(np.dot(CORNERS[c] - centre, v), np.dot(CORNERS[c] - centre, u)) for c in idx]
            faces.append([idx[t] for t in np.argsort(ang)])
    return faces


def _edge_of(a, b):
    for e, (p, q) in enumerate(EDGES):
        if {p, q} == {a, b}:
            return e
    raise KeyError((a, b))


def generate_case_table():
    """Returns a list of 256 lists of triangles (edge-index triples)."""
    faces = _faces_ccw()
    table = []
    for case in range(256):
        inside = [(case >> c) & 1 == 1 for c in range(8)]
        nxt = {}
        for f in faces:
            ring = [(f[t], f[(t + 1) % 4]) for t in range(4)]
            marks = []  # (position, kind, edge)
            for t, (a, b) in enumerate(ring):
                if inside[a] != inside[b]:
                    marks.append((t, "exit" if inside[a] else "entry", _edge_of(a, b)))
            for m, (t, kind, e) in enumerate(marks):
                if kind != "entry":
                    continue
                # the next exit edge walking counter-clockwise
                for step in range(1, len(marks)):
                    t2, kind2, e2 = marks[(m + step) % len(marks)]
                    if kind2 == "exit":
                        nxt[e] = e2
                        break
        tris = []
        seen = set()
        for start in sorted(nxt):
            if start in seen:
                continue
            cyc = [start]
            seen.add(start)
            e = nxt[start]
            while e != start:
                cyc.append(e)
                seen.add(e)
                e = nxt[e]
            for t in range(1, len(cyc) - 1):
                tris.append((cyc[0], cyc[t], cyc[t + 1]))
        table.append(tris)
    return table


_TABLE = None


def case_table():
    global _TABLE
    if _TABLE is None:
        _TABLE = generate_case_table()
    return _TABLE


def cell_cases(values, c):
    """values [N, 8] corner values -> case index [N] (bit i set iff v_i < c)."""
    bits = (np.asarray(values) < c).astype(np.int64)
    return (bits << np.arange(8, dtype=np.int64)[None, :]).sum(axis=1)


def march(cell_ijk, values, c, depth, lo=(-1.0,) * 3, hi=(1.0,) * 3):
    """Marching cubes over cells of the level-``depth`` grid.

    cell_ijk [N, 3] integer cell coordinates, values [N, 8] float64 corner
    values in corner order, c the iso-value.  Returns a dict with
    ``keys`` uint64 [T, 3] global edge ids (grid point linear index * 3 +
    axis, grid of (2^depth + 1)^3 points), ``pos`` float64 [T, 3, 3] vertex
    positions, ``cell`` int64 [T] the row of the cell that emitted each
    triangle.  Triangles are listed cell by cell in input order, in table
    order within a cell.
    """
    cell_ijk = np.asarray(cell_ijk, dtype=np.int64).reshape(-1, 3)
    values = np.asarray(values, dtype=np.float64).reshape(-1, 8)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    R1 = (1 << depth) + 1
    s = (hi - lo) / (1 << depth)
    table = case_table()
    cases = cell_cases(values, c)
    ntri = np.array([len(table[k]) for k in range(256)])[cases]
    T = int(ntri.sum())
    keys = np.zeros((T, 3), dtype=np.uint64)
    pos = np.zeros((T, 3, 3))
    cell = np.repeat(np.arange(cell_ijk.shape[0]), ntri)
    first = np.concatenate([[0], np.cumsum(ntri)[:-1]])
    for k in np.unique(cases):
        tris = table[k]
        if not tris:
            continue
        rows = np.nonzero(cases == k)[0]
        for t, tri in enumerate(tris):
            out = first[rows] + t
            for v, e in enumerate(tri):
                p, q = EDGES[e]
                ax = EDGE_AXIS[e]
                vp = values[rows, p]
                vq = values[rows, q]
                frac = (c - vp) / (vq - vp)
                g = cell_ijk[rows] + CORNERS[p][None, :]
                keys[out, v] = ((g[:, 0] + R1 * (g[:, 1] + R1 * g[:, 2])) * 3 + ax).astype(np.uint64)
                P = lo[None, :] + g * s[None, :]
                P[:, ax] += frac * s[ax]
                pos[out, v] = P
    return dict(keys=keys, pos=pos, cell=cell)


def corner_values(f, cell_ijk, depth, lo=(-1.0,) * 3, hi=(1.0,) * 3):
    """Evaluate ``f`` (points [M,3] -> [M]) at the 8 corners of each cell."""
    cell_ijk = np.asarray(cell_ijk, dtype=np.int64).reshape(-1, 3)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    s = (hi - lo) / (1 << depth)
    g = cell_ijk[:, None, :] + CORNERS[None, :, :]
    pts = lo[None, None, :] + g * s[None, None, :]
    return f(pts.reshape(-1, 3)).reshape(-1, 8)


def dense_grid(f, depth, lo=(-1.0,) * 3, hi=(1.0,) * 3):
    """Values of ``f`` on all (2^depth+1)^3 grid points, indexed [i, j, k]."""
    R1 = (1 << depth) + 1
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    ax = [lo[a] + np.arange(R1) * (hi[a] - lo[a]) / (1 << depth) for a in range(3)]
    X, Y, Z = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
    return f(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)).reshape(R1, R1, R1)


def dense_cells(grid):
    """All cells of a dense grid: (ijk [N,3], corner values [N,8])."""
    R = grid.shape[0] - 1
    i, j, k = np.meshgrid(np.arange(R), np.arange(R), np.arange(R), indexing="ij")
    ijk = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    vals = np.stack(
        [grid[ijk[:, 0] + dx, ijk[:, 1] + dy, ijk[:, 2] + dz] for dx, dy, dz in CORNERS], axis=1
    )
    return ijk, vals


def iso_voxels(values, c):
    """Cells the surface crosses (the paper's iso-voxels): case not 0/255."""
    cases = cell_cases(values, c)
    return (cases != 0) & (cases != 255)


def triangle_area(pos):
    a = pos[:, 1] - pos[:, 0]
    b = pos[:, 2] - pos[:, 0]
    return 0.5 * np.linalg.norm(np.cross(a, b), axis=1)
