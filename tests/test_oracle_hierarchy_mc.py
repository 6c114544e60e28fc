"""Pins for the oracle's octree search (Alg. 1) and marching cubes.

* Morton ids: round trip and child order.
* Alg. 1's test keeps a node whose bound touches the iso-value.
* Monotone in t: a larger t never drops a cell.
* AA is sound, so its hierarchical leaves contain every dense iso-voxel and
  its leaf surface equals the brute-force dense surface exactly.
* For the plane x+y+z+d, UP with t = 3 predicts the exact active set
  (3 * ||h||_2 / sqrt3 * sqrt3 = the exact range 3h of x+y+z over a cube).
* The generated case table uses exactly the sign-change edges, once each.
* The exact ReLU octahedron |x|+|y|+|z| = r: MC on a grid that contains the
  kink planes reproduces the surface exactly (area 4 sqrt3 r^2), watertight,
  with outward normals.
"""

import numpy as np
import pytest

from oracle import mc
from oracle.mlp import mlp_forward
from oracle.metrics import fpr_fnr, set_recall
from oracle.octree import cell_boxes, classify, extract_active, morton_decode, morton_encode
from oracle.propagate import AA, UP
from oracle.propagate import propagate
from workloads import he_normal_mlp, uniform_points


def test_morton_roundtrip_and_children():
    rng = np.random.default_rng(0)
    i, j, k = rng.integers(0, 1024, (3, 1000))
    code = morton_encode(i, j, k)
    i2, j2, k2 = morton_decode(code)
    np.testing.assert_array_equal(i, i2)
    np.testing.assert_array_equal(j, j2)
    np.testing.assert_array_equal(k, k2)
    # children of (i,j,k) are (2i+dx, 2j+dy, 2k+dz) with child index dz<<2|dy<<1|dx
    p = morton_encode(5, 9, 3)
    for c in range(8):
        ci, cj, ck = morton_decode(np.uint64(p) * np.uint64(8) + np.uint64(c))
        assert (ci, cj, ck) == (10 + (c & 1), 18 + ((c >> 1) & 1), 6 + ((c >> 2) & 1))


def test_cell_boxes_level_geometry():
    c, h = cell_boxes(2, morton_encode(np.array([0, 3]), np.array([0, 1]), np.array([0, 2])))
    np.testing.assert_array_equal(c, [[-0.75, -0.75, -0.75], [0.75, -0.25, 0.25]])
    np.testing.assert_array_equal(h, 0.25)


def test_classify_closed_interval():
    # Alg. 1 drops a node only if mu + t sigma < c or mu - t sigma > c
    centre = np.array([0.0, 0.0, 0.0, 0.0])
    spread = np.array([1.0, 1.0, 1.0, 1.0])
    m = classify(centre, spread, 2.0, [2.0, -2.0, 2.0 + 1e-12, -3.0], 0b1111)
    assert m[0] == 0b0011  # touching either end keeps the iso bit


def _net():
    return he_normal_mlp([3, 24, 24, 1], seed=3)


@pytest.mark.parametrize("depth", [4, 5])
def test_aa_hierarchy_equals_dense_surface(depth):
    mlp = _net()
    iso = float(np.median(mlp_forward(mlp, np.random.default_rng(1).uniform(-1, 1, (4000, 3)))))
    levels = extract_active(mlp, AA, [iso], depth)
    leaves = levels[-1]["ids"][levels[-1]["mask"] != 0]
    grid = mc.dense_grid(lambda p: mlp_forward(mlp, p), depth)
    ijk_all, vals_all = mc.dense_cells(grid)
    truth = mc.iso_voxels(vals_all, iso)
    true_ids = morton_encode(*ijk_all[truth].T)
    assert set_recall(leaves, true_ids) == 1.0
    # surface from AA leaves == dense surface (same triangles, same vertices)
    li, lj, lk = morton_decode(leaves)
    lijk = np.stack([li, lj, lk], 1)
    lv = mc.corner_values(lambda p: mlp_forward(mlp, p), lijk, depth)
    hier = mc.march(lijk, lv, iso, depth)
    dense = mc.march(ijk_all[truth], vals_all[truth], iso, depth)
    hk = {tuple(sorted(t)) for t in map(tuple, hier["keys"])}
    dk = {tuple(sorted(t)) for t in map(tuple, dense["keys"])}
    assert hk == dk
    assert hier["keys"].shape[0] == dense["keys"].shape[0]
    np.testing.assert_allclose(mc.triangle_area(hier["pos"]).sum(), mc.triangle_area(dense["pos"]).sum(), rtol=1e-12)


def test_monotone_in_t():
    mlp = _net()
    isos = [-0.2, 0.3]
    prev = None
    for t in (1.0, 2.0, 3.0, 5.0):
        lv = extract_active(mlp, UP, isos, 4, k=t)
        active = [set(l["ids"][l["mask"] != 0].tolist()) for l in lv]
        if prev is not None:
            for a, b in zip(prev, active):
                assert a <= b
        prev = active


def test_plane_up_t3_is_exact():
    # f(x) = x + y + z + d written as a 3 -> 1 -> 1 ReLU net that is affine on the domain
    d = 0.123
    layers = [(np.array([[1.0, 1.0, 1.0]]), np.array([10.0])), (np.array([[1.0]]), np.array([d - 10.0]))]
    depth = 5
    lv = extract_active(layers, UP, [0.0], depth, k=3.0)
    got = set(lv[-1]["ids"][lv[-1]["mask"] != 0].tolist())
    # exact active set: cells whose closed range of x+y+z+d contains 0
    R = 1 << depth
    i, j, k = np.meshgrid(np.arange(R), np.arange(R), np.arange(R), indexing="ij")
    s = 2.0 / R
    low = -3.0 + (i + j + k) * s + d
    high = low + 3 * s
    want = morton_encode(i[(low <= 0) & (high >= 0)], j[(low <= 0) & (high >= 0)], k[(low <= 0) & (high >= 0)])
    assert got == set(want.tolist())


def test_case_table_uses_each_crossed_edge_once():
    table = mc.case_table()
    for case in range(256):
        inside = [(case >> c) & 1 for c in range(8)]
        crossed = {e for e, (p, q) in enumerate(mc.EDGES) if inside[p] != inside[q]}
        used = [e for tri in table[case] for e in tri]
        assert set(used) == crossed
        # fan triangulation of closed polygons: vertex count = sum over cycles
        # of (len - 2) triangles; every crossed edge lies on exactly one cycle
        assert len(table[case]) == len(crossed) - 2 * _n_cycles(table[case])


def _n_cycles(tris):
    # cycles are fanned from their first vertex: a new cycle starts at a new apex
    return len({t[0] for t in tris})


def _octahedron_net(r):
    # |x| + |y| + |z| - r = sum relu(+-x_i) - r : exact 3 -> 6 -> 1 ReLU net
    W1 = np.concatenate([np.eye(3), -np.eye(3)])
    return [(W1, np.zeros(6)), (np.ones((1, 6)), np.array([-r]))]


@pytest.mark.parametrize("depth,r", [(4, 0.7), (5, 0.55)])
def test_octahedron_area_watertight_and_oriented(depth, r):
    layers = _octahedron_net(r)
    f = lambda p: mlp_forward(layers, p)
    grid = mc.dense_grid(f, depth)
    ijk, vals = mc.dense_cells(grid)
    out = mc.march(ijk, vals, 0.0, depth)
    # exact area of the octahedron: 8 equilateral faces of side r sqrt2
    assert mc.triangle_area(out["pos"]).sum() == pytest.approx(4 * np.sqrt(3) * r * r, rel=1e-12)
    # vertices lie on the surface
    np.testing.assert_allclose(np.abs(out["pos"]).sum(-1), r, atol=1e-12)
    # watertight and consistently oriented: each directed edge appears once,
    # and its reverse appears once
    directed = {}
    for t in out["keys"]:
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            directed[(a, b)] = directed.get((a, b), 0) + 1
    assert all(v == 1 for v in directed.values())
    assert all((b, a) in directed for (a, b) in directed)
    # outward normals (toward increasing f), checked on non-degenerate triangles
    p = out["pos"]
    n = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    cen = p.mean(1)
    big = np.linalg.norm(n, axis=1) > 1e-12
    assert np.all((n[big] * np.sign(cen[big])).sum(1) > 0)


def test_dense_plane_vertices_exact():
    d = 0.123
    layers = [(np.array([[1.0, 1.0, 1.0]]), np.array([10.0])), (np.array([[1.0]]), np.array([d - 10.0]))]
    grid = mc.dense_grid(lambda p: mlp_forward(layers, p), 3)
    ijk, vals = mc.dense_cells(grid)
    out = mc.march(ijk, vals, 0.0, 3)
    np.testing.assert_allclose(out["pos"].sum(-1), -d, atol=1e-12)


def test_fpr_fnr_hand_counted():
    pred = np.array([1, 1, 0, 0, 1, 0, 1], dtype=bool)
    true = np.array([1, 0, 1, 0, 1, 0, 0], dtype=bool)
    # TP=2, FP=2, FN=1, TN=2
    fpr, fnr = fpr_fnr(pred, true)
    assert fpr == pytest.approx(2 / 4)
    assert fnr == pytest.approx(1 / 3)


def _kd_recursive(layers, method, iso, depth, k, c, h, node, d, out):
    """Alg. 1 as printed: depth-first recursion on one node."""
    from oracle.octree import kd_split, widest_axis

    cen, spr = propagate(layers, c[None, :], h[None, :], method)
    kk = 1.0 if method == AA else k
    if not (cen[0] - kk * spr[0] <= iso <= cen[0] + kk * spr[0]):
        return
    if d == depth:
        out.add(int(node))
        return
    lower, upper = kd_split(c, h, widest_axis(h))
    _kd_recursive(layers, method, iso, depth, k, *lower, 2 * node, d + 1, out)
    _kd_recursive(layers, method, iso, depth, k, *upper, 2 * node + 1, d + 1, out)


@pytest.mark.parametrize("method", [AA, UP])
def test_kd_tree_breadth_first_equals_recursion(method):
    """The level-by-level k-d search equals the depth-first recursion of
    Alg. 1 on a tiny net (every node's decision depends on its box only)."""
    from oracle.octree import extract_active_kd

    mlp = he_normal_mlp([3, 16, 16, 1], seed=2)
    iso = float(np.median(mlp_forward(mlp, uniform_points(2000, seed=1))))
    lv = extract_active_kd(mlp, method, [iso], 6, k=3.0)
    bfs = set(lv[-1]["ids"][lv[-1]["mask"] != 0].tolist())
    rec = set()
    _kd_recursive(mlp, method, iso, 6, 3.0, np.zeros(3), np.ones(3), 0, 0, rec)
    assert bfs == rec and len(bfs) > 0


def test_kd_tree_splits_cycle_and_leaves_are_octree_cells():
    """On a cube the widest-dimension rule with ties x, y, z splits x, y, z in
    turn; depth 3D nodes are the octree cells of level D (k-d id -> Morton)."""
    from oracle.octree import cell_boxes, extract_active_kd, kd_to_morton, widest_axis

    assert widest_axis([1.0, 1.0, 1.0]) == 0
    assert widest_axis([0.5, 1.0, 1.0]) == 1
    assert widest_axis([0.5, 0.5, 1.0]) == 2
    layers = [(np.eye(3)[:1] * 0.0, np.array([0.0])), (np.array([[1.0]]), np.array([0.0]))]  # constant 0: all active
    lv = extract_active_kd(layers, AA, [0.0], 6)
    ids = lv[6]["ids"]
    assert ids.size == 64
    c_oct, h_oct = cell_boxes(2, kd_to_morton(ids, 2))
    np.testing.assert_allclose(lv[6]["centre_box"], c_oct)
    np.testing.assert_allclose(lv[6]["half"], h_oct)


@pytest.mark.parametrize("method", [AA, UP])
def test_kd_leaves_within_octree_leaves_and_aa_covers_dense(method):
    """Cube nodes of the k-d tree have the octree cells' boxes, so they get
    the same test; a k-d leaf also needs its half and quarter ancestors, so
    the k-d leaves at depth 3D are a subset of the octree leaves at D.  For
    AA (sound), both contain the dense grid's iso-voxels."""
    from oracle.octree import extract_active_kd, kd_to_morton

    mlp = he_normal_mlp([3, 32, 32, 1], seed=3)
    iso = float(np.median(mlp_forward(mlp, uniform_points(4000, seed=1))))
    D = 4
    kd = extract_active_kd(mlp, method, [iso], 3 * D, k=3.0)
    oc = extract_active(mlp, method, [iso], D, k=3.0)
    kd_leaves = set(kd_to_morton(kd[-1]["ids"][kd[-1]["mask"] != 0], D).tolist())
    oc_leaves = set(oc[-1]["ids"][oc[-1]["mask"] != 0].tolist())
    assert kd_leaves <= oc_leaves
    if method == AA:
        grid = mc.dense_grid(lambda p: mlp_forward(mlp, p), D)
        ijk, cv = mc.dense_cells(grid)
        act = mc.iso_voxels(cv, iso)
        dense = set(morton_encode(ijk[act, 0], ijk[act, 1], ijk[act, 2]).tolist())
        assert dense <= kd_leaves
