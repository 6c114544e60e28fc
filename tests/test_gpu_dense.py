"""GPU: the dense baseline (isx_extract_dense) -- the INR at every grid corner
and marching cubes on every cell -- against the oracle's brute-force dense
surface, and against the hierarchical extraction with sound (margin-widened)
affine arithmetic, which must keep every cell the surface crosses.

Tolerances: triangle sets (grid-edge keys per iso-value) exact; with the
same float32 corner evaluation on both sides, vertex positions bit-exact.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mc
from oracle.mlp import mlp_forward
from workloads import he_normal_mlp, uniform_points

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2402_13861_amd as isx

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = isx.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _isos(mlp, qs, seed=1):
    vals = mlp_forward(mlp, uniform_points(4000, seed=seed))
    return [float(np.float32(np.quantile(vals, q))) for q in qs]


def _tri_set(pos, keys, iso):
    """{(iso, sorted edge keys): vertex positions in key order}"""
    out = {}
    for p, k, i in zip(pos, keys, iso):
        order = np.argsort(k)
        out[(int(i),) + tuple(int(x) for x in k[order])] = p[order].tobytes()
    return out


def test_dense_equals_dense_oracle_fp64(ctx):
    """Float64 corner values: the same triangles (grid-edge keys) as the
    oracle's dense marching cubes, for two iso-values."""
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp([3, 32, 32, 1], seed=3)
    depth = 5
    isos = _isos(mlp, [0.3, 0.7])
    mid = ctx.load_weights(mlp)
    try:
        ctx.set_isovalues(mid, isos)
        mesh = ctx.extract_dense(mid, depth, isx.FP64)
        assert mesh.n_leaves == 8 ** depth
        assert mesh.n_corners == (2 ** depth + 1) ** 3
        assert mesh.n_levels == 0
        _, keys, iso = mesh.triangles()
        grid = mc.dense_grid(lambda p: mlp_forward(mlp, p), depth)
        ijk, cv = mc.dense_cells(grid)
        for q, c in enumerate(isos):
            act = mc.iso_voxels(cv, c)
            dense = mc.march(ijk[act], cv[act], c, depth)
            gk = sorted(tuple(sorted(map(int, t))) for t in keys[iso == q])
            dk = sorted(tuple(sorted(map(int, t))) for t in dense["keys"])
            assert gk == dk, q
    finally:
        ctx.unload_mlp(mid)


@pytest.mark.parametrize("widths,depth", [([3, 64, 64, 64, 1], 6), ([3, 256, 256, 1], 5)])
def test_dense_equals_sound_hierarchy_fp32(ctx, widths, depth):
    """Affine arithmetic with the rounding margin keeps every crossed cell,
    so its surface is the dense surface: the same triangles with the same
    float32 vertices (both evaluate the corners with the same kernel)."""
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp(widths, seed=5)
    isos = _isos(mlp, [0.25, 0.5, 0.75], seed=2)
    mid = ctx.load_weights(mlp)
    try:
        ctx.set_isovalues(mid, isos)
        ctx.set_option(isx.AA_MARGIN, 1)
        h = ctx.extract(mid, isx.AA, isx.FP32, k=1.0, max_depth=depth)
        ctx.set_option(isx.AA_MARGIN, 0)
        d = ctx.extract_dense(mid, depth, isx.FP32)
        assert d.n_tris == h.n_tris > 0
        assert _tri_set(*d.triangles()) == _tri_set(*h.triangles())
        # the hierarchy's leaves are a subset of the dense grid's cells
        hid, _ = h.leaves()
        did, dm = d.leaves()
        assert np.array_equal(did, np.arange(8 ** depth, dtype=np.uint32))
        assert np.all(dm == 7)
        assert np.all(np.diff(hid.astype(np.int64)) > 0) and hid[-1] < 8 ** depth
    finally:
        ctx.set_option(isx.AA_MARGIN, 0)
        ctx.unload_mlp(mid)


def test_dense_errors(ctx):
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp([3, 32, 32, 1], seed=3)
    mid = ctx.load_weights(mlp)
    try:
        with pytest.raises(isx.IsxError) as e:
            ctx.extract_dense(mid, 4, isx.FP32)  # no iso-values yet
        assert e.value.status == -1
        ctx.set_isovalues(mid, [0.0])
        with pytest.raises(isx.IsxError) as e:
            ctx.extract_dense(mid, 10, isx.FP32)  # 2^30 cells
        assert e.value.status == -4
        with pytest.raises(isx.IsxError) as e:
            ctx.extract_dense(mid, 11, isx.FP32)
        assert e.value.status == -1
        with pytest.raises(isx.IsxError) as e:
            ctx.extract_dense(mid, 4, 7)
        assert e.value.status == -1
        m0 = ctx.extract_dense(mid, 0, isx.FP32)
        assert m0.n_leaves == 1 and m0.n_corners == 8
    finally:
        ctx.unload_mlp(mid)


@pytest.mark.parametrize("level", [3, 4])
def test_dense_from_level_contains_full_refinement(ctx, level):
    """Range analysis down to `level`, dense subtrees below: the levels down
    to `level` are those of the full refinement, the leaves are every cell
    below its active level-`level` cells, and the surface contains the full
    refinement's surface, vertex for vertex."""
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp([3, 64, 64, 64, 1], seed=7)
    depth = 6
    isos = _isos(mlp, [0.3, 0.6], seed=4)
    mid = ctx.load_weights(mlp)
    try:
        ctx.set_isovalues(mid, isos)
        full = ctx.extract(mid, isx.UP, isx.FP32, k=3.0, max_depth=depth)
        ctx.set_option(isx.DENSE_FROM_LEVEL, level)
        hyb = ctx.extract(mid, isx.UP, isx.FP32, k=3.0, max_depth=depth)
        ctx.set_option(isx.DENSE_FROM_LEVEL, 0)
        fl, hl = full.levels(), hyb.levels()
        assert len(hl) == level + 1
        assert [(x["cells"], x["active"]) for x in hl] == [(x["cells"], x["active"]) for x in fl[:level + 1]]
        assert hyb.n_leaves == hl[level]["active"] * 8 ** (depth - level)
        ids, masks = hyb.leaves()
        assert np.all(np.diff(ids.astype(np.int64)) > 0)
        fids, fmasks = full.leaves()
        pos = np.minimum(np.searchsorted(ids, fids), ids.size - 1)
        assert np.array_equal(ids[pos], fids)
        assert np.all((fmasks & ~masks[pos]) == 0)  # a leaf's isos are its ancestor's
        ht, ft = _tri_set(*hyb.triangles()), _tri_set(*full.triangles())
        assert ft.items() <= ht.items()
        assert hyb.n_tris >= full.n_tris > 0
    finally:
        ctx.set_option(isx.DENSE_FROM_LEVEL, 0)
        ctx.unload_mlp(mid)


def test_dense_from_level_sound_aa_is_dense(ctx):
    """With sound affine arithmetic above the dense level, the surface is the
    dense baseline's."""
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp([3, 64, 64, 64, 1], seed=5)
    depth = 6
    isos = _isos(mlp, [0.25, 0.5, 0.75], seed=2)
    mid = ctx.load_weights(mlp)
    try:
        ctx.set_isovalues(mid, isos)
        ctx.set_option(isx.AA_MARGIN, 1)
        ctx.set_option(isx.DENSE_FROM_LEVEL, 3)
        h = ctx.extract(mid, isx.AA, isx.FP32, k=1.0, max_depth=depth)
        ctx.set_option(isx.DENSE_FROM_LEVEL, 0)
        ctx.set_option(isx.AA_MARGIN, 0)
        d = ctx.extract_dense(mid, depth, isx.FP32)
        assert _tri_set(*h.triangles()) == _tri_set(*d.triangles())
    finally:
        ctx.set_option(isx.DENSE_FROM_LEVEL, 0)
        ctx.set_option(isx.AA_MARGIN, 0)
        ctx.unload_mlp(mid)


def test_dense_from_level_edges(ctx):
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp([3, 32, 32, 1], seed=3)
    mid = ctx.load_weights(mlp)
    try:
        ctx.set_isovalues(mid, [0.0])
        with pytest.raises(isx.IsxError) as e:
            ctx.set_option(isx.DENSE_FROM_LEVEL, 11)
        assert e.value.status == -1
        full = ctx.extract(mid, isx.UP, isx.FP32, k=3.0, max_depth=4)
        ctx.set_option(isx.DENSE_FROM_LEVEL, 4)  # not above max_depth: the full refinement
        same = ctx.extract(mid, isx.UP, isx.FP32, k=3.0, max_depth=4)
        assert same.n_levels == full.n_levels and same.n_leaves == full.n_leaves
        assert _tri_set(*same.triangles()) == _tri_set(*full.triangles())
        ctx.set_option(isx.DENSE_FROM_LEVEL, 2)
        with pytest.raises(isx.IsxError) as e:
            ctx.extract(mid, isx.UP, isx.FP32, k=3.0, max_depth=4, kd_tree=True)
        assert e.value.status == -7
    finally:
        ctx.set_option(isx.DENSE_FROM_LEVEL, 0)
        ctx.unload_mlp(mid)


def test_every_option_takes_its_default(ctx):
    """isx_set_option accepts every documented option at its default value."""
    import paper_2402_13861_amd as isx

    defaults = [(isx.KEEP_LEVELS, 0), (isx.HIDDEN_KERNEL, 0), (isx.PROFILE, 0), (isx.SCRATCH_BYTES, 16 << 30),
                (isx.VERBOSE, 0), (isx.BF16_VARIANT, 0), (isx.UP_FORM, 0), (isx.LIN_PRECISION, 1),
                (isx.AA_MARGIN, 0), (isx.BATCH_WORKERS, 4), (isx.CANCEL_CHECK, 1), (isx.AUTOTUNE, 0),
                (isx.BF16_READOFF, 0), (isx.RECHECK_CASCADE, 0), (isx.DENSE_FROM_LEVEL, 0),
                (isx.RECHECK_SPLIT, 0)]
    assert sorted(o for o, _ in defaults) == list(range(1, 17))
    for opt, val in defaults:
        ctx.set_option(opt, val)
    ctx.set_option(isx.RECHECK_CASCADE, 1)
    ctx.set_option(isx.RECHECK_CASCADE, 0)
    with pytest.raises(isx.IsxError) as e:
        ctx.set_option(99, 0)
    assert e.value.status == -1


@pytest.mark.parametrize("prec_name,n", [("fp32", (1 << 26) + 1000), ("fp64", (1 << 25) + 1000)])
def test_eval_points_past_one_launch(ctx, prec_name, n):
    """More points than one launch of the vector-ALU evaluation takes (a
    launch stays below 2^32 work-items: 2^26 points in float32, 2^25 in
    float64 for a 256-wide net): points on both sides of every split and at
    the ends match the oracle (a sine net takes the vector-ALU kernel)."""
    import paper_2402_13861_amd as isx
    from workloads.weights import siren_mlp

    mlp = siren_mlp([3, 256, 256, 1], 5, 6.0)
    prec = {"fp32": isx.FP32, "fp64": isx.FP64}[prec_name]
    per = 1 << (26 if prec_name == "fp32" else 25)
    mid = ctx.load_weights(mlp)
    try:
        ctx.set_activation(mid, isx.SINE)
        g = torch.Generator(device="cuda").manual_seed(3)
        pts = torch.rand((n, 3), device="cuda", generator=g) * 2 - 1
        vals = torch.full((n,), float("nan"), device="cuda")
        ctx.eval_points(mid, prec, pts, vals)
        torch.cuda.synchronize()
        pick = np.concatenate([np.arange(0, 300), np.arange(per - 300, per + 300), np.arange(n - 300, n)])
        p = pts[torch.from_numpy(pick).cuda()].double().cpu().numpy()
        ref = mlp_forward(mlp, p, act="sine")
        got = vals[torch.from_numpy(pick).cuda()].double().cpu().numpy()
        S = float(np.std(mlp_forward(mlp, uniform_points(4000, seed=1), act="sine")))
        err = np.abs(got - ref) / np.maximum(np.abs(ref), S)
        assert np.all(np.isfinite(got)) and err.max() <= (1e-5 if prec_name == "fp32" else 1e-7), err.max()
    finally:
        ctx.unload_mlp(mid)
