"""Alg. 1 as printed -- its binary k-d tree with widest-dimension splits --
and the RA-UA read-off of Sec. IV-A (Eq. 5), on the GPU against the float64
oracle.

* RA-UA propagation: float32 within 1e-5 of max(|o|, S) on the bounds
  x0 -/+ t sigma (sigma within 1e-4 relative), float64 within 1e-10, BF16
  within the AA tolerance of the BF16 tests.
* k-d extraction: per node depth, the active node sets equal the oracle's
  except nodes that are, or descend from, a node whose oracle bound endpoint
  lies within 1e-4 S of an iso-value; the k-d leaves are a subset of the
  octree leaves (same tests at cube nodes, plus the half and quarter nodes).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.metrics import margin
from oracle.mlp import mlp_forward
from oracle.octree import extract_active_kd, kd_to_morton
from oracle.propagate import AA, RAUA, UP, propagate
from workloads import he_normal_mlp, random_boxes, uniform_points

from _parity import assert_pair_close, output_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2402_13861_amd as isx

    assert torch.cuda.is_available()
    c = isx.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _prop(ctx, mid, method, prec, c, h, kernel=0):
    import paper_2402_13861_amd as isx

    ctx.set_option(isx.HIDDEN_KERNEL, kernel)
    try:
        out = torch.full((c.shape[0], 2), float("nan"), dtype=torch.float32, device="cuda")
        out64 = torch.full((c.shape[0], 2), float("nan"), dtype=torch.float64, device="cuda") if prec == isx.FP64 \
            else None
        ctx.propagate(mid, method, prec, torch.from_numpy(c).cuda(), torch.from_numpy(h).cuda(), out, out64)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(isx.HIDDEN_KERNEL, 0)
    return out.cpu().numpy(), (out64.cpu().numpy() if out64 is not None else None)


@pytest.mark.parametrize("widths", [[3, 64, 64, 64, 1], [3, 48, 40, 1], [3, 256, 256, 256, 256, 256, 1]],
                         ids=lambda w: "x".join(map(str, w)))
def test_raua_propagation_matches_oracle(ctx, widths):
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp(widths, seed=4)
    S = output_scale(mlp)
    c, h, _ = random_boxes(150, range(0, 10), seed=12)
    ref = propagate(mlp, c, h, RAUA)
    mid = ctx.load_weights(mlp)
    try:
        for kern, kname in ((0, "mfma"), (1, "simt")):
            g, _ = _prop(ctx, mid, isx.RAUA, isx.FP32, c, h, kern)
            assert_pair_close(g, ref, S, 1e-5, f"raua fp32 {kname} {widths}", k=3.0)
            _, g64 = _prop(ctx, mid, isx.RAUA, isx.FP64, c, h, kern)
            assert_pair_close(g64, ref, S, 1e-10, f"raua fp64 {kname} {widths}", k=3.0)
        gb, _ = _prop(ctx, mid, isx.RAUA, isx.BF16, c, h)
        assert_pair_close(gb, ref, S, 2e-2, f"raua bf16 {widths}", k=3.0, spread_rtol=1.5e-2)
        # the centre is AA's centre (both through the vector-ALU read-off)
        ga, _ = _prop(ctx, mid, isx.AA, isx.FP32, c, h, 1)
        g, _ = _prop(ctx, mid, isx.RAUA, isx.FP32, c, h, 1)
        np.testing.assert_array_equal(g[:, 0], ga[:, 0])
    finally:
        ctx.unload_mlp(mid)


def _kd_unexcused(gpu_levels, oracle_levels, S, k, isos, band_rel=1e-4):
    """Per node depth, differences of the active node sets not excused by a
    borderline node (oracle margin <= band_rel S) at that depth or above."""
    close = []
    for lv in oracle_levels:
        m = margin(lv["centre"], lv["spread"], k, isos)
        close.append(set(lv["ids"][m <= band_rel * S].tolist()))
    bad = []
    for d, (g, o) in enumerate(zip(gpu_levels, oracle_levels)):
        g_ids, _, g_mask = g
        ga = set(g_ids[g_mask != 0].tolist())
        oa = set(o["ids"][o["mask"] != 0].tolist())
        for node in ga ^ oa:
            if not any((int(node) >> (d - e)) in close[e] for e in range(d + 1)):
                bad.append((d, int(node)))
    return bad


@pytest.mark.parametrize("mname", ["up", "aa", "raua"])
def test_kd_tree_extraction_matches_oracle(ctx, mname):
    """3->64x3->1 He-normal (seed 0), iso = median over 10^4 points, k-d tree
    to node depth 12 (octree depth 4); t = 3."""
    import paper_2402_13861_amd as isx

    method, gm = {"up": (UP, isx.UP), "aa": (AA, isx.AA), "raua": (RAUA, isx.RAUA)}[mname]
    mlp = he_normal_mlp([3, 64, 64, 64, 1], seed=0)
    vals = mlp_forward(mlp, uniform_points(10_000, seed=1))
    iso = [float(np.float32(np.median(vals)))]
    S = float(vals.std())
    D = 4
    mid = ctx.load_weights(mlp)
    try:
        ctx.set_isovalues(mid, iso)
        ctx.set_option(isx.KEEP_LEVELS, 1)
        mesh = ctx.extract(mid, gm, isx.FP32, k=3.0, max_depth=D, kd_tree=True)
        oct_mesh = ctx.extract(mid, gm, isx.FP32, k=3.0, max_depth=D)
        ctx.set_option(isx.KEEP_LEVELS, 0)
        assert mesh.n_levels == 3 * D + 1
        gl = [mesh.level_cells(d) for d in range(mesh.n_levels)]
        ol = extract_active_kd(mlp, method, iso, 3 * D, k=3.0)
        kk = 1.0 if mname == "aa" else 3.0
        bad = _kd_unexcused(gl, ol, S, kk, iso)
        print(f"k-d {mname}: active per depth gpu {[int((g[2] != 0).sum()) for g in gl]} "
              f"oracle {[int((o['mask'] != 0).sum()) for o in ol]}", flush=True)
        assert not bad, bad[:5]
        leaves, _ = mesh.leaves()
        o_leaves = kd_to_morton(ol[-1]["ids"][ol[-1]["mask"] != 0], D)
        oct_leaves, _ = oct_mesh.leaves()
        print(f"k-d leaves gpu {leaves.size} oracle {o_leaves.size}; octree leaves {oct_leaves.size}; "
              f"triangles k-d {mesh.n_tris} octree {oct_mesh.n_tris}", flush=True)
        assert set(leaves.tolist()) <= set(oct_leaves.tolist())
        assert mesh.n_tris > 0
        mesh.free()
        oct_mesh.free()
    finally:
        ctx.unload_mlp(mid)


def test_kd_tree_needs_a_cube_domain_and_no_surrogate(ctx):
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp([3, 32, 32, 1], seed=3)
    mid = ctx.load_weights(mlp)
    try:
        ctx.set_isovalues(mid, [0.0])
        ctx.set_domain(mid, (-1, -1, -1), (1, 1, 2))
        with pytest.raises(isx.IsxError) as e:
            ctx.extract(mid, isx.UP, isx.FP32, max_depth=3, kd_tree=True)
        assert e.value.status == -7
    finally:
        ctx.unload_mlp(mid)
