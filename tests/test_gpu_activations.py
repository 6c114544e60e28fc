"""Sine (SIREN) and ELU networks (App. D table, Sine and ELU rows) on the
GPU against the float64 oracle.

* Propagation, UP / AA / RA-UA: float32 (FP32-MFMA and vector-ALU kernels)
  within 1e-5 of max(|o|, S) on the bounds (spread 1e-4 relative), float64
  within 1e-10, on dyadic cells of levels 0..9.
* Point evaluation: float32 within 1e-5 of max(|f|, S), float64 1e-12.
* Extraction (UP, t = 3, octree depth 5): per-level active sets equal the
  oracle's except borderline cells (oracle margin <= 1e-4 S, or an ancestor
  with one).
* BF16 propagation (covariance form and coefficient form for UP, the
  coefficient form for AA): bounds, spread and centre within the BF16
  tolerances below, relative to max(|o|, S); with a float64 re-check band
  wider than that error, BF16 extraction reproduces the oracle's active
  sets except cells within 1e-9 S of an iso-value.
* Paths written for ReLU only report ISX_EUNSUPPORTED.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.mlp import mlp_forward
from oracle.octree import extract_active
from oracle.propagate import AA, RAUA, UP, propagate
from workloads import he_normal_mlp, random_boxes, uniform_points
from workloads.weights import MLPWeights

from _parity import assert_pair_close, close_sets, unexcused_level_diffs

pytestmark = pytest.mark.gpu


def siren(widths, seed, w0=3.0):
    """Sine net in the SIREN layout, w0 folded into the first layer."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for li, (i, o) in enumerate(zip(widths[:-1], widths[1:])):
        lim = w0 / i if li == 0 else np.sqrt(6.0 / i)
        Ws.append(rng.uniform(-lim, lim, (o, i)).astype(np.float32))
        bs.append(rng.uniform(-lim, lim, o).astype(np.float32))
    return MLPWeights(Ws=Ws, bs=bs)


NETS = {
    "sine-64x3": ("sine", lambda: siren([3, 64, 64, 64, 1], 1, w0=6.0)),
    "sine-128x4": ("sine", lambda: siren([3, 128, 128, 128, 128, 1], 2, w0=3.0)),
    "elu-64x3": ("elu", lambda: he_normal_mlp([3, 64, 64, 64, 1], seed=3)),
    "elu-48x40": ("elu", lambda: he_normal_mlp([3, 48, 40, 1], seed=4)),
}


@pytest.fixture(scope="module")
def ctx():
    import paper_2402_13861_amd as isx

    assert torch.cuda.is_available()
    c = isx.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _load(ctx, name):
    import paper_2402_13861_amd as isx

    act, make = NETS[name]
    mlp = make()
    mid = ctx.load_weights(mlp)
    ctx.set_activation(mid, {"sine": isx.SINE, "elu": isx.ELU}[act])
    return act, mlp, mid


def _scale(mlp, act):
    return float(np.std(mlp_forward(mlp, uniform_points(10_000, 1), act=act)))


def _prop(ctx, mid, method, prec, c, h, kernel=0):
    import paper_2402_13861_amd as isx

    ctx.set_option(isx.HIDDEN_KERNEL, kernel)
    try:
        out = torch.full((c.shape[0], 2), float("nan"), dtype=torch.float32, device="cuda")
        out64 = torch.full((c.shape[0], 2), float("nan"), dtype=torch.float64, device="cuda") \
            if prec == isx.FP64 else None
        ctx.propagate(mid, method, prec, torch.from_numpy(c).cuda(), torch.from_numpy(h).cuda(), out, out64)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(isx.HIDDEN_KERNEL, 0)
    return out.cpu().numpy(), (out64.cpu().numpy() if out64 is not None else None)


@pytest.mark.parametrize("name", list(NETS))
@pytest.mark.parametrize("mname", ["up", "aa", "raua"])
def test_propagation_matches_oracle(ctx, name, mname):
    import paper_2402_13861_amd as isx

    method, gm, k = {"up": (UP, isx.UP, 3.0), "aa": (AA, isx.AA, 1.0), "raua": (RAUA, isx.RAUA, 3.0)}[mname]
    act, mlp, mid = _load(ctx, name)
    try:
        S = _scale(mlp, act)
        c, h, _ = random_boxes(200, range(0, 10), seed=31)
        ref = propagate(mlp, c, h, method, act=act)
        for kern, kname in ((0, "mfma"), (1, "simt")):
            g32, _ = _prop(ctx, mid, gm, isx.FP32, c, h, kern)
            assert_pair_close(g32, ref, S, 1e-5, f"{name} {mname} fp32 {kname}", k=k)
            _, g64 = _prop(ctx, mid, gm, isx.FP64, c, h, kern)
            assert_pair_close(g64, ref, S, 1e-10, f"{name} {mname} fp64 {kname}", k=k)
    finally:
        ctx.unload_mlp(mid)


@pytest.mark.parametrize("name", ["sine-64x3", "elu-64x3"])
def test_point_evaluation_matches_oracle(ctx, name):
    import paper_2402_13861_amd as isx

    act, mlp, mid = _load(ctx, name)
    try:
        x = uniform_points(4099, seed=5).astype(np.float32)
        ref = mlp_forward(mlp, x.astype(np.float64), act=act)
        S = float(ref.std())
        for prec, tol in ((isx.FP32, 1e-5), (isx.FP64, 1e-7)):
            v = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
            ctx.eval_points(mid, prec, torch.from_numpy(x).cuda(), v)
            torch.cuda.synchronize()
            err = np.abs(v.cpu().numpy() - ref) / np.maximum(np.abs(ref), S)
            print(f"{name} eval precision {prec}: max rel err {err.max():.3e}", flush=True)
            assert err.max() <= tol
    finally:
        ctx.unload_mlp(mid)


@pytest.mark.parametrize("name", ["sine-64x3", "elu-64x3"])
def test_extraction_matches_oracle(ctx, name):
    import paper_2402_13861_amd as isx

    act, mlp, mid = _load(ctx, name)
    try:
        vals = mlp_forward(mlp, uniform_points(10_000, seed=1), act=act)
        iso = [float(np.float32(np.median(vals)))]
        S = float(vals.std())
        ctx.set_isovalues(mid, iso)
        ctx.set_option(isx.KEEP_LEVELS, 1)
        mesh = ctx.extract(mid, isx.UP, isx.FP32, k=3.0, max_depth=5)
        ctx.set_option(isx.KEEP_LEVELS, 0)
        gl = [mesh.level_cells(L) for L in range(mesh.n_levels)]
        ol = extract_active(mlp, UP, iso, 5, k=3.0, act=act)
        bad = unexcused_level_diffs(gl, ol, close_sets(ol, UP, 3.0, iso, S))
        print(f"{name}: active per level gpu {[l['active'] for l in mesh.levels()]} oracle "
              f"{[int((l['mask'] != 0).sum()) for l in ol]}; triangles {mesh.n_tris}", flush=True)
        assert not bad, bad
        assert mesh.n_tris > 0
        mesh.free()
    finally:
        ctx.unload_mlp(mid)


# BF16 tolerances relative to max(|o|, S): (bounds, spread, centre), about
# twice the largest error measured over NETS on the device (UP, both forms:
# bounds 1.55e-3, spread 5.7e-4, centre 9.3e-4; AA: bounds 1.50e-3, spread
# 1.0e-3, centre 1.47e-3)
BF16_TOL = {"up": (3e-3, 1.2e-3, 2e-3), "aa": (3e-3, 2e-3, 3e-3)}


@pytest.mark.parametrize("name", list(NETS))
@pytest.mark.parametrize("mname", ["up", "aa"])
def test_bf16_propagation_error_against_oracle(ctx, name, mname):
    """BF16 operands, FP32 accumulation, the activation's rule in float64:
    the bound error against the FP64 oracle, reported and bounded."""
    import paper_2402_13861_amd as isx

    method, gm, k = {"up": (UP, isx.UP, 3.0), "aa": (AA, isx.AA, 1.0)}[mname]
    act, mlp, mid = _load(ctx, name)
    try:
        S = _scale(mlp, act)
        c, h, _ = random_boxes(257, range(0, 10), seed=11)
        ref = propagate(mlp, c, h, method, act=act)
        tol, stol, ctol = BF16_TOL[mname]
        for form in ((0, 1) if mname == "up" else (0,)):
            ctx.set_option(isx.UP_FORM, form)
            g, _ = _prop(ctx, mid, gm, isx.BF16, c, h)
            worst, _ = assert_pair_close(g, ref, S, tol, f"bf16 {name} {mname} form {form}", k=k, spread_rtol=stol)
            assert worst["centre"] <= ctol
    finally:
        ctx.set_option(isx.UP_FORM, 0)
        ctx.unload_mlp(mid)


@pytest.mark.parametrize("name", ["sine-64x3", "elu-64x3"])
def test_bf16_extraction_with_band_matches_oracle(ctx, name):
    """BF16 UP extraction with a float64 re-check band wider than the BF16
    bound error: every classification is decided as in float64."""
    import paper_2402_13861_amd as isx

    act, mlp, mid = _load(ctx, name)
    try:
        vals = mlp_forward(mlp, uniform_points(10_000, seed=1), act=act)
        isos = [float(np.float32(np.quantile(vals, q))) for q in (0.3, 0.6)]
        S = float(vals.std())
        ctx.set_isovalues(mid, isos)
        ctx.set_option(isx.KEEP_LEVELS, 1)
        mesh = ctx.extract(mid, isx.UP, isx.BF16, k=3.0, max_depth=5, fp64_band=5e-2 * S)
        ctx.set_option(isx.KEEP_LEVELS, 0)
        assert sum(l["rechecked"] for l in mesh.levels()) > 0
        ol = extract_active(mlp, UP, isos, 5, k=3.0, act=act)
        close = close_sets(ol, UP, 3.0, isos, S, band_rel=1e-9)
        bad = unexcused_level_diffs([mesh.level_cells(L) for L in range(mesh.n_levels)], ol, close)
        assert not bad, bad
    finally:
        ctx.set_option(isx.KEEP_LEVELS, 0)
        ctx.unload_mlp(mid)


def test_relu_only_paths_report_unsupported(ctx):
    import paper_2402_13861_amd as isx

    act, mlp, mid = _load(ctx, "sine-64x3")
    try:
        c, h, _ = random_boxes(4, [3], seed=1)
        out = torch.empty((4, 2), device="cuda")
        with pytest.raises(isx.IsxError) as e:
            ctx.linearize(mid, torch.from_numpy(c).cuda(), torch.from_numpy(h).cuda(), out)
        assert e.value.status == -7
        ctx.set_option(isx.AA_MARGIN, 1)
        with pytest.raises(isx.IsxError) as e:
            _prop(ctx, mid, isx.AA, isx.FP32, c, h)
        assert e.value.status == -7
    finally:
        ctx.set_option(isx.AA_MARGIN, 0)
        ctx.unload_mlp(mid)


@pytest.mark.parametrize("name", ["sine-64x3", "sine-128x4", "elu-64x3"])
def test_split_fp32_products_against_oracle(ctx, name):
    """Float32 UP with its products as split bf16 MFMAs (ISX_HIDDEN_KERNEL 3,
    the re-check cascade's first stage) on sine and ELU nets: bounds within
    1e-5 of max(|o|, S) and spread within 1e-4 relative, the float32 MFMA
    path's tolerances (measured: bounds 3.4e-6, spread 2.6e-6 at most)."""
    import paper_2402_13861_amd as isx

    act, mlp, mid = _load(ctx, name)
    try:
        S = _scale(mlp, act)
        c, h, _ = random_boxes(257, range(0, 10), seed=17)
        ref = propagate(mlp, c, h, UP, act=act)
        g, _ = _prop(ctx, mid, isx.UP, isx.FP32, c, h, kernel=3)
        assert_pair_close(g, ref, S, 1e-5, f"split fp32 {name}", k=3.0, spread_rtol=1e-4)
    finally:
        ctx.unload_mlp(mid)
