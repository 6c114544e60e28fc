"""GPU parity at the benchmark's network shape, against the float64 oracle.

Nets: the 3->256x5->1 ReLU INR fitted to the synthetic Fourier field (the
benchmark's INR) and a He-normal 3->256x5->1 (seed 0).  Checked here:
* float32 (MFMA and vector-ALU kernels) and float64 propagation, both
  methods, at 1e-5 / 1e-10 of max(|o|, S) on the bounds (spread: 1e-4 / 1e-9
  relative), on dyadic cells of every octree level 0..9;
* the BF16 paths' bound error against the oracle per octree level, in units
  of S, with the float64 re-check band shown to exceed it where the band is
  meant to protect the classification (levels >= 6);
* extraction at depth 7 with the three iso-values: the float32 + band and
  the BF16 + band leaf sets against the float64 extraction (the plain-UP set
  the recall target refers to); with the band widened per cell by 2^-6 of
  its sigma, the BF16 sets equal the float64 sets exactly.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.propagate import AA, UP, propagate
from workloads import he_normal_mlp, random_boxes

from _parity import assert_pair_close, output_scale

pytestmark = pytest.mark.gpu

METHODS = {"up": (UP, 1), "aa": (AA, 0)}
INR = "relu256x5_fourier"

# Largest BF16 endpoint error against the oracle over levels 0..9 of the
# 3->256x5->1 INR, about twice the largest value measured on the device:
# UP in units of S (covariance form 4.2e-3, coefficient form 1.14e-2, both at
# levels 0-2); AA relative to max(|endpoint|, S), since its ranges at the top
# levels are hundreds of S wide.
BF16_ENDPOINT_TOL = {"up-cov": 8e-3, "up-coef": 2.5e-2, "aa": 1e-2}
BAND_REL = 1e-3  # the float64 re-check band of the benchmark, in units of S
# its per-cell widening by a multiple of the cell's spread (isx_params.fp64_band_rel): the BF16 endpoint error
# measured on the device, in units of the oracle's sigma of the cell, peaks near 8e-3 at levels 3-5
BAND_REL_SPREAD = 2.0 ** -6


@pytest.fixture(scope="module")
def ctx():
    import paper_2402_13861_amd as isx

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = isx.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _net(name):
    from workloads.configs import load_mlp

    if name == "fourier-inr":
        return load_mlp(INR)
    return he_normal_mlp([3, 256, 256, 256, 256, 256, 1], seed=0)


def _gpu_prop(ctx, mid, method, precision, c, h, kernel=0, form=0):
    import paper_2402_13861_amd as isx

    ctx.set_option(isx.HIDDEN_KERNEL, kernel)
    ctx.set_option(isx.UP_FORM, form)
    n = c.shape[0]
    out = torch.full((n, 2), float("nan"), dtype=torch.float32, device="cuda")
    out64 = torch.full((n, 2), float("nan"), dtype=torch.float64, device="cuda") if precision == isx.FP64 else None
    try:
        ctx.propagate(mid, method, precision, torch.from_numpy(c).cuda(), torch.from_numpy(h).cuda(), out, out64)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(isx.HIDDEN_KERNEL, 0)
        ctx.set_option(isx.UP_FORM, 0)
    return out.cpu().numpy(), (out64.cpu().numpy() if out64 is not None else None)


@pytest.mark.parametrize("net", ["fourier-inr", "he-normal"])
@pytest.mark.parametrize("mname", ["up", "aa"])
def test_propagate_256x5_fp32_and_fp64_match_oracle(ctx, net, mname):
    import paper_2402_13861_amd as isx

    method, gm = METHODS[mname]
    mlp = _net(net)
    S = output_scale(mlp)
    k = 3.0 if mname == "up" else 1.0
    c, h, _ = random_boxes(200, range(0, 10), seed=41)
    print(f"oracle {mname} on {net}: 200 cells, levels 0..9", flush=True)
    ref = propagate(mlp, c, h, method)
    mid = ctx.load_weights(mlp)
    try:
        for kern, kname in ((0, "mfma"), (1, "simt")):
            g32, _ = _gpu_prop(ctx, mid, gm, isx.FP32, c, h, kernel=kern)
            assert_pair_close(g32, ref, S, 1e-5, f"fp32 {kname} {mname} {net}", k=k)
            _, g64 = _gpu_prop(ctx, mid, gm, isx.FP64, c, h, kernel=kern)
            assert_pair_close(g64, ref, S, 1e-10, f"fp64 {kname} {mname} {net}", k=k)
    finally:
        ctx.unload_mlp(mid)


def _endpoint_err(g, oc, os_, k, S, relative=False):
    """Largest endpoint error per cell, in units of S, or relative to
    max(|endpoint|, S)."""
    g = np.asarray(g, np.float64)
    lo_o, hi_o = oc - k * os_, oc + k * os_
    lo = np.abs((g[:, 0] - k * g[:, 1]) - lo_o)
    hi = np.abs((g[:, 0] + k * g[:, 1]) - hi_o)
    if relative:
        return np.maximum(lo / np.maximum(np.abs(lo_o), S), hi / np.maximum(np.abs(hi_o), S))
    return np.maximum(lo, hi) / S


def test_bf16_error_per_level_on_the_benchmark_inr(ctx):
    """BF16 bound error against the oracle on 80 cells per octree level
    0..9 (800 cells), per level max and 99.9th percentile in units of S
    (AA: relative to max(|endpoint|, S)).
    Both UP forms and AA stay within BF16_ENDPOINT_TOL; for UP (the
    benchmark's method) the band 1e-3 S exceeds the largest error at every
    level from 6 on, so that a cell classified differently in BF16 and in
    float64 there is always inside the band and re-decided in float64; with
    the band widened by 2^-6 of each cell's sigma (fp64_band_rel) it covers
    the error of every cell at every level."""
    import paper_2402_13861_amd as isx
    from workloads.configs import isovalues

    mlp = _net("fourier-inr")
    _, S = isovalues(INR)
    rng_levels = np.repeat(np.arange(10), 80)
    cs, hs = [], []
    for L in range(10):
        c, h, _ = random_boxes(80, [L], seed=100 + L)
        cs.append(c)
        hs.append(h)
    c, h = np.concatenate(cs), np.concatenate(hs)
    print("oracle UP and AA on 800 cells of the 3->256x5->1 INR", flush=True)
    mu, sg = propagate(mlp, c, h, UP)
    x0, r = propagate(mlp, c, h, AA)
    mid = ctx.load_weights(mlp)
    try:
        results = {
            "up-cov": _endpoint_err(_gpu_prop(ctx, mid, isx.UP, isx.BF16, c, h, form=0)[0], mu, sg, 3.0, S),
            "up-coef": _endpoint_err(_gpu_prop(ctx, mid, isx.UP, isx.BF16, c, h, form=1)[0], mu, sg, 3.0, S),
            "aa": _endpoint_err(_gpu_prop(ctx, mid, isx.AA, isx.BF16, c, h)[0], x0, r, 1.0, S, relative=True),
            "up-fp32": _endpoint_err(_gpu_prop(ctx, mid, isx.UP, isx.FP32, c, h)[0], mu, sg, 3.0, S),
        }
    finally:
        ctx.unload_mlp(mid)
    for name, e in results.items():
        per = [(L, float(e[rng_levels == L].max()), float(np.quantile(e[rng_levels == L], 0.999)))
               for L in range(10)]
        unit = "relative" if name == "aa" else "units of S"
        print(f"bf16 error vs oracle [{name}] ({unit}): max {e.max():.3e} p99.9 {np.quantile(e, 0.999):.3e}; "
              + ", ".join(f"L{L} {m:.2e}/{q:.2e}" for L, m, q in per), flush=True)
    for name, tol in BF16_ENDPOINT_TOL.items():
        assert results[name].max() <= tol, (name, float(results[name].max()))
    for name in ("up-cov", "up-coef"):
        deep = results[name][rng_levels >= 6]
        assert deep.max() < BAND_REL, (name, float(deep.max()))
        # with the relative term the band covers the error at every level and every cell
        assert np.all(results[name] * S < BAND_REL * S + BAND_REL_SPREAD * sg), name
    assert results["up-fp32"].max() < 1e-2 * BAND_REL


def test_band_leaf_sets_equal_fp64_extraction_depth7(ctx):
    """Depth 7 (128^3), 3 iso-values, t = 3 on the benchmark INR: the float32
    and the BF16 extractions with the 1e-3 S float64 re-check band give the
    float64 extraction's leaves (the plain-UP set the recall target refers
    to).  float32: exactly, since its bound error (1e-5 of max(|o|, S)) is far
    inside the band and band cells are decided by the same float64 kernels.
    BF16: recall and precision at least 99.99 %, every difference counted."""
    import paper_2402_13861_amd as isx
    from workloads.configs import isovalues

    mlp = _net("fourier-inr")
    isos, S = isovalues(INR)
    mid = ctx.load_weights(mlp)
    try:
        ctx.set_isovalues(mid, isos)
        kw = dict(k=3.0, max_depth=7)
        m64 = ctx.extract(mid, isx.UP, isx.FP64, **kw)
        ids64, masks64 = m64.leaves()
        m64.free()
        m32 = ctx.extract(mid, isx.UP, isx.FP32, fp64_band=BAND_REL * S, **kw)
        ids32, masks32 = m32.leaves()
        m32.free()
        mbf = ctx.extract(mid, isx.UP, isx.BF16, fp64_band=BAND_REL * S, **kw)
        idsbf, _ = mbf.leaves()
        rc = sum(l["rechecked"] for l in mbf.levels())
        mbf.free()
        mrel = ctx.extract(mid, isx.UP, isx.BF16, fp64_band=BAND_REL * S, fp64_band_rel=BAND_REL_SPREAD, **kw)
        idsrel, masksrel = mrel.leaves()
        rc_rel = sum(l["rechecked"] for l in mrel.levels())
        mrel.free()
        # the two-stage re-check: float32 for the band, float64 within an eighth of it
        ctx.set_option(isx.RECHECK_CASCADE, 1)
        try:
            mcas = ctx.extract(mid, isx.UP, isx.BF16, fp64_band=BAND_REL * S, **kw)
        finally:
            ctx.set_option(isx.RECHECK_CASCADE, 0)
        idscas, maskscas = mcas.leaves()
        lv = mcas.levels()
        rc_cas, rc_cas64 = sum(l["rechecked"] for l in lv), sum(l["rechecked_fp64"] for l in lv)
        mcas.free()
        # the same with the float32 stage's products as split bf16 MFMAs
        ctx.set_option(isx.RECHECK_CASCADE, 1)
        ctx.set_option(isx.RECHECK_SPLIT, 1)
        try:
            msp = ctx.extract(mid, isx.UP, isx.BF16, fp64_band=BAND_REL * S, **kw)
        finally:
            ctx.set_option(isx.RECHECK_CASCADE, 0)
            ctx.set_option(isx.RECHECK_SPLIT, 0)
        idssp, maskssp = msp.leaves()
        lv = msp.levels()
        rc_sp, rc_sp64 = sum(l["rechecked"] for l in lv), sum(l["rechecked_fp64"] for l in lv)
        msp.free()
    finally:
        ctx.unload_mlp(mid)
    common = np.intersect1d(idsbf, ids64).size
    print(f"depth 7 leaves: fp64 {ids64.size}, fp32+band {ids32.size}, bf16+band {idsbf.size} "
          f"(common with fp64 {common}, bf16 re-checked {rc}); bf16 + relative band {idsrel.size} "
          f"(re-checked {rc_rel})", flush=True)
    np.testing.assert_array_equal(ids32, ids64)
    np.testing.assert_array_equal(masks32, masks64)
    assert common >= 0.9999 * ids64.size
    assert common >= 0.9999 * idsbf.size
    # the error-aware band re-decides every cell BF16 could misclassify: the float64 sets exactly
    np.testing.assert_array_equal(idsrel, ids64)
    np.testing.assert_array_equal(masksrel, masks64)
    print(f"two-stage re-check: {rc_cas} band cells, {rc_cas64} of them in float64; leaves {idscas.size}", flush=True)
    assert rc_cas == rc and rc_cas64 < 0.5 * rc_cas
    # the float32 decisions outside the inner band are the float64 ones: same sets as the one-stage band
    np.testing.assert_array_equal(idscas, idsbf)
    assert common >= 0.9999 * ids64.size and np.intersect1d(idscas, ids64).size == common
    # split products in the first stage: the same band cells, and their decisions are the float64 ones too
    print(f"two-stage re-check, split products: {rc_sp} band cells, {rc_sp64} in float64; leaves {idssp.size}",
          flush=True)
    assert rc_sp == rc
    np.testing.assert_array_equal(idssp, idsbf)
    np.testing.assert_array_equal(maskssp, maskscas)


# the split products' endpoint error must stay well inside the cascade's inner
# band (1/8 of the 1e-3 S band): allowed 2.5e-5 S, a fifth of it
SPLIT_TOL = 2.5e-5


def test_split_fp32_products_error_per_level(ctx):
    """Float32 UP with its products as split bfloat16 MFMAs (ISX_HIDDEN_KERNEL
    3, the cascade's first stage with ISX_RECHECK_SPLIT) on 80 cells per
    octree level 0..9 of the benchmark INR: endpoint error against the oracle
    in units of S, per level, below SPLIT_TOL; the float32 MFMA path for
    comparison."""
    import paper_2402_13861_amd as isx
    from workloads.configs import isovalues

    mlp = _net("fourier-inr")
    _, S = isovalues(INR)
    rng_levels = np.repeat(np.arange(10), 80)
    cs, hs = [], []
    for L in range(10):
        c, h, _ = random_boxes(80, [L], seed=200 + L)
        cs.append(c)
        hs.append(h)
    c, h = np.concatenate(cs), np.concatenate(hs)
    print("oracle UP on 800 cells of the 3->256x5->1 INR", flush=True)
    mu, sg = propagate(mlp, c, h, UP)
    mid = ctx.load_weights(mlp)
    try:
        e_split = _endpoint_err(_gpu_prop(ctx, mid, isx.UP, isx.FP32, c, h, kernel=3)[0], mu, sg, 3.0, S)
        e_f32 = _endpoint_err(_gpu_prop(ctx, mid, isx.UP, isx.FP32, c, h, kernel=2)[0], mu, sg, 3.0, S)
    finally:
        ctx.unload_mlp(mid)
    for name, e in (("split", e_split), ("fp32", e_f32)):
        per = ", ".join(f"L{L} {e[rng_levels == L].max():.2e}" for L in range(10))
        print(f"endpoint error vs oracle [{name}] (units of S): max {e.max():.3e}; {per}", flush=True)
    assert e_split.max() <= SPLIT_TOL, float(e_split.max())
    assert e_f32.max() <= SPLIT_TOL
