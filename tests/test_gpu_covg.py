"""BF16 uncertainty propagation in covariance form with the per-cell N x N
matrices in device memory (Eq. 8-9 through covariances), against the float64
oracle.

The form runs by default (ISX_UP_FORM = 0) for nets whose hidden layers all
have width 512 or 1024, and with ISX_UP_FORM = 2 also at width 256.  Checked
here:
* bounds, spread and centre against the oracle on dyadic cells of octree
  levels 0..9, ReLU, sine (SIREN) and ELU nets of widths 256, 512 and 1024
  (the largest hidden width), with two and more hidden layers (layer 2 in
  rank-3 form, and as the last layer), within the BF16 tolerances below;
* a batch split into many chunks gives the one-chunk result bit for bit;
* extraction with the float64 re-check band against the float64 extraction.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.mlp import mlp_forward
from oracle.propagate import UP, propagate
from workloads import he_normal_mlp, random_boxes, uniform_points
from workloads.weights import siren_mlp

from _parity import assert_pair_close

pytestmark = pytest.mark.gpu

# (bounds, centre) relative to max(|o|, S): the tolerances of the on-chip
# BF16 forms; the spread relative to itself within 2^-8, two units of
# bfloat16 rounding (the variance sums take bfloat16 products of matrices
# stored in bfloat16)
TOL = (3e-3, 2.0 ** -8, 2e-3)

NETS = {
    "relu-256x5": ("relu", lambda: he_normal_mlp([3, 256, 256, 256, 256, 256, 1], seed=0), 2),
    "relu-512x3": ("relu", lambda: he_normal_mlp([3, 512, 512, 512, 1], seed=2), 2),
    "relu-1024x2": ("relu", lambda: he_normal_mlp([3, 1024, 1024, 1], seed=5), 0),
    "relu-512x2": ("relu", lambda: he_normal_mlp([3, 512, 512, 1], seed=8), 0),  # layer 2 rank-3 and last
    "sine-1024x2": ("sine", lambda: siren_mlp([3, 1024, 1024, 1], seed=9, w0=6.0), 0),
    "sine-512x3": ("sine", lambda: siren_mlp([3, 512, 512, 512, 1], seed=6, w0=6.0), 2),
    "elu-512x3": ("elu", lambda: he_normal_mlp([3, 512, 512, 512, 1], seed=7), 2),
}


@pytest.fixture(scope="module")
def ctx():
    import paper_2402_13861_amd as isx

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = isx.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _load(ctx, name):
    import paper_2402_13861_amd as isx

    act, make, form = NETS[name]
    mlp = make()
    mid = ctx.load_weights(mlp)
    if act != "relu":
        ctx.set_activation(mid, {"sine": isx.SINE, "elu": isx.ELU}[act])
    return act, mlp, mid, form


def _prop(ctx, mid, c, h, form):
    import paper_2402_13861_amd as isx

    ctx.set_option(isx.UP_FORM, form)
    out = torch.full((c.shape[0], 2), float("nan"), dtype=torch.float32, device="cuda")
    try:
        ctx.propagate(mid, isx.UP, isx.BF16, torch.from_numpy(c).cuda(), torch.from_numpy(h).cuda(), out)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(isx.UP_FORM, 0)
    return out.cpu().numpy()


@pytest.mark.parametrize("name", list(NETS))
def test_device_memory_covariance_form_against_oracle(ctx, name):
    act, mlp, mid, form = _load(ctx, name)
    try:
        S = float(np.std(mlp_forward(mlp, uniform_points(10_000, 1), act=act)))
        c, h, _ = random_boxes(96, range(0, 10), seed=13)
        print(f"oracle UP on {name}: 96 cells, levels 0..9", flush=True)
        ref = propagate(mlp, c, h, UP, act=act)
        g = _prop(ctx, mid, c, h, form)
        assert np.isfinite(g).all()
        tol, stol, ctol = TOL
        worst, _ = assert_pair_close(g, ref, S, tol, f"bf16 up device-memory cov {name}", k=3.0, spread_rtol=stol)
        assert worst["centre"] <= ctol
    finally:
        ctx.unload_mlp(mid)


def test_device_memory_covariance_form_chunks_match_one_chunk(ctx):
    """An 8 MiB scratch budget (7 cells of width 512 per chunk) against one
    chunk: identical results, bit for bit."""
    import paper_2402_13861_amd as isx

    _, mlp, mid, _ = _load(ctx, "relu-512x3")
    c, h, _ = random_boxes(300, range(0, 10), seed=21)
    try:
        a = _prop(ctx, mid, c, h, 2)
        ctx.set_option(isx.SCRATCH_BYTES, 8 << 20)
        b = _prop(ctx, mid, c, h, 2)
        np.testing.assert_array_equal(a, b)
        # form 1 (coefficient form) still answers at this width, to its own tolerance
        ref = propagate(mlp, c[:64], h[:64], UP)
        S = float(np.std(mlp_forward(mlp, uniform_points(10_000, 1))))
        assert_pair_close(_prop(ctx, mid, c[:64], h[:64], 1), ref, S, TOL[0], "bf16 up coefficient form 512", k=3.0,
                          spread_rtol=TOL[1])
    finally:
        ctx.set_option(isx.SCRATCH_BYTES, 16 << 30)
        ctx.unload_mlp(mid)


def test_device_memory_covariance_extraction_with_band(ctx):
    """Depth 6, t = 3, iso-values at the 30 / 60 % quantiles of a 3->512x3->1
    net: the BF16 extraction with a float64 re-check band of 1e-3 S against
    the float64 extraction, recall and precision at least 99.99 %."""
    import paper_2402_13861_amd as isx

    _, mlp, mid, _ = _load(ctx, "relu-512x3")
    try:
        vals = mlp_forward(mlp, uniform_points(10_000, seed=1))
        S = float(vals.std())
        isos = [float(np.float32(np.quantile(vals, q))) for q in (0.3, 0.6)]
        ctx.set_isovalues(mid, isos)
        kw = dict(k=3.0, max_depth=6)
        m64 = ctx.extract(mid, isx.UP, isx.FP64, **kw)
        ids64, _ = m64.leaves()
        m64.free()
        ctx.set_option(isx.UP_FORM, 2)
        try:
            mbf = ctx.extract(mid, isx.UP, isx.BF16, fp64_band=1e-3 * S, **kw)
        finally:
            ctx.set_option(isx.UP_FORM, 0)
        idsbf, _ = mbf.leaves()
        mbf.free()
        a, b = set(ids64.tolist()), set(idsbf.tolist())
        both = len(a & b)
        print(f"leaves fp64 {len(a)}, bf16 {len(b)}, common {both}", flush=True)
        assert len(a) > 1000
        assert both >= 0.9999 * len(a) and both >= 0.9999 * len(b)
    finally:
        ctx.unload_mlp(mid)


def test_device_memory_covariance_form_unsupported_net(ctx):
    """ISX_UP_FORM = 2 on a net whose hidden widths differ reports
    ISX_EUNSUPPORTED."""
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp([3, 512, 256, 512, 1], seed=9)
    mid = ctx.load_weights(mlp)
    c, h, _ = random_boxes(8, range(0, 4), seed=1)
    try:
        with pytest.raises(isx.IsxError) as e:
            _prop(ctx, mid, c, h, 2)
        assert e.value.status == -7  # ISX_EUNSUPPORTED
    finally:
        ctx.unload_mlp(mid)
