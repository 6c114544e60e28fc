"""Segments, RA-Fixed and ray casting (App. A) on the GPU against the
float64 oracle.

* Segment bounds (AA, UP, RA-UA, RA-Fixed): float32 within 1e-5 of
  max(|o|, S), float64 within 1e-10, on random segments of many lengths
  (RA-Fixed's float32 spread within 5e-4 of max(spread, 1e-3 S)).
* RA-Fixed on boxes: the same tolerances.
* Ray casting a 20x20 image (3->32x3->1 He-normal net, iso = median): with
  float64 bounds every ray whose decisions all clear the iso-value by more
  than 1e-9 S takes the oracle's steps and hits at the same float32 t; with
  float32 bounds, the same for rays clearing it by 1e-4 S.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.mlp import mlp_forward
from oracle.propagate import AA, RAFIXED, RAUA, UP, propagate_rafixed, propagate_segments
from oracle.raycast import cast
from workloads import he_normal_mlp, random_boxes

from _parity import assert_pair_close, output_scale

pytestmark = pytest.mark.gpu

METHODS = {"aa": AA, "up": UP, "raua": RAUA, "rafixed": RAFIXED}


@pytest.fixture(scope="module")
def ctx():
    import paper_2402_13861_amd as isx

    assert torch.cuda.is_available()
    c = isx.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _gm(isx, name):
    return {"aa": isx.AA, "up": isx.UP, "raua": isx.RAUA, "rafixed": isx.RAFIXED}[name]


def _segments(n, seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-0.9, 0.9, (n, 3)).astype(np.float32)
    d = rng.normal(0, 1, (n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    length = 2.0 ** rng.uniform(-12, 0, n)
    return c, (d * length[:, None]).astype(np.float32)


@pytest.mark.parametrize("widths", [[3, 64, 64, 64, 1], [3, 48, 40, 1], [3, 256, 256, 256, 1]],
                         ids=lambda w: "x".join(map(str, w)))
@pytest.mark.parametrize("name", list(METHODS))
def test_segment_bounds_match_oracle(ctx, widths, name):
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp(widths, seed=11)
    S = output_scale(mlp)
    c, v = _segments(300, 5)
    ref = propagate_segments(mlp, c, v, METHODS[name])
    k = 1.0 if name in ("aa", "rafixed") else 3.0
    mid = ctx.load_weights(mlp)
    try:
        for prec, tol in ((isx.FP32, 1e-5), (isx.FP64, 1e-10)):
            out = torch.full((c.shape[0], 2), float("nan"), device="cuda")
            out64 = torch.full((c.shape[0], 2), float("nan"), dtype=torch.float64, device="cuda") \
                if prec == isx.FP64 else None
            ctx.propagate_segments(mid, _gm(isx, name), prec, torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda(),
                                   out, out64)
            torch.cuda.synchronize()
            got = out64.cpu().numpy() if out64 is not None else out.cpu().numpy()
            # RA-Fixed's error term adds |W| |gamma| over every straddling neuron, and gamma = -alpha l / 2
            # carries the float32 centre's absolute rounding (~1e-7 S): on segments whose spread is near the
            # 1e-3 S floor that is a few 1e-4 of it, without the sign cancellation AA's separate symbols get
            srtol = 5e-4 if (name == "rafixed" and prec == isx.FP32) else None
            assert_pair_close(got, ref, S, tol, f"segments {name} {widths} prec {prec}", k=k, spread_rtol=srtol)
    finally:
        ctx.unload_mlp(mid)


def test_rafixed_boxes_match_oracle(ctx):
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp([3, 64, 64, 64, 1], seed=12)
    S = output_scale(mlp)
    c, h, _ = random_boxes(200, range(0, 10), seed=4)
    F0 = np.zeros((c.shape[0], 3, 3))
    for a in range(3):
        F0[:, a, a] = h[:, a]
    ref = propagate_rafixed(mlp, c, F0)
    mid = ctx.load_weights(mlp)
    try:
        for prec, tol in ((isx.FP32, 1e-5), (isx.FP64, 1e-10)):
            out = torch.empty((c.shape[0], 2), device="cuda")
            out64 = torch.empty((c.shape[0], 2), dtype=torch.float64, device="cuda") if prec == isx.FP64 else None
            ctx.propagate(mid, isx.RAFIXED, prec, torch.from_numpy(c).cuda(), torch.from_numpy(h).cuda(), out, out64)
            torch.cuda.synchronize()
            got = out64.cpu().numpy() if out64 is not None else out.cpu().numpy()
            assert_pair_close(got, ref, S, tol, f"rafixed boxes prec {prec}", k=1.0)
    finally:
        ctx.unload_mlp(mid)


def _camera(res):
    o = np.array([0.15, -0.1, 2.6], np.float32)
    u = (np.arange(res) + 0.5) / res * 1.2 - 0.6
    X, Y = np.meshgrid(u, u, indexing="xy")
    d = np.stack([X.ravel(), Y.ravel(), -np.full(res * res, 2.0)], axis=1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    org = np.tile(o, (res * res, 1))
    # the unit cube's slabs
    with np.errstate(divide="ignore"):
        inv = 1.0 / d
    t0 = (-1.0 - o) * inv
    t1 = (1.0 - o) * inv
    tn = np.maximum(np.minimum(t0, t1).max(axis=1), 0.0)
    tf = np.maximum(t0, t1).min(axis=1)
    return org, d.astype(np.float32), tn.astype(np.float32), np.maximum(tf, tn).astype(np.float32)


@pytest.mark.parametrize("name", ["up", "aa", "rafixed", "raua"])
def test_raycast_matches_oracle(ctx, name):
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp([3, 32, 32, 32, 1], seed=13)
    vals = mlp_forward(mlp, np.random.default_rng(2).uniform(-1, 1, (4000, 3)))
    iso = float(np.float32(np.median(vals)))
    S = float(vals.std())
    org, d, tn, tf = _camera(20)
    kw = dict(k=3.0, iso=iso, step0=1 / 16, step_min=1 / 1024, step_max=0.5, max_iter=400)
    ref_t, ref_steps, margin = cast(mlp, org, d, tn, tf, METHODS[name], kw["k"], iso, kw["step0"], kw["step_min"],
                                    kw["step_max"], kw["max_iter"])
    mid = ctx.load_weights(mlp)
    try:
        dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
        for prec, clear in ((isx.FP64, 1e-9), (isx.FP32, 1e-4)):
            thit, steps, nseg, nsteps = ctx.raycast(mid, dev(org), dev(d), dev(tn), dev(tf), method=_gm(isx, name),
                                                   precision=prec, **kw)
            torch.cuda.synchronize()
            g_t, g_s = thit.cpu().numpy(), steps.cpu().numpy()
            ok = margin > clear * S
            hits = np.isfinite(ref_t)
            print(f"raycast {name} prec {prec}: {hits.sum()} hits of {len(ref_t)} rays, {nseg} segments, "
                  f"{nsteps} steps; rays clear of the level {ok.sum()}", flush=True)
            assert ok.mean() > 0.8
            np.testing.assert_array_equal(g_s[ok], ref_steps[ok])
            np.testing.assert_array_equal(np.isfinite(g_t[ok]), hits[ok])
            np.testing.assert_array_equal(g_t[ok & hits], ref_t[ok & hits])
            assert nseg == int(g_s.sum())
    finally:
        ctx.unload_mlp(mid)


def test_raycast_rejects_bf16_and_bad_steps(ctx):
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp([3, 16, 16, 1], seed=1)
    mid = ctx.load_weights(mlp)
    try:
        org, d, tn, tf = (torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in _camera(4))
        with pytest.raises(isx.IsxError) as e:
            ctx.raycast(mid, org, d, tn, tf, precision=isx.BF16)
        assert e.value.status == -7
        with pytest.raises(isx.IsxError) as e:
            ctx.raycast(mid, org, d, tn, tf, step0=0.1, step_max=0.05)
        assert e.value.status == -1
        # an empty interval is a miss after no step
        thit, steps, nseg, _ = ctx.raycast(mid, org[:1], d[:1], tf[:1], tn[:1])
        assert np.isnan(thit.cpu().numpy()[0]) and steps.cpu().numpy()[0] == 0 and nseg == 0
    finally:
        ctx.unload_mlp(mid)
