"""Batched extraction (isx_extract_batch): many INRs of uneven width and
depth, each with its own iso-values, extracted on several streams at once.
Every mesh must equal the one isx_extract returns for that INR alone."""

import time

import numpy as np
import pytest
import torch

from _parity import close_sets, unexcused_level_diffs
from oracle.mlp import mlp_forward
from oracle.octree import extract_active
from oracle.propagate import UP
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


def _uneven_inrs(n, seed, widths=(64, 128, 256), depths=(2, 3, 4, 5)):
    """n ReLU INRs with hidden width and depth drawn per INR (He-normal
    weights, per-INR seed) and 2 iso-values at random output quantiles."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        w = int(rng.choice(widths))
        d = int(rng.choice(depths))
        mlp = he_normal_mlp([3] + [w] * d + [1], seed=1000 + i)
        vals = mlp_forward(mlp, uniform_points(4000, seed=2000 + i))
        isos = [float(np.quantile(vals, q)) for q in np.sort(rng.uniform(0.1, 0.9, 2))]
        out.append((mlp, isos))
    return out


@pytest.mark.parametrize("prec_name,widths", [("fp32", (64, 128, 256, 512)), ("bf16", (64, 128, 256))])
def test_extract_batch_equals_single_extractions(ctx, prec_name, widths):
    import paper_2402_13861_amd as isx

    prec = isx.FP32 if prec_name == "fp32" else isx.BF16
    inrs = _uneven_inrs(8, seed=5 if prec_name == "fp32" else 6, widths=widths)
    ids = []
    try:
        for mlp, isos in inrs:
            mid = ctx.load_weights(mlp)
            ctx.set_isovalues(mid, isos)
            ids.append(mid)
        kw = dict(method=isx.UP, precision=prec, k=3.0, max_depth=5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        singles = [ctx.extract(mid, **kw) for mid in ids]
        t_single = time.perf_counter() - t0
        for workers in (1, 4):
            ctx.set_option(isx.BATCH_WORKERS, workers)
            t0 = time.perf_counter()
            batch = ctx.extract_batch(ids, **kw)
            t_batch = time.perf_counter() - t0
            assert len(batch) == len(ids)
            for i, (a, b) in enumerate(zip(singles, batch)):
                assert (a.n_tris, a.n_leaves, a.n_corners) == (b.n_tris, b.n_leaves, b.n_corners), (workers, i)
                la, lb = a.leaves(), b.leaves()
                assert all(np.array_equal(x, y) for x, y in zip(la, lb)), (workers, i)
                ta, tb = a.triangles(), b.triangles()
                assert all(np.array_equal(x, y) for x, y in zip(ta, tb)), (workers, i)
                assert [l["active"] for l in a.levels()] == [l["active"] for l in b.levels()]
            print(f"{prec_name}: {len(ids)} INRs, {workers} worker(s): batch {t_batch * 1e3:.1f} ms, "
                  f"one by one {t_single * 1e3:.1f} ms", flush=True)
            for m in batch:
                m.free()
        for m in singles:
            m.free()
    finally:
        ctx.set_option(isx.BATCH_WORKERS, 4)
        for mid in ids:
            ctx.unload_mlp(mid)


def test_extract_batch_matches_oracle(ctx):
    """Every INR of a batch (uneven widths and depths, own iso-values, four
    worker streams) against the oracle's octree search: per-level active
    sets equal except cells that are, or descend from, cells whose oracle
    bound endpoint lies within 1e-4 S of an iso-value."""
    import paper_2402_13861_amd as isx

    inrs = _uneven_inrs(6, seed=11, widths=(32, 64, 96), depths=(2, 3))
    depth = 4
    ids = []
    try:
        for mlp, isos in inrs:
            mid = ctx.load_weights(mlp)
            ctx.set_isovalues(mid, [float(np.float32(c)) for c in isos])
            ids.append(mid)
        ctx.set_option(isx.KEEP_LEVELS, 1)
        ctx.set_option(isx.BATCH_WORKERS, 4)
        meshes = ctx.extract_batch(ids, method=isx.UP, precision=isx.FP32, k=3.0, max_depth=depth)
        ctx.set_option(isx.KEEP_LEVELS, 0)
        for i, ((mlp, isos), m) in enumerate(zip(inrs, meshes)):
            isos32 = [float(np.float32(c)) for c in isos]
            S = float(mlp_forward(mlp, uniform_points(10_000, seed=1)).std())
            gl = [m.level_cells(L) for L in range(m.n_levels)]
            ol = extract_active(mlp, UP, isos32, depth, k=3.0)
            bad = unexcused_level_diffs(gl, ol, close_sets(ol, UP, 3.0, isos32, S))
            assert not bad, (i, bad)
            m.free()
    finally:
        ctx.set_option(isx.KEEP_LEVELS, 0)
        ctx.set_option(isx.BATCH_WORKERS, 4)
        for mid in ids:
            ctx.unload_mlp(mid)


def test_extract_batch_reports_a_bad_inr(ctx):
    import paper_2402_13861_amd as isx

    mlp = he_normal_mlp([3, 32, 32, 1], seed=3)
    mid = ctx.load_weights(mlp)
    try:
        ctx.set_isovalues(mid, [0.0])
        with pytest.raises(isx.IsxError):
            ctx.extract_batch([mid, mid + 100], method=isx.UP, precision=isx.FP32, max_depth=3)
        # the context still works afterwards
        ms = ctx.extract_batch([mid, mid], method=isx.UP, precision=isx.FP32, max_depth=3)
        assert ms[0].n_leaves == ms[1].n_leaves
    finally:
        ctx.unload_mlp(mid)


def test_extract_batch_overlaps_small_inrs(ctx):
    """32 small INRs (3->64x3->1, depth 6, BF16): the level loops are
    launch- and sync-bound, so running them on several streams at once is
    faster than one after another.  Prints both times; the meshes agree."""
    import paper_2402_13861_amd as isx

    ids = []
    try:
        for i in range(32):
            mlp = he_normal_mlp([3, 64, 64, 64, 1], seed=6400 + i)
            vals = mlp_forward(mlp, uniform_points(2000, seed=6500 + i))
            mid = ctx.load_weights(mlp)
            ctx.set_isovalues(mid, [float(np.median(vals))])
            ids.append(mid)
        kw = dict(method=isx.UP, precision=isx.BF16, k=3.0, max_depth=6)
        for m in [ctx.extract(i, **kw) for i in ids]:
            m.free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        singles = [ctx.extract(i, **kw) for i in ids]
        t_single = time.perf_counter() - t0
        times = {}
        for workers in (1, 4, 8):
            ctx.set_option(isx.BATCH_WORKERS, workers)
            for m in ctx.extract_batch(ids, **kw):
                m.free()
            t0 = time.perf_counter()
            batch = ctx.extract_batch(ids, **kw)
            times[workers] = time.perf_counter() - t0
            assert [m.n_tris for m in batch] == [m.n_tris for m in singles]
            for m in batch:
                m.free()
        print("32 INRs 3->64x3->1, depth 6, BF16: one by one %.1f ms; batch %s" %
              (t_single * 1e3, ", ".join(f"{w} workers {t * 1e3:.1f} ms" for w, t in times.items())), flush=True)
        for m in singles:
            m.free()
    finally:
        ctx.set_option(isx.BATCH_WORKERS, 4)
        for mid in ids:
            ctx.unload_mlp(mid)
