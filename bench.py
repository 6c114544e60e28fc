#!/usr/bin/env python3
"""Benchmark of hierarchical iso-surface extraction on one MI355X.

Workload (default): ReLU MLP 3->256x5->1 fitted to a synthetic Fourier field
(k^-5/3 spectrum), octree to depth 9 (512^3 effective resolution), iso-values
at the 25/50/75 % output quantiles, uncertainty propagation with t = 3 and a
float64 re-check band of 1e-3 S.  One step = one full extraction (every octree
level: propagation, classification, compaction; then leaf-corner evaluation
and marching cubes), with the weights resident and nothing cached between
steps.

Prints one JSON line (stdout).  Progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--precision fp32|bf16]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "iso-surface ms @512³, cells/s; plain vs BF16+surrogate at ≥99.9% cell recall"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp64": 78.6}
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# hidden-layer kernel kinds: (kernel name, source file, MFMA dtype, formulation)
HIDDEN_KINDS = {
    "hidden_fp32": ("hidden_mfma_f32_kernel", "kernels_mfma.hip", "fp32", "coefficient"),
    "hidden_bf16": ("hidden_mfma_bf16_kernel", "kernels_bf16.hip", "bf16", "coefficient"),
    "hidden_cov_bf16": ("up_cov_bf16_kernel", "kernels_cov.hip", "bf16", "covariance"),
    "hidden_fp64": ("hidden_mfma_f64_kernel", "kernels_mfma64.hip", "fp64", "coefficient"),
}
# the covariance form with the per-cell matrices in device memory (hidden
# widths 512 and 1024) reports under the same kind
COV_GLOBAL = ("covg_layer_kernel", "kernels_covg.hip", "bf16", "covariance (device memory)")


def kind_info(kind: str, widths) -> tuple:
    """(kernel, source file, dtype, formulation) of a hidden-layer kind for a
    net: the covariance kind runs in device memory above width 256."""
    if kind == "hidden_cov_bf16" and max(widths[1:-1]) > 256:
        return COV_GLOBAL
    return HIDDEN_KINDS[kind]


def alg_flops_coefficient(widths):
    """Algorithmic flops of one cell's hidden-layer products in coefficient
    form: sum over hidden layers h >= 2 of 2 n_h n_{h-1} (D_h + 1), where
    D_2 = 3 and D_{h+1} = D_h + n_h symbol columns enter layer h (+1 for the
    centre column)."""
    hid = widths[1:-1]
    D, f = 3, 0.0
    for h in range(1, len(hid)):
        f += 2.0 * hid[h] * hid[h - 1] * (D + 1)
        D += hid[h - 1]
    return f


def alg_flops_cov_hybrid(widths):
    """Algorithmic flops of the cheapest exact formulation of uncertainty
    propagation per cell: layer by layer the cheaper of the coefficient
    product (2 n_h n_{h-1} D_h) and the covariance update W Sigma W^T
    (2 n^3 for W Sigma plus n^3 for the symmetric half of the second
    product), paying once for Sigma = F F^T (n^2 D, symmetric) where the
    covariance form takes over.  3->256x5->1: 168.7 MFLOP."""
    hid = widths[1:-1]
    D, f, cov = 3, 0.0, False
    for h in range(1, len(hid)):
        n_o, n_i = hid[h], hid[h - 1]
        coef = 2.0 * n_o * n_i * D
        full = 2.0 * n_o * n_i * n_i + 1.0 * n_o * n_o * n_i
        if not cov and full < coef:
            f += 1.0 * n_i * n_i * D
            cov = True
        f += full if cov else coef
        D += n_i
    return f


def kernel_source_hash(kind: str, src_name: str = None) -> str:
    src = ROOT / "paper_2402_13861_amd" / "csrc" / (src_name or HIDDEN_KINDS[kind][1])
    return hashlib.sha256(src.read_bytes()).hexdigest()[:16]


def traffic_from_profiles(kind: str, cells_per_launch: float, src_name: str = None):
    """HBM bytes per launch of the dominant kernel: the committed rocprofv3
    counter summary's bytes per propagated cell (all hidden-layer launches of
    a cell; taken on the current kernel source, else None) times the
    propagated cells per launch of this run (propagated cells / launches).
    A kind's kernel in another source file (the device-memory covariance
    form) has its own summary, named after that file."""
    default = not src_name or src_name == HIDDEN_KINDS[kind][1]
    name = f"{kind}_traffic.json" if default else f"{kind}_{Path(src_name).stem}_traffic.json"
    f = ROOT / "profiles" / name
    if not f.exists():
        return None
    t = json.loads(f.read_text())
    if t.get("kernel_source_sha256_16") != kernel_source_hash(kind, None if default else src_name):
        return None
    return t["hbm_bytes_per_cell"] * cells_per_launch


def host_cpu():
    """(logical cores, CPU model) of the host."""
    model = "unknown"
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def cpu_baseline(mlp, depth: int, budget_s: float, seed: int = 0, act: str = "relu"):
    """The float64 oracle on a bounded sample: random cells drawn uniformly
    over octree levels 3..depth (the oracle's cost per cell does not depend on
    the level), timed on the host's BLAS threads.  Returns the rate and the
    sample with its oracle (mu, sigma), which also serves to measure the GPU
    paths' error against the oracle."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle.propagate import UP, propagate
    from workloads import random_boxes

    rng = np.random.default_rng(seed)
    levels = list(range(min(3, depth), depth + 1))
    cs, hs, ls, mus, sgs = [], [], [], [], []
    done, t_used = 0, 0.0
    batch = 32
    while t_used < budget_s:
        c, h, L = random_boxes(batch, levels, seed=int(rng.integers(1 << 30)))
        t0 = time.perf_counter()
        mu, sg = propagate(mlp, c, h, UP, act=act)
        t_used += time.perf_counter() - t0
        done += batch
        cs.append(c)
        hs.append(h)
        ls.append(L)
        mus.append(mu)
        sgs.append(sg)
    rate = done / t_used
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    sample = dict(centres=np.concatenate(cs), halves=np.concatenate(hs), levels=np.concatenate(ls),
                  mu=np.concatenate(mus), sigma=np.concatenate(sgs))
    return rate, done, t_used, threads, sample


def error_vs_oracle(ctx, mid, mlp, sample, S, k, n_aa, log, act="relu"):
    """Error of the GPU's BF16 bounds (UP covariance form, UP coefficient form,
    AA) and FP32 UP bounds against the float64 oracle, per octree level: max
    and 99.9th percentile of |endpoint_gpu - endpoint_oracle| / S over both
    endpoints centre -/+ k spread (AA: k = 1), and the max of the same error
    over the oracle's spread of the cell.  AA is measured on the first
    n_aa cells of the sample (the oracle's AA is run here, untimed)."""
    import numpy as np
    import torch

    import paper_2402_13861_amd as isx
    from oracle.propagate import AA, propagate

    def gpu(method, prec, c, h, form=0):
        ctx.set_option(isx.UP_FORM, form)
        out = torch.empty((c.shape[0], 2), dtype=torch.float32, device="cuda")
        ctx.propagate(mid, method, prec, torch.from_numpy(c).cuda(), torch.from_numpy(h).cuda(), out)
        torch.cuda.synchronize()
        ctx.set_option(isx.UP_FORM, 0)
        return out.cpu().numpy().astype(np.float64)

    def stats(g, oc, os_, kk, lv):
        ea = np.maximum(np.abs((g[:, 0] - kk * g[:, 1]) - (oc - kk * os_)),
                        np.abs((g[:, 0] + kk * g[:, 1]) - (oc + kk * os_)))
        e = ea / S
        er = ea / np.maximum(os_, 1e-30)  # in units of the cell's own spread
        per = {}
        for L in np.unique(lv):
            sel = lv == L
            per[int(L)] = {"n": int(sel.sum()), "max": float(e[sel].max()),
                           "p999": float(np.quantile(e[sel], 0.999)), "max_over_spread": float(er[sel].max())}
        return {"max": float(e.max()), "p999": float(np.quantile(e, 0.999)), "max_over_spread": float(er.max()),
                "levels": per}

    c, h, lv = sample["centres"], sample["halves"], sample["levels"]
    mu, sg = sample["mu"], sample["sigma"]
    out = {"unit": "S (output scale)", "n_cells": int(c.shape[0]), "k": k}
    out["up_bf16_cov"] = stats(gpu(isx.UP, isx.BF16, c, h, 0), mu, sg, k, lv)
    out["up_bf16_coef"] = stats(gpu(isx.UP, isx.BF16, c, h, 1), mu, sg, k, lv)
    out["up_fp32"] = stats(gpu(isx.UP, isx.FP32, c, h), mu, sg, k, lv)
    na = min(n_aa, c.shape[0])
    x0, r = propagate(mlp, c[:na], h[:na], AA, act=act)
    out["aa_bf16"] = stats(gpu(isx.AA, isx.BF16, c[:na], h[:na]), x0, r, 1.0, lv[:na])
    out["aa_fp32"] = stats(gpu(isx.AA, isx.FP32, c[:na], h[:na]), x0, r, 1.0, lv[:na])
    for key in ("up_bf16_cov", "up_bf16_coef", "up_fp32", "aa_bf16", "aa_fp32"):
        v = out[key]
        log(f"error vs oracle {key}: max {v['max']:.3e} S, p99.9 {v['p999']:.3e} S, max {v['max_over_spread']:.3e} "
            f"of the spread; per level max " +
            ", ".join(f"L{L} {d['max']:.2e} ({d['max_over_spread']:.1e})" for L, d in v["levels"].items()))
    return out



def dense_truth(ctx, mid, depth, isos):
    """Iso-voxels of the dense (2^D)^3 grid: cells whose 8 corner values
    (library float32 evaluation of the INR at every grid point) straddle an
    iso-value (some < c, some >= c), as a bool tensor [iso, i, j, k] on the
    device."""
    import torch

    import paper_2402_13861_amd as isx

    R = (1 << depth) + 1
    g = torch.linspace(-1.0, 1.0, R, device="cuda", dtype=torch.float64).float()
    vals = torch.empty(R ** 3, dtype=torch.float32, device="cuda")
    plane = torch.empty((R * R, 3), dtype=torch.float32, device="cuda")
    jj, ii = torch.meshgrid(g, g, indexing="ij")
    plane[:, 0] = ii.reshape(-1)
    plane[:, 1] = jj.reshape(-1)
    for kz in range(R):  # one z-plane of grid points per call (index i + R (j + R k))
        plane[:, 2] = g[kz]
        ctx.eval_points(mid, isx.FP32, plane, vals[kz * R * R:(kz + 1) * R * R])
    v = vals.view(R, R, R)  # [k, j, i]
    out = []
    for c in isos:
        below = v < c
        any_b = torch.zeros((R - 1,) * 3, dtype=torch.bool, device="cuda")
        all_b = torch.ones((R - 1,) * 3, dtype=torch.bool, device="cuda")
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    s_ = below[dz:dz + R - 1, dy:dy + R - 1, dx:dx + R - 1]
                    any_b |= s_
                    all_b &= s_
        out.append((any_b & ~all_b).permute(2, 1, 0).contiguous())  # [i, j, k]
    return torch.stack(out)


def leaf_rates(ids, masks, truth, depth):
    """FPR and FNR (Sec. V-A-3) of the active (leaf, iso) pairs against the
    dense iso-voxels, over all (2^D)^3 x n_iso pairs."""
    import numpy as np
    import torch

    code = torch.from_numpy(np.asarray(ids, dtype=np.int64)).cuda()
    ijk = []
    for axis in range(3):  # Morton ids, x bit lowest
        v = torch.zeros_like(code)
        for t_ in range(depth):
            v |= ((code >> (3 * t_ + axis)) & 1) << t_
        ijk.append(v)
    ii, jj, kk = ijk
    n_iso = truth.shape[0]
    m = torch.from_numpy(np.asarray(masks, dtype=np.int64)).cuda()
    tp = fp = 0
    for q in range(n_iso):
        pred = ((m >> q) & 1).bool()
        t = truth[q, ii, jj, kk]
        tp += int((pred & t).sum())
        fp += int((pred & ~t).sum())
    pos = int(truth.sum())
    total = truth.numel()
    fn = pos - tp
    tn = total - pos - fp
    return fp / max(fp + tn, 1), fn / max(fn + tp, 1)


def t_sweep(a, log):
    """Sec. V-B's sweep of t (time against missed iso-voxels) on the
    benchmark INR at depth a.depth (default 8, 256^3): BF16 with the float64
    band; UP on the octree and on Alg. 1's k-d tree, RA-UA on the octree, and
    AA (the hard range) once.  Prints one JSON line."""
    import numpy as np
    import torch

    import paper_2402_13861_amd as isx
    from workloads.configs import WORKLOADS, isovalues, load_mlp

    w = WORKLOADS[a.workload]
    depth = a.depth if a.depth is not None else 8
    mlp = load_mlp(a.workload)
    isos, S = isovalues(a.workload)
    ctx = isx.Context(0)
    ctx.set_option(isx.SCRATCH_BYTES, 48 << 30)
    mid = ctx.load_weights(mlp)
    ctx.set_isovalues(mid, isos)
    t0 = time.perf_counter()
    truth = dense_truth(ctx, mid, depth, isos)
    torch.cuda.synchronize()
    dense_s = time.perf_counter() - t0
    log(f"t-sweep: dense truth at {1 << depth}^3 in {dense_s:.2f} s, {int(truth.sum())} iso-voxel pairs")
    band = w.get("band_rel", 0.0) * S
    rows = []
    runs = [("up", isx.UP, False, t) for t in (1, 2, 3, 4, 5, 6, 8, 10)]
    runs += [("up-kd", isx.UP, True, t) for t in (2, 3, 5, 10)]
    runs += [("raua", isx.RAUA, False, t) for t in (1, 2, 3, 5, 10)]
    runs += [("aa", isx.AA, False, 1.0)]
    for name, meth, kd, t in runs:
        ctx.extract(mid, meth, isx.BF16, k=float(t), max_depth=depth, fp64_band=band, kd_tree=kd).free()  # warm
        t1 = time.perf_counter()
        m = ctx.extract(mid, meth, isx.BF16, k=float(t), max_depth=depth, fp64_band=band, kd_tree=kd)
        ms = 1e3 * (time.perf_counter() - t1)
        ids, masks = m.leaves()
        fpr, fnr = leaf_rates(ids, masks, truth, depth)
        prop = sum(l["propagated"] for l in m.levels())
        rows.append(dict(method=name, t=t, ms=round(ms, 2), leaves=int(m.n_leaves), propagated=int(prop),
                         fpr=fpr, fnr=fnr))
        log(f"t-sweep {name} t={t}: {ms:.1f} ms, {m.n_leaves} leaves, FPR {fpr:.4f}, FNR {fnr:.2e}")
        m.free()
    print(json.dumps({"t_sweep": rows, "workload": a.workload, "depth": depth, "precision": "bf16",
                      "fp64_band_S": w.get("band_rel", 0.0), "dense_truth_s": round(dense_s, 2)}), flush=True)
    ctx.close()
    return 0


def kl_report(a, log):
    """Sec. V-E's evaluation of the estimated distribution on the benchmark
    INR: a.kl_blocks random octree blocks of level a.kl_level (default 100 of
    level 5, seed a.kl_seed), 10^6 Monte Carlo samples each, a 100-bin
    histogram, and the KL divergence of Eq. 11 from UP's Gaussian, RA-UA's
    and the Gaussian fitted to 100 samples (the SAMPLE baseline).  Prints one
    JSON line."""
    import numpy as np
    import torch

    import paper_2402_13861_amd as isx
    from workloads.configs import load_mlp

    mlp = load_mlp(a.workload)
    rng = np.random.default_rng(a.kl_seed)
    L = a.kl_level
    idx = rng.integers(0, 1 << L, (a.kl_blocks, 3))
    h = 1.0 / (1 << L)
    centres = (-1.0 + (2 * idx + 1) * h).astype(np.float32)
    halves = np.full((a.kl_blocks, 3), h, np.float32)
    ctx = isx.Context(0)
    mid = ctx.load_weights(mlp)
    args = dict(n_samples=a.kl_samples, n_bins=100, n_fit=100, seed=a.kl_seed)
    c, hh = torch.from_numpy(centres).cuda(), torch.from_numpy(halves).cuda()
    ctx.distribution_kl(mid, c[:1], hh[:1], **args)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = ctx.distribution_kl(mid, c, hh, **args)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = out.cpu().numpy()
    cols = {f: i for i, f in enumerate(isx.DIST_FIELDS)}
    res = {}
    for name in ("up", "raua", "fit"):
        kl = r[:, cols[f"kl_{name}"]]
        ok = np.isfinite(kl)
        res[name] = dict(mean=float(kl[ok].mean()), median=float(np.median(kl[ok])), max=float(kl[ok].max()),
                         finite=int(ok.sum()))
    log(f"kl report: {a.kl_blocks} blocks of level {L}, {a.kl_samples} samples each, {dt:.2f} s; mean KL "
        + ", ".join(f"{k} {v['mean']:.4f}" for k, v in res.items()))
    print(json.dumps({"kl_report": res, "workload": a.workload, "blocks": a.kl_blocks, "level": L,
                      "samples_per_block": a.kl_samples, "bins": 100, "fit_samples": 100, "seconds": round(dt, 3),
                      "samples_per_s": a.kl_blocks * a.kl_samples / dt}), flush=True)
    ctx.close()
    return 0


def batch_bench(a, log):
    """The batched workload (64 INRs of uneven width and depth, 4 iso-values
    each, octree depth 8, BF16 UP, t = 3): isx_extract_batch on
    a.batch_workers worker streams against the INRs extracted one after
    another.  Prints one JSON line."""
    import numpy as np
    import torch

    import paper_2402_13861_amd as isx
    from workloads.batch import DEPTH, batch_mlps, batch_shapes

    table = json.loads((ROOT / "workloads" / "isovalues.json").read_text())["batch64"]
    n = a.batch_inrs
    mlps = batch_mlps(n)
    ctx = isx.Context(0)
    ctx.set_option(isx.SCRATCH_BYTES, 48 << 30)
    ctx.set_option(isx.DENSE_FROM_LEVEL, a.dense_from_level)
    ids = []
    for mlp, t in zip(mlps, table[:n]):
        mid = ctx.load_weights(mlp)
        ctx.set_isovalues(mid, t["iso"])
        ids.append(mid)
    depth = a.depth if a.depth is not None else DEPTH
    prec = {"fp32": isx.FP32, "bf16": isx.BF16}[a.precision]
    kw = dict(method=isx.UP, precision=prec, k=3.0, max_depth=depth)
    if a.autotune:
        # tile shapes of the coefficient-form kernel, timed per INR (printed by the library)
        ctx.set_option(isx.AUTOTUNE, 1)
        ctx.set_option(isx.VERBOSE, 1)
        t0 = time.perf_counter()
        for m in ctx.extract_batch(ids, **dict(kw, max_depth=1)):
            m.free()
        ctx.set_option(isx.VERBOSE, 0)
        log(f"batch: tile shapes timed in {time.perf_counter() - t0:.2f} s")
    # warm-up (code objects, scratch)
    for m in ctx.extract_batch(ids[:4], **kw):
        m.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    singles = []
    for mid in ids:
        m = ctx.extract(mid, **kw)
        singles.append(dict(leaves=int(m.n_leaves), tris=int(m.n_tris),
                            propagated=int(sum(l["propagated"] for l in m.levels())), ms=m.times()["total_ms"]))
        m.free()
    t_seq = time.perf_counter() - t0
    propagated = sum(x["propagated"] for x in singles)
    log(f"batch: {n} INRs one after another in {t_seq * 1e3:.1f} ms, {propagated} propagated cells")
    res = {}
    for workers in a.batch_workers:
        ctx.set_option(isx.BATCH_WORKERS, workers)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms = ctx.extract_batch(ids, **kw)
        dt = time.perf_counter() - t0
        same = all(m.n_leaves == x["leaves"] and m.n_tris == x["tris"] for m, x in zip(ms, singles))
        for m in ms:
            m.free()
        res[workers] = dict(ms=round(dt * 1e3, 2), cells_per_s=propagated / dt, same_meshes_as_single=same)
        log(f"batch: {workers} workers {dt * 1e3:.1f} ms, same meshes {same}")
    shapes = [w for w, _ in batch_shapes(n)]
    print(json.dumps({"batch": res, "sequential_ms": round(t_seq * 1e3, 2), "inrs": n, "depth": depth,
                      "autotune": bool(a.autotune), "dense_from_level": a.dense_from_level,
                      "precision": a.precision, "propagated_cells": propagated,
                      "per_inr": [dict(widths=f"{w[1]}x{len(w) - 2}", **x) for w, x in zip(shapes, singles)]}),
          flush=True)
    ctx.close()
    return 0


def camera_rays(res: int, eye=(1.3, 0.8, 2.3), fov_deg: float = 42.0):
    """Pinhole camera looking at the origin (up = +y), one ray per pixel
    centre, clipped to the domain [-1, 1]^3 by the slab test; float32 arrays
    (origins, unit directions, t_near, t_far)."""
    import numpy as np

    eye = np.array(eye, np.float64)
    fwd = -eye / np.linalg.norm(eye)
    right = np.cross(fwd, [0.0, 1.0, 0.0])
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    half = np.tan(np.radians(fov_deg) / 2)
    u = ((np.arange(res) + 0.5) / res * 2 - 1) * half
    X, Y = np.meshgrid(u, -u, indexing="xy")
    d = fwd[None, :] + X.reshape(-1, 1) * right[None, :] + Y.reshape(-1, 1) * up[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t0 = (-1.0 - eye) * inv
        t1 = (1.0 - eye) * inv
    tn = np.maximum(np.nanmax(np.minimum(t0, t1), axis=1), 0.0)
    tf = np.nanmin(np.maximum(t0, t1), axis=1)
    tf = np.maximum(tf, tn)
    org = np.tile(eye, (res * res, 1))
    return org.astype(np.float32), d.astype(np.float32), tn.astype(np.float32), tf.astype(np.float32)


def raycast_bench(a, log):
    """App. A's ray casting on the two SDF INRs (ReLU 3->64->64->48->1 at
    512^2, ELU 3->128->128->96->1 at 400^2): frame time, segments bounded and
    agreement with RA-Full's image, for UP at several t, RA-Full (AA) and
    RA-Fixed, float32.  Prints one JSON line."""
    import numpy as np
    import torch

    import paper_2402_13861_amd as isx
    from workloads.configs import WORKLOADS, load_mlp

    ctx = isx.Context(0)
    res_all = {}
    for name, res in (("relu_sdf_7k", 512), ("elu_sdf_29k", 400)):
        w = WORKLOADS[name]
        mlp = load_mlp(name, a.sdf_weights_dir)
        mid = ctx.load_weights(mlp)
        if w.get("act") == "elu":
            ctx.set_activation(mid, isx.ELU)
        org, d, tn, tf = (torch.from_numpy(x).cuda() for x in camera_rays(res))
        runs = [("ra-full", isx.AA, 1.0), ("ra-fixed", isx.RAFIXED, 1.0)]
        runs += [(f"up-t{t}", isx.UP, float(t)) for t in (2, 3, 4, 5)]
        ref = None
        rows = []
        for label, meth, t in runs:
            kw = dict(method=meth, precision=isx.FP32, k=t, iso=0.0, step0=1 / 16, step_min=1 / 2048, step_max=0.5,
                      max_iter=2000)
            ctx.raycast(mid, org, d, tn, tf, **kw)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            thit, steps, nseg, nsteps = ctx.raycast(mid, org, d, tn, tf, **kw)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            th = thit.cpu().numpy()
            hit = np.isfinite(th)
            row = dict(method=label, t=t, ms=round(ms, 2), segments=nseg, max_steps=nsteps, hits=int(hit.sum()))
            if ref is None:
                ref = th
            else:
                rh = np.isfinite(ref)
                row["missing_vs_ra_full"] = int((rh & ~hit).sum())
                row["extra_vs_ra_full"] = int((~rh & hit).sum())
                both = rh & hit
                row["mean_abs_dt_vs_ra_full"] = float(np.abs(th[both] - ref[both]).mean()) if both.any() else None
            rows.append(row)
            log(f"raycast {name} {res}^2 {label}: {ms:.1f} ms, {nseg} segments, {int(hit.sum())} hits")
        res_all[name] = dict(resolution=res, widths=mlp.widths, act=w.get("act", "relu"), runs=rows)
        ctx.unload_mlp(mid)
    print(json.dumps({"raycast": res_all, "precision": "fp32", "step0": 1 / 16, "step_min": 1 / 2048,
                      "step_max": 0.5}), flush=True)
    ctx.close()
    return 0


def copy_probe(nbytes: int, reps: int = 5):
    """A plain device-to-device copy of known size: the reference that scales
    the HBM byte counters (FETCH_SIZE, WRITE_SIZE) read for the kernels."""
    import torch

    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes": nbytes, "reps": reps, "ms": 1e3 * dt,
                      "GBps_read_plus_write": 2 * nbytes / dt / 1e9}), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="relu256x5_fourier")
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16"])
    ap.add_argument("--no-surrogate", action="store_true", help="headline path without the learned surrogate")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 reference run")
    ap.add_argument("--dense-from-level", type=int, default=0,
                    help="range analysis down to this level only, dense subtrees below (0: the full refinement)")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the dense baseline (the INR at every grid corner and marching cubes on every cell)")
    ap.add_argument("--accept-leaves", type=int, default=1,
                    help="let the surrogate accept leaves it is confident about (recall is unaffected)")
    ap.add_argument("--sur-base", type=int, default=1,
                    help="1: the surrogate predicts corrections to the INR's centre linearisation; "
                         "0: standardised (mean, log sigma) targets")
    ap.add_argument("--sur-pairs", type=int, default=5_000_000)
    ap.add_argument("--sur-holdout", type=int, default=1_000_000,
                    help="held-out (cell, propagated) pairs for the error and band calibration")
    ap.add_argument("--sur-steps", type=int, default=2000)
    ap.add_argument("--sur-miss-target", type=float, default=3e-4,
                    help="held-out rate of cells the prune band may drop that the plain test keeps, per level")
    ap.add_argument("--sur-accept-target", type=float, default=1e-2,
                    help="held-out rate of cells the accept band may accept that the plain test rejects")
    ap.add_argument("--depth", type=int, default=None)
    ap.add_argument("--cpu-baseline-seconds", type=float, default=30.0)
    ap.add_argument("--no-bf16-only", action="store_true",
                    help="skip the BF16 extraction without the surrogate (its recall is reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--t-sweep", action="store_true",
                    help="only run the sweep of t (time against missed iso-voxels) and exit")
    ap.add_argument("--raycast", action="store_true",
                    help="only run ray casting of the two SDF INRs (UP, RA-Full, RA-Fixed) and exit")
    ap.add_argument("--sdf-weights-dir", default=None, help="directory of the SDF weight files (default: workloads/data)")
    ap.add_argument("--batch", action="store_true",
                    help="only run the batched 64-INR workload (isx_extract_batch) and exit")
    ap.add_argument("--batch-inrs", type=int, default=64)
    ap.add_argument("--batch-workers", type=int, nargs="+", default=[1, 4, 8])
    ap.add_argument("--autotune", type=int, default=0,
                    help="time the BF16 coefficient kernel's tile shapes per INR (switched off in the library)")
    ap.add_argument("--kl-report", action="store_true",
                    help="only run the distribution-quality report (KL of Eq. 11 over random blocks) and exit")
    ap.add_argument("--kl-blocks", type=int, default=100)
    ap.add_argument("--kl-level", type=int, default=5)
    ap.add_argument("--kl-samples", type=int, default=1_000_000)
    ap.add_argument("--kl-seed", type=int, default=0)
    ap.add_argument("--recheck-cascade", type=int, default=1,
                    help="BF16: re-check band cells in float32 first and in float64 only within 1/8 of the band")
    ap.add_argument("--recheck-split", type=int, default=1,
                    help="with --recheck-cascade: the float32 stage's products as split bf16 MFMAs (hi/lo parts; "
                         "endpoint error <= 2.5e-5 S on the benchmark INR, against the inner band of 1.25e-4 S)")
    ap.add_argument("--band-rel", type=float, default=0.0,
                    help="BF16: widen each cell's float64 re-check band by this multiple of its spread (2^-6 "
                         "covers the BF16 endpoint error measured at every level)")
    ap.add_argument("--subtree", type=int, default=0,
                    help="extract only inside the level-L octree cell [0, 2/2^L]^3 of the domain, to the same "
                         "leaf size (depth - L levels below it)")
    ap.add_argument("--copy-probe-bytes", type=int, default=0,
                    help="only run a plain copy of this many bytes (counter calibration) and exit")
    a = ap.parse_args(argv)

    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 (the library has no multi-GPU path)"}))
        return 2
    if a.copy_probe_bytes:
        return copy_probe(a.copy_probe_bytes)
    if a.t_sweep:
        return t_sweep(a, log)
    if a.kl_report:
        return kl_report(a, log)
    if a.batch:
        return batch_bench(a, log)
    if a.raycast:
        return raycast_bench(a, log)

    import numpy as np
    import torch

    import paper_2402_13861_amd as isx
    from paper_2402_13861_amd.surrogate import train_surrogate
    from workloads.configs import WORKLOADS, isovalues, load_mlp

    w = WORKLOADS[a.workload]
    full_depth = a.depth if a.depth is not None else w["depth"]
    depth = full_depth - a.subtree
    mlp = load_mlp(a.workload)
    isos, S = isovalues(a.workload)
    import json as _json

    mu_bar = _json.loads((ROOT / "workloads" / "isovalues.json").read_text())[a.workload]["mean"]
    prec = {"fp32": isx.FP32, "bf16": isx.BF16}[a.precision]
    band = w.get("band_rel", 0.0) * S
    use_sur = not a.no_surrogate
    log(f"bench: {a.workload} widths {mlp.widths} depth {depth} isos {isos} precision {a.precision} "
        f"surrogate {use_sur} band {band:.3g}")

    ctx = isx.Context(0)
    ctx.set_option(isx.SCRATCH_BYTES, 48 << 30)
    ctx.set_option(isx.VERBOSE, 1)
    ctx.set_option(isx.RECHECK_CASCADE, a.recheck_cascade)
    ctx.set_option(isx.RECHECK_SPLIT, a.recheck_split)
    ctx.set_option(isx.DENSE_FROM_LEVEL, a.dense_from_level)
    mid = ctx.load_weights(mlp)
    act = w.get("act", "relu")
    if act != "relu":
        ctx.set_activation(mid, {"sine": isx.SINE, "elu": isx.ELU}[act])
        if use_sur and a.sur_base:
            raise SystemExit(f"bench: the surrogate's linearisation base needs a ReLU net ({a.workload} is {act}); "
                             "pass --no-surrogate or --sur-base 0")
    ctx.set_isovalues(mid, isos)
    sub_hi = 2.0 / (1 << a.subtree) if a.subtree else None
    if a.subtree:
        ctx.set_domain(mid, (0.0, 0.0, 0.0), (sub_hi, sub_hi, sub_hi))
    base = dict(method=isx.UP, k=w["k"], max_depth=depth, fp64_band=band,
                fp64_band_rel=a.band_rel if a.precision == "bf16" else 0.0)

    # 1. plain FP32 reference: the speedup baseline, the recall reference and
    #    the source of visited cells for the surrogate's training set
    plain = None
    if not a.no_plain or use_sur:
        ctx.set_option(isx.KEEP_LEVELS, 1 if use_sur else 0)
        t0 = time.perf_counter()
        m = ctx.extract(mid, precision=isx.FP32, **base)
        plain_s = time.perf_counter() - t0
        ctx.set_option(isx.KEEP_LEVELS, 0)
        plain_ids, _ = m.leaves()
        plain = dict(ms=1e3 * plain_s, leaves=int(m.n_leaves), tris=int(m.n_tris),
                     propagated=sum(l["cells"] for l in m.levels()), phases=m.times())
        log(f"plain fp32: {1e3 * plain_s:.1f} ms, {m.n_leaves} leaves")
        if use_sur:
            visited = m  # its kept levels seed the surrogate's training cells
        else:
            m.free()

    # 1b. BF16 without the surrogate: separates the BF16 error's share of the
    #     leaf differences from the surrogate's
    bf16_only = None
    if plain is not None and a.precision == "bf16" and use_sur and not a.no_bf16_only:
        t0 = time.perf_counter()
        m = ctx.extract(mid, precision=isx.BF16, **base)
        dt = time.perf_counter() - t0
        ids_b, _ = m.leaves()
        common = np.intersect1d(plain_ids, ids_b).size
        bf16_only = dict(ms=1e3 * dt, leaves=int(m.n_leaves), recall_vs_plain=common / max(plain_ids.size, 1),
                         false_active_vs_plain=(ids_b.size - common) / max(ids_b.size, 1),
                         rechecked=sum(l["rechecked"] for l in m.levels()))
        log(f"bf16 without surrogate: {bf16_only}")
        m.free()

    # 2. surrogate training (once per INR, not part of the timed extraction)
    sur_info = None
    if use_sur:
        t0 = time.perf_counter()
        info = train_surrogate(ctx, mid, depth, mu_bar, S, visited=visited, n_pairs=a.sur_pairs, steps=a.sur_steps,
                               holdout=a.sur_holdout, k=w["k"], accept_leaves=bool(a.accept_leaves),
                               base=bool(a.sur_base), miss_target=a.sur_miss_target,
                               accept_target=a.sur_accept_target, log=log)
        sur_info = dict(train_total_s=round(time.perf_counter() - t0, 2),
                        pairs=info.n_pairs, steps=info.steps, final_loss=info.final_loss, z=info.z,
                        z_accept=info.z_accept, z_levels=info.z_levels, z_accept_levels=info.z_accept_levels,
                        holdout_miss=info.holdout_miss, miss_target=a.sur_miss_target,
                        accept_target=a.sur_accept_target,
                        holdout_false_accept=info.holdout_false_accept,
                        accept_leaves=bool(a.accept_leaves), base=bool(a.sur_base),
                        err_mu=[round(x, 5) for x in info.err_mu], err_logsig=[round(x, 4) for x in info.err_logsig])
        visited.free()

    kw = dict(base, precision=prec, use_surrogate=use_sur)
    for i in range(a.warmup):
        t0 = time.perf_counter()
        m = ctx.extract(mid, **kw)
        log(f"warmup {i}: {1e3 * (time.perf_counter() - t0):.1f} ms, {m.n_leaves} leaves, {m.n_tris} triangles")
        m.free()

    ctx.set_option(isx.PROFILE, 1)
    ctx.profile(reset=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    runs = []
    last_ids = None
    for i in range(a.steps):
        t0 = time.perf_counter()
        m = ctx.extract(mid, **kw)
        dt = time.perf_counter() - t0
        runs.append(dict(wall_s=dt, levels=m.levels(), times=m.times(), leaves=m.n_leaves, tris=m.n_tris,
                         corners=m.n_corners))
        log(f"step {i}: {1e3 * dt:.1f} ms, leaves {m.n_leaves}, triangles {m.n_tris}, corners {m.n_corners}, "
            f"phases {m.times()}")
        if i == a.steps - 1:
            last_ids, _ = m.leaves()
        m.free()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = ctx.profile(reset=True)
    ctx.set_option(isx.PROFILE, 0)

    K = a.steps
    eff_cells = float((1 << depth) ** 3)  # leaves of the extracted domain at full resolution
    ms_per_step = 1e3 * elapsed / K
    value = eff_cells * K / elapsed
    levels = runs[-1]["levels"]
    examined = sum(l["cells"] for l in levels)
    propagated = sum(l["propagated"] for l in levels)
    acp_s = np.mean([r["times"]["acp_ms"] for r in runs]) / 1e3
    log("levels (cells, propagated, active, re-checked):",
        [(l["cells"], l["propagated"], l["active"], l["rechecked"]) for l in levels])

    quality = None
    if plain is not None:
        common = np.intersect1d(plain_ids, last_ids).size
        quality = dict(recall_vs_plain=common / max(plain_ids.size, 1),
                       false_active_vs_plain=(last_ids.size - common) / max(last_ids.size, 1),
                       plain_leaves=int(plain_ids.size), leaves=int(last_ids.size))
        log("quality:", quality)

    # dense baseline (context, outside the timed region): the INR at every
    # corner of the (2^D)^3 grid and marching cubes on every cell, float32
    dense = None
    if not a.no_dense:
        ctx.extract_dense(mid, depth, isx.FP32).free()  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dm = ctx.extract_dense(mid, depth, isx.FP32)
        dense_s = time.perf_counter() - t0
        dense = dict(ms=round(1e3 * dense_s, 1), phases={k_: round(v_, 2) for k_, v_ in dm.times().items()},
                     corners=dm.n_corners, tris=dm.n_tris,
                     ratio_to_step=round(1e3 * dense_s / ms_per_step, 3))
        dm.free()
        log(f"dense baseline: {dense}")
    # dense subtrees below level depth - 2 (the same extraction otherwise;
    # context, outside the timed region)
    hybrid = None
    if not a.no_dense and a.dense_from_level == 0 and depth >= 3:
        hl = depth - 2
        ctx.set_option(isx.DENSE_FROM_LEVEL, hl)
        ctx.extract(mid, **kw).free()  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hm = ctx.extract(mid, **kw)
        hyb_s = time.perf_counter() - t0
        ctx.set_option(isx.DENSE_FROM_LEVEL, 0)
        hybrid = dict(dense_from_level=hl, ms=round(1e3 * hyb_s, 1),
                      phases={k_: round(v_, 2) for k_, v_ in hm.times().items()}, leaves=hm.n_leaves,
                      corners=hm.n_corners, tris=hm.n_tris, ratio_to_step=round(1e3 * hyb_s / ms_per_step, 3))
        hm.free()
        log(f"dense subtrees below level {hl}: {hybrid}")

    # per hidden-layer kernel kind: achieved rate at the algorithmic flop count
    # of its formulation (coefficient form: alg_flops_coefficient per cell;
    # covariance form: the cheapest exact formulation, alg_flops_cov_hybrid),
    # and at the flops the kernel executes (the library's own count)
    rechecked = sum(l["rechecked"] for l in levels)
    rechecked64 = sum(l["rechecked_fp64"] for l in levels)
    per_kernel = {}
    split_recheck = a.precision == "bf16" and a.recheck_cascade and a.recheck_split
    for kname in HIDDEN_KINDS:
        kern, src, dt, form = kind_info(kname, mlp.widths)
        v = prof[kname]
        if not v["launches"] or v["ms"] <= 0:
            continue
        executed = v["flops"]
        if kname == "hidden_cov_bf16":
            alg = propagated * K * alg_flops_cov_hybrid(mlp.widths)
        elif kname == "hidden_fp64":
            alg = rechecked64 * K * alg_flops_coefficient(mlp.widths)
        else:
            alg = v["flops"]
        if kname == "hidden_fp32" and split_recheck:
            # the timed steps run only the re-check's float32 stage, whose
            # products are three bf16 MFMAs each: bf16 MFMA peak, three times
            # the float32 products' flops executed
            kern, dt, form = kern + " (SPLIT)", "bf16", form + ", split bf16 products"
            executed = 3 * v["flops"]
        sec = v["ms"] * 1e-3
        per_kernel[kname] = {
            "kernel": kern, "dtype": dt, "formulation": form, "ms_per_step": round(v["ms"] / K, 2),
            "launches_per_step": v["launches"] / K, "alg_flops_per_step": alg / K,
            "achieved_TFLOPs": round(alg / sec / 1e12, 2), "frac": round(alg / sec / 1e12 / PEAK_TFLOPS[dt], 4),
            "executed_flops_per_step": executed / K,
            "executed_TFLOPs": round(executed / sec / 1e12, 2),
            "frac_executed": round(executed / sec / 1e12 / PEAK_TFLOPS[dt], 4),
        }
    # the dominant hidden-layer kernel: the kind with the most device time
    kind = max(per_kernel, key=lambda k_: prof[k_]["ms"])
    kp = prof[kind]
    pk = per_kernel[kind]
    launches = max(kp["launches"], 1)
    avg_ms = kp["ms"] / launches
    alg_per_launch = pk["alg_flops_per_step"] * K / launches
    cells_kind = rechecked64 if kind == "hidden_fp64" else propagated
    cells_per_launch = cells_kind / (kp["launches"] / K) if kp["launches"] else 0.0
    kinfo = kind_info(kind, mlp.widths)
    traffic = traffic_from_profiles(kind, cells_per_launch, kinfo[1])
    roofline = {
        "bound": "mfma",
        "kernel": kinfo[0],
        "achieved": round(alg_per_launch / (avg_ms * 1e-3) / 1e12, 3),
        "peak": PEAK_TFLOPS[kinfo[2]],
        "unit": "TFLOP/s",
        "frac": pk["frac"],
        "traffic": traffic,
        "launches": kp["launches"],
        "avg_launch_ms": round(avg_ms, 4),
        "alg_flops_per_launch": alg_per_launch,
        "cells_per_launch": cells_per_launch,
        "frac_executed": pk["frac_executed"],
        "alg_bytes_per_launch": kp["bytes"] / launches,
        "alg_hbm_GBps": round(kp["bytes"] / launches / (avg_ms * 1e-3) / 1e9, 1) if avg_ms > 0 else 0.0,
        "per_kernel": per_kernel,
    }
    kernels = {}
    for name, v in prof.items():
        if v["launches"]:
            kernels[name] = {"ms_per_step": round(v["ms"] / K, 2), "launches_per_step": v["launches"] / K,
                             "TFLOPs": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2) if v["ms"] > 0 else None}
    log("kernel time per step:", kernels)
    log("roofline per kernel:", per_kernel)

    cpu = None
    err_oracle = None
    if not a.no_cpu_baseline:
        rate, done, t_used, threads, sample = cpu_baseline(mlp, depth, a.cpu_baseline_seconds, act=act)
        total_plain = plain["propagated"] if plain is not None else examined
        est_s = total_plain / rate
        n_cores, cpu_model = host_cpu()
        cpu = {
            "value": eff_cells / est_s,
            "unit": "cells/s",
            "cores": threads,
            "host_cores": n_cores,
            "cpu_model": cpu_model,
            "kind": "oracle",
            "sample": (f"float64 oracle propagation of {done} random cells drawn uniformly over octree levels "
                       f"3..{depth} ({t_used:.1f} s on {threads} BLAS threads, {rate:.1f} cells/s; the oracle's "
                       f"cost per cell does not depend on the level); plain-method extraction time extrapolated "
                       f"from propagation of its {int(total_plain)} cells alone ({est_s:.0f} s)"),
        }
        err_oracle = error_vs_oracle(ctx, mid, mlp, sample, S, w["k"], 2000, log, act=act)
        err_oracle["band_S"] = w.get("band_rel", 0.0)
        err_oracle["levels_where_band_exceeds_bf16_max"] = [
            L for L, d in err_oracle["up_bf16_cov"]["levels"].items() if d["max"] < w.get("band_rel", 0.0)]

    name = ("bf16+surrogate" if use_sur else "bf16") if a.precision == "bf16" else ("fp32+surrogate" if use_sur
                                                                                     else "fp32")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.precision,
        "data": "synthetic",
        "config": {
            "workload": f"{a.workload}: {dict(relu='ReLU', sine='sine', elu='ELU')[act]} MLP "
                        f"{'x'.join(map(str, mlp.widths))}, octree depth {depth} "
                        f"({1 << depth}^3 effective cells), {len(isos)} iso-values, UP t={w['k']}, "
                        f"fp64 band {w.get('band_rel', 0)} S"
                        + (f" + {a.band_rel:g} of the cell's spread" if a.precision == "bf16" and a.band_rel else "")
                        + ((" (float32 re-check" + (" with split bf16 products" if a.recheck_split else "")
                            + ", float64 within 1/8 of the band)") if a.precision == "bf16" and a.recheck_cascade
                           else "")
                        + (f"; domain [0, {sub_hi:g}]^3, the level-{a.subtree} subtree of [-1, 1]^3 at "
                           f"{1 << full_depth}^3 effective resolution" if a.subtree else ""),
            "path": name,
        },
        "value_definition": "effective cells (2^depth)^3 per second of full extraction",
        "plain_fp32": plain and {k: v for k, v in plain.items() if k != "phases"},
        "speedup_vs_plain_fp32": (plain["ms"] / ms_per_step) if plain else None,
        "quality": quality,
        "bf16_only": bf16_only,
        "dense_gpu": dense,
        "dense_subtrees_gpu": hybrid,
        "bf16_err_vs_oracle": err_oracle,
        "surrogate": sur_info,
        "examined_cells": examined,
        "propagated_cells": propagated,
        "rechecked_cells": int(rechecked),
        "rechecked_fp64_cells": int(rechecked64),
        "propagated_cells_per_s": propagated / acp_s if acp_s > 0 else None,
        "active_leaves": runs[-1]["leaves"],
        "triangles": runs[-1]["tris"],
        "phase_ms": {k: round(float(np.mean([r["times"][k] for r in runs])), 2) for k in runs[-1]["times"]},
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
