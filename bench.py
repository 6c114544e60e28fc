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


# hidden-layer kernel kinds: (kernel name, source file, MFMA dtype)
HIDDEN_KINDS = {
    "hidden_fp32": ("hidden_mfma_f32_kernel", "kernels_mfma.hip", "fp32"),
    "hidden_bf16": ("hidden_mfma_bf16_kernel", "kernels_bf16.hip", "bf16"),
    "hidden_cov_bf16": ("up_cov_bf16_kernel", "kernels_cov.hip", "bf16"),
}


def kernel_source_hash(kind: str) -> str:
    src = ROOT / "paper_2402_13861_amd" / "csrc" / HIDDEN_KINDS[kind][1]
    return hashlib.sha256(src.read_bytes()).hexdigest()[:16]


def traffic_from_profiles(kind: str, cells_per_launch: float):
    """HBM bytes per launch of the dominant kernel: the committed rocprofv3
    counter summary's bytes per propagated cell (all hidden-layer launches of
    a cell; taken on the current kernel source, else None) times the
    propagated cells per launch of this run (propagated cells / launches)."""
    f = ROOT / "profiles" / f"{kind}_traffic.json"
    if not f.exists():
        return None
    t = json.loads(f.read_text())
    if t.get("kernel_source_sha256_16") != kernel_source_hash(kind):
        return None
    return t["hbm_bytes_per_cell"] * cells_per_launch


def cpu_baseline(mlp, levels, budget_s: float):
    """The float64 oracle on a bounded sample: random cells drawn level by
    level in proportion to the GPU run's propagated cells, timed on the host;
    the extraction time is extrapolated from that rate."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle.propagate import UP, propagate
    from workloads import random_boxes

    counts = np.array([l["cells"] for l in levels], dtype=np.float64)
    total = counts.sum()
    p = counts / total
    rng = np.random.default_rng(0)
    done, t_used = 0, 0.0
    batch = 16
    while t_used < budget_s:
        lv = int(rng.choice(len(p), p=p))
        c, h, _ = random_boxes(batch, [lv], seed=int(rng.integers(1 << 30)))
        t0 = time.perf_counter()
        propagate(mlp, c, h, UP)
        t_used += time.perf_counter() - t0
        done += batch
    rate = done / t_used
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return rate, done, t_used, threads, total


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
    ap.add_argument("--accept-leaves", type=int, default=1,
                    help="let the surrogate accept leaves it is confident about (recall is unaffected)")
    ap.add_argument("--sur-base", type=int, default=1,
                    help="1: the surrogate predicts corrections to the INR's centre linearisation; "
                         "0: standardised (mean, log sigma) targets")
    ap.add_argument("--sur-pairs", type=int, default=5_000_000)
    ap.add_argument("--sur-holdout", type=int, default=1_000_000,
                    help="held-out (cell, propagated) pairs for the error and band calibration")
    ap.add_argument("--sur-steps", type=int, default=2000)
    ap.add_argument("--depth", type=int, default=None)
    ap.add_argument("--cpu-baseline-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-bytes", type=int, default=0,
                    help="only run a plain copy of this many bytes (counter calibration) and exit")
    a = ap.parse_args(argv)

    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        return 2
    if a.copy_probe_bytes:
        return copy_probe(a.copy_probe_bytes)

    import numpy as np
    import torch

    import paper_2402_13861_amd as isx
    from paper_2402_13861_amd.surrogate import train_surrogate
    from workloads.configs import WORKLOADS, isovalues, load_mlp

    w = WORKLOADS[a.workload]
    depth = a.depth if a.depth is not None else w["depth"]
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
    mid = ctx.load_weights(mlp)
    ctx.set_isovalues(mid, isos)
    base = dict(method=isx.UP, k=w["k"], max_depth=depth, fp64_band=band)

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
        visited = [m.level_cells(L)[0] for L in range(m.n_levels)] if use_sur else None
        plain = dict(ms=1e3 * plain_s, leaves=int(m.n_leaves), tris=int(m.n_tris),
                     propagated=sum(l["cells"] for l in m.levels()), phases=m.times())
        log(f"plain fp32: {1e3 * plain_s:.1f} ms, {m.n_leaves} leaves")
        m.free()

    # 2. surrogate training (once per INR, not part of the timed extraction)
    sur_info = None
    if use_sur:
        t0 = time.perf_counter()
        info = train_surrogate(ctx, mid, depth, mu_bar, S, visited=visited, n_pairs=a.sur_pairs, steps=a.sur_steps,
                               holdout=a.sur_holdout,
                               isos=isos, k=w["k"], accept_leaves=bool(a.accept_leaves), base=bool(a.sur_base),
                               log=log)
        sur_info = dict(train_total_s=round(time.perf_counter() - t0, 2), train_kernel_s=round(info.train_seconds, 3),
                        pairs=info.n_pairs, steps=info.steps, final_loss=info.final_loss, z=info.z,
                        z_accept=info.z_accept, z_levels=info.z_levels, z_accept_levels=info.z_accept_levels,
                        holdout_miss=info.holdout_miss,
                        holdout_false_accept=info.holdout_false_accept,
                        accept_leaves=bool(a.accept_leaves), base=bool(a.sur_base),
                        err_mu=[round(x, 5) for x in info.err_mu], err_logsig=[round(x, 4) for x in info.err_logsig])
        del visited

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
    eff_cells = float((1 << depth) ** 3)
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

    # the dominant hidden-layer kernel: the kind with the most device time
    kind = max(HIDDEN_KINDS, key=lambda k_: prof[k_]["ms"])
    kp = prof[kind]
    launches = max(kp["launches"], 1)
    avg_ms = kp["ms"] / launches
    flops_per_launch = kp["flops"] / launches
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    peak = PEAK_TFLOPS[HIDDEN_KINDS[kind][2]]
    cells_per_launch = propagated / (kp["launches"] / K) if kp["launches"] else 0.0
    traffic = traffic_from_profiles(kind, cells_per_launch)
    roofline = {
        "bound": "mfma",
        "kernel": HIDDEN_KINDS[kind][0],
        "achieved": round(achieved, 3),
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": traffic,
        "launches": kp["launches"],
        "avg_launch_ms": round(avg_ms, 4),
        "flops_per_launch": flops_per_launch,
        "alg_bytes_per_launch": kp["bytes"] / launches,
        "alg_hbm_GBps": round(kp["bytes"] / launches / (avg_ms * 1e-3) / 1e9, 1) if avg_ms > 0 else 0.0,
    }
    kernels = {}
    for name, v in prof.items():
        if v["launches"]:
            kernels[name] = {"ms_per_step": round(v["ms"] / K, 2), "launches_per_step": v["launches"] / K,
                             "TFLOPs": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2) if v["ms"] > 0 else None}
    log("kernel time per step:", kernels)

    cpu = None
    if not a.no_cpu_baseline:
        rate, done, t_used, threads, total = cpu_baseline(mlp, levels, a.cpu_baseline_seconds)
        total_plain = plain["propagated"] if plain is not None else total
        est_s = total_plain / rate
        cpu = {
            "value": eff_cells / est_s,
            "unit": "cells/s",
            "cores": threads,
            "kind": "oracle",
            "sample": (f"float64 oracle propagation of {done} random cells drawn over octree levels in proportion "
                       f"to the extraction's cells ({t_used:.1f} s, {rate:.1f} cells/s); plain-method extraction "
                       f"time extrapolated from propagation of its {int(total_plain)} cells alone ({est_s:.0f} s)"),
        }

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
            "workload": f"{a.workload}: ReLU MLP {'x'.join(map(str, mlp.widths))}, octree depth {depth} "
                        f"({1 << depth}^3 effective cells), {len(isos)} iso-values, UP t={w['k']}, "
                        f"fp64 band {w.get('band_rel', 0)} S",
            "path": name,
        },
        "value_definition": "effective cells (2^depth)^3 per second of full extraction",
        "plain_fp32": plain and {k: v for k, v in plain.items() if k != "phases"},
        "speedup_vs_plain_fp32": (plain["ms"] / ms_per_step) if plain else None,
        "quality": quality,
        "surrogate": sur_info,
        "examined_cells": examined,
        "propagated_cells": propagated,
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
