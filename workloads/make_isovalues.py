"""Write workloads/isovalues.json: iso-values and output scales of the
synthetic workloads, computed by the float64 oracle MLP.

Protocol: points ``default_rng(weight_seed + 1).uniform(-1, 1, (10000, 3))``;
the iso-value is the median (numpy's mean of the two middle values) or the
given quantiles (``np.quantile``, linear); S is the standard deviation of the
same outputs.  Values are rounded to float32, the precision both sides read.

    python -m workloads.make_isovalues
"""

from __future__ import annotations

import json
from pathlib import Path

import numpy as np

from oracle.mlp import mlp_forward

from .batch import batch_mlps, batch_shapes
from .cells import uniform_points
from .configs import WORKLOADS, load_mlp

OUT = Path(__file__).resolve().parent / "isovalues.json"


def main():
    table = {}
    for name, w in WORKLOADS.items():
        if w.get("iso_quantiles") is None:
            continue
        mlp = load_mlp(name)
        vals = mlp_forward(mlp, uniform_points(10_000, w["weight_seed"] + 1), act=w.get("act", "relu"))
        qs = w["iso_quantiles"]
        if qs == "median":
            isos = [float(np.median(vals))]
        else:
            isos = [float(v) for v in np.quantile(vals, qs, method="linear")]
        table[name] = dict(
            iso=[float(np.float32(v)) for v in isos],
            scale=float(np.std(vals)),
            mean=float(np.mean(vals)),
        )
        print(name, table[name])
    # the batched workload: per INR, iso-values at its own quantile levels
    # over the points of seed 3 + i + 1
    batch = []
    for i, (mlp, (_, qs)) in enumerate(zip(batch_mlps(), batch_shapes())):
        vals = mlp_forward(mlp, uniform_points(10_000, 3 + i + 1))
        isos = [float(np.float32(v)) for v in np.quantile(vals, qs, method="linear")]
        batch.append(dict(iso=isos, scale=float(np.std(vals)), mean=float(np.mean(vals))))
    table["batch64"] = batch
    print("batch64:", len(batch), "INRs")
    OUT.write_text(json.dumps(table, indent=1) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
