"""The synthetic workloads: MLP shapes, weight sources, iso-value protocol and
octree depth.  Inputs only; no method arithmetic here.

* ``relu64x3_he``: ReLU MLP 3->64->64->64->1, He-normal weights and biases
  (seed 0) on [-1,1]^3, octree depth 6 (64^3 leaves), iso = median of the MLP
  over 10^4 uniform points, t = 3.
* ``relu256x5_fourier``: ReLU MLP 3->256x5->1 fitted (2000 Adam steps, batch
  65536, lr 1e-3, He-normal init seed 0) to a standardised sum of 512 random
  Fourier modes with a k^(-5/3) amplitude spectrum, |k| <= 16, sampled on
  256^3 points (field seed 2); octree depth 9 (512^3 effective resolution);
  iso-values at the 25/50/75 % output quantiles; t = 3; float64 re-check band
  1e-3 S.
* ``relu512x8_blobs``: ReLU MLP 3->512x8->1 fitted (4000 Adam steps, batch
  65536, lr 1e-3, He-normal init seed 0; ``workloads.fit_gpu``) to a field
  of 4096 random anisotropic Gaussian blobs (seed 5) plus a 0.25-weighted
  unit-std Fourier background (512 modes, k^(-5/3), seed 6), standardised,
  sampled at random points of the 512^3 grid; octree depth 10 (1024^3
  effective resolution); 8 iso-values at the 1/9 .. 8/9 output quantiles;
  t = 3; float64 re-check band 1e-3 S.
* ``sine256x5_siren``: sine network 3->256x5->1 (the paper's INR family) in
  the SIREN initialisation (seed 0, first-layer frequency 6), octree depth 9;
  iso-values at the 25/50/75 % output quantiles; t = 3; float64 re-check band
  1e-3 S.  Random weights: a stand-in for a fitted SIREN of the same shape.
* ``relu_sdf_7k`` / ``elu_sdf_29k``: signed distance functions of a small
  analytic scene (a sphere, a torus and a box; ``workloads.fit_gpu --target
  sdf``) fitted by a ReLU 3->64->64->48->1 (7.6k parameters) and an ELU
  3->128->128->96->1 (29.5k parameters) net (3000 Adam steps, batch 65536,
  lr 1e-3, He-normal init seed 0); the level set f = 0 is ray cast (App. A's
  experiment, whose networks have 7.6k and 29k parameters).
"""

from __future__ import annotations

import json
from pathlib import Path

from .weights import he_normal_mlp, read_weights, siren_mlp

DATA = Path(__file__).resolve().parent / "data"
ISO_JSON = Path(__file__).resolve().parent / "isovalues.json"

WORKLOADS = {
    "relu64x3_he": dict(
        widths=[3, 64, 64, 64, 1], weight_seed=0, weights=None, depth=6, k=3.0, iso_quantiles="median",
    ),
    "relu256x5_fourier": dict(
        widths=[3, 256, 256, 256, 256, 256, 1], weight_seed=0, weights="relu_256x5_fourier.isxw", depth=9, k=3.0,
        iso_quantiles=[0.25, 0.5, 0.75], band_rel=1e-3,
    ),
    "relu_sdf_7k": dict(
        widths=[3, 64, 64, 48, 1], weight_seed=0, weights="relu_sdf_7k.isxw", depth=8, k=3.0, iso_quantiles=None,
        act="relu",
    ),
    "elu_sdf_29k": dict(
        widths=[3, 128, 128, 96, 1], weight_seed=0, weights="elu_sdf_29k.isxw", depth=8, k=3.0, iso_quantiles=None,
        act="elu",
    ),
    "sine256x5_siren": dict(
        widths=[3, 256, 256, 256, 256, 256, 1], weight_seed=0, weights="siren:6.0", depth=9, k=3.0,
        iso_quantiles=[0.25, 0.5, 0.75], band_rel=1e-3, act="sine",
    ),
    "relu512x8_blobs": dict(
        widths=[3] + [512] * 8 + [1], weight_seed=0, weights="relu_512x8_blobs.isxw", depth=10, k=3.0,
        iso_quantiles=[i / 9 for i in range(1, 9)], band_rel=1e-3,
    ),
}


def load_mlp(name: str, data_dir=None):
    w = WORKLOADS[name]
    if w["weights"] is None:
        return he_normal_mlp(w["widths"], w["weight_seed"])
    if w["weights"].startswith("siren:"):
        return siren_mlp(w["widths"], w["weight_seed"], float(w["weights"].split(":")[1]))
    mlp = read_weights(Path(data_dir or DATA) / w["weights"])
    assert mlp.widths == w["widths"], (mlp.widths, w["widths"])
    return mlp


def isovalues(name: str):
    """(iso list, output scale S) as written by make_isovalues."""
    t = json.loads(ISO_JSON.read_text())[name]
    return t["iso"], t["scale"]
