"""Quality of the predicted output distribution over a block (Sec. V-E,
Eq. 11): Monte Carlo histogram of the INR over the block, the Gaussian that
UP predicts, the one RA-UA predicts, and a Gaussian fitted to a few samples
(the paper's SAMPLE baseline), each scored by the KL divergence of the
histogram from it.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014; the finaliser constants of
  Vigna's public-domain splitmix64.c).  Output n (n = 0, 1, ...) of the
  stream with seed s is mix(s + (n + 1) * 0x9E3779B97F4A7C15) mod 2^64, i.e.
  the n-th value of the sequential generator started at s.
* Sample i of block b, axis a: counter n = (b * n_samples + i) * 3 + a,
  u = (output >> 40) * 2^-24 (a multiple of 2^-24 in [0, 1)), coordinate
  c_a + h_a (2u - 1) computed in float64 (product, then sum) and rounded to
  float32.  For dyadic blocks (octree cells) every step before the float32
  rounding is exact.
* Histogram: n_bins equal bins on [lo, hi] = [min, max] of the samples; a
  value v falls in bin floor((v - lo) / (hi - lo) * n_bins), clamped to
  n_bins - 1.
* Eq. 11 with p the histogram density (P_b / w on bin b, w = (hi - lo) /
  n_bins, P_b = count_b / N) and q the Gaussian density N(mu, sigma^2); the
  integral over each bin is closed-form because ln q is a quadratic:
    KL = sum_{P_b > 0} P_b [ln(P_b / w) + ln(sigma sqrt(2 pi))
                            + ((e_{b+1} - mu)^3 - (e_b - mu)^3) / (6 sigma^2 w)],
  e_b = lo + b w, the last term evaluated as (a^2 + a c + c^2) / (6 sigma^2)
  with a = e_{b+1} - mu, c = e_b - mu (the same value, without
  cancellation).  A block whose samples are all equal (w = 0) or a Gaussian
  with sigma = 0 gives NaN.
* SAMPLE: the maximum-likelihood Gaussian of the block's first n_fit samples
  (mean, and the root of the mean squared deviation).
"""

from __future__ import annotations

import numpy as np

from .mlp import mlp_forward
from .propagate import RAUA, UP, propagate

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# column order of a block's report (the library writes the same order)
FIELDS = ("mc_mean", "mc_std", "lo", "hi", "up_mu", "up_sigma", "raua_mu", "raua_sigma", "fit_mu", "fit_sigma",
          "kl_up", "kl_raua", "kl_fit")


def splitmix64(seed: int, counters) -> np.ndarray:
    """Outputs number ``counters`` (uint64 array) of the SplitMix64 stream
    started at ``seed``."""
    n = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (n + np.uint64(1)) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def block_samples(centre, half, n_samples: int, seed: int, block: int) -> np.ndarray:
    """The n_samples float32 sample points [N, 3] of block number ``block``."""
    i = np.arange(n_samples, dtype=np.uint64)
    pts = np.empty((n_samples, 3), dtype=np.float32)
    for a in range(3):
        n = (np.uint64(block) * np.uint64(n_samples) + i) * np.uint64(3) + np.uint64(a)
        u = (splitmix64(seed, n) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
        s = 2.0 * u - 1.0
        pts[:, a] = (np.float64(centre[a]) + np.float64(half[a]) * s).astype(np.float32)
    return pts


def histogram(values, n_bins: int):
    """(counts [n_bins], lo, hi) of ``values`` as the module docstring bins them."""
    v = np.asarray(values, dtype=np.float64)
    lo, hi = float(v.min()), float(v.max())
    w = hi - lo
    if w > 0:
        idx = np.floor((v - lo) / w * n_bins).astype(np.int64)
        idx = np.clip(idx, 0, n_bins - 1)
    else:
        idx = np.zeros(v.shape, dtype=np.int64)
    return np.bincount(idx, minlength=n_bins).astype(np.int64), lo, hi


def kl_histogram_gaussian(counts, lo: float, hi: float, mu: float, sigma: float) -> float:
    """Eq. 11: KL divergence of the histogram density from N(mu, sigma^2)."""
    counts = np.asarray(counts, dtype=np.float64)
    nb = counts.size
    w = (hi - lo) / nb
    if not (w > 0) or not (sigma > 0):
        return float("nan")
    P = counts / counts.sum()
    b = np.arange(nb, dtype=np.float64)
    e0 = lo + b * w
    e1 = lo + (b + 1.0) * w
    a, c = e1 - mu, e0 - mu
    cube = (a * a + a * c + c * c) / (6.0 * sigma * sigma)  # ((a^3 - c^3) / (a - c)) / (6 sigma^2)
    keep = P > 0
    terms = P[keep] * (np.log(P[keep] / w) + np.log(sigma * np.sqrt(2.0 * np.pi)) + cube[keep])
    return float(terms.sum())


def gaussian_fit(values):
    """Maximum-likelihood Gaussian (mean, root mean squared deviation)."""
    v = np.asarray(values, dtype=np.float64)
    m = v.mean()
    return float(m), float(np.sqrt(np.mean((v - m) ** 2)))


def block_report(layers, centres, halves, n_samples: int, n_bins: int, n_fit: int, seed: int,
                 act: str = "relu", values_out=None):
    """Per block: the FIELDS row (float64 [B, 13]) and the histogram counts
    (int64 [B, n_bins]).  UP and RA-UA are the oracle's float64 propagation
    (t-independent: the Gaussian itself); MC values are the float64 MLP at the
    float32 sample points.  ``values_out``: optional list that receives each
    block's sample values."""
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    halves = np.asarray(halves, dtype=np.float64).reshape(-1, 3)
    B = centres.shape[0]
    up_mu, up_s = propagate(layers, centres, halves, UP, act=act)
    ra_mu, ra_s = propagate(layers, centres, halves, RAUA, act=act)
    rows = np.zeros((B, len(FIELDS)))
    hists = np.zeros((B, n_bins), dtype=np.int64)
    for b in range(B):
        pts = block_samples(centres[b], halves[b], n_samples, seed, b)
        v = mlp_forward(layers, pts.astype(np.float64), act=act)
        if values_out is not None:
            values_out.append(v)
        counts, lo, hi = histogram(v, n_bins)
        fm, fs = gaussian_fit(v[:n_fit])
        mm, ms = gaussian_fit(v)
        rows[b] = [mm, ms, lo, hi, up_mu[b], up_s[b], ra_mu[b], ra_s[b], fm, fs,
                   kl_histogram_gaussian(counts, lo, hi, up_mu[b], up_s[b]),
                   kl_histogram_gaussian(counts, lo, hi, ra_mu[b], ra_s[b]),
                   kl_histogram_gaussian(counts, lo, hi, fm, fs)]
        hists[b] = counts
    return rows, hists
