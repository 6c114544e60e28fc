"""Pins for the oracle's distribution-quality report (Sec. V-E, Eq. 11).

* SplitMix64 against the published outputs of the reference generator
  (seeds 0 and 1234567), and the counter form against the sequential one.
* Sample points: inside their block, on the 2^-24 grid, and uniform
  (chi-square over 8 octants).
* KL of Eq. 11 in the continuum limit, where it has closed forms: a linear
  field over a cube has a uniform (one active axis) or triangular (two equal
  axes) output density, and UP is exact for linear nets, so
  KL(uniform || N) = (ln(pi/6) + 1)/2 and KL(triangular || N) = ln(pi/3)/2.
* The binned KL equals scipy's relative entropy of the bin masses when q is
  replaced by a step density; the SAMPLE fit is numpy's mean and std.
"""

import numpy as np
import pytest

from oracle.distribution import (block_report, block_samples, gaussian_fit, histogram, kl_histogram_gaussian,
                                 splitmix64)
from workloads.weights import MLPWeights


def test_splitmix64_published_outputs():
    assert [int(x) for x in splitmix64(0, np.arange(5))] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC, 0x1B39896A51A8749B]
    assert [int(x) for x in splitmix64(1234567, np.arange(5))] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431, 16408922859458223821]


def test_samples_inside_block_on_grid_and_uniform():
    c = np.array([0.25, -0.5, 0.125])
    h = np.array([0.125, 0.25, 0.0625])
    p = block_samples(c, h, 80_000, seed=3, block=5).astype(np.float64)
    assert np.all(np.abs(p - c) <= h)
    grid = (p - c) / h * 2.0 ** 23  # 2u - 1 on a 2^-23 grid
    assert np.all(grid == np.round(grid))
    octant = ((p > c) * np.array([1, 2, 4])).sum(axis=1)
    counts = np.bincount(octant, minlength=8)
    chi2 = ((counts - 10_000) ** 2 / 10_000).sum()
    assert chi2 < 24.3  # 7 degrees of freedom, p = 0.001
    # a different block or seed gives different points
    assert not np.array_equal(p, block_samples(c, h, 80_000, seed=3, block=6))
    assert not np.array_equal(p, block_samples(c, h, 80_000, seed=4, block=5))


def _linear_net(a):
    W = [np.array([a], dtype=np.float32), np.array([[1.0]], dtype=np.float32)]
    b = [np.zeros(1, np.float32), np.zeros(1, np.float32)]
    # one hidden neuron kept on the identity side of its ReLU by a large bias
    b[0] = np.array([50.0], np.float32)
    b[1] = np.array([-50.0], np.float32)
    return MLPWeights(Ws=W, bs=b)


@pytest.mark.parametrize("axes,expected", [([1.0, 0.0, 0.0], 0.5 * (np.log(np.pi / 6) + 1.0)),
                                           ([1.0, 1.0, 0.0], 0.5 * np.log(np.pi / 3))])
def test_kl_of_linear_fields_matches_closed_form(axes, expected):
    net = _linear_net(axes)
    c = np.array([[0.0, 0.0, 0.0]])
    h = np.array([[0.5, 0.5, 0.5]])
    rows, hist = block_report(net, c, h, n_samples=400_000, n_bins=64, n_fit=100, seed=11)
    kl_up = rows[0, 10]
    kl_raua = rows[0, 11]
    # plug-in bias (bins - 1) / (2 N) and the histogram's own binning keep it within 3e-3
    assert abs(kl_up - expected) < 3e-3, (kl_up, expected)
    # RA-UA is exact on linear nets too (same sigma)
    assert abs(kl_raua - kl_up) < 1e-9
    assert hist.sum() == 400_000


def test_binned_kl_against_relative_entropy_of_bin_masses():
    """With q replaced by its bin-averaged log density the closed form is the
    relative entropy of the bin masses P against exp(mean ln q) w."""
    from scipy.stats import entropy
    rng = np.random.default_rng(0)
    v = rng.gamma(2.0, 1.5, 50_000) - 2.0
    counts, lo, hi = histogram(v, 40)
    mu, s = 1.0, 3.0
    kl = kl_histogram_gaussian(counts, lo, hi, mu, s)
    w = (hi - lo) / 40
    e = lo + w * np.arange(41)
    # mean of ln q over each bin by Gauss-Legendre quadrature (exact for the quadratic)
    x, wt = np.polynomial.legendre.leggauss(4)
    mids, halfw = 0.5 * (e[1:] + e[:-1]), 0.5 * w
    lnq = np.array([np.sum(wt * (-0.5 * ((m + halfw * x - mu) / s) ** 2 - np.log(s * np.sqrt(2 * np.pi)))) / 2
                    for m in mids])
    P = counts / counts.sum()
    Qstep = np.exp(lnq) * w  # not normalised
    keep = P > 0
    ref = float(np.sum(P[keep] * np.log(P[keep] / Qstep[keep])))
    assert kl == pytest.approx(ref, rel=1e-12, abs=1e-12)
    # relative entropy with scipy (it normalises Q, so compare after removing that)
    assert float(entropy(P, Qstep)) == pytest.approx(ref + np.log(Qstep.sum()), rel=1e-10)


def test_gaussian_fit_and_histogram_edges():
    v = np.array([1.0, 2.0, 4.0, 7.0])
    m, s = gaussian_fit(v)
    assert m == pytest.approx(np.mean(v)) and s == pytest.approx(np.std(v))
    counts, lo, hi = histogram(v, 3)  # edges 1, 3, 5, 7: the maximum goes to the last bin
    assert (lo, hi) == (1.0, 7.0) and counts.tolist() == [2, 1, 1]
    counts, lo, hi = histogram(np.full(5, 2.0), 4)
    assert counts.tolist() == [5, 0, 0, 0]
    assert np.isnan(kl_histogram_gaussian(counts, lo, hi, 2.0, 1.0))
    assert np.isnan(kl_histogram_gaussian([1, 2], 0.0, 1.0, 0.5, 0.0))
