"""Pins for the oracle's segment forms, RA-Fixed and ray casting (App. A).

* A segment along an axis is the box with the other two half-sizes 0, for
  every method.
* Linear nets: every method's range of a segment is exact (AA, RA-Fixed:
  mu -/+ |a . v|; UP: sigma = |a . v| / sqrt 3), and ray casting hits within
  step_min / 2 of the analytic crossing (UP: k / sqrt 3 times that).
* Soundness: RA-Fixed's range contains AA's, which contains dense samples of
  the segment; on a net whose neurons keep their sign over the segment both
  are exact and equal.
* Ray casting with a sound method never steps over the first sign change a
  dense scan of the ray finds.
"""

import numpy as np
import pytest

from oracle.mlp import mlp_forward
from oracle.propagate import AA, RAFIXED, RAUA, UP, propagate, propagate_rafixed, propagate_segments
from oracle.raycast import cast
from workloads import he_normal_mlp
from workloads.weights import MLPWeights


def _linear_net(a, b0):
    # a ReLU net that is affine on [-1, 1]^3: hidden neurons biased far positive
    W1 = np.array([a, [0.0, 0.0, 0.0]], dtype=np.float32)
    b1 = np.array([10.0, 10.0], dtype=np.float32)
    W2 = np.array([[1.0, 0.0]], dtype=np.float32)
    b2 = np.array([b0 - 10.0], dtype=np.float32)
    return MLPWeights(Ws=[W1, W2], bs=[b1, b2])


@pytest.mark.parametrize("method", [AA, UP, RAUA, RAFIXED])
def test_axis_segment_is_a_degenerate_box(method):
    mlp = he_normal_mlp([3, 32, 32, 1], seed=2)
    rng = np.random.default_rng(0)
    c = rng.uniform(-0.8, 0.8, (50, 3))
    for ax in range(3):
        v = np.zeros((50, 3))
        v[:, ax] = rng.uniform(0.001, 0.3, 50)
        got = propagate_segments(mlp, c, v, method)
        if method == RAFIXED:
            F0 = np.zeros((50, 3, 3))
            F0[:, ax, ax] = v[:, ax]
            ref = propagate_rafixed(mlp, c, F0)
        else:
            ref = propagate(mlp, c, np.abs(v), method)
        np.testing.assert_allclose(got[0], ref[0], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(got[1], ref[1], rtol=1e-12, atol=1e-12)


def test_linear_net_segments_are_exact():
    a = np.array([0.7, -0.4, 0.25])
    mlp = _linear_net(a, 0.1)
    rng = np.random.default_rng(1)
    c = rng.uniform(-0.5, 0.5, (40, 3))
    v = rng.normal(0, 0.2, (40, 3))
    av = np.abs(v @ a)
    for method, spread in ((AA, av), (RAFIXED, av), (UP, av / np.sqrt(3)), (RAUA, av / np.sqrt(3))):
        mu, sp = propagate_segments(mlp, c, v, method)
        np.testing.assert_allclose(mu, c @ a + 0.1, rtol=0, atol=1e-6)
        np.testing.assert_allclose(sp, spread, rtol=1e-6, atol=1e-12)


def test_rafixed_contains_aa_contains_samples():
    mlp = he_normal_mlp([3, 24, 24, 24, 1], seed=5)
    rng = np.random.default_rng(2)
    c = rng.uniform(-0.7, 0.7, (30, 3))
    v = rng.normal(0, 0.15, (30, 3))
    ma, ra = propagate_segments(mlp, c, v, AA)
    mf, rf = propagate_segments(mlp, c, v, RAFIXED)
    assert np.all(mf - rf <= ma - ra + 1e-12) and np.all(mf + rf >= ma + ra - 1e-12)
    e = np.linspace(-1, 1, 401)
    for i in range(30):
        vals = mlp_forward(mlp, c[i] + e[:, None] * v[i])
        assert vals.min() >= ma[i] - ra[i] - 1e-9 and vals.max() <= ma[i] + ra[i] + 1e-9
    # a short segment inside one linear region: both exact and equal
    mu_a, r_a = propagate_segments(mlp, c[:1], v[:1] * 1e-7, AA)
    mu_f, r_f = propagate_segments(mlp, c[:1], v[:1] * 1e-7, RAFIXED)
    assert mu_a[0] == pytest.approx(mu_f[0], abs=1e-12) and r_a[0] == pytest.approx(r_f[0], rel=1e-9)


def _rays(n, seed):
    rng = np.random.default_rng(seed)
    org = np.tile(np.array([0.1, -0.2, 2.5], np.float32), (n, 1))
    tgt = rng.uniform(-0.8, 0.8, (n, 3))
    d = tgt - org
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return org, d.astype(np.float32), np.full(n, 1.0, np.float32), np.full(n, 4.0, np.float32)


@pytest.mark.parametrize("method", [AA, RAFIXED, UP])
def test_linear_field_ray_hits_at_the_crossing(method):
    a = np.array([0.3, 0.5, 0.8])
    mlp = _linear_net(a, -0.05)
    org, d, tn, tf = _rays(64, 3)
    thit, steps, _ = cast(mlp, org, d, tn, tf, method, 3.0, 0.0, 1 / 16, 1 / 1024, 0.5, 2000)
    o64, d64 = org.astype(np.float64), d.astype(np.float64)
    tstar = (0.05 - o64 @ a) / (d64 @ a)
    crosses = (tstar >= tn) & (tstar <= tf)
    assert crosses.sum() > 20
    np.testing.assert_array_equal(np.isfinite(thit), crosses)
    # a segment of length de <= step_min whose bound (centre -/+ q |f'| de / 2,
    # q = 1 for the exact range, k / sqrt 3 for UP's soft bound) holds the
    # level has its midpoint within q de / 2 of the crossing
    q = 3.0 / np.sqrt(3.0) if method == UP else 1.0
    assert np.all(np.abs(thit[crosses] - tstar[crosses]) <= q * 0.5 / 1024 + 1e-6)


@pytest.mark.parametrize("method", [AA, RAFIXED])
def test_sound_ray_casting_never_skips_the_first_crossing(method):
    mlp = he_normal_mlp([3, 32, 32, 1], seed=7)
    iso = float(np.median(mlp_forward(mlp, np.random.default_rng(8).uniform(-1, 1, (4000, 3)))))
    org, d, tn, tf = _rays(48, 9)
    thit, steps, _ = cast(mlp, org, d, tn, tf, method, 1.0, iso, 1 / 16, 1 / 512, 0.5, 3000)
    ts = np.linspace(1.0, 4.0, 30001)
    for i in range(org.shape[0]):
        f = mlp_forward(mlp, org[i].astype(np.float64) + ts[:, None] * d[i].astype(np.float64)) - np.float32(iso)
        sc = np.nonzero(np.sign(f[1:]) != np.sign(f[:-1]))[0]
        if sc.size:
            assert np.isfinite(thit[i]) and thit[i] <= ts[sc[0] + 1] + 1.0 / 1024
