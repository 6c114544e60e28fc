"""Pins for the oracle's centre linearisation.

Fixed by things other than its own formula: central finite differences of the
plain MLP (exact for a piecewise-linear function inside one linear region),
the uncertainty propagation on tiny boxes (every neuron decided, so the
propagation becomes the tangent map), nets that are affine on the whole
domain, and a one-neuron net whose kink passes through the centre.
"""

import numpy as np
import pytest

from oracle.linearize import linearize
from oracle.mlp import mlp_forward
from oracle.propagate import UP, propagate
from workloads import he_normal_mlp, random_boxes, uniform_points

from test_oracle_propagate import _affine_on_domain_net


@pytest.mark.parametrize("widths", [[3, 16, 16, 1], [3, 64, 64, 64, 1], [3, 32, 24, 40, 1]])
def test_gradient_matches_finite_differences(widths):
    mlp = he_normal_mlp(widths, seed=7)
    c = uniform_points(300, seed=3)
    h = np.random.default_rng(4).uniform(1e-3, 0.2, (300, 3))
    f, s, margin = linearize(mlp, c, h, return_margin=True)
    np.testing.assert_allclose(f, mlp_forward(mlp, c), rtol=1e-12, atol=1e-12)
    d = 1e-6
    ok = margin > 1e-3  # no kink within +-d of the centre along any axis
    assert ok.mean() > 0.5
    grad = np.stack([(mlp_forward(mlp, c + d * e) - mlp_forward(mlp, c - d * e)) / (2 * d) for e in np.eye(3)], 1)
    s_fd = np.sqrt(np.sum((grad * h / np.sqrt(3.0)) ** 2, axis=1))
    np.testing.assert_allclose(s[ok], s_fd[ok], rtol=1e-6, atol=1e-9)


def test_tiny_boxes_equal_uncertainty_propagation():
    # on a box far smaller than the distance to the nearest kink every
    # neuron's Gaussian rule is the identity or zero, so the propagation is
    # exactly the tangent map
    mlp = he_normal_mlp([3, 32, 32, 32, 1], seed=11)
    c = uniform_points(200, seed=12)
    h = np.full((200, 3), 1e-8)
    f, s, margin = linearize(mlp, c, h, return_margin=True)
    ok = margin > 1e-4
    mu, sigma = propagate(mlp, c[ok], h[ok], UP)
    np.testing.assert_allclose(mu, f[ok], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(sigma, s[ok], rtol=1e-9)


@pytest.mark.parametrize("seed", [0, 1])
def test_affine_net_is_its_own_linearisation(seed):
    layers, A, a = _affine_on_domain_net(seed)
    c, h, _ = random_boxes(64, range(0, 6), seed=20 + seed)
    c = c.astype(np.float64)
    h = h.astype(np.float64)
    f, s = linearize(layers, c, h)
    np.testing.assert_allclose(f, c @ A + a, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(s, np.sqrt(np.sum((A * h) ** 2, axis=1) / 3.0), rtol=1e-12)
    mu, sigma = propagate(layers, c, h, UP)
    np.testing.assert_allclose(s, sigma, rtol=1e-9)


def test_kink_through_the_centre_counts_as_inactive():
    layers = [(np.array([[1.0, 0.0, 0.0]]), np.array([0.0])), (np.array([[2.0]]), np.array([0.5]))]
    c = np.array([[0.0, 0.3, 0.1], [0.25, 0.0, 0.0], [-0.25, 0.0, 0.0]])
    h = np.full((3, 3), 0.1)
    f, s = linearize(layers, c, h)
    np.testing.assert_allclose(f, [0.5, 1.0, 0.5])
    np.testing.assert_allclose(s, [0.0, 2.0 * 0.1 / np.sqrt(3.0), 0.0])
