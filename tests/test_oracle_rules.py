"""Pins for the oracle's ReLU linearisation rules.

The UP rule is checked against Eq. 10 solved by numerical quadrature (the
least-squares normal equations integrated against the Gaussian density), not
against its own closed form; the AA rule against the Chebyshev equioscillation
property and a brute-force minimax fit.
"""

import numpy as np
import pytest
from scipy import integrate
from scipy.optimize import linprog

from oracle.rules import relu_aa_rule, relu_up_rule, relu_up_rule_table_form


def _lsq_by_quadrature(mu, sigma):
    """argmin_{a,b} E[(relu(X) - a X - b)^2], X ~ N(mu, sigma^2), by quadrature
    of the moments, and the residual mean square at the optimum."""
    pdf = lambda x: np.exp(-0.5 * ((x - mu) / sigma) ** 2) / (sigma * np.sqrt(2 * np.pi))
    lim = (mu - 40 * sigma, mu + 40 * sigma)

    def E(g):
        pts = [0.0] if lim[0] < 0 < lim[1] else None
        return integrate.quad(lambda x: g(x) * pdf(x), *lim, points=pts, epsabs=0, epsrel=1e-12, limit=400)[0]

    relu = lambda x: max(x, 0.0)
    m1 = E(lambda x: x)
    m2 = E(lambda x: x * x)
    ef = E(relu)
    exf = E(lambda x: x * relu(x))
    # normal equations [[m2, m1],[m1, 1]] [a, b] = [exf, ef]
    a, b = np.linalg.solve(np.array([[m2, m1], [m1, 1.0]]), np.array([exf, ef]))
    mse = E(lambda x: (relu(x) - a * x - b) ** 2)
    return a, b, mse


@pytest.mark.parametrize("mu,sigma", [(0.0, 1.0), (0.3, 1.0), (-0.7, 0.5), (2.0, 1.5), (-3.0, 2.0), (1e-3, 2e-3),
                                      (4.0, 1.0), (-4.5, 1.0), (10.0, 7.0)])
def test_up_rule_matches_quadrature_of_eq10(mu, sigma):
    a, b, g2 = relu_up_rule(mu, sigma)
    qa, qb, qg2 = _lsq_by_quadrature(mu, sigma)
    assert abs(a - qa) < 1e-9
    assert abs(b - qb) < 1e-9 * max(1.0, sigma)
    assert abs(g2 - qg2) < 1e-9 * sigma ** 2


def test_up_rule_special_value():
    # mu = 0, sigma = 1: alpha = 1/2, beta = 1/sqrt(2 pi), gamma^2 = 1/4 - 1/(2 pi)
    a, b, g2 = relu_up_rule(0.0, 1.0)
    assert a == pytest.approx(0.5, abs=1e-15)
    assert b == pytest.approx(0.3989422804014327, abs=1e-15)
    assert g2 == pytest.approx(0.25 - 1.0 / (2 * np.pi), abs=1e-15)


def test_up_rule_symmetry():
    # relu(x) - relu(-x) = x  =>  alpha(mu)+alpha(-mu) = 1, beta and gamma^2 even in mu
    mu = np.linspace(-6, 6, 97)
    s = np.full_like(mu, 1.3)
    a1, b1, g1 = relu_up_rule(mu, s)
    a2, b2, g2 = relu_up_rule(-mu, s)
    np.testing.assert_allclose(a1 + a2, 1.0, atol=1e-15)
    np.testing.assert_allclose(b1, b2, rtol=1e-14)
    np.testing.assert_allclose(g1, g2, rtol=1e-9, atol=1e-300)


def test_up_rule_scale_equivariance():
    mu = np.linspace(-3, 3, 13)
    s = np.full_like(mu, 0.8)
    a1, b1, g1 = relu_up_rule(mu, s)
    a2, b2, g2 = relu_up_rule(5.0 * mu, 5.0 * s)
    np.testing.assert_allclose(a1, a2, rtol=1e-14)
    np.testing.assert_allclose(5.0 * b1, b2, rtol=1e-14)
    np.testing.assert_allclose(25.0 * g1, g2, rtol=1e-12)


def test_up_rule_equals_printed_table_in_well_conditioned_range():
    mu = np.linspace(-2.5, 2.5, 41)
    s = np.full_like(mu, 1.0)
    a, b, g = relu_up_rule(mu, s)
    ta, tb, tg = relu_up_rule_table_form(mu, s)
    np.testing.assert_allclose(a, ta, atol=1e-15)
    np.testing.assert_allclose(b, tb, atol=1e-15)
    np.testing.assert_allclose(g, tg, atol=1e-13)


def test_up_rule_degenerate_sigma():
    a, b, g = relu_up_rule(np.array([2.0, -2.0, 0.0]), np.zeros(3))
    np.testing.assert_array_equal(a, [1.0, 0.0, 0.5])
    np.testing.assert_array_equal(b, [0.0, 0.0, 0.0])
    np.testing.assert_array_equal(g, [0.0, 0.0, 0.0])


def test_up_rule_far_tails_nonnegative_and_small():
    mu = np.array([-12.0, -8.0, 8.0, 12.0, 40.0])
    a, b, g = relu_up_rule(mu, np.ones_like(mu))
    assert np.all(g >= 0.0)
    assert np.all(g < 1e-12)


def test_aa_rule_hand_example():
    # x = 1 + 2 eps -> [l, u] = [-1, 3]: 0.75 x + 0.375 + 0.375 eps', range [-0.75, 3]
    a, b, g = relu_aa_rule(1.0, 2.0)
    assert (a, b, g) == (0.75, 0.375, 0.375)
    centre = a * 1.0 + b
    radius = a * 2.0 + g
    assert (centre - radius, centre + radius) == (-0.75, 3.0)


def test_aa_rule_one_sided_ranges_are_exact():
    a, b, g = relu_aa_rule(np.array([-3.0, 3.0, -1.0, 1.0]), np.array([1.0, 1.0, 1.0, 1.0]))
    np.testing.assert_array_equal(a, [0.0, 1.0, 0.0, 1.0])
    np.testing.assert_array_equal(b, 0.0)
    np.testing.assert_array_equal(g, 0.0)


@pytest.mark.parametrize("l,u", [(-1.0, 3.0), (-2.0, 0.5), (-0.01, 5.0), (-7.0, 7.0)])
def test_aa_rule_is_minimax(l, u):
    a, b, g = relu_aa_rule((l + u) / 2, (u - l) / 2)
    x = np.linspace(l, u, 20001)
    err = np.maximum(x, 0) - (a * x + b)
    # sound: every error within gamma, and gamma is attained (equioscillation at l, 0, u)
    assert np.max(np.abs(err)) <= g * (1 + 1e-12)
    e = lambda t: max(t, 0.0) - (a * t + b)
    np.testing.assert_allclose([e(l), -e(0.0), e(u)], g, rtol=1e-12)
    # optimal: brute-force minimax line by LP over the sample points
    xs = np.union1d(np.linspace(l, u, 2001), [0.0])
    fx = np.maximum(xs, 0)
    # variables (a, b, t): minimise t s.t. |f - a x - b| <= t
    A = np.concatenate([np.stack([-xs, -np.ones_like(xs), -np.ones_like(xs)], 1),
                        np.stack([xs, np.ones_like(xs), -np.ones_like(xs)], 1)])
    rhs = np.concatenate([-fx, fx])
    res = linprog([0, 0, 1], A_ub=A, b_ub=rhs, bounds=[(None, None)] * 3)
    assert res.status == 0
    assert g == pytest.approx(res.x[2], rel=1e-5, abs=1e-8)
