"""Pins for the oracle's Sine and ELU rules (App. D table, Sine and ELU rows).

UP: the closed forms against Eq. 10 solved by numerical quadrature (the
least-squares normal equations integrated against the Gaussian density) and
special values; the printed ELU gamma^2 is shown to disagree with that
quadrature.  AA: soundness on dense samples of the range and, for the convex
ELU, optimality against a brute-force minimax fit.  Propagation: Monte Carlo
moments on tiny boxes, AA soundness under dense sampling, coefficient form
equal to covariance form.
"""

import numpy as np
import pytest
from scipy import integrate
from scipy.optimize import linprog

from oracle.mlp import mlp_forward
from oracle.propagate import AA, UP, propagate, propagate_up_covariance
from oracle.rules import activation, elu_aa_rule, elu_up_rule, sine_aa_rule, sine_up_rule
from workloads import he_normal_mlp, random_boxes

F = {"sine": np.sin, "elu": lambda x: x if x > 0 else np.expm1(x)}


def _lsq_by_quadrature(f, mu, sigma, kink=None):
    pdf = lambda x: np.exp(-0.5 * ((x - mu) / sigma) ** 2) / (sigma * np.sqrt(2 * np.pi))
    lim = (mu - 40 * sigma, mu + 40 * sigma)
    pts = [kink] if kink is not None and lim[0] < kink < lim[1] else None

    def E(g):
        return integrate.quad(lambda x: g(x) * pdf(x), *lim, points=pts, epsabs=0, epsrel=1e-12, limit=800)[0]

    m1, m2 = E(lambda x: x), E(lambda x: x * x)
    ef, exf = E(f), E(lambda x: x * f(x))
    a, b = np.linalg.solve(np.array([[m2, m1], [m1, 1.0]]), np.array([exf, ef]))
    return a, b, E(lambda x: (f(x) - a * x - b) ** 2)


@pytest.mark.parametrize("mu,sigma", [(0.0, 1.0), (0.3, 0.2), (-2.0, 0.7), (5.0, 2.0), (1.2, 0.05), (-0.4, 3.0)])
def test_sine_up_rule_matches_quadrature(mu, sigma):
    a, b, g2 = sine_up_rule(mu, sigma)
    qa, qb, qg2 = _lsq_by_quadrature(np.sin, mu, sigma)
    assert abs(a - qa) < 1e-9
    assert abs(b - qb) < 1e-9 * max(1.0, abs(mu))
    assert abs(g2 - qg2) < 1e-9


@pytest.mark.parametrize("sigma", [1e-7, 1e-5, 3e-4, 1e-2, 0.3, 0.999, 1.0, 1.7, 6.0])
def test_sine_residual_keeps_its_digits_for_small_cells(sigma):
    """gamma^2 = Var sin X - alpha^2 sigma^2 is O(sigma^4) (O(sigma^6) where
    sin mu = 0) while its two terms are O(sigma^2): the definition evaluated
    with 60-digit arithmetic, from E sin X = sin(mu) e^{-t/2} and
    E sin^2 X = (1 - cos(2 mu) e^{-2t})/2, t = sigma^2, pins the oracle's
    cancellation-free form to 1e-13 relative, at the series/closed-form switch
    (t = 1) too."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 60
    for mu in (0.0, 0.37, 1.0, np.pi / 2, -2.5, 7.0):
        _, _, g2 = sine_up_rule(mu, sigma)
        m, t = mp.mpf(mu), mp.mpf(sigma) ** 2
        mean = mp.sin(m) * mp.exp(-t / 2)
        var = (1 - mp.cos(2 * m) * mp.exp(-2 * t)) / 2 - mean ** 2
        ref = var - (mp.cos(m) * mp.exp(-t / 2)) ** 2 * t
        assert abs(g2 - float(ref)) <= 1e-13 * float(ref), (mu, sigma, g2, float(ref))


@pytest.mark.parametrize("mu,sigma", [(0.0, 1.0), (0.3, 0.2), (-2.0, 0.7), (5.0, 2.0), (-0.1, 0.05), (-4.0, 3.0)])
def test_elu_up_rule_matches_quadrature(mu, sigma):
    a, b, g2 = elu_up_rule(mu, sigma)
    qa, qb, qg2 = _lsq_by_quadrature(F["elu"], mu, sigma, kink=0.0)
    assert abs(a - qa) < 1e-9
    assert abs(b - qb) < 1e-9 * max(1.0, sigma)
    assert abs(g2 - qg2) < 1e-9 * max(1.0, sigma ** 2)


def test_printed_elu_gamma2_disagrees_with_the_integrals():
    """At mu = 0, sigma = 1 the quadrature gives gamma^2 = 0.0392 (this
    rule), while the table's printed expression evaluates to about -0.045,
    a negative variance; the rule therefore takes gamma^2 from the moments."""
    _, _, g2 = elu_up_rule(0.0, 1.0)
    _, _, qg2 = _lsq_by_quadrature(F["elu"], 0.0, 1.0, kink=0.0)
    assert g2 == pytest.approx(qg2, abs=1e-10)
    assert 0.039 < g2 < 0.0395


def test_sine_and_elu_special_values():
    # sin at mu = 0: alpha = e^{-s^2/2}, beta = 0, gamma^2 = (1 - e^{-2 s^2})/2 - s^2 e^{-s^2}
    s = 0.8
    a, b, g2 = sine_up_rule(0.0, s)
    assert a == pytest.approx(np.exp(-s * s / 2), abs=1e-15) and b == pytest.approx(0.0, abs=1e-15)
    assert g2 == pytest.approx(0.5 * (1 - np.exp(-2 * s * s)) - s * s * np.exp(-s * s), abs=1e-14)
    # ELU far on the positive side is the identity; a zero-width input is the tangent
    a, b, g2 = elu_up_rule(50.0, 1.0)
    assert a == pytest.approx(1.0, abs=1e-15) and abs(b) < 1e-12 and g2 < 1e-12
    a, b, g2 = elu_up_rule(-1.5, 0.0)
    assert a == pytest.approx(np.exp(-1.5)) and b == pytest.approx(np.expm1(-1.5) + 1.5 * np.exp(-1.5))
    assert g2 == 0.0


@pytest.mark.parametrize("name,l,u", [("sine", -0.3, 0.9), ("sine", 1.0, 4.0), ("sine", -5.0, 0.5), ("elu", -2.0, 1.5),
                                      ("elu", -4.0, -1.0), ("elu", 0.5, 2.0), ("sine", 2.0, 2.0)])
def test_aa_rules_sound_on_dense_samples(name, l, u):
    rule = {"sine": sine_aa_rule, "elu": elu_aa_rule}[name]
    a, b, g = rule((l + u) / 2, (u - l) / 2)
    x = np.linspace(l, u, 20001)
    err = activation(name, x) - (a * x + b)
    assert np.max(np.abs(err)) <= g * (1 + 1e-12) + 1e-15


@pytest.mark.parametrize("l,u", [(-2.0, 1.5), (-4.0, -1.0), (-0.3, 0.1)])
def test_elu_aa_rule_is_minimax(l, u):
    a, b, g = elu_aa_rule((l + u) / 2, (u - l) / 2)
    xs = np.linspace(l, u, 4001)
    fx = activation("elu", xs)
    A = np.concatenate([np.stack([-xs, -np.ones_like(xs), -np.ones_like(xs)], 1),
                        np.stack([xs, np.ones_like(xs), -np.ones_like(xs)], 1)])
    res = linprog([0, 0, 1], A_ub=A, b_ub=np.concatenate([-fx, fx]), bounds=[(None, None)] * 3)
    assert res.status == 0
    assert g == pytest.approx(res.x[2], rel=1e-5, abs=1e-9)


def _siren(widths, seed, w0=3.0):
    """A sine network in the SIREN layout (first layer scaled by w0, hidden
    layers U(-sqrt(6/n), sqrt(6/n))), w0 folded into the weights."""
    from workloads.weights import MLPWeights

    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for li, (i, o) in enumerate(zip(widths[:-1], widths[1:])):
        lim = w0 / i if li == 0 else np.sqrt(6.0 / i)
        Ws.append(rng.uniform(-lim, lim, (o, i)).astype(np.float32))
        bs.append(rng.uniform(-lim, lim, o).astype(np.float32))
    return MLPWeights(Ws=Ws, bs=bs)


@pytest.mark.parametrize("act", ["sine", "elu"])
def test_up_matches_monte_carlo_on_tiny_boxes(act):
    """On a tiny box a smooth activation is nearly affine, so UP's mean and
    sigma equal the Monte Carlo moments of f over the box (10^6 samples)."""
    mlp = _siren([3, 32, 32, 1], 4) if act == "sine" else he_normal_mlp([3, 32, 32, 1], seed=5)
    c, h, _ = random_boxes(3, [12], seed=6)
    mu, sigma = propagate(mlp, c, h, UP, act=act)
    rng = np.random.default_rng(7)
    for i in range(3):
        x = c[i].astype(float) + rng.uniform(-1, 1, (1_000_000, 3)) * h[i].astype(float)
        v = mlp_forward(mlp, x, act=act)
        assert abs(mu[i] - v.mean()) < 6 * v.std() / 1000 + 1e-12
        assert sigma[i] == pytest.approx(v.std(), rel=5e-3)


@pytest.mark.parametrize("act", ["sine", "elu"])
def test_aa_sound_and_forms_agree(act):
    mlp = _siren([3, 16, 16, 1], 8) if act == "sine" else he_normal_mlp([3, 16, 16, 1], seed=9)
    c, h, _ = random_boxes(30, range(0, 5), seed=10)
    x0, r = propagate(mlp, c, h, AA, act=act)
    unit = np.random.default_rng(11).uniform(-1, 1, (3000, 3))
    corners = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], dtype=float)
    unit = np.concatenate([unit, corners])
    for i in range(c.shape[0]):
        v = mlp_forward(mlp, c[i].astype(float) + unit * h[i].astype(float), act=act)
        tol = 1e-12 * max(1.0, abs(x0[i]) + r[i])
        assert v.min() >= x0[i] - r[i] - tol and v.max() <= x0[i] + r[i] + tol
    mu, sg = propagate(mlp, c, h, UP, act=act)
    mu2, sg2 = propagate_up_covariance(mlp, c, h, act=act)
    np.testing.assert_allclose(mu2, mu, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(sg2, sg, rtol=1e-10)
