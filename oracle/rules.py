"""ReLU linearisation rules, float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Two rules replace ReLU(x) on a form with centre ``mu`` by
``alpha * x + beta`` plus one new independent symbol with coefficient
``gamma``:

* affine arithmetic (Sec. III-A, Eq. 4): the minimax (Chebyshev) line over
  the hard range [l, u]; ``gamma`` is the maximum error;
* uncertainty propagation (Sec. IV-B, Eq. 9-10, App. D table, ReLU row): the
  least-squares line under X ~ N(mu, sigma^2); ``gamma^2`` is the variance of
  the residual.
"""

from __future__ import annotations

from math import factorial

import numpy as np
from scipy.special import erf, erfc

_SQRT2 = np.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / np.sqrt(2.0 * np.pi)


def relu_aa_rule(x0, r):
    """Chebyshev / minimax line for ReLU on [x0 - r, x0 + r] (Eq. 4).

    The paper names the Chebyshev approximation but does not print it for
    ReLU.  Reading: for l < 0 < u the best uniform line is the chord slope
    alpha = u/(u-l), shifted down by half of the chord's largest gap (at x=0),
    so beta = gamma = -alpha*l/2.  Wholly non-positive ranges map to 0,
    wholly non-negative ranges to the identity (both exact, gamma = 0).
    Returns (alpha, beta, gamma) arrays.
    """
    x0 = np.asarray(x0, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    l = x0 - r
    u = x0 + r
    alpha = np.zeros(np.broadcast(x0, r).shape)
    beta = np.zeros_like(alpha)
    gamma = np.zeros_like(alpha)
    pos = l >= 0.0
    straddle = (u > 0.0) & (l < 0.0)
    alpha[pos] = 1.0
    a = u[straddle] / (u[straddle] - l[straddle])
    alpha[straddle] = a
    beta[straddle] = -a * l[straddle] / 2.0
    gamma[straddle] = beta[straddle]
    return alpha, beta, gamma


def relu_up_rule(mu, sigma):
    """Gaussian least-squares line for ReLU (Eq. 10; App. D table, ReLU row).

    With r = mu/sigma, Phi/phi the standard normal cdf/pdf and Q = 1 - Phi:
      alpha   = Phi(r)                       (= (1 - a)/2, a = erf(-r/sqrt2))
      beta    = sigma * phi(r)
      gamma^2 = sigma^2 [ (r^2+1) Phi Q + r phi (Q - Phi) - phi^2 ]
    which is the table's expression with (1 - a^2)/4 written as Phi*Q from
    erfc (no 1 - erf^2 cancellation) and clamped at 0.  A zero-width input
    (sigma <= 1e-30 max(1,|mu|)) takes the exact limit: alpha = [mu > 0]
    (1/2 at mu = 0), beta = gamma = 0.
    Returns (alpha, beta, gamma2).
    """
    mu = np.asarray(mu, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    mu, sigma = np.broadcast_arrays(mu, sigma)
    alpha = np.empty(mu.shape)
    beta = np.zeros(mu.shape)
    gamma2 = np.zeros(mu.shape)
    degen = sigma <= 1e-30 * np.maximum(1.0, np.abs(mu))
    alpha[degen] = np.where(mu[degen] > 0, 1.0, np.where(mu[degen] < 0, 0.0, 0.5))
    ok = ~degen
    s = sigma[ok]
    r = mu[ok] / s
    Phi = 0.5 * erfc(-r / _SQRT2)
    Q = 0.5 * erfc(r / _SQRT2)
    phi = _INV_SQRT_2PI * np.exp(-0.5 * r * r)
    alpha[ok] = Phi
    beta[ok] = s * phi
    g2 = s * s * ((r * r + 1.0) * Phi * Q + r * phi * (Q - Phi) - phi * phi)
    gamma2[ok] = np.maximum(g2, 0.0)
    return alpha, beta, gamma2


def relu_up_rule_table_form(mu, sigma):
    """The App. D ReLU row exactly as printed (erf-based), for comparison:
    a = erf(-mu/(sqrt2 sigma)), alpha = (1-a)/2,
    beta = sigma/sqrt(2 pi) exp(-mu^2/(2 sigma^2)),
    gamma^2 = (1-a^2)(mu^2+sigma^2)/4 + a mu beta - beta^2."""
    mu = np.asarray(mu, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    a = erf(-mu / (_SQRT2 * sigma))
    alpha = 0.5 * (1.0 - a)
    beta = sigma * _INV_SQRT_2PI * np.exp(-mu * mu / (2.0 * sigma * sigma))
    gamma2 = 0.25 * (1.0 - a * a) * (mu * mu + sigma * sigma) + a * mu * beta - beta * beta
    return alpha, beta, gamma2


# ------------------------------------------------------------ Sine and ELU
# Both rules come from the definition of the Gaussian least-squares line
# (Eq. 10): under X ~ N(mu, sigma^2) the line alpha X + beta minimising
# E[(f(X) - alpha X - beta)^2] has alpha = Cov(X, f(X)) / sigma^2,
# beta = E f(X) - alpha mu, and residual variance
# gamma^2 = Var f(X) - alpha^2 sigma^2 (clamped at 0).  The moments are the
# standard Gaussian integrals written out below (App. D table, Sine and ELU
# rows; the table's ELU gamma^2 is replaced by this one, since the printed
# expression disagrees with the integrals).

def sine_up_rule(mu, sigma):
    """Gaussian least-squares line for sin (App. D table, Sine row).
    E sin X = sin(mu) e^{-s^2/2}; Cov(X, sin X) = s^2 cos(mu) e^{-s^2/2};
    E sin^2 X = (1 - cos(2 mu) e^{-2 s^2}) / 2.  Returns (alpha, beta, gamma2)."""
    mu = np.asarray(mu, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    e1 = np.exp(-0.5 * s * s)
    alpha = np.cos(mu) * e1
    mean = np.sin(mu) * e1
    beta = mean - alpha * mu
    # gamma^2 = Var sin X - alpha^2 t, t = s^2.  With Var sin X =
    # (1 - e^{-2t} cos 2 mu)/2 - e^{-t} sin^2 mu and cos 2 mu = 1 - 2 sin^2 mu it
    # equals e^{-t} (sinh t - t) + sin^2(mu) e^{-t} (e^{-t} - 1 + t): two
    # non-negative terms, so no digits are lost to cancellation for small t.
    t = s * s
    S = np.sin(mu) ** 2
    et = np.exp(-t)
    ts = np.minimum(t, 1.0)
    sh = np.zeros_like(ts)  # sinh t - t = sum_{k >= 1} t^(2k+1) / (2k+1)!
    for k in range(1, 13):
        sh = sh + ts ** (2 * k + 1) / factorial(2 * k + 1)
    em = np.zeros_like(ts)  # e^{-t} - 1 + t = sum_{k >= 2} (-t)^k / k!
    for k in range(2, 26):
        em = em + (-ts) ** k / factorial(k)
    small = t < 1.0
    q = np.where(small, et * sh, 0.5 * (1.0 - np.exp(-2.0 * t)) - t * et)  # e^{-t} (sinh t - t)
    bt = np.where(small, em, et - 1.0 + t)
    gamma2 = q + S * et * bt
    return alpha, beta, np.maximum(gamma2, 0.0)


def _phi_cdf(x):
    return 0.5 * erfc(-x / _SQRT2)


def elu_moments(mu, sigma):
    """E f, E f^2 and E f'(X) for ELU f(x) = x (x > 0), e^x - 1 (x <= 0)
    under X ~ N(mu, sigma^2), r = mu / sigma:
      E[X; X > 0]       = mu Phi(r) + sigma phi(r)
      E[X^2; X > 0]     = (mu^2 + sigma^2) Phi(r) + mu sigma phi(r)
      E[e^{cX}; X <= 0] = e^{c mu + c^2 sigma^2 / 2} Phi(-r - c sigma)."""
    mu = np.asarray(mu, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    r = mu / s
    Phi, Qm = _phi_cdf(r), _phi_cdf(-r)
    phi = _INV_SQRT_2PI * np.exp(-0.5 * r * r)
    e1 = np.exp(mu + 0.5 * s * s) * _phi_cdf(-r - s)
    e2 = np.exp(2.0 * mu + 2.0 * s * s) * _phi_cdf(-r - 2.0 * s)
    m1 = mu * Phi + s * phi + e1 - Qm
    m2 = (mu * mu + s * s) * Phi + mu * s * phi + e2 - 2.0 * e1 + Qm
    dmean = Phi + e1  # E f'(X): 1 on X > 0, e^X on X <= 0
    return m1, m2, dmean


def elu_up_rule(mu, sigma):
    """Gaussian least-squares line for ELU (App. D table, ELU row, with
    gamma^2 from the moments): by Stein's identity Cov(X, f(X)) =
    sigma^2 E f'(X), so alpha = E f'(X), beta = E f - alpha mu and
    gamma^2 = E f^2 - (E f)^2 - alpha^2 sigma^2.  A zero-width input takes
    the exact limit (alpha = f'(mu), beta = f(mu) - alpha mu, gamma = 0)."""
    mu = np.asarray(mu, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    mu, s = np.broadcast_arrays(mu, s)
    alpha = np.where(mu > 0, 1.0, np.exp(np.minimum(mu, 0.0)))
    beta = np.where(mu > 0, 0.0, np.expm1(np.minimum(mu, 0.0)) - alpha * mu)
    gamma2 = np.zeros(mu.shape)
    ok = s > 1e-30 * np.maximum(1.0, np.abs(mu))
    m1, m2, dm = elu_moments(mu[ok], s[ok])
    alpha = alpha.copy()
    beta = beta.copy()
    alpha[ok] = dm
    beta[ok] = m1 - dm * mu[ok]
    gamma2[ok] = np.maximum(m2 - m1 * m1 - dm * dm * s[ok] * s[ok], 0.0)
    return alpha, beta, gamma2


def elu_aa_rule(x0, r):
    """Minimax line for ELU on [l, u] = [x0 - r, x0 + r] (Eq. 4).  ELU is
    convex, so the chord lies above it and the best uniform line is the chord
    (slope alpha = (f(u) - f(l)) / (u - l)) lowered by half its largest gap,
    reached where f'(x*) = alpha (x* = ln alpha <= 0 when l < 0): gamma =
    gap/2.  l >= 0 is the identity; r = 0 is the tangent at x0."""
    shape = np.broadcast(np.asarray(x0), np.asarray(r)).shape
    x0, r = (np.atleast_1d(np.broadcast_to(np.asarray(v, dtype=np.float64), shape)).ravel() for v in (x0, r))
    f = lambda x: np.where(x > 0, x, np.expm1(np.minimum(x, 0.0)))
    l, u = x0 - r, x0 + r
    alpha = np.where(x0 > 0, 1.0, np.exp(np.minimum(x0, 0.0)))
    beta = f(x0) - alpha * x0
    gamma = np.zeros(x0.shape)
    pos = l >= 0
    alpha = np.where(pos, 1.0, alpha)
    beta = np.where(pos, 0.0, beta)
    w = (~pos) & (r > 0)
    if w.any():
        lw, uw = l[w], u[w]
        a = (f(uw) - f(lw)) / (uw - lw)
        xs = np.log(a)  # f'(xs) = a, xs in (l, 0]
        gap = f(lw) + a * (xs - lw) - f(xs)
        alpha[w] = a
        beta[w] = f(lw) - a * lw - 0.5 * gap
        gamma[w] = 0.5 * gap
    return alpha.reshape(shape), beta.reshape(shape), gamma.reshape(shape)


def sine_aa_rule(x0, r):
    """A sound linearisation of sin on [l, u] = [x0 - r, x0 + r] (Eq. 4 form):
    the chord slope alpha = (sin u - sin l) / (u - l) and, from the exact
    extremes of the error e(x) = sin x - alpha x over [l, u] (end points and
    the points where cos x = alpha), beta = (max e + min e) / 2 and gamma =
    (max e - min e) / 2.  Ranges wider than 2 pi take alpha = 0, beta = 0,
    gamma = 1 (sin's whole range); r = 0 is the tangent at x0."""
    shape = np.broadcast(np.asarray(x0), np.asarray(r)).shape
    x0, r = (np.atleast_1d(np.broadcast_to(np.asarray(v, dtype=np.float64), shape)).ravel() for v in (x0, r))
    alpha = np.cos(x0)
    beta = np.sin(x0) - alpha * x0
    gamma = np.zeros(x0.shape)
    wide = 2.0 * r > 2.0 * np.pi
    alpha = np.where(wide, 0.0, alpha)
    beta = np.where(wide, 0.0, beta)
    gamma = np.where(wide, 1.0, gamma)
    for idx in np.nonzero((~wide) & (r > 0))[0]:
        l, u = x0[idx] - r[idx], x0[idx] + r[idx]
        a = (np.sin(u) - np.sin(l)) / (u - l)
        pts = [l, u]
        base = np.arccos(np.clip(a, -1.0, 1.0))
        for sgn in (1.0, -1.0):
            k0 = np.ceil((l - sgn * base) / (2.0 * np.pi))
            x = sgn * base + 2.0 * np.pi * k0
            while x <= u:
                pts.append(x)
                x += 2.0 * np.pi
        e = np.sin(np.array(pts)) - a * np.array(pts)
        alpha[idx] = a
        beta[idx] = 0.5 * (e.max() + e.min())
        gamma[idx] = 0.5 * (e.max() - e.min())
    return alpha.reshape(shape), beta.reshape(shape), gamma.reshape(shape)


ACTIVATIONS = ("relu", "sine", "elu")


def activation(name, x):
    """The activation itself: ReLU, sin, or ELU (x for x > 0, e^x - 1 else)."""
    x = np.asarray(x, dtype=np.float64)
    if name == "relu":
        return np.maximum(x, 0.0)
    if name == "sine":
        return np.sin(x)
    if name == "elu":
        return np.where(x > 0, x, np.expm1(np.minimum(x, 0.0)))
    raise ValueError(name)


def up_rule(name, mu, sigma):
    return {"relu": relu_up_rule, "sine": sine_up_rule, "elu": elu_up_rule}[name](mu, sigma)


def aa_rule(name, x0, r):
    return {"relu": relu_aa_rule, "sine": sine_aa_rule, "elu": elu_aa_rule}[name](x0, r)
