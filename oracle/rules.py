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
