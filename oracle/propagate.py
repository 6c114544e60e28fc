"""Layer-by-layer range analysis (AA) and uncertainty propagation (UP) of a
box through a ReLU MLP, float64, by explicit coefficient tracking.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A form is a centre vector x0 [n] and a coefficient matrix F [n, N] whose
column i multiplies symbol i (Eq. 1 for AA, eps_i in [-1, 1]; Eq. 6 for UP,
Z_i zero-mean, unit-variance, independent).

* Input form of a box with centre c and half-widths h (Sec. III-B for AA;
  Sec. IV-C and Alg. 1 for UP): x0 = c, F = diag(h) for AA and
  F = diag(h / sqrt 3) for UP (a uniform variable on [-h, h] has std h/sqrt 3).
* Linear layer y = W x + b (Eq. 3 / Eq. 8, exact): x0 <- W x0 + b, F <- W F.
* Activation (ReLU; or sine / ELU, App. D rows), per neuron j (Eq. 4 /
  Eq. 9): take (alpha_j, beta_j, gamma_j) from the rule, then x0_j <- alpha_j x0_j + beta_j, row j of F <- alpha_j * row j, and
  append one new symbol column whose only nonzero entry is gamma_j in row j.
  The rule's input is (x0_j, r_j = sum_i |F_ji|) for AA (Eq. 2 hard range)
  and (mu_j = x0_j, sigma_j = sqrt(sum_i F_ji^2)) for UP (Eq. 7, CLT).
* Output read-off: AA range [x0 - r, x0 + r] (Eq. 2); UP N(x0, sum F^2)
  (Eq. 7), whose soft bound is [mu - t sigma, mu + t sigma] (Alg. 1).

Both return (centre, spread): AA (x0, r), UP (mu, sigma), so that the bound
is centre -/+ k * spread with k = 1 for AA and k = t for UP.

Rounding margin for AA (``margin=True``; the paper assumes exact arithmetic,
this is the reading that keeps float bounds sound).  A linear layer computed
in floating point with unit roundoff u (and operands rounded with u_b) lands
within m_j = c (sum_k |W_jk| (rho_k + |x0_k|) + |b_j|) of the exact form,
with c = 2 u_b + u_b^2 + g_{K+1} (1 + u_b)^2 and g_n = n u / (1 - n u)
(K = layer input width, rho_k = sum_i |F_ki|).  That error is one more
independent symbol per neuron:
* the radius entering the ReLU rule is r_j (1 + 2 g_D) + m_j (the first
  factor covers the rounding of the D-term sum r_j itself);
* after the rule the error symbol is scaled by alpha_j and merged into the
  new symbol, gamma_j + alpha_j m_j, plus a slack of 8 u (alpha_j (|x0_j| +
  r_j) + |beta_j|) for the rounding of the rule, the centre update and the
  row scaling;
* the output radius gets the same widening, plus 4 u_32 (|x0| + r) so that a
  float32 read-off x0 -/+ r still contains the range.
The oracle applies it with float64 arithmetic (u = 2^-53, u_b = 0).
"""

from __future__ import annotations

import numpy as np

from .mlp import as_f64_layers
from .rules import aa_rule, relu_aa_rule, relu_up_rule, up_rule

AA = "aa"
UP = "up"
RAUA = "raua"  # AA propagation, uniform-assumption read-off (Sec. IV-A)
RAFIXED = "rafixed"  # input symbols kept, created symbols folded into one error term (App. A)


def _chunk_for(layers, budget_bytes=2.0e8):
    n_max = max(W.shape[0] for W, _ in layers)
    d_max = 3 + sum(W.shape[0] for W, _ in layers[:-1])
    return max(1, int(budget_bytes // (8 * n_max * d_max)))


U64 = 2.0 ** -53
U32 = 2.0 ** -24


def gamma_n(n, u):
    """n u / (1 - n u): the relative error bound of an n-term float sum."""
    return n * u / (1.0 - n * u)


def margin_const(K, u, u_b=0.0):
    """c of the AA rounding margin for a length-K product (bias included)."""
    return 2.0 * u_b + u_b * u_b + gamma_n(K + 1, u) * (1.0 + u_b) ** 2


def _track(layers, centres, halves, method, keep_hidden=False, margin=False, act="relu", F0=None):
    """Coefficient tracking for one chunk of boxes; returns (centre, spread)
    and optionally per-hidden-layer (pre-activation centre, row statistic).
    F0: an input coefficient block [C, 3, N0] in place of the box's
    diag(halves) (UP's 1/sqrt 3 included by the caller)."""
    C = centres.shape[0]
    s = 1.0 if method in (AA, RAUA) else 1.0 / np.sqrt(3.0)
    x0 = centres.copy()
    if F0 is not None:
        F = np.array(F0, dtype=np.float64)
    else:
        F = np.zeros((C, 3, 3))
        for i in range(3):
            F[:, i, i] = halves[:, i] * s
    hidden = []
    last = len(layers) - 1
    for li, (W, b) in enumerate(layers):
        m = None
        if margin:
            rho = np.abs(F).sum(axis=2)
            m = margin_const(W.shape[1], U64) * ((rho + np.abs(x0)) @ np.abs(W).T + np.abs(b))
        x0 = x0 @ W.T + b
        F = np.matmul(W, F)
        if li == last:
            break
        n = W.shape[0]
        if method == UP:
            stat = np.sqrt(np.einsum("cnd,cnd->cn", F, F))
            alpha, beta, gamma2 = up_rule(act, x0, stat)
            gamma = np.sqrt(gamma2)
        else:
            stat = np.abs(F).sum(axis=2)
            if margin:
                stat = stat * (1.0 + 2.0 * gamma_n(F.shape[2], U64)) + m
            alpha, beta, gamma = aa_rule(act, x0, stat)
            if margin:
                gamma = gamma + alpha * m + 8.0 * U64 * (alpha * (np.abs(x0) + stat) + np.abs(beta))
        if keep_hidden:
            hidden.append((x0.copy(), stat.copy()))
        x0 = alpha * x0 + beta
        F = alpha[:, :, None] * F
        G = np.zeros((C, n, n))
        G[:, np.arange(n), np.arange(n)] = gamma
        F = np.concatenate([F, G], axis=2)
    row = F[:, 0, :]
    if method == UP:
        spread = np.sqrt(np.einsum("cd,cd->c", row, row))
    elif method == AA:
        spread = np.abs(row).sum(axis=1)
        if margin:
            spread = spread * (1.0 + 2.0 * gamma_n(row.shape[1], U64)) + m[:, 0]
            spread = spread + 4.0 * U32 * (np.abs(x0[:, 0]) + spread)
    else:  # RA-UA: uniform variables on [-|x_i|, |x_i|] have variance x_i^2/3
        spread = np.sqrt(np.einsum("cd,cd->c", row, row) / 3.0)
    return x0[:, 0], spread, hidden


def propagate(layers, centres, halves, method: str, chunk: int | None = None, margin: bool = False,
              act: str = "relu"):
    """Propagate boxes through the MLP.

    centres, halves: [C, 3] (box centre and per-axis half-widths).
    method: ``AA`` (range analysis), ``UP`` (uncertainty propagation) or
    ``RAUA`` (range analysis with the uniform assumption read-off).
    margin: AA only, apply the rounding margin (module docstring).
    act: the hidden activation, ``relu``, ``sine`` or ``elu`` (App. D rows).
    Returns float64 (centre [C], spread [C]).
    """
    if margin and (method != AA or act != "relu"):
        raise ValueError("the rounding margin applies to AA on ReLU nets")
    layers = as_f64_layers(layers)
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    halves = np.asarray(halves, dtype=np.float64).reshape(-1, 3)
    chunk = chunk or _chunk_for(layers)
    cs, ss = [], []
    for a in range(0, centres.shape[0], chunk):
        c, s, _ = _track(layers, centres[a : a + chunk], halves[a : a + chunk], method, margin=margin, act=act)
        cs.append(c)
        ss.append(s)
    if not cs:
        return np.zeros(0), np.zeros(0)
    return np.concatenate(cs), np.concatenate(ss)


def propagate_segments(layers, centres, halfvecs, method: str, act: str = "relu"):
    """Propagate line segments {c + e v : e in [-1, 1]} (App. A's ray
    casting): one input symbol e, coefficient v (range analysis) or v/sqrt 3
    (UP: e uniform on [-1, 1]).  ``method``: AA, UP, RAUA or RAFIXED.
    Returns float64 (centre [C], spread [C])."""
    layers = as_f64_layers(layers)
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    v = np.asarray(halfvecs, dtype=np.float64).reshape(-1, 3)
    if method == RAFIXED:
        return propagate_rafixed(layers, centres, v[:, :, None], act=act)
    s = 1.0 if method in (AA, RAUA) else 1.0 / np.sqrt(3.0)
    if centres.shape[0] == 0:
        return np.zeros(0), np.zeros(0)
    c, sp, _ = _track(layers, centres, None, method, act=act, F0=v[:, :, None] * s)
    return c, sp


def propagate_rafixed(layers, centres, F0, act: str = "relu"):
    """RA-Fixed (the reduced affine form App. A compares with): the input
    symbols' coefficients A [C, n, N0] are tracked exactly, every symbol an
    activation creates is folded into one error magnitude e [C, n] per
    neuron.  Linear: x0 <- W x0 + b, A <- W A, e <- |W| e.  Activation: the
    affine rule of Eq. 4 on the range x0 -/+ (sum |A| + e), then
    x0 <- alpha x0 + beta, A <- alpha A, e <- |alpha| e + |gamma|.  Output:
    (x0, sum |A| + e), the hard range's centre and radius."""
    layers = as_f64_layers(layers)
    x0 = np.asarray(centres, dtype=np.float64).reshape(-1, 3).copy()
    A = np.array(F0, dtype=np.float64)
    e = np.zeros(x0.shape)
    last = len(layers) - 1
    for li, (W, b) in enumerate(layers):
        x0 = x0 @ W.T + b
        A = np.matmul(W, A)
        e = e @ np.abs(W).T
        r = np.abs(A).sum(axis=2) + e
        if li == last:
            return x0[:, 0], r[:, 0]
        alpha, beta, gamma = aa_rule(act, x0, r)
        x0 = alpha * x0 + beta
        A = alpha[:, :, None] * A
        e = np.abs(alpha) * e + np.abs(gamma)
    raise AssertionError("unreachable")


def propagate_hidden(layers, centres, halves, method: str, act: str = "relu"):
    """As ``propagate`` but also returns, per hidden layer, the pre-activation
    centre [C, n] and row statistic [C, n] (sigma for UP, r for AA)."""
    layers = as_f64_layers(layers)
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    halves = np.asarray(halves, dtype=np.float64).reshape(-1, 3)
    return _track(layers, centres, halves, method, keep_hidden=True, act=act)


def propagate_up_covariance(layers, centres, halves, act: str = "relu"):
    """UP written with the covariance of the symbols instead of the symbols.

    Since the symbols are independent with unit variance, only
    Sigma = F F^T enters sigma_j^2 = Sigma_jj (Eq. 7).  The rules become
    Sigma <- W Sigma W^T (linear) and
    Sigma <- D_alpha Sigma D_alpha + diag(gamma^2) (ReLU, Eq. 9).
    Exactly equal to coefficient tracking; used as an internal cross-check.
    """
    layers = as_f64_layers(layers)
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    halves = np.asarray(halves, dtype=np.float64).reshape(-1, 3)
    C = centres.shape[0]
    x0 = centres.copy()
    S = np.zeros((C, 3, 3))
    for i in range(3):
        S[:, i, i] = halves[:, i] ** 2 / 3.0
    last = len(layers) - 1
    for li, (W, b) in enumerate(layers):
        x0 = x0 @ W.T + b
        S = np.matmul(np.matmul(W, S), W.T)
        if li == last:
            break
        n = W.shape[0]
        sigma = np.sqrt(np.maximum(S[:, np.arange(n), np.arange(n)], 0.0))
        alpha, beta, gamma2 = up_rule(act, x0, sigma)
        x0 = alpha * x0 + beta
        S = alpha[:, :, None] * S * alpha[:, None, :]
        S[:, np.arange(n), np.arange(n)] += gamma2
    return x0[:, 0], np.sqrt(np.maximum(S[:, 0, 0], 0.0))


def bounds(centre, spread, k):
    """Bound read-off centre -/+ k * spread (AA: k = 1, Eq. 2; UP: k = t,
    Alg. 1 soft bound)."""
    return centre - k * spread, centre + k * spread
