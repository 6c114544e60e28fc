"""Pins for the oracle's layer-by-layer AA and UP propagation.

Each check is fixed by something other than the oracle's own formulas:
closed forms for nets that are affine on the box, the exact range of a tiny
net by linear programming over its activation patterns, dense sampling
(soundness of AA), invariances of the function (neuron rescaling and
permutation), a one-neuron net whose UP output equals the exact Gaussian
moments of ReLU by quadrature, Monte Carlo moments on tiny boxes, and the
exact centre of one-hidden-layer nets under UP's Gaussian input model on
boxes of any size.
"""

import itertools

import numpy as np
import pytest
from scipy import integrate
from scipy.optimize import linprog

from oracle.mlp import mlp_forward
from oracle.propagate import AA, UP, propagate, propagate_hidden, propagate_up_covariance
from workloads import he_normal_mlp, random_boxes
from workloads.weights import siren_mlp


def _affine_on_domain_net(seed, widths=(3, 8, 8, 1)):
    """An MLP whose every hidden pre-activation is > 0 on [-1,1]^3 (biases
    lifted above an interval bound), so ReLU is the identity there and the
    net is the affine map A x + a.  The lift is large enough that the UP
    rule also sees every neuron as fully on."""
    rng = np.random.default_rng(seed)
    layers = []
    lo, hi = -np.ones(3), np.ones(3)
    for li, (i, o) in enumerate(zip(widths[:-1], widths[1:])):
        W = rng.standard_normal((o, i))
        b = rng.standard_normal(o)
        if li + 1 < len(widths) - 1:
            Wp, Wn = np.maximum(W, 0), np.minimum(W, 0)
            pre_lo = Wp @ lo + Wn @ hi + b
            # every neuron positive on the box, and so far from 0 (mu/sigma >= 60)
            # that the Gaussian rule's alpha = Phi(mu/sigma) is 1 in float64
            width = (Wp @ hi + Wn @ lo - (Wp @ lo + Wn @ hi)).max()
            b = b - pre_lo.min() + 60.0 * width + 0.5
            pre_lo = Wp @ lo + Wn @ hi + b
            pre_hi = Wp @ hi + Wn @ lo + b
            lo, hi = pre_lo, pre_hi
            assert np.all(lo > 0)
        layers.append((W, b))
    A = np.eye(3)
    a = np.zeros(3)
    for W, b in layers:
        A = W @ A
        a = W @ a + b
    return layers, A[0], a[0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_affine_net_closed_forms(seed):
    layers, A, a = _affine_on_domain_net(seed)
    c, h, _ = random_boxes(64, range(0, 6), seed=10 + seed)
    c = c.astype(np.float64)
    h = h.astype(np.float64)
    mu, sigma = propagate(layers, c, h, UP)
    x0, r = propagate(layers, c, h, AA)
    f = c @ A + a
    np.testing.assert_allclose(mu, f, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(x0, f, rtol=1e-12, atol=1e-12)
    # UP: X_i uniform on [c_i - h_i, c_i + h_i] -> var = sum (A_i h_i)^2 / 3 (Eq. 8 exact)
    np.testing.assert_allclose(sigma, np.sqrt(((A * h) ** 2).sum(1) / 3.0), rtol=1e-12)
    # AA: the exact range of an affine function over the box (Eq. 3 exact)
    np.testing.assert_allclose(r, np.abs(A * h).sum(1), rtol=1e-12)


def test_dead_layer_gives_constant():
    rng = np.random.default_rng(3)
    W1 = rng.standard_normal((6, 3))
    b1 = -1000.0 * np.ones(6)  # all neurons off on [-1,1]^3, far beyond the Gaussian tails
    W2 = rng.standard_normal((1, 6))
    b2 = np.array([0.25])
    c, h, _ = random_boxes(16, range(0, 4), seed=4)
    for m in (UP, AA):
        cen, spr = propagate([(W1, b1), (W2, b2)], c, h, m)
        np.testing.assert_array_equal(cen, 0.25)
        np.testing.assert_array_equal(spr, 0.0)


def _exact_range_tiny(layers, c, h):
    """Exact [min, max] of a 3->n->1 ReLU net over a box by LP per pattern."""
    (W1, b1), (W2, b2) = layers
    n = W1.shape[0]
    lo_all, hi_all = np.inf, -np.inf
    bounds = [(c[i] - h[i], c[i] + h[i]) for i in range(3)]
    for pat in itertools.product([0, 1], repeat=n):
        s = np.array(pat, dtype=float)
        # on pattern s: f = W2 diag(s) (W1 x + b1) + b2, with (W1 x + b1)_j >= 0 iff s_j
        g = (W2[0] * s) @ W1
        g0 = (W2[0] * s) @ b1 + b2[0]
        # constraints: s_j=1 -> -(W1 x + b1) <= 0 ; s_j=0 -> W1 x + b1 <= 0
        sign = np.where(s > 0, -1.0, 1.0)
        A_ub = sign[:, None] * W1
        b_ub = -sign * b1
        rmin = linprog(g, A_ub=A_ub, b_ub=b_ub, bounds=bounds)
        if rmin.status != 0:
            continue  # pattern infeasible on this machine
        rmax = linprog(-g, A_ub=A_ub, b_ub=b_ub, bounds=bounds)
        lo_all = min(lo_all, rmin.fun + g0)
        hi_all = max(hi_all, -rmax.fun + g0)
    return lo_all, hi_all


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_aa_contains_exact_range_of_tiny_net(seed):
    mlp = he_normal_mlp([3, 4, 1], seed=seed)
    layers = [(W.astype(float), b.astype(float)) for W, b in mlp.layers()]
    c, h, _ = random_boxes(6, range(0, 3), seed=100 + seed)
    x0, r = propagate(layers, c, h, AA)
    for i in range(c.shape[0]):
        lo, hi = _exact_range_tiny(layers, c[i].astype(float), h[i].astype(float))
        assert x0[i] - r[i] <= lo + 1e-12
        assert hi <= x0[i] + r[i] + 1e-12


@pytest.mark.parametrize("seed", [0, 5])
def test_aa_sound_under_dense_sampling(seed):
    mlp = he_normal_mlp([3, 16, 16, 16, 1], seed=seed)
    c, h, _ = random_boxes(40, range(0, 5), seed=200 + seed)
    x0, r = propagate(mlp, c, h, AA)
    g = np.linspace(-1, 1, 17)
    grid = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    rnd = np.random.default_rng(seed).uniform(-1, 1, (4000, 3))
    unit = np.concatenate([grid, rnd])
    for i in range(c.shape[0]):
        pts = c[i].astype(float) + unit * h[i].astype(float)
        v = mlp_forward(mlp, pts)
        tol = 1e-12 * max(1.0, abs(x0[i]) + r[i])
        assert v.min() >= x0[i] - r[i] - tol
        assert v.max() <= x0[i] + r[i] + tol


@pytest.mark.parametrize("widths", [(3, 16, 16, 1), (3, 32, 32, 32, 1), (3, 8, 8, 8, 8, 8, 1)])
def test_up_coefficient_form_equals_covariance_form(widths):
    mlp = he_normal_mlp(list(widths), seed=7)
    c, h, _ = random_boxes(50, range(0, 7), seed=8)
    mu, sigma = propagate(mlp, c, h, UP)
    mu2, sigma2 = propagate_up_covariance(mlp, c, h)
    np.testing.assert_allclose(mu, mu2, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(sigma, sigma2, rtol=1e-9, atol=1e-13)


@pytest.mark.parametrize("method", [UP, AA])
def test_neuron_rescaling_invariance(method):
    # relu(l x) = l relu(x) for l > 0: scaling row j of (W_l, b_l) by l_j and
    # column j of W_{l+1} by 1/l_j leaves the function AND both propagations unchanged
    mlp = he_normal_mlp([3, 16, 16, 1], seed=11)
    layers = [(W.astype(float), b.astype(float)) for W, b in mlp.layers()]
    lam = np.random.default_rng(0).uniform(0.25, 4.0, 16)
    scaled = [list(p) for p in layers]
    scaled[1] = [layers[1][0] * lam[:, None], layers[1][1] * lam]
    scaled[2] = [layers[2][0] / lam[None, :], layers[2][1]]
    c, h, _ = random_boxes(40, range(0, 6), seed=12)
    a = propagate(layers, c, h, method)
    b = propagate([tuple(p) for p in scaled], c, h, method)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(a[1], b[1], rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("method", [UP, AA])
def test_neuron_permutation_invariance(method):
    mlp = he_normal_mlp([3, 12, 12, 1], seed=13)
    layers = [(W.astype(float), b.astype(float)) for W, b in mlp.layers()]
    p = np.random.default_rng(1).permutation(12)
    perm = [(layers[0][0][p], layers[0][1][p]), (layers[1][0][:, p], layers[1][1]), layers[2]]
    c, h, _ = random_boxes(30, range(0, 6), seed=14)
    a = propagate(layers, c, h, method)
    b = propagate(perm, c, h, method)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(a[1], b[1], rtol=1e-12, atol=1e-12)


def test_single_neuron_up_matches_gaussian_relu_moments():
    # 3 -> 1 -> 1: the output form is w (alpha Y + beta) + b + w gamma Z, whose
    # mean / variance must be w E[relu(Y)] + b and w^2 Var[relu(Y)] for
    # Y ~ N(mu_Y, sigma_Y^2) (least squares keeps the first two moments).
    W1 = np.array([[0.7, -1.2, 0.4]])
    b1 = np.array([0.1])
    w2 = np.array([[-1.7]])
    b2 = np.array([0.3])
    c = np.array([[0.05, -0.1, 0.2], [0.6, 0.6, -0.6], [-0.3, 0.8, 0.1]])
    h = np.array([[0.3, 0.3, 0.3], [0.05, 0.05, 0.05], [0.6, 0.6, 0.6]])
    mu, sigma = propagate([(W1, b1), (w2, b2)], c, h, UP)
    for i in range(3):
        my = W1[0] @ c[i] + b1[0]
        sy = np.sqrt(((W1[0] * h[i]) ** 2).sum() / 3.0)
        pdf = lambda x: np.exp(-0.5 * ((x - my) / sy) ** 2) / (sy * np.sqrt(2 * np.pi))
        lim = (my - 40 * sy, my + 40 * sy)
        pts = [0.0] if lim[0] < 0 < lim[1] else None
        m1 = integrate.quad(lambda x: max(x, 0) * pdf(x), *lim, points=pts, epsabs=0, epsrel=1e-12, limit=300)[0]
        m2 = integrate.quad(lambda x: max(x, 0) ** 2 * pdf(x), *lim, points=pts, epsabs=0, epsrel=1e-12, limit=300)[0]
        assert mu[i] == pytest.approx(w2[0, 0] * m1 + b2[0], rel=1e-10, abs=1e-12)
        assert sigma[i] == pytest.approx(abs(w2[0, 0]) * np.sqrt(m2 - m1 ** 2), rel=1e-8)


def test_up_matches_monte_carlo_on_tiny_boxes():
    # Tiny boxes with no kink inside: f is affine there, so UP must equal the
    # Monte Carlo mean/std of f(X), X uniform in the box (10^6 samples, Sec. V-E).
    mlp = he_normal_mlp([3, 32, 32, 1], seed=21)
    c, h, _ = random_boxes(64, [14], seed=22)
    mu, sigma = propagate(mlp, c, h, UP)
    rng = np.random.default_rng(23)
    checked = 0
    for i in range(c.shape[0]):
        x = c[i].astype(float) + rng.uniform(-1, 1, (1_000_000, 3)) * h[i].astype(float)
        # kink check: activation pattern constant over the samples
        pre = x @ mlp.Ws[0].astype(float).T + mlp.bs[0].astype(float)
        if not (np.all(pre > 0, axis=0) | np.all(pre < 0, axis=0)).all():
            continue
        v = mlp_forward(mlp, x)
        se = v.std() / np.sqrt(v.size)
        assert abs(mu[i] - v.mean()) < 6 * se + 1e-12
        assert sigma[i] == pytest.approx(v.std(), rel=5e-3)
        checked += 1
        if checked == 4:
            break
    assert checked >= 2


def test_up_close_to_monte_carlo_on_wide_box():
    # Sanity (not exact): on a wide box the Gaussian estimate is near the MC
    # moments for a random 3->64->64->1 net (Sec. V-E reports small KL).
    mlp = he_normal_mlp([3, 64, 64, 1], seed=0)
    c = np.array([[0.1, -0.2, 0.3]])
    h = np.array([[0.25, 0.25, 0.25]])
    mu, sigma = propagate(mlp, c, h, UP)
    x = c + np.random.default_rng(1).uniform(-1, 1, (400_000, 3)) * h
    v = mlp_forward(mlp, x)
    assert abs(mu[0] - v.mean()) < 0.25 * v.std()
    assert 0.5 < sigma[0] / v.std() < 2.0


def test_hidden_statistics_shapes_and_first_layer_closed_form():
    mlp = he_normal_mlp([3, 10, 10, 1], seed=2)
    c, h, _ = random_boxes(5, range(0, 4), seed=3)
    _, _, hidden = propagate_hidden(mlp, c, h, UP)
    assert len(hidden) == 2
    y1, s1 = hidden[0]
    W1 = mlp.Ws[0].astype(float)
    np.testing.assert_allclose(y1, c @ W1.T + mlp.bs[0], rtol=1e-12)
    np.testing.assert_allclose(s1, np.sqrt((W1[None] * h[:, None, :] ** 2 * W1[None]).sum(-1) / 3), rtol=1e-12)


@pytest.mark.parametrize("seed", [0, 3])
def test_aa_margin_widens_by_a_tiny_amount(seed):
    """The rounding margin (float64 arithmetic, float32 read-off slack)
    contains the unwidened AA range and moves it by about 1e-7 relative."""
    mlp = he_normal_mlp([3, 32, 32, 32, 1], seed=seed)
    c, h, _ = random_boxes(60, range(0, 8), seed=300 + seed)
    x0, r = propagate(mlp, c, h, AA)
    x0m, rm = propagate(mlp, c, h, AA, margin=True)
    scale = np.abs(x0) + r
    # a wider ReLU range gives a slightly different line, so the centre moves
    # too; the widened range contains the plain one
    assert (x0m - rm <= x0 - r).all() and (x0m + rm >= x0 + r).all()
    assert (np.abs(x0m - x0) + np.abs(rm - r) <= 1e-6 * scale).all()


def test_aa_margin_keeps_tight_ranges_sound_in_float32():
    """On boxes where the net is affine (every neuron active), AA is exact
    and its range is attained at box corners.  The same arithmetic in float32
    then misses corner values by a rounding error, which the margin covers."""
    from oracle.mlp import as_f64_layers

    rng = np.random.default_rng(11)
    widths = [3, 24, 24, 24, 1]
    layers = []
    for a, b in zip(widths[:-1], widths[1:]):
        W = rng.uniform(0.0, 1.0, (b, a)) / a
        layers.append((W, rng.uniform(0.5, 1.0, b)))
    layers = as_f64_layers(layers)
    c = rng.uniform(-0.5, 0.5, (40, 3))
    h = np.full((40, 3), 0.25)
    x0, r = propagate(layers, c, h, AA)
    x0m, rm = propagate(layers, c, h, AA, margin=True)
    corners = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], dtype=float)
    for i in range(c.shape[0]):
        v = mlp_forward(layers, c[i] + corners * h[i])
        # exact: the range is attained
        assert abs(v.max() - (x0[i] + r[i])) <= 1e-12 * (abs(x0[i]) + r[i])
        assert abs(v.min() - (x0[i] - r[i])) <= 1e-12 * (abs(x0[i]) + r[i])
        # the widened float64 range contains it with room for float32 read-off
        lo32, hi32 = np.float32(x0m[i]) - np.float32(rm[i]), np.float32(x0m[i]) + np.float32(rm[i])
        assert lo32 <= v.min() and v.max() <= hi32


def _bf16(x):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("K", [3, 64, 256, 1027])
def test_aa_margin_constant_bounds_float32_and_bf16_products(K):
    """c of the margin bounds the error of a float32 dot product (sequential
    float32 sum, optional bfloat16 operands) against the exact product of the
    unrounded operands: |fl(w.x + b) - (w.x + b)| <= c (sum |w||x| + |b|)."""
    from oracle.propagate import U32, margin_const

    rng = np.random.default_rng(K)
    for trial in range(200):
        w = rng.standard_normal(K).astype(np.float32)
        x = (rng.standard_normal(K) * rng.uniform(0.1, 10)).astype(np.float32)
        b = np.float32(rng.standard_normal())
        exact = float(np.dot(w.astype(np.float64), x.astype(np.float64))) + float(b)
        scale = float(np.abs(w.astype(np.float64)) @ np.abs(x.astype(np.float64))) + abs(float(b))
        for u_b in (0.0, 2.0 ** -8):
            wr, xr = (w, x) if u_b == 0 else (_bf16(w).astype(np.float32), _bf16(x).astype(np.float32))
            acc = np.float32(0)
            for k in range(K):  # float32 products and sums, in order
                acc = np.float32(acc + np.float32(wr[k] * xr[k]))
            acc = np.float32(acc + b)
            assert abs(float(acc) - exact) <= margin_const(K, U32, u_b) * scale, (trial, u_b)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_raua_affine_net_closed_form(seed):
    """RA-UA (Sec. IV-A, Eq. 5): affine-arithmetic coefficients read off as
    independent uniform variables, variance x_i^2 / 3 each.  On a net that is
    affine on the box the AA coefficients are exactly A_i h_i, so the read-off
    is N(f(c), sum (A_i h_i)^2 / 3) -- the exact mean and variance of f under
    a uniform input on the box."""
    from oracle.propagate import RAUA

    layers, A, a = _affine_on_domain_net(seed)
    c, h, _ = random_boxes(64, range(0, 6), seed=20 + seed)
    c = c.astype(np.float64)
    h = h.astype(np.float64)
    mu, sigma = propagate(layers, c, h, RAUA)
    np.testing.assert_allclose(mu, c @ A + a, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(sigma, np.sqrt(((A * h) ** 2).sum(1) / 3.0), rtol=1e-12)


def test_raua_one_kink_hand_example():
    """One ReLU neuron on the pre-activation 1 + 2 eps_1 (range [-1, 3]):
    the Chebyshev rule gives 0.75 x + 0.375 + 0.375 eps', so the output form
    is 1.125 + 1.5 eps_1 + 0.375 eps'.  RA-UA reads it as mean 1.125 and
    variance (1.5^2 + 0.375^2) / 3 = 0.796875; AA's radius is 1.875."""
    from oracle.propagate import RAUA

    layers = [(np.array([[1.0, 0.0, 0.0]]), np.array([0.0])), (np.array([[1.0]]), np.array([0.0]))]
    c = np.array([[1.0, 0.3, -0.2]])
    h = np.array([[2.0, 0.5, 0.25]])
    mu, sigma = propagate(layers, c, h, RAUA)
    assert mu[0] == pytest.approx(1.125, abs=1e-15)
    assert sigma[0] == pytest.approx(np.sqrt(0.796875), rel=1e-15)
    x0, r = propagate(layers, c, h, AA)
    assert x0[0] == pytest.approx(1.125, abs=1e-15)
    assert r[0] == pytest.approx(1.875, rel=1e-15)


@pytest.mark.parametrize("seed", [3, 4])
def test_raua_between_aa_radius_bounds(seed):
    """RA-UA and AA share the coefficients x_i (N of them), so by the norm
    inequalities r / sqrt(3 N) <= sigma_RAUA <= r / sqrt(3) with r = sum |x_i|,
    and the centres are equal."""
    from oracle.propagate import RAUA

    widths = [3, 16, 16, 1]
    mlp = he_normal_mlp(widths, seed=seed)
    c, h, _ = random_boxes(200, range(0, 6), seed=seed)
    mu, sigma = propagate(mlp, c, h, RAUA)
    x0, r = propagate(mlp, c, h, AA)
    np.testing.assert_array_equal(mu, x0)
    n_sym = 3 + sum(widths[1:-1])
    assert np.all(sigma <= r / np.sqrt(3.0) * (1 + 1e-12))
    assert np.all(sigma >= r / np.sqrt(3.0 * n_sym) * (1 - 1e-12))


@pytest.mark.parametrize("act", ["relu", "sine", "elu"])
def test_up_mean_exact_for_one_hidden_layer_under_gaussian_input(act):
    # UP models the box as a Gaussian with the uniform variable's mean and
    # variance (Eq. 6 with the input scale h/sqrt(3)).  With one hidden layer
    # every pre-activation is then exactly Gaussian, each per-neuron rule
    # keeps the mean of the activation (App. D), and the output layer is
    # linear, so UP's centre equals E[f(X)], X ~ N(c, diag(h^2/3)), on boxes
    # of any size, kinks and sine periods inside included.  Checked against
    # Monte Carlo at 6 standard errors on the whole domain and half of it.
    if act == "sine":
        mlp = siren_mlp([3, 64, 1], seed=4, w0=12.0)
    else:
        mlp = he_normal_mlp([3, 64, 1], seed=4)
    c = np.array([[0.0, 0.0, 0.0], [0.5, -0.5, 0.5], [-0.3, 0.2, 0.1]])
    h = np.array([[1.0, 1.0, 1.0], [0.5, 0.5, 0.5], [0.25, 0.5, 1.0]])
    mu, sigma = propagate(mlp, c, h, UP, act=act)
    rng = np.random.default_rng(31)
    for i in range(c.shape[0]):
        x = c[i] + rng.standard_normal((2_000_000, 3)) * (h[i] / np.sqrt(3.0))
        v = mlp_forward(mlp, x, act=act)
        se = v.std() / np.sqrt(v.size)
        assert abs(mu[i] - v.mean()) < 6 * se, (act, i, mu[i], v.mean(), se)
        # the spread is not exact (cross terms of the linearised neurons), but
        # stays near the Gaussian-input standard deviation
        assert 0.5 < sigma[i] / v.std() < 2.0


def test_up_mean_misses_monte_carlo_with_two_hidden_layers():
    # The exactness above rests on the single hidden layer: with two, layer 2
    # sees a non-Gaussian input, and on the whole domain the centre differs
    # from the Gaussian-input mean by many standard errors.  This keeps the
    # test above from passing on a Monte Carlo tolerance that is too loose.
    mlp = he_normal_mlp([3, 64, 64, 1], seed=4)
    c = np.zeros((1, 3))
    h = np.ones((1, 3))
    mu, _ = propagate(mlp, c, h, UP)
    x = np.random.default_rng(31).standard_normal((2_000_000, 3)) / np.sqrt(3.0)
    v = mlp_forward(mlp, x)
    assert abs(mu[0] - v.mean()) > 20 * v.std() / np.sqrt(v.size)
