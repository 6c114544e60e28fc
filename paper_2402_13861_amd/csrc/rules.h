// Linearisation rules of the activations (Eq. 4 for affine arithmetic,
// Eq. 9-10 and the App. D table for uncertainty propagation), shared by every
// propagation kernel in float32 and float64.
//
// Each rule replaces f(x) on a form with centre y by alpha x + beta plus one
// new independent symbol with coefficient gamma.
//  UP (Gaussian least squares under X ~ N(y, sigma^2)): alpha = Cov(X, f)/sigma^2,
//    beta = E f - alpha y, gamma^2 = Var f - alpha^2 sigma^2 (clamped at 0):
//    ReLU  alpha = Phi(r), beta = sigma phi(r), r = y / sigma,
//          gamma^2 = sigma^2 [(r^2+1) Phi Q + r phi (Q - Phi) - phi^2], Q = 1 - Phi
//          (one erfc: the smaller tail, the other as its complement);
//    sine  alpha = cos(y) e^{-s^2/2}, E f = sin(y) e^{-s^2/2},
//          E f^2 = (1 - cos(2y) e^{-2 s^2}) / 2;
//    ELU   (x for x > 0, e^x - 1 else) alpha = E f'(X) = Phi(r) + e^{y + s^2/2} Phi(-r - s),
//          E f = y Phi(r) + s phi(r) + e^{y + s^2/2} Phi(-r - s) - Phi(-r),
//          E f^2 = (y^2 + s^2) Phi(r) + y s phi(r) + e^{2y + 2s^2} Phi(-r - 2s)
//                  - 2 e^{y + s^2/2} Phi(-r - s) + Phi(-r);
//    a zero-width input takes the exact limit (the tangent; ReLU's alpha is
//    1/2 at y = 0).
//  AA (range [l, u] = [y - r, y + r]):
//    ReLU  the minimax line: alpha = u/(u-l), beta = gamma = -alpha l / 2 for
//          l < 0 < u, identity if l >= 0, 0 if u <= 0;
//    ELU   convex: the chord lowered by half its largest gap, which lies at
//          x* = ln(alpha) (identity if l >= 0);
//    sine  the chord slope, with beta and gamma from the exact extremes of
//          sin x - alpha x over [l, u] (end points and the points where
//          cos x = alpha); a range wider than 2 pi gives 0 +/- 1.
// The sine and ELU rules run in float64 (also inside float32 kernels), with
// the sine residual as a sum of non-negative terms and chord slopes in
// product forms, which avoid differences of nearly equal terms.
#pragma once

#include <hip/hip_runtime.h>

#include "isx.h"

namespace isx {

template <typename T>
struct RM;
template <>
struct RM<float> {
  __device__ static float erfc_(float x) { return erfcf(x); }
  __device__ static float exp_(float x) { return expf(x); }
  __device__ static float expm1_(float x) { return expm1f(x); }
  __device__ static float sqrt_(float x) { return sqrtf(x); }
  __device__ static float abs_(float x) { return fabsf(x); }
  __device__ static float sin_(float x) { return sinf(x); }
  __device__ static float cos_(float x) { return cosf(x); }
  __device__ static float sinh_(float x) { return sinhf(x); }
  __device__ static float acos_(float x) { return acosf(x); }
  __device__ static float log_(float x) { return logf(x); }
  __device__ static float ceil_(float x) { return ceilf(x); }
};
template <>
struct RM<double> {
  __device__ static double erfc_(double x) { return erfc(x); }
  __device__ static double exp_(double x) { return exp(x); }
  __device__ static double expm1_(double x) { return expm1(x); }
  __device__ static double sqrt_(double x) { return sqrt(x); }
  __device__ static double abs_(double x) { return fabs(x); }
  __device__ static double sin_(double x) { return sin(x); }
  __device__ static double cos_(double x) { return cos(x); }
  __device__ static double sinh_(double x) { return sinh(x); }
  __device__ static double acos_(double x) { return acos(x); }
  __device__ static double log_(double x) { return log(x); }
  __device__ static double ceil_(double x) { return ceil(x); }
};

// The activation itself (dense evaluation).
template <typename T>
__device__ __forceinline__ T activate(int act, T x) {
  if (act == ISX_SINE) return RM<T>::sin_(x);
  if (act == ISX_ELU) return x > T(0) ? x : RM<T>::expm1_(x);
  return x > T(0) ? x : T(0);
}

// Standard normal cdf from one erfc.
template <typename T>
__device__ __forceinline__ T norm_cdf(T x) {
  return T(0.5) * RM<T>::erfc_(-x * T(0.70710678118654752440));
}

template <typename T>
__device__ __forceinline__ void up_rule(int act, T y, T var, T& a, T& b, T& g) {
  using M = RM<T>;
  const T sigma = M::sqrt_(var > T(0) ? var : T(0));
  const T ay = M::abs_(y);
  if (!(sigma > T(1e-30) * (ay > T(1) ? ay : T(1)))) {  // zero width: the tangent
    if (act == ISX_SINE) {
      a = M::cos_(y);
      b = M::sin_(y) - a * y;
    } else if (act == ISX_ELU) {
      a = y > T(0) ? T(1) : M::exp_(y);
      b = y > T(0) ? T(0) : M::expm1_(y) - a * y;
    } else {
      a = y > T(0) ? T(1) : (y < T(0) ? T(0) : T(0.5));
      b = T(0);
    }
    g = T(0);
    return;
  }
  if (act == ISX_SINE) {
    const T e1 = M::exp_(T(-0.5) * var);
    const T sn = M::sin_(y), cs = M::cos_(y);
    a = cs * e1;
    const T mean = sn * e1;
    b = mean - a * y;
    // Var f - alpha^2 t (t = sigma^2) rewritten as a sum of non-negative
    // terms, e^{-t} [(sinh t - t) + S (e^{-t} - 1 + t)], S = sin^2 y, so that
    // small cells keep every digit
    const T t = var, S = sn * sn, et = M::exp_(-t);
    T q, bt;  // e^{-t} (sinh t - t) and e^{-t} - 1 + t
    if (t < T(1)) {
      const T t2 = t * t;
      // sinh t - t by its series (the first dropped term is below 1e-19 of the sum)
      const T sh = t * t2 / T(6) *
                   (T(1) + t2 / T(20) *
                               (T(1) + t2 / T(42) *
                                           (T(1) + t2 / T(72) *
                                                       (T(1) + t2 / T(110) *
                                                                   (T(1) + t2 / T(156) *
                                                                               (T(1) + t2 / T(210) *
                                                                                           (T(1) + t2 / T(272) * (T(1) + t2 / T(342)))))))));
      const T h = M::sinh_(T(0.5) * t);
      q = et * sh;
      bt = T(2) * h * h - sh;  // cosh t - 1 - (sinh t - t)
    } else {
      q = T(-0.5) * M::expm1_(T(-2) * t) - t * et;
      bt = M::expm1_(-t) + t;
    }
    const T g2 = q + S * et * bt;
    g = g2 > T(0) ? M::sqrt_(g2) : T(0);
    return;
  }
  const T r = y / sigma;
  const T phi = T(0.39894228040143267794) * M::exp_(T(-0.5) * r * r);
  if (act == ISX_ELU) {
    if (r >= T(8)) {  // the whole Gaussian on the identity side (tail < 7e-16)
      a = T(1);
      b = T(0);
      g = T(0);
      return;
    }
    if (r <= T(-8)) {
      // on the exponential side: lognormal moments, E e^X = e^{y + t/2},
      // Var e^X = e^{2y + t} (e^t - 1), alpha = E e^X, gamma^2 = e^{2y + t} (e^t - 1 - t)
      const T t = var;
      const T em = M::exp_(y + T(0.5) * t);
      a = em;
      b = (em - T(1)) - a * y;
      const T d = t < T(0.01) ? t * t * (T(0.5) + t * (T(1) / T(6) + t * (T(1) / T(24) + t / T(120))))
                              : M::expm1_(t) - t;
      const T g2 = em * em * d;
      g = g2 > T(0) ? M::sqrt_(g2) : T(0);
      return;
    }
    const T P = norm_cdf(r), Pm = norm_cdf(-r);
    const T e1 = M::exp_(y + T(0.5) * var) * norm_cdf(-r - sigma);
    const T e2 = M::exp_(T(2) * y + T(2) * var) * norm_cdf(-r - T(2) * sigma);
    const T m1 = y * P + sigma * phi + e1 - Pm;
    const T m2 = (y * y + var) * P + y * sigma * phi + e2 - T(2) * e1 + Pm;
    a = P + e1;
    b = m1 - a * y;
    const T g2 = m2 - m1 * m1 - a * a * var;
    g = g2 > T(0) ? M::sqrt_(g2) : T(0);
    return;
  }
  const T tail = T(0.5) * M::erfc_(M::abs_(r) * T(0.70710678118654752440));
  const T Phi = r >= T(0) ? T(1) - tail : tail;
  const T Q = r >= T(0) ? tail : T(1) - tail;
  a = Phi;
  b = sigma * phi;
  const T g2 = var * ((r * r + T(1)) * Phi * Q + r * phi * (Q - Phi) - phi * phi);
  g = g2 > T(0) ? M::sqrt_(g2) : T(0);
}

template <typename T>
__device__ __forceinline__ T elu_f(T x) {
  return x > T(0) ? x : RM<T>::expm1_(x);
}

template <typename T>
__device__ __forceinline__ void aa_rule_act(int act, T y, T rad, T& a, T& b, T& g) {
  using M = RM<T>;
  const T l = y - rad, u = y + rad;
  if (act == ISX_SINE) {
    if (!(rad > T(0))) {
      a = M::cos_(y);
      b = M::sin_(y) - a * y;
      g = T(0);
      return;
    }
    if (u - l > T(6.28318530717958647693)) {
      a = T(0);
      b = T(0);
      g = T(1);
      return;
    }
    // chord slope without the difference of sines: (sin u - sin l)/(u - l)
    // = cos(y) sin(rad)/rad; errors taken relative to the centre,
    // e(y + d) - e(y) = 2 cos(y + d/2) sin(d/2) - alpha d
    const T al = M::cos_(y) * (M::sin_(rad) / rad);
    auto ed = [&](T d) { return T(2) * M::cos_(y + T(0.5) * d) * M::sin_(T(0.5) * d) - al * d; };
    T emax = ed(-rad), emin = emax;
    const T eu = ed(rad);
    emax = eu > emax ? eu : emax;
    emin = eu < emin ? eu : emin;
    const T base = M::acos_(al > T(1) ? T(1) : (al < T(-1) ? T(-1) : al));
    const T two_pi = T(6.28318530717958647693);
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
      const T off = sg == 0 ? base : -base;
      T x = off + two_pi * M::ceil_((l - off) / two_pi);
      for (int it = 0; it < 3 && x <= u; ++it, x += two_pi) {
        const T e = ed(x - y);
        emax = e > emax ? e : emax;
        emin = e < emin ? e : emin;
      }
    }
    a = al;
    b = M::sin_(y) - al * y + T(0.5) * (emax + emin);
    g = T(0.5) * (emax - emin);
    return;
  }
  if (act == ISX_ELU) {
    if (l >= T(0)) {
      a = T(1);
      b = T(0);
      g = T(0);
      return;
    }
    if (!(rad > T(0))) {
      a = y > T(0) ? T(1) : M::exp_(y);
      b = elu_f(y) - a * y;
      g = T(0);
      return;
    }
    const T fl = elu_f(l);
    if (u <= T(0)) {
      // all on the exponential side: alpha = e^y sinh(rad)/rad and, with
      // e^{x*} = alpha, gap = alpha (e^dl - 1 - dl), dl = l - x* (no differences of
      // nearly equal exponentials)
      const T sh = rad < T(1e-2) ? T(1) + rad * rad / T(6) * (T(1) + rad * rad / T(20))
                                 : T(0.5) * (M::exp_(rad) - M::exp_(-rad)) / rad;
      const T al = M::exp_(y) * sh;
      const T dl = l - M::log_(al);
      const T em = M::abs_(dl) < T(1e-2) ? dl * dl * (T(0.5) + dl * (T(1) / T(6) + dl / T(24)))
                                         : M::expm1_(dl) - dl;
      const T gap = al * em;
      a = al;
      b = fl - al * l - T(0.5) * gap;
      g = T(0.5) * gap;
      return;
    }
    const T al = (elu_f(u) - fl) / (u - l);
    const T xs = M::log_(al);
    const T gap = fl + al * (xs - l) - elu_f(xs);
    a = al;
    b = fl - al * l - T(0.5) * gap;
    g = T(0.5) * gap;
    return;
  }
  if (u <= T(0)) {
    a = b = g = T(0);
  } else if (l >= T(0)) {
    a = T(1);
    b = g = T(0);
  } else {
    a = u / (u - l);
    b = -a * l * T(0.5);
    g = b;
  }
}

// Rule of METHOD (ISX_UP: stat = variance; otherwise AA: stat = radius).
// The sine and ELU rules are evaluated in float64 also for float32 kernels:
// their moments are differences of O(1) terms whose float32 rounding would
// dominate the O(sigma^2) results (one evaluation per neuron, beside the
// layer's products).
template <typename T, int METHOD>
__device__ __forceinline__ void apply_rule(int act, T y, T stat, T& a, T& b, T& g) {
  if (act != ISX_RELU && sizeof(T) == 4) {
    double ad, bd, gd;
    if (METHOD == ISX_UP)
      up_rule<double>(act, (double)y, (double)stat, ad, bd, gd);
    else
      aa_rule_act<double>(act, (double)y, (double)stat, ad, bd, gd);
    a = (T)ad;
    b = (T)bd;
    g = (T)gd;
    return;
  }
  if (METHOD == ISX_UP)
    up_rule<T>(act, y, stat, a, b, g);
  else
    aa_rule_act<T>(act, y, stat, a, b, g);
}

}  // namespace isx
