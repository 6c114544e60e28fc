// Rounding margin of affine arithmetic in floating point (the paper assumes
// exact arithmetic for Eq. 1-4; this keeps the float32 / bfloat16 / float64
// ranges sound).
//
// A linear layer z -> W z + b evaluated with unit roundoff u (operands rounded
// with u_b) lands within
//   m_j = c sum_k |W_jk| rho_k + c_z (sum_k |W_jk| |z_k| + |b_j|),
//   c = 2 u_b + u_b^2 + g_{K+1} (1 + u_b)^2,   g_n = n u / (1 - n u),
// of the exact form, where z and rho_k (the sum of |coefficients| of input
// component k) describe the layer's input form.  The operand rounding u_b
// applies only to products whose operands are rounded: the bfloat16 path
// multiplies coefficients with bfloat16 operands but computes the centre
// W z + b with float32 weights, so its centre term takes c_z = g_{K+1}
// (c_z = c wherever u_b = 0).  That error is one more
// independent symbol per neuron, so after the hidden kernel has written the
// pre-activation centre y_j and its float row statistic r_j:
//   * the ReLU rule (Eq. 4) is applied to the radius r_j (1 + 2 g_D) + m_j
//     (the factor covers the rounding of the D-term sum r_j);
//   * the error symbol, scaled by alpha_j, is merged into the new symbol:
//     gamma_j + alpha_j m_j, plus a slack of 8 u (alpha_j (|y_j| + r_j) +
//     |beta_j|) for the rounding of the rule, the centre update and the row
//     scaling;
//   * R_j = alpha_j max(r_j, sum_k |W_jk| R_k) + gamma_j' is carried as rho_j
//     of the next layer: it bounds the sum of |coefficients| of neuron j both
//     as computed and along the absolute-value chain, which is what the
//     output's error bound needs.
// The coefficient blocks the hidden kernels store do not depend on the same
// layer's rule (alpha, beta and gamma are applied by the next layer), so this
// pass runs between the layer kernels and overwrites (alpha, beta, gamma).
// The output read-off computes the spread through the chain of downward row
// vectors v_{h-1} = (v_h . alpha_h) W_h; its rounding error is at most
// (number of layers + 1) g_{K+1} times the same chain taken with |W|, and
// that chain's spread is sum_k |w_k| R_k.  So the output radius becomes
//   r_out (1 + 2 g_D) + c_out (sum_k |w_k| (R_k + |z_k|) + |b|),
// c_out = (n_linear + 1) g_{Kmax+1}, plus 4 u_32 (|x0| + r) so that a float32
// read-off x0 -/+ r still contains the range.
#include "isx_internal.h"
#include "rules.h"

namespace isx {


// (sum_k |W_jk| R_k, sum_k |W_jk| |z_k| + |b_j|) for the input form of a
// layer: the previous hidden layer's post-rule vectors, or for layer 1 the
// box (z = centre, R = half-widths)
template <typename T>
__device__ __forceinline__ void aa_margin_sums(int64_t cell, int j, int n_in, int n_out, const T* __restrict__ Wt,
                                               const T* __restrict__ bias, const T* __restrict__ Yp,
                                               const T* __restrict__ Ap, const T* __restrict__ Bp,
                                               const T* __restrict__ Rp, const float* __restrict__ centres,
                                               const float* __restrict__ halves, T& sr, T& sz) {
  sr = T(0);
  sz = fabs(bias[j]);
  if (Yp) {
    const int64_t base = cell * n_in;
    for (int k = 0; k < n_in; ++k) {
      const T w = fabs(Wt[(int64_t)k * n_out + j]);
      sr += w * Rp[base + k];
      sz += w * fabs(Ap[base + k] * Yp[base + k] + Bp[base + k]);
    }
  } else {
    for (int k = 0; k < 3; ++k) {
      const T w = fabs(Wt[(int64_t)k * n_out + j]);
      sr += w * T(halves[cell * 3 + k]);
      sz += w * fabs(T(centres[cell * 3 + k]));
    }
  }
}

template <typename T>
__global__ void aa_margin_hidden_kernel(int64_t C, int n_in, int n_out, const T* __restrict__ Wt,
                                        const T* __restrict__ bias, const T* __restrict__ Yp,
                                        const T* __restrict__ Ap, const T* __restrict__ Bp,
                                        const T* __restrict__ Rp, const float* __restrict__ centres,
                                        const float* __restrict__ halves, const T* __restrict__ Y,
                                        const T* __restrict__ S, T* __restrict__ A, T* __restrict__ B,
                                        T* __restrict__ G, T* __restrict__ R, AaMargin<T> k) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= C * n_out) return;
  const int64_t cell = idx / n_out;
  const int j = (int)(idx - cell * n_out);
  T sr, sz;
  aa_margin_sums<T>(cell, j, n_in, n_out, Wt, bias, Yp, Ap, Bp, Rp, centres, halves, sr, sz);
  sr *= k.infl_m;
  const T m = (k.c * sr + k.c_z * sz) * k.infl_m;
  const T y = Y[idx];
  const T r = S[idx] * k.infl_s + m;
  T a, b, g;
  aa_rule_act<T>(ISX_RELU, y, r, a, b, g);
  g = g + a * m + k.slack * (a * (fabs(y) + r) + fabs(b));
  A[idx] = a;
  B[idx] = b;
  G[idx] = g;
  R[idx] = (a * (r > sr ? r : sr) + g) * (T(1) + k.slack);
}

template <typename T>
__global__ void aa_margin_output_kernel(int64_t C, int n_in, const T* __restrict__ Wt, const T* __restrict__ bias,
                                        const T* __restrict__ Yp, const T* __restrict__ Ap,
                                        const T* __restrict__ Bp, const T* __restrict__ Rp,
                                        const float* __restrict__ centres, const float* __restrict__ halves,
                                        float* __restrict__ out32, double* __restrict__ out64, AaMargin<T> k) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= C) return;
  T sr, sz;
  aa_margin_sums<T>(cell, 0, n_in, 1, Wt, bias, Yp, Ap, Bp, Rp, centres, halves, sr, sz);
  const T m = (k.c * sr + k.c_z * sz) * k.infl_m;
  const T x0 = out64 ? T(out64[cell * 2]) : T(out32[cell * 2]);
  const T r0 = out64 ? T(out64[cell * 2 + 1]) : T(out32[cell * 2 + 1]);
  T r = r0 * k.infl_s + m;
  r += T(4.0 / 16777216.0) * (fabs(x0) + r);
  if (out64) out64[cell * 2 + 1] = (double)r;
  if (out32) out32[cell * 2 + 1] = (float)r;
}

template <typename T>
AaMargin<T> aa_margin_consts(double u, double u_b, int K, int64_t D) {
  auto gn = [u](double n) { return n * u / (1.0 - n * u); };
  AaMargin<T> k;
  k.c = (T)(2.0 * u_b + u_b * u_b + gn(K + 1) * (1.0 + u_b) * (1.0 + u_b));
  k.c_z = (T)gn(K + 1);
  k.infl_m = (T)(1.0 + 2.0 * gn(K + 4));
  k.infl_s = (T)(1.0 + 2.0 * gn((double)D + 1));
  k.slack = (T)(8.0 * u);
  return k;
}
template AaMargin<float> aa_margin_consts<float>(double, double, int, int64_t);
template AaMargin<double> aa_margin_consts<double>(double, double, int, int64_t);

template <typename T>
hipError_t launch_aa_margin_hidden(int64_t C, int n_in, int n_out, const T* Wt, const T* bias, const T* Yp,
                                   const T* Ap, const T* Bp, const T* Rp, const float* centres, const float* halves,
                                   const T* Y, const T* S, T* A, T* B, T* G, T* R, const AaMargin<T>& k,
                                   hipStream_t s) {
  if (C <= 0) return hipSuccess;
  const int64_t n = C * n_out;
  hipLaunchKernelGGL((aa_margin_hidden_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, n_in, n_out,
                     Wt, bias, Yp, Ap, Bp, Rp, centres, halves, Y, S, A, B, G, R, k);
  return hipGetLastError();
}
template hipError_t launch_aa_margin_hidden<float>(int64_t, int, int, const float*, const float*, const float*,
                                                   const float*, const float*, const float*, const float*,
                                                   const float*, const float*, const float*, float*, float*, float*,
                                                   float*, const AaMargin<float>&, hipStream_t);
template hipError_t launch_aa_margin_hidden<double>(int64_t, int, int, const double*, const double*, const double*,
                                                    const double*, const double*, const double*, const float*,
                                                    const float*, const double*, const double*, double*, double*,
                                                    double*, double*, const AaMargin<double>&, hipStream_t);

template <typename T>
hipError_t launch_aa_margin_output(int64_t C, int n_in, const T* Wt, const T* bias, const T* Yp, const T* Ap,
                                   const T* Bp, const T* Rp, const float* centres, const float* halves, float* out32,
                                   double* out64, const AaMargin<T>& k, hipStream_t s) {
  if (C <= 0) return hipSuccess;
  hipLaunchKernelGGL((aa_margin_output_kernel<T>), dim3((unsigned)((C + 255) / 256)), dim3(256), 0, s, C, n_in, Wt,
                     bias, Yp, Ap, Bp, Rp, centres, halves, out32, out64, k);
  return hipGetLastError();
}
template hipError_t launch_aa_margin_output<float>(int64_t, int, const float*, const float*, const float*,
                                                   const float*, const float*, const float*, const float*,
                                                   const float*, float*, double*, const AaMargin<float>&,
                                                   hipStream_t);
template hipError_t launch_aa_margin_output<double>(int64_t, int, const double*, const double*, const double*,
                                                    const double*, const double*, const double*, const float*,
                                                    const float*, float*, double*, const AaMargin<double>&,
                                                    hipStream_t);

}  // namespace isx
