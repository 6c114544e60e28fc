// Propagation of boxes through a ReLU MLP: affine arithmetic (Sec. III,
// Eq. 1-4) and uncertainty propagation with probabilistic affine forms
// (Sec. IV-B/C, Eq. 6-10), plus plain MLP evaluation.
//
// Formulation (per cell).  The pre-activation form of hidden layer h is a
// centre y_h [n_h] and a coefficient block F_h [n_h x N_h]; the linear rule
// (Eq. 3 / Eq. 8) maps it exactly, and each ReLU (Eq. 4 / Eq. 9) replaces
// neuron j by alpha_j x + beta_j plus a new symbol gamma_j Z_j.  So
//   y_h   = W_h (alpha_{h-1} . y_{h-1} + beta_{h-1}) + b_h
//   F_h   = [ W_h diag(alpha_{h-1}) F_{h-1} | W_h diag(gamma_{h-1}) ]
// and the ReLU of layer h needs only the row statistic of F_h: the sum of
// squares (UP: sigma^2, Eq. 7) or of absolute values (AA: r, Eq. 2).
//   * alpha is applied when the next layer loads F (no extra pass);
//   * the centre travels as column 0 of F (its B-load adds beta);
//   * the last hidden layer only needs its row statistics, so its F is never
//     written;
//   * the output layer's coefficient of every symbol equals the product of
//     the linearised layers above it (a row vector v propagated downward:
//     v_L = w_out, v_{h-1} = (v_h . alpha_h) W_h), so the output spread is
//     sum over layers and neurons of stat(v_h[j] gamma_h[j]) plus the input
//     symbols' terms -- a few matrix-vector products per cell instead of
//     another wide product.  Each symbol's output coefficient is the same
//     number the forward tracking would give, so this is exact.
#include "isx_internal.h"
#include "rules.h"

#include <algorithm>

namespace isx {

// (the activation rules, Eq. 4 and Eq. 9-10 with the App. D rows, are in rules.h)

// row statistic terms: squares for UP and for the RA-UA read-off, magnitudes for AA
template <typename T, int METHOD>
__device__ __forceinline__ T stat_term(T v) {
  return METHOD != ISX_AA ? v * v : RM<T>::abs_(v);
}

// ---------------------------------------------------------------- layer 1
// Input form of a box (Sec. III-B / Sec. IV-C; the input box of Alg. 1): centre c,
// one symbol per axis with coefficient h_i (AA) or h_i/sqrt(3) (UP: a uniform
// variable on [-h, h] has standard deviation h/sqrt 3).  One thread per
// (cell, neuron).
// A segment (seg != 0; App. A's ray casting) {c + v e : e in [-1, 1]} has one
// input symbol, e (uniform on [-1, 1] for UP, coefficient v/sqrt 3): its
// column holds W1 v s and the other two input columns are 0; `halves` then
// holds the half-vectors v.
template <typename T, int METHOD>
__global__ void layer1_kernel(int64_t C, int n, const float* __restrict__ centres,
                              const float* __restrict__ halves, const T* __restrict__ W1,
                              const T* __restrict__ b1, T* __restrict__ Fout, T* __restrict__ Y,
                              T* __restrict__ A, T* __restrict__ B, T* __restrict__ G, T* __restrict__ S, int act,
                              int seg) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= C * n) return;
  const int64_t cell = idx / n;
  const int m = (int)(idx - cell * n);
  const T s = METHOD == ISX_UP ? T(0.57735026918962576451) : T(1);
  T f[3];
  T y = b1[m];
  T stat = T(0);
  if (seg) {
    T wv = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T w = W1[m * 3 + i];
      y += w * T(centres[cell * 3 + i]);
      wv += w * T(halves[cell * 3 + i]);
    }
    f[0] = wv * s;
    f[1] = f[2] = T(0);
    stat = stat_term<T, METHOD>(f[0]);
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T w = W1[m * 3 + i];
      y += w * T(centres[cell * 3 + i]);
      f[i] = w * (T(halves[cell * 3 + i]) * s);
      stat += stat_term<T, METHOD>(f[i]);
    }
  }
  T a, b, g;
  apply_rule<T, METHOD>(act, y, stat, a, b, g);
  Y[idx] = y;
  A[idx] = a;
  B[idx] = b;
  G[idx] = g;
  if (S) S[idx] = stat;
  if (Fout) {
    T* col = Fout + cell * (int64_t)kHeadCols * n + m;
    col[0] = y;
    col[(int64_t)1 * n] = f[0];
    col[(int64_t)2 * n] = f[1];
    col[(int64_t)3 * n] = f[2];
#pragma unroll
    for (int c = 4; c < kHeadCols; ++c) col[(int64_t)c * n] = T(0);
  }
}

// ----------------------------------------------------- hidden layer (SIMT)
// Reference kernel: one workgroup per cell, one thread per output neuron m;
// the cell's columns stream through LDS in tiles of CT (alpha-scaled on load,
// beta added to the centre column); thread m accumulates its full row
// statistic, appends the new symbol block W diag(gamma_{h-1}), and applies
// the ReLU rule.
template <typename T, int METHOD, int CT>
__global__ void hidden_simt_kernel(int64_t C, int n_in, int n_out, int64_t cols_in,
                                   const T* __restrict__ Wt, const T* __restrict__ bias,
                                   const T* __restrict__ Fin, const T* __restrict__ Ain,
                                   const T* __restrict__ Bin, const T* __restrict__ Gin,
                                   T* __restrict__ Fout, T* __restrict__ Y, T* __restrict__ A,
                                   T* __restrict__ B, T* __restrict__ G, T* __restrict__ S, int act_fn) {
  extern __shared__ unsigned char smem_raw[];
  T* Bs = reinterpret_cast<T*>(smem_raw);  // [n_in][CT]
  const int64_t cell = blockIdx.x;
  const int m = threadIdx.x;
  const bool act = m < n_out;
  const int64_t cols_out = cols_in + n_in;
  const T* fin = Fin + cell * cols_in * n_in;
  T* fout = Fout ? Fout + cell * cols_out * n_out : nullptr;
  const T* ain = Ain + cell * n_in;
  const T* bin = Bin + cell * n_in;
  const T* gin = Gin + cell * n_in;
  const T bm = act ? bias[m] : T(0);
  T y = T(0), stat = T(0);
  for (int64_t c0 = 0; c0 < cols_in; c0 += CT) {
    const int nc = (int)((cols_in - c0) < CT ? (cols_in - c0) : CT);
    for (int i = threadIdx.x; i < CT * n_in; i += blockDim.x) {
      const int col = i / n_in;
      const int k = i - col * n_in;
      T v = T(0);
      if (col < nc) {
        v = ain[k] * fin[(c0 + col) * n_in + k];
        if (c0 + col == 0) v += bin[k];
      }
      Bs[k * CT + col] = v;
    }
    __syncthreads();
    if (act) {
      T acc[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[c] = T(0);
      for (int k = 0; k < n_in; ++k) {
        const T w = Wt[(int64_t)k * n_out + m];
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c] += w * Bs[k * CT + c];
      }
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        if (c < nc) {
          const int64_t col = c0 + c;
          T v = acc[c];
          if (col == 0) {
            v += bm;
            y = v;
          } else {
            stat += stat_term<T, METHOD>(v);
          }
          if (fout) fout[col * n_out + m] = v;
        }
      }
    }
    __syncthreads();
  }
  if (act) {
    for (int j = 0; j < n_in; ++j) {
      const T v = Wt[(int64_t)j * n_out + m] * gin[j];
      stat += stat_term<T, METHOD>(v);
      if (fout) fout[(cols_in + j) * n_out + m] = v;
    }
    T a, b, g;
    apply_rule<T, METHOD>(act_fn, y, stat, a, b, g);
    const int64_t o = cell * n_out + m;
    Y[o] = y;
    A[o] = a;
    B[o] = b;
    G[o] = g;
    if (S) S[o] = stat;
  }
}

// ------------------------------------------------------------ output layer
// Output read-off (Eq. 2 for AA, Eq. 7 for UP) by the downward row vector
// described at the top of this file.  One workgroup (256 threads) handles
// CPB cells: each weight of the chain is loaded once for all of them (the
// chain's weights are the read-off's main traffic).  Every cell's sums run in
// the same order for any CPB.  LDS: v and u of the CPB cells, [CPB][nmax]
// each (nmax = the widest hidden layer).
template <typename T, int METHOD, int CPB>
__global__ __launch_bounds__(256) void output_kernel(int64_t C, NetView<T> net, int nmax,
                                                     const float* __restrict__ halves, float* __restrict__ out32,
                                                     double* __restrict__ out64, int seg) {
  extern __shared__ float4 outk_smem4[];
  T* v = reinterpret_cast<T*>(outk_smem4);  // [CPB][nmax]
  T* u = v + CPB * nmax;                    // [CPB][nmax]
  __shared__ T red[2][CPB][256 / 64];
  const int64_t cell0 = (int64_t)blockIdx.x * CPB;
  const int t = threadIdx.x;
  const int L = net.n_linear;
  const int Lh = L - 1;
  const int nL = net.n[Lh];
  const T* wout = net.W[L - 1];
  int64_t cl[CPB];  // the cell, clamped to a valid one for cells past the end
#pragma unroll
  for (int c = 0; c < CPB; ++c) cl[c] = cell0 + c < C ? cell0 + c : C - 1;
  T mu_p[CPB], acc_p[CPB];
#pragma unroll
  for (int c = 0; c < CPB; ++c) mu_p[c] = acc_p[c] = T(0);
#pragma unroll
  for (int c = 0; c < CPB; ++c) {
    const T* Yh = net.Y[Lh] + cl[c] * nL;
    const T* Ah = net.A[Lh] + cl[c] * nL;
    const T* Bh = net.B[Lh] + cl[c] * nL;
    const T* Gh = net.G[Lh] + cl[c] * nL;
    for (int j = t; j < nL; j += blockDim.x) {
      const T w = wout[j];
      mu_p[c] += w * (Ah[j] * Yh[j] + Bh[j]);
      acc_p[c] += stat_term<T, METHOD>(w * Gh[j]);
      v[c * nmax + j] = w;
    }
  }
  __syncthreads();
  for (int h = Lh; h >= 2; --h) {
    const int nh = net.n[h], np = net.n[h - 1];
#pragma unroll
    for (int c = 0; c < CPB; ++c) {
      const T* Ah = net.A[h] + cl[c] * nh;
      for (int j = t; j < nh; j += blockDim.x) u[c * nmax + j] = v[c * nmax + j] * Ah[j];
    }
    __syncthreads();
    const T* Wl = net.W[h - 1];  // [nh][np]
    for (int i = t; i < np; i += blockDim.x) {
      T sv[CPB];
#pragma unroll
      for (int c = 0; c < CPB; ++c) sv[c] = T(0);
      for (int j = 0; j < nh; ++j) {
        const T w = Wl[(int64_t)j * np + i];
#pragma unroll
        for (int c = 0; c < CPB; ++c) sv[c] += u[c * nmax + j] * w;
      }
#pragma unroll
      for (int c = 0; c < CPB; ++c) {
        v[c * nmax + i] = sv[c];
        acc_p[c] += stat_term<T, METHOD>(sv[c] * net.G[h - 1][cl[c] * np + i]);
      }
    }
    __syncthreads();
  }
  {
    const int n1 = net.n[1];
#pragma unroll
    for (int c = 0; c < CPB; ++c) {
      const T* A1 = net.A[1] + cl[c] * n1;
      for (int j = t; j < n1; j += blockDim.x) u[c * nmax + j] = v[c * nmax + j] * A1[j];
    }
    __syncthreads();
    const T* W0 = net.W[0];  // [n1][3]
    const T sc = METHOD == ISX_UP ? T(0.57735026918962576451) : T(1);
    if (!seg && t < 3) {
#pragma unroll
      for (int c = 0; c < CPB; ++c) {
        T s = T(0);
        for (int j = 0; j < n1; ++j) s += u[c * nmax + j] * W0[j * 3 + t];
        acc_p[c] += stat_term<T, METHOD>(s * (T(halves[cl[c] * 3 + t]) * sc));
      }
    } else if (seg && t == 0) {
      // the segment's one input symbol: coefficient (u^T W0) . v
#pragma unroll
      for (int c = 0; c < CPB; ++c) {
        T sv = T(0);
        for (int a = 0; a < 3; ++a) {
          T s = T(0);
          for (int j = 0; j < n1; ++j) s += u[c * nmax + j] * W0[j * 3 + a];
          sv += s * T(halves[cl[c] * 3 + a]);
        }
        acc_p[c] += stat_term<T, METHOD>(sv * sc);
      }
    }
  }
  // block reductions of (mu_p, acc_p)
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform
#pragma unroll
  for (int c = 0; c < CPB; ++c) {
    for (int off = 32; off > 0; off >>= 1) {
      mu_p[c] += __shfl_xor(mu_p[c], off);
      acc_p[c] += __shfl_xor(acc_p[c], off);
    }
    if ((t & 63) == 0) {
      red[0][c][wave] = mu_p[c];
      red[1][c][wave] = acc_p[c];
    }
  }
  __syncthreads();
  if (t < CPB && cell0 + t < C) {
    const int c = t;
    T mu = T(0), acc = T(0);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      mu += red[0][c][w];
      acc += red[1][c][w];
    }
    mu += net.b[L - 1][0];
    // RA-UA (Eq. 5): the AA coefficients read as uniform variables, variance x_i^2 / 3
    const T spread = METHOD == ISX_UP ? RM<T>::sqrt_(acc)
                                      : (METHOD == ISX_RAUA ? RM<T>::sqrt_(acc) * T(0.57735026918962576451) : acc);
    const int64_t cell = cell0 + c;
    out32[cell * 2 + 0] = (float)mu;
    out32[cell * 2 + 1] = (float)spread;
    if (out64) {
      out64[cell * 2 + 0] = (double)mu;
      out64[cell * 2 + 1] = (double)spread;
    }
  }
}

// Launch of the read-off with CPB cells per workgroup.
template <typename T, int METHOD, int CPB>
static hipError_t launch_output_simt(const Model& m, int64_t C, const NetView<T>& view, const float* halves,
                                     float* out32, double* out64, hipStream_t s, int seg = 0) {
  int nmax = 3;
  for (int h = 1; h < m.n_linear; ++h) nmax = std::max(nmax, m.pw[h]);
  const size_t lds = (size_t)2 * CPB * nmax * sizeof(T);
  {
    hipError_t e = ensure_lds_limit(reinterpret_cast<const void*>(&output_kernel<T, METHOD, CPB>), (int)(2 * CPB * ISX_MAX_WIDTH * sizeof(T)));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((output_kernel<T, METHOD, CPB>), dim3((unsigned)((C + CPB - 1) / CPB)), dim3(256), lds, s, C,
                     view, nmax, halves, out32, out64, seg);
  return hipGetLastError();
}

// ------------------------------------------------------- MLP evaluation
// Plain forward pass (Sec. III-B) on tiles of PT points; one thread per
// neuron, activations of the tile in LDS.
template <typename T, int PT>
__global__ void mlp_eval_kernel(int64_t n, NetView<T> net, int n_max, const float* __restrict__ pts,
                                float* __restrict__ vals) {
  extern __shared__ unsigned char smem_raw[];
  T* h0 = reinterpret_cast<T*>(smem_raw);  // [n_max][PT]
  T* h1 = h0 + (size_t)n_max * PT;
  const int64_t p0 = (int64_t)blockIdx.x * PT;
  const int t = threadIdx.x;
  for (int i = t; i < 3 * PT; i += blockDim.x) {
    const int p = i / 3, a = i - p * 3;
    h0[a * PT + p] = (p0 + p < n) ? T(pts[(p0 + p) * 3 + a]) : T(0);
  }
  __syncthreads();
  T* hin = h0;
  T* hout = h1;
  for (int l = 0; l < net.n_linear; ++l) {
    const int ni = net.n[l], no = net.n[l + 1];
    const T* W = net.W[l];
    for (int m = t; m < no; m += blockDim.x) {
      T acc[PT];
      const T bm = net.b[l][m];
#pragma unroll
      for (int p = 0; p < PT; ++p) acc[p] = bm;
      for (int k = 0; k < ni; ++k) {
        const T w = W[(int64_t)m * ni + k];
#pragma unroll
        for (int p = 0; p < PT; ++p) acc[p] += w * hin[k * PT + p];
      }
      const bool hidden = l + 1 < net.n_linear;
#pragma unroll
      for (int p = 0; p < PT; ++p) hout[m * PT + p] = hidden ? activate<T>(net.act, acc[p]) : acc[p];
    }
    __syncthreads();
    T* tmp = hin;
    hin = hout;
    hout = tmp;
  }
  if (t < PT && p0 + t < n) vals[p0 + t] = (float)hin[t];
}

// ================================================================ host side
size_t prop_F_elems(const Model& m, int64_t C) {
  size_t best = 1;
  for (int h = 1; h < m.hidden(); ++h) best = std::max(best, (size_t)(m.cols(h) * m.pw[h]));
  return best * (size_t)C;
}

// Per hidden layer h: Y, A, B, G (each [C][n_h]) in layer order, then (with
// the AA rounding margin) the row statistics S and the absolute radii R of
// every layer.
size_t prop_vec_elems(const Model& m, int64_t C, bool with_margin) {
  size_t s = 0;
  for (int h = 1; h <= m.hidden(); ++h) s += (with_margin ? 6 : 4) * (size_t)m.pw[h];
  return s * (size_t)C;
}

template <typename T>
static void margin_ptrs(const Model& m, int64_t C, T* vec, T** S, T** R) {
  size_t tot = 0;
  for (int h = 1; h <= m.hidden(); ++h) tot += (size_t)m.pw[h] * C;
  size_t off = 4 * tot;
  for (int h = 1; h <= m.hidden(); ++h) {
    const size_t n = (size_t)m.pw[h] * C;
    S[h] = vec + off;
    R[h] = vec + off + tot;
    off += n;
  }
}

template <typename T>
static void layer_ptrs(const Model& m, int64_t C, T* vec, T** Y, T** A, T** B, T** G) {
  size_t off = 0;
  for (int h = 1; h <= m.hidden(); ++h) {
    const size_t n = (size_t)m.pw[h] * C;
    Y[h] = vec + off;
    A[h] = vec + off + n;
    B[h] = vec + off + 2 * n;
    G[h] = vec + off + 3 * n;
    off += 4 * n;
  }
}

template <typename T>
static const T* wptr(const Layer& l);
template <>
const float* wptr<float>(const Layer& l) {
  return l.W;
}
template <>
const double* wptr<double>(const Layer& l) {
  return l.Wd;
}
template <typename T>
static const T* wtptr(const Layer& l);
template <>
const float* wtptr<float>(const Layer& l) {
  return l.Wt;
}
template <>
const double* wtptr<double>(const Layer& l) {
  return l.Wtd;
}
template <typename T>
static const T* bptr(const Layer& l);
template <>
const float* bptr<float>(const Layer& l) {
  return l.b;
}
template <>
const double* bptr<double>(const Layer& l) {
  return l.bd;
}

template <typename T>
static NetView<T> make_view(const Model& m) {
  NetView<T> v{};
  v.n_linear = m.n_linear;
  v.act = m.act;
  for (int i = 0; i <= m.n_linear; ++i) v.n[i] = m.pw[i];
  for (int l = 0; l < m.n_linear; ++l) {
    v.W[l] = wptr<T>(m.L[l]);
    v.b[l] = bptr<T>(m.L[l]);
  }
  return v;
}

template <>
NetView<float> net_view<float>(const Model& m) {
  return make_view<float>(m);
}
template <>
NetView<double> net_view<double>(const Model& m) {
  return make_view<double>(m);
}


hipError_t launch_hidden_mfma_f32(int method, int64_t C, int n_in, int n_out, int64_t cols_in, const float* Wt,
                                  const float* Wrow, const float* bias, const float* Fin, const float* Ain,
                                  const float* Bin, const float* Gin, float* Fout, float* Y, float* A, float* B,
                                  float* G, float* S, hipStream_t s);
hipError_t launch_hidden_mfma_f64(int method, int64_t C, int n_in, int n_out, int64_t cols_in, const double* Wt,
                                  const double* bias, const double* Fin, const double* Ain, const double* Bin,
                                  const double* Gin, double* Fout, double* Y, double* A, double* B, double* G,
                                  double* S, hipStream_t s);
bool mfma_supported(const Model& m);

template <typename T>
static hipError_t hidden_mfma(int, int64_t, int, int, int64_t, const T*, const T*, const T*, const T*, const T*,
                              const T*, const T*, T*, T*, T*, T*, T*, T*, hipStream_t) {
  return hipErrorNotSupported;
}
template <>
hipError_t hidden_mfma<float>(int method, int64_t C, int n_in, int n_out, int64_t cols_in, const float* Wt,
                              const float* Wrow, const float* bias, const float* Fin, const float* Ain,
                              const float* Bin, const float* Gin, float* Fout, float* Y, float* A, float* B,
                              float* G, float* S, hipStream_t s) {
  return launch_hidden_mfma_f32(method, C, n_in, n_out, cols_in, Wt, Wrow, bias, Fin, Ain, Bin, Gin, Fout, Y, A, B,
                                G, S, s);
}
template <>
hipError_t hidden_mfma<double>(int method, int64_t C, int n_in, int n_out, int64_t cols_in, const double* Wt,
                               const double*, const double* bias, const double* Fin, const double* Ain, const double* Bin,
                               const double* Gin, double* Fout, double* Y, double* A, double* B, double* G,
                               double* S, hipStream_t s) {
  return launch_hidden_mfma_f64(method, C, n_in, n_out, cols_in, Wt, bias, Fin, Ain, Bin, Gin, Fout, Y, A, B, G, S, s);
}

template <typename T, int METHOD>
static hipError_t propagate_impl(const PropArgs& a, PropWork<T>& w, bool use_mfma) {
  const Model& m = *a.m;
  const int Lh = m.hidden();
  const int64_t C = a.C;
  T *Y[ISX_MAX_LINEAR] = {}, *A[ISX_MAX_LINEAR] = {}, *B[ISX_MAX_LINEAR] = {}, *G[ISX_MAX_LINEAR] = {};
  T *S[ISX_MAX_LINEAR] = {}, *R[ISX_MAX_LINEAR] = {};
  layer_ptrs<T>(m, C, w.vec, Y, A, B, G);
  // AA rounding margin: the kernels also write their row statistics, and a
  // pass after each layer re-applies the rule to the widened radius
  const bool marg = METHOD == ISX_AA && a.aa_margin && a.method == ISX_AA;
  const double u = sizeof(T) == 8 ? 0x1p-53 : 0x1p-24;
  if (marg) margin_ptrs<T>(m, C, w.vec, S, R);
  int64_t D = 3;  // symbol columns summed by the row statistic of the layer
  int cur = 0;
  {
    const int n1 = m.pw[1];
    const int64_t threads = C * n1;
    const int bs = 256;
    hipLaunchKernelGGL((layer1_kernel<T, METHOD>), dim3((unsigned)((threads + bs - 1) / bs)), dim3(bs), 0,
                       a.stream, C, n1, a.centres, a.halves, wptr<T>(m.L[0]), bptr<T>(m.L[0]),
                       Lh >= 2 ? w.F[cur] : (T*)nullptr, Y[1], A[1], B[1], G[1], S[1], m.act, a.seg);
    if (marg) {
      hipError_t e = launch_aa_margin_hidden<T>(C, 3, n1, wtptr<T>(m.L[0]), bptr<T>(m.L[0]), nullptr, nullptr, nullptr,
                                                nullptr, a.centres, a.halves, Y[1], S[1], A[1], B[1], G[1], R[1],
                                                aa_margin_consts<T>(u, 0.0, 3, D), a.stream);
      if (e != hipSuccess) return e;
    }
  }
  for (int h = 2; h <= Lh; ++h) {
    const int n_in = m.pw[h - 1], n_out = m.pw[h];
    const int64_t cols_in = m.cols(h - 1);
    T* Fout = h < Lh ? w.F[cur ^ 1] : nullptr;
    Profiler::Rec rec{};
    bool prof = false;
    if (a.prof && a.prof->on) {
      int64_t real_cols = 4;
      for (int i = 1; i <= h - 2; ++i) real_cols += m.widths[i];
      const double flops = 2.0 * m.widths[h] * m.widths[h - 1] * (double)real_cols * (double)C;
      const double bytes = (double)sizeof(T) * C *
                           ((double)real_cols * m.widths[h - 1] +
                            (h < Lh ? (double)(real_cols + m.widths[h - 1]) * m.widths[h] : 0.0));
      const int kind = sizeof(T) == 8 ? ISX_KERNEL_HIDDEN_FP64
                                      : (use_mfma ? ISX_KERNEL_HIDDEN_FP32 : ISX_KERNEL_HIDDEN_SIMT_FP32);
      prof = a.prof->begin(rec, kind, flops, bytes, a.stream);
    }
    if (use_mfma) {
      // (bit 8: float32 products as split bfloat16 MFMAs, where asked for)
      const int word = METHOD | (m.act << 4) | (sizeof(T) == 4 && a.f32_split ? 256 : 0);
      hipError_t e = hidden_mfma<T>(word, C, n_in, n_out, cols_in, wtptr<T>(m.L[h - 1]), wptr<T>(m.L[h - 1]),
                                    bptr<T>(m.L[h - 1]), w.F[cur], A[h - 1], B[h - 1], G[h - 1], Fout, Y[h], A[h],
                                    B[h], G[h], S[h], a.stream);
      if (e != hipSuccess) return e;
    } else {
      constexpr int CT = sizeof(T) == 8 ? 8 : 16;
      const int bs = std::max(64, (n_out + 63) / 64 * 64);
      const size_t lds = (size_t)CT * n_in * sizeof(T);
      hipLaunchKernelGGL((hidden_simt_kernel<T, METHOD, CT>), dim3((unsigned)C), dim3(bs), lds, a.stream, C, n_in,
                         n_out, cols_in, wtptr<T>(m.L[h - 1]), bptr<T>(m.L[h - 1]), w.F[cur], A[h - 1], B[h - 1],
                         G[h - 1], Fout, Y[h], A[h], B[h], G[h], S[h], m.act);
    }
    if (prof) a.prof->end(rec, a.stream);
    D += n_in;
    if (marg) {
      hipError_t e = launch_aa_margin_hidden<T>(C, n_in, n_out, wtptr<T>(m.L[h - 1]), bptr<T>(m.L[h - 1]), Y[h - 1],
                                                A[h - 1], B[h - 1], R[h - 1], a.centres, a.halves, Y[h], S[h], A[h],
                                                B[h], G[h], R[h], aa_margin_consts<T>(u, 0.0, n_in, D), a.stream);
      if (e != hipSuccess) return e;
    }
    cur ^= 1;
  }
  Profiler::Rec rec{};
  const bool prof = a.prof && a.prof->begin(rec, ISX_KERNEL_OUTPUT, output_flops_per_cell(m) * (double)C,
                                            (double)sizeof(T) * C * 4.0 * (double)m.pw[1] * Lh, a.stream);
  if (a.method == ISX_RAUA) {
    // RA-UA: the AA vectors with the uniform-assumption read-off
    NetView<T> view = make_view<T>(m);
    for (int h = 1; h <= Lh; ++h) {
      view.Y[h] = Y[h];
      view.A[h] = A[h];
      view.B[h] = B[h];
      view.G[h] = G[h];
    }
    hipError_t e = sizeof(T) == 8
                       ? launch_output_simt<T, ISX_RAUA, 4>(m, C, view, a.halves, a.out32, a.out64, a.stream, a.seg)
                       : launch_output_simt<T, ISX_RAUA, 1>(m, C, view, a.halves, a.out32, a.out64, a.stream, a.seg);
    if (e != hipSuccess) return e;
  } else if (use_mfma && sizeof(T) == 4 && a.out64 == nullptr && !a.seg) {
    hipError_t e = launch_output_mfma(m, (isx_method)METHOD, C, reinterpret_cast<float* const*>(Y),
                                      reinterpret_cast<float* const*>(A), reinterpret_cast<float* const*>(B),
                                      reinterpret_cast<float* const*>(G), a.halves, a.out32, a.stream);
    if (e != hipSuccess) return e;
  } else {
    NetView<T> view = make_view<T>(m);
    for (int h = 1; h <= Lh; ++h) {
      view.Y[h] = Y[h];
      view.A[h] = A[h];
      view.B[h] = B[h];
      view.G[h] = G[h];
    }
    // float64 (the re-check band) batches 4 cells per workgroup
    hipError_t e = sizeof(T) == 8
                       ? launch_output_simt<T, METHOD, 4>(m, C, view, a.halves, a.out32, a.out64, a.stream, a.seg)
                       : launch_output_simt<T, METHOD, 1>(m, C, view, a.halves, a.out32, a.out64, a.stream, a.seg);
    if (e != hipSuccess) return e;
  }
  if (prof) a.prof->end(rec, a.stream);
  if (marg) {
    int kmax = 3;
    for (int h = 1; h <= Lh; ++h) kmax = std::max(kmax, m.pw[h]);
    AaMargin<T> k = aa_margin_consts<T>(u, 0.0, m.pw[Lh], D + m.pw[Lh]);
    // the downward read-off: (layers + 1) products of length <= kmax
    k.c = (T)((m.n_linear + 1) * ((kmax + 1) * u / (1.0 - (kmax + 1) * u)));
    hipError_t e = launch_aa_margin_output<T>(C, m.pw[Lh], wtptr<T>(m.L[Lh]), bptr<T>(m.L[Lh]), Y[Lh], A[Lh], B[Lh],
                                              R[Lh], a.centres, a.halves, a.out32, a.out64, k, a.stream);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// Output read-off for paths that keep float32 vectors (used by the bf16 path).
hipError_t launch_output_f32(const Model& m, isx_method method, int64_t C, float* vec, const float* halves,
                             float* out32, hipStream_t s) {
  float *Y[ISX_MAX_LINEAR] = {}, *A[ISX_MAX_LINEAR] = {}, *B[ISX_MAX_LINEAR] = {}, *G[ISX_MAX_LINEAR] = {};
  layer_ptrs<float>(m, C, vec, Y, A, B, G);
  NetView<float> view = make_view<float>(m);
  for (int h = 1; h <= m.hidden(); ++h) {
    view.Y[h] = Y[h];
    view.A[h] = A[h];
    view.B[h] = B[h];
    view.G[h] = G[h];
  }
  return method == ISX_UP     ? launch_output_simt<float, ISX_UP, 1>(m, C, view, halves, out32, nullptr, s)
         : method == ISX_RAUA ? launch_output_simt<float, ISX_RAUA, 1>(m, C, view, halves, out32, nullptr, s)
                              : launch_output_simt<float, ISX_AA, 1>(m, C, view, halves, out32, nullptr, s);
}

hipError_t propagate_f32(const PropArgs& a, PropWork<float>& w) {
  if (a.C <= 0) return hipSuccess;
  const bool use_mfma = a.kernel_choice != 1 && mfma_supported(*a.m);
  return a.method == ISX_UP ? propagate_impl<float, ISX_UP>(a, w, use_mfma)
                            : propagate_impl<float, ISX_AA>(a, w, use_mfma);
}

hipError_t propagate_f64(const PropArgs& a, PropWork<double>& w) {
  if (a.C <= 0) return hipSuccess;
  const bool use_mfma = a.kernel_choice != 1 && mfma_supported(*a.m);
  return a.method == ISX_UP ? propagate_impl<double, ISX_UP>(a, w, use_mfma)
                            : propagate_impl<double, ISX_AA>(a, w, use_mfma);
}

template <typename T, int PT>
static hipError_t eval_points_t(const Model& m, int64_t n, const float* pts, float* vals, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int n_max = 3;
  for (int i = 0; i <= m.n_linear; ++i) n_max = std::max(n_max, m.pw[i]);
  const int bs = std::min(1024, std::max(64, (n_max + 63) / 64 * 64));
  const size_t lds = 2 * (size_t)n_max * PT * sizeof(T);
  NetView<T> view = make_view<T>(m);
  // a launch's work-items (blocks x bs) must stay below 2^32: at most 2^31 / bs
  // blocks of PT points each per launch
  const int64_t per_launch = ((int64_t(1) << 31) / bs) * PT;
  for (int64_t o = 0; o < n; o += per_launch) {
    const int64_t c = std::min(per_launch, n - o);
    hipLaunchKernelGGL((mlp_eval_kernel<T, PT>), dim3((unsigned)((c + PT - 1) / PT)), dim3(bs), lds, s, c, view,
                       n_max, pts + 3 * o, vals + o);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t eval_points_f32(const Model& m, int64_t n, const float* pts, float* vals, hipStream_t s) {
  return eval_points_t<float, 8>(m, n, pts, vals, s);
}
hipError_t eval_points_f64(const Model& m, int64_t n, const float* pts, float* vals, hipStream_t s) {
  return eval_points_t<double, 4>(m, n, pts, vals, s);
}

}  // namespace isx
