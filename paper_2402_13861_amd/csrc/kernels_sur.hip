// Learned surrogate of the propagation: a small ReLU MLP mapping a cell
// (centre, log2 size) to a predicted (mean, sigma), trained on the GPU by the
// kernels below (bf16 MFMA products with float32 accumulation, float32 master
// weights, Adam), and used during extraction to decide cells whose outcome
// it predicts confidently; every other cell falls back to propagation.
#include "isx_internal.h"

#include <algorithm>

namespace isx {

typedef __bf16 sbf16x8 __attribute__((ext_vector_type(8)));
typedef float sv16f __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------------ GEMM
// C[m][n] = epilogue( sum_k A(m,k) B(k,n) ), operands rounded to bf16 when
// staged, float32 accumulation.  A(m,k) = ta ? A[k*lda+m] : A[m*lda+k];
// B(k,n) = tb ? B[n*ldb+k] : B[k*ldb+n].  Epilogue: + bias[n], ReLU, times
// (mask[m*ldm+n] > 0).  64x64 tiles, 4 waves of 32x32 (32x32x16 bf16 MFMA).
// Split K: workgroup z sums k in [z kc, (z+1) kc) and writes its partial
// tile, without the epilogue, to part[z][M][N]; a second kernel adds the
// partials in z order (deterministic).
constexpr int GT = 64;       // tile edge
constexpr int GK = 32;       // K chunk
constexpr int GKP = GK + 8;  // padded bf16 row in LDS

__global__ __launch_bounds__(256) void sur_gemm_kernel(int M, int N, int K, const float* __restrict__ A, int lda,
                                                       int ta, const float* __restrict__ B, int ldb, int tb,
                                                       float* __restrict__ Cm, int ldc, const float* __restrict__ bias,
                                                       int relu, const float* __restrict__ mask, int ldm, int kc,
                                                       float* __restrict__ part) {
  __shared__ __bf16 As[GT * GKP];
  __shared__ __bf16 Bs[GT * GKP];
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform
  const int wr = wave & 1, wc = wave >> 1;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  sv16f acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  const int kbeg = blockIdx.z * kc, kend = min(K, kbeg + kc);
  for (int k0 = kbeg; k0 < kend; k0 += GK) {
    for (int i = t; i < GT * GK; i += 256) {
      // consecutive threads walk the contiguous index of each operand
      int r, kk;
      if (ta) {
        kk = i / GT;
        r = i - kk * GT;
      } else {
        r = i / GK;
        kk = i - r * GK;
      }
      const int m = m0 + r, k = k0 + kk;
      float v = 0.f;
      if (m < M && k < kend) v = ta ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k];
      As[r * GKP + kk] = (__bf16)v;
    }
    for (int i = t; i < GT * GK; i += 256) {
      int c, kk;
      if (tb) {
        c = i / GK;
        kk = i - c * GK;
      } else {
        kk = i / GT;
        c = i - kk * GT;
      }
      const int n = n0 + c, k = k0 + kk;
      float v = 0.f;
      if (n < N && k < kend) v = tb ? B[(int64_t)n * ldb + k] : B[(int64_t)k * ldb + n];
      Bs[c * GKP + kk] = (__bf16)v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GK / 16; ++ks) {
      const sbf16x8 a = *reinterpret_cast<const sbf16x8*>(As + (wr * 32 + (lane & 31)) * GKP + 16 * ks + 8 * (lane >> 5));
      const sbf16x8 b = *reinterpret_cast<const sbf16x8*>(Bs + (wc * 32 + (lane & 31)) * GKP + 16 * ks + 8 * (lane >> 5));
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int n = n0 + wc * 32 + (lane & 31);
  if (n < N) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = m0 + wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (m < M && part) {
        part[((int64_t)blockIdx.z * M + m) * N + n] = acc[r];
      } else if (m < M) {
        float v = acc[r];
        if (bias) v += bias[n];
        if (relu) v = v > 0.f ? v : 0.f;
        if (mask && !(mask[(int64_t)m * ldm + n] > 0.f)) v = 0.f;
        Cm[(int64_t)m * ldc + n] = v;
      }
    }
  }
}

// C[m][n] = sum_z part[z][m][n], z in order
__global__ void sur_splitk_sum_kernel(int M, int N, int splits, const float* __restrict__ part, float* __restrict__ C,
                                      int ldc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  const int m = (int)(i / N), n = (int)(i - (int64_t)m * N);
  float v = 0.f;
  for (int z = 0; z < splits; ++z) v += part[(int64_t)z * M * N + i];
  C[(int64_t)m * ldc + n] = v;
}

hipError_t sur_gemm(int M, int N, int K, const float* A, int lda, bool ta, const float* B, int ldb, bool tb, float* C,
                    int ldc, const float* bias, bool relu, const float* mask, int ldm, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  hipLaunchKernelGGL(sur_gemm_kernel, grid, dim3(256), 0, s, M, N, K, A, lda, (int)ta, B, ldb, (int)tb, C, ldc, bias,
                     (int)relu, mask, ldm, K, (float*)nullptr);
  return hipGetLastError();
}

int sur_gemm_splits(int M, int N, int K) {
  const int tiles = ((N + GT - 1) / GT) * ((M + GT - 1) / GT);
  // at least two K chunks per workgroup, and about 256 workgroups in all
  const int by_k = std::max(1, K / (2 * GK));
  const int want = std::max(1, (256 + tiles - 1) / tiles);
  const int splits = std::min(by_k, want);
  if (splits <= 1) return 1;
  const int kc = ((K + splits - 1) / splits + GK - 1) / GK * GK;
  return (K + kc - 1) / kc;
}

hipError_t sur_gemm_splitk(int M, int N, int K, const float* A, int lda, bool ta, const float* B, int ldb, bool tb,
                           float* C, int ldc, float* work, size_t work_elems, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int splits = sur_gemm_splits(M, N, K);
  if (splits <= 1 || !work || work_elems < (size_t)splits * M * N)
    return sur_gemm(M, N, K, A, lda, ta, B, ldb, tb, C, ldc, nullptr, false, nullptr, 0, s);
  const int kc = ((K + splits - 1) / splits + GK - 1) / GK * GK;
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, splits);
  hipLaunchKernelGGL(sur_gemm_kernel, grid, dim3(256), 0, s, M, N, K, A, lda, (int)ta, B, ldb, (int)tb, C, ldc,
                     (const float*)nullptr, 0, (const float*)nullptr, 0, kc, work);
  const int64_t mn = (int64_t)M * N;
  hipLaunchKernelGGL(sur_splitk_sum_kernel, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, M, N, splits,
                     (const float*)work, C, ldc);
  return hipGetLastError();
}

// ---------------------------------------------------------- elementwise
// Features x = (c_x, c_y, c_z, a * log2(2 h_x) + b) of rows [r0, r0+B) of a
// data set of n cells (wrapping around), and optionally the targets: the
// standardised ((mu - mu_bar)/S, ln sigma) or, with a base (f, s) per cell,
// the corrections to that base ((mu - f)/s_b, ln(sigma/s_b)), s_b =
// max(s, s_floor).
__global__ void sur_features_kernel(int64_t n, int64_t r0, int B, const float* __restrict__ centres,
                                    const float* __restrict__ halves, float a, float b, float* __restrict__ X,
                                    const float* __restrict__ mu_sigma, float mu_bar, float scale,
                                    const float* __restrict__ base, float s_floor, float* __restrict__ T) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const int64_t row = (r0 + i) % n;
  X[i * 4 + 0] = centres[row * 3 + 0];
  X[i * 4 + 1] = centres[row * 3 + 1];
  X[i * 4 + 2] = centres[row * 3 + 2];
  X[i * 4 + 3] = a * log2f(2.f * halves[row * 3 + 0]) + b;
  if (T) {
    const float mu = mu_sigma[row * 2 + 0];
    const float sg = fmaxf(mu_sigma[row * 2 + 1], 1e-12f * scale);
    if (base) {
      const float sb = fmaxf(base[row * 2 + 1], s_floor);
      T[i * 2 + 0] = (mu - base[row * 2 + 0]) / sb;
      T[i * 2 + 1] = logf(sg / sb);
    } else {
      T[i * 2 + 0] = (mu - mu_bar) / scale;
      T[i * 2 + 1] = logf(sg);
    }
  }
}

hipError_t sur_features(int64_t n, int64_t r0, int B, const float* centres, const float* halves, float a, float b,
                        float* X, const float* mu_sigma, float mu_bar, float scale, const float* base,
                        float s_floor, float* T, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(sur_features_kernel, dim3((B + 255) / 256), dim3(256), 0, s, n, r0, B, centres, halves, a, b, X,
                     mu_sigma, mu_bar, scale, base, s_floor, T);
  return hipGetLastError();
}

// d loss / d out = (out - T) / B, and the loss 0.5 * sum (out - T)^2 / B
// (one block, fixed summation order).
__global__ void sur_loss_kernel(int B, const float* __restrict__ out, const float* __restrict__ T,
                                float* __restrict__ dout, float* __restrict__ loss_out) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < 2 * B; i += 256) {
    const float d = out[i] - T[i];
    dout[i] = d / (float)B;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss_out) *loss_out = 0.5f * red[0] / (float)B;
}

hipError_t sur_loss(int B, const float* out, const float* T, float* dout, float* loss_out, hipStream_t s) {
  hipLaunchKernelGGL(sur_loss_kernel, dim3(1), dim3(256), 0, s, B, out, T, dout, loss_out);
  return hipGetLastError();
}

// db[n] = sum_m dY[m][n] (one block per column, fixed order)
__global__ void sur_colsum_kernel(int M, int N, const float* __restrict__ dY, float* __restrict__ db) {
  __shared__ float red[256];
  const int n = blockIdx.x;
  float s = 0.f;
  for (int m = threadIdx.x; m < M; m += 256) s += dY[(int64_t)m * N + n];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[n] = red[0];
}

hipError_t sur_colsum(int M, int N, const float* dY, float* db, hipStream_t s) {
  hipLaunchKernelGGL(sur_colsum_kernel, dim3(N), dim3(256), 0, s, M, N, dY, db);
  return hipGetLastError();
}

// Adam with bias correction (Kingma & Ba): m = b1 m + (1-b1) g,
// v = b2 v + (1-b2) g^2, p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
__global__ void sur_adam_kernel(int n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t sur_adam(int n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sur_adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, p, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

// Network outputs -> (mu_hat, sigma_hat) in field units: standardised
// outputs, or corrections to a base (f, s) per cell (then the base scale s_b
// is also written to sb_out if given).
__global__ void sur_unstd_kernel(int64_t n, const float* __restrict__ o, float mu_bar, float scale,
                                 const float* __restrict__ base, float s_floor, float* __restrict__ out,
                                 float* __restrict__ sb_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (base) {
    const float sb = fmaxf(base[i * 2 + 1], s_floor);
    out[i * 2 + 0] = base[i * 2 + 0] + sb * o[i * 2 + 0];
    out[i * 2 + 1] = sb * expf(o[i * 2 + 1]);
    if (sb_out) sb_out[i] = sb;
  } else {
    out[i * 2 + 0] = mu_bar + scale * o[i * 2 + 0];
    out[i * 2 + 1] = expf(o[i * 2 + 1]);
  }
}

hipError_t sur_unstd(int64_t n, const float* o, float mu_bar, float scale, const float* base, float s_floor,
                     float* out, float* sb_out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sur_unstd_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, o, mu_bar, scale, base,
                     s_floor, out, sb_out);
  return hipGetLastError();
}

// ------------------------------------------------------------ partition
// Decide a cell from the surrogate when every iso-value it still carries is
// confidently inside or outside the soft bound, allowing z standard deviations
// of the surrogate's own per-level error (err_mu in field units, or in units
// of the per-cell base scale mu_unit[i] when given; err_ls in log-sigma
// units), z_p for pruning and z_a for accepting:
//   prune bit j   if |mu_hat - c_j| - z_p err_mu > t sigma_hat e^{+z_p err_ls}
//   accept bit j  if |mu_hat - c_j| + z_a err_mu < t sigma_hat e^{-z_a err_ls}
// and fall back to propagation otherwise (always at the leaf level unless
// accept_leaves).  Writes mask (decided cells) and fallback flags.
__global__ void sur_partition_kernel(int64_t n, const float* __restrict__ pred, const float* __restrict__ mu_unit,
                                     float k, IsoList iso, const uint32_t* __restrict__ pmask, float err_mu,
                                     float err_ls, float z, float z_acc,
                                     int leaf, int accept_leaves, uint32_t* __restrict__ mask,
                                     uint32_t* __restrict__ fallback) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float mu = pred[2 * i], sg = pred[2 * i + 1];
  const float hi_s = k * sg * expf(z * err_ls), lo_s = k * sg * expf(-z_acc * err_ls);
  const float unit = err_mu * (mu_unit ? mu_unit[i] : 1.f);
  const float e = z * unit, ea = z_acc * unit;
  const uint32_t pm = pmask[i];
  uint32_t acc_bits = 0;
  bool unsure = false;
  for (int j = 0; j < iso.n; ++j) {
    if (!((pm >> j) & 1u)) continue;
    const float d = fabsf(mu - iso.c[j]);
    if (d - e > hi_s) continue;                 // confidently outside
    if (d + ea < lo_s) acc_bits |= 1u << j;     // confidently inside
    else unsure = true;
  }
  if (!isfinite(mu) || !isfinite(sg)) unsure = true;  // non-finite predictions fall back
  const bool fb = unsure || (leaf && !accept_leaves && acc_bits != 0u);
  fallback[i] = fb ? 1u : 0u;
  mask[i] = fb ? 0u : acc_bits;
}

hipError_t sur_partition(int64_t n, const float* pred, const float* mu_unit, float k, const IsoList& iso,
                         const uint32_t* pmask, float err_mu, float err_ls, float z, float z_acc, int leaf,
                         int accept_leaves, uint32_t* mask, uint32_t* fallback, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sur_partition_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, pred, mu_unit, k, iso,
                     pmask, err_mu, err_ls, z, z_acc, leaf, accept_leaves, mask, fallback);
  return hipGetLastError();
}

__global__ void gather_u32_kernel(int64_t n, const uint32_t* __restrict__ idx, const uint32_t* __restrict__ src,
                                  uint32_t* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[idx[t]];
}

hipError_t gather_u32(int64_t n, const uint32_t* idx, const uint32_t* src, uint32_t* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, idx, src, dst);
  return hipGetLastError();
}

__global__ void scatter_u32_kernel(int64_t n, const uint32_t* __restrict__ idx, const uint32_t* __restrict__ src,
                                   uint32_t* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[idx[t]] = src[t];
}

hipError_t scatter_u32(int64_t n, const uint32_t* idx, const uint32_t* src, uint32_t* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, idx, src, dst);
  return hipGetLastError();
}

__global__ void scatter_u64_kernel(int64_t n, const uint32_t* __restrict__ idx, const uint64_t* __restrict__ src,
                                   uint64_t* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[idx[t]] = src[t];
}

hipError_t scatter_u64(int64_t n, const uint32_t* idx, const uint64_t* src, uint64_t* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, idx, src, dst);
  return hipGetLastError();
}

}  // namespace isx
