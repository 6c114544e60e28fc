// Quality of the predicted output distribution over a block (Sec. V-E,
// Eq. 11): Monte Carlo samples of the INR over the block, their histogram,
// and the KL divergence of that histogram from a Gaussian.
//
// * Sample i of block b, axis a: u = (splitmix64 output number
//   (b * ns + i) * 3 + a) >> 40) * 2^-24, coordinate c_a + h_a (2u - 1) in
//   float64 (product, then sum, each correctly rounded), rounded to float32.
// * Statistics per block (one workgroup, fixed-order sums in float64): mean,
//   root mean squared deviation, min, max of the sample values, and the
//   maximum-likelihood Gaussian of the first n_fit samples (the few-sample
//   baseline the paper calls SAMPLE).
// * Histogram: n_bins equal bins on [min, max]; v falls in bin
//   floor((v - lo) / (hi - lo) * n_bins) (float64), clamped to n_bins - 1.
//   Counts in LDS (integer atomics: order-independent).
// * Eq. 11 with p the histogram density and q = N(mu, sigma^2): ln q is a
//   quadratic, so each bin integrates in closed form,
//     KL = sum_{P_b > 0} P_b [ln(P_b / w) + ln(sigma sqrt(2 pi))
//                             + (a^2 + a c + c^2) / (6 sigma^2)],
//   w = (hi - lo) / n_bins, a = e_{b+1} - mu, c = e_b - mu, e_b = lo + b w
//   ((a^2 + a c + c^2) w equals a^3 - c^3, without its cancellation).
//   NaN when w = 0 (all samples equal) or sigma = 0.
#include "isx_internal.h"

#include <cmath>

namespace isx {

namespace {

constexpr int kDistBlock = 1024;
constexpr int kDistFields = 13;

__global__ __launch_bounds__(256) void dist_points_kernel(int64_t total, int64_t b0, int64_t ns, uint64_t seed,
                                                          const float* __restrict__ centres,
                                                          const float* __restrict__ halves, float* __restrict__ pts) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int64_t bl = idx / ns;
  const int64_t i = idx - bl * ns;
  const int64_t gb = b0 + bl;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint64_t n = ((uint64_t)gb * (uint64_t)ns + (uint64_t)i) * 3ull + (uint64_t)a;
    const uint64_t r = splitmix64(seed + n * 0x9E3779B97F4A7C15ull);
    const double s = (double)(r >> 40) * 0x1.0p-23 - 1.0;  // 2u - 1, exact
    const double x = __dadd_rn((double)centres[gb * 3 + a], __dmul_rn((double)halves[gb * 3 + a], s));
    pts[idx * 3 + a] = (float)x;
  }
}

// fixed-order tree reduction of kDistBlock doubles in LDS (sum, min or max)
template <int OP>
__device__ inline double block_reduce(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int off = kDistBlock / 2; off > 0; off >>= 1) {
    if (t < off) {
      const double a = red[t], b = red[t + off];
      red[t] = OP == 0 ? a + b : (OP == 1 ? fmin(a, b) : fmax(a, b));
    }
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// one workgroup per block: stats[b] = (mean, std, lo, hi, fit_mu, fit_sigma)
__global__ __launch_bounds__(kDistBlock) void dist_stats_kernel(int64_t ns, int n_fit, const float* __restrict__ vals,
                                                                double* __restrict__ stats) {
  __shared__ double red[kDistBlock];
  const int t = threadIdx.x;
  const float* v = vals + (int64_t)blockIdx.x * ns;
  double s = 0.0, lo = INFINITY, hi = -INFINITY;
  for (int64_t i = t; i < ns; i += kDistBlock) {
    const double x = (double)v[i];
    s += x;
    lo = fmin(lo, x);
    hi = fmax(hi, x);
  }
  s = block_reduce<0>(s, red);
  lo = block_reduce<1>(lo, red);
  hi = block_reduce<2>(hi, red);
  const double mean = s / (double)ns;
  double q = 0.0;
  for (int64_t i = t; i < ns; i += kDistBlock) {
    const double d = (double)v[i] - mean;
    q += d * d;
  }
  q = block_reduce<0>(q, red);
  if (t == 0) {
    const int nf = (int)(n_fit < ns ? n_fit : ns);
    double fs = 0.0;
    for (int i = 0; i < nf; ++i) fs += (double)v[i];
    const double fm = fs / (double)nf;
    double fq = 0.0;
    for (int i = 0; i < nf; ++i) {
      const double d = (double)v[i] - fm;
      fq += d * d;
    }
    double* o = stats + (int64_t)blockIdx.x * 6;
    o[0] = mean;
    o[1] = sqrt(q / (double)ns);
    o[2] = lo;
    o[3] = hi;
    o[4] = fm;
    o[5] = sqrt(fq / (double)nf);
  }
}

// the bin term of Eq. 11 for bin b of a Gaussian (mu, sigma)
__device__ inline double kl_bin(double P, int b, double lo, double w, double mu, double sigma) {
  const double c = lo + (double)b * w - mu;
  const double a = lo + (double)(b + 1) * w - mu;
  return P * (log(P / w) + log(sigma * 2.50662827463100050242) + (a * a + a * c + c * c) / (6.0 * sigma * sigma));
}

// one workgroup per block: histogram in LDS, then the three KL sums
__global__ __launch_bounds__(kDistBlock) void dist_hist_kl_kernel(int64_t ns, int n_bins, const float* __restrict__ vals,
                                                                  const double* __restrict__ stats,
                                                                  const double* __restrict__ up64,
                                                                  const double* __restrict__ raua64,
                                                                  double* __restrict__ out, uint32_t* __restrict__ hist) {
  extern __shared__ uint32_t cnt[];  // [n_bins]
  __shared__ double red[kDistBlock];
  const int t = threadIdx.x;
  const int64_t b = blockIdx.x;
  const float* v = vals + b * ns;
  const double* st = stats + b * 6;
  const double lo = st[2], hi = st[3];
  const double width = hi - lo;
  for (int i = t; i < n_bins; i += kDistBlock) cnt[i] = 0u;
  __syncthreads();
  for (int64_t i = t; i < ns; i += kDistBlock) {
    int k = 0;
    if (width > 0.0) {
      const double f = floor(((double)v[i] - lo) / width * (double)n_bins);
      k = f >= 0.0 ? (f < (double)(n_bins - 1) ? (int)f : n_bins - 1) : 0;  // (a NaN lands in bin 0)
    }
    atomicAdd(&cnt[k], 1u);
  }
  __syncthreads();
  if (hist)
    for (int i = t; i < n_bins; i += kDistBlock) hist[b * n_bins + i] = cnt[i];
  const double w = width / (double)n_bins;
  const double g_mu[3] = {up64[b * 2], raua64[b * 2], st[4]};
  const double g_sd[3] = {up64[b * 2 + 1], raua64[b * 2 + 1], st[5]};
  double kl[3];
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    double acc = 0.0;
    if (w > 0.0 && g_sd[g] > 0.0)
      for (int i = t; i < n_bins; i += kDistBlock) {
        if (cnt[i] == 0u) continue;
        acc += kl_bin((double)cnt[i] / (double)ns, i, lo, w, g_mu[g], g_sd[g]);
      }
    acc = block_reduce<0>(acc, red);
    kl[g] = (w > 0.0 && g_sd[g] > 0.0) ? acc : NAN;
  }
  if (t == 0) {
    double* o = out + b * kDistFields;
    o[0] = st[0];
    o[1] = st[1];
    o[2] = lo;
    o[3] = hi;
    o[4] = g_mu[0];
    o[5] = g_sd[0];
    o[6] = g_mu[1];
    o[7] = g_sd[1];
    o[8] = g_mu[2];
    o[9] = g_sd[2];
    o[10] = kl[0];
    o[11] = kl[1];
    o[12] = kl[2];
  }
}

}  // namespace

hipError_t launch_dist_points(int64_t nb, int64_t b0, int64_t ns, uint64_t seed, const float* centres,
                              const float* halves, float* pts, hipStream_t s) {
  const int64_t total = nb * ns;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(dist_points_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, b0, ns, seed,
                     centres, halves, pts);
  return hipGetLastError();
}

hipError_t launch_dist_stats(int64_t nb, int64_t ns, int n_fit, const float* vals, double* stats, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(dist_stats_kernel, dim3((unsigned)nb), dim3(kDistBlock), 0, s, ns, n_fit, vals, stats);
  return hipGetLastError();
}

hipError_t launch_dist_hist_kl(int64_t nb, int64_t ns, int n_bins, const float* vals, const double* stats,
                               const double* up64, const double* raua64, double* out, uint32_t* hist, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(dist_hist_kl_kernel, dim3((unsigned)nb), dim3(kDistBlock), (size_t)n_bins * 4, s, ns, n_bins,
                     vals, stats, up64, raua64, out, hist);
  return hipGetLastError();
}

}  // namespace isx
