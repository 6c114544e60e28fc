// Training-set sampling and safety-band calibration of the learned surrogate.
//
// Cells: half (on average) are drawn uniformly from the cells a plain
// extraction visited, the rest are uniform random cells of a random octree
// level in [level_lo, level_hi] (uniform level, uniform integer position).
// Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast
// splittable pseudorandom number generators", OOPSLA 2014) evaluated at
// counter seed + (4 i + stream) * golden gamma, so every cell's draw depends
// only on (seed, i).
//
// Calibration on held-out cells with known propagated (mu, sigma):
//   1. per octree level, the root-mean-square error of the prediction in mu
//      (in units of the base scale s_b when the surrogate has a base) and in
//      ln sigma -- sums per thread in a fixed cell order, then a fixed-order
//      reduction per block; the host adds the block partials in order;
//   2. per level and per band z of a fixed ladder, integer counts of cells
//      the plain soft-bound test keeps (|mu - c| <= t sigma for some carried
//      iso-value), of those the prune rule at z would drop for an iso-value
//      the plain test keeps (misses), and of cells the accept rule at z would
//      accept for an iso-value the plain test rejects (false accepts).
// The host picks the smallest band whose rate meets the target.
#include "isx_internal.h"

namespace isx {

// uniform double in [0, 1) from draw `stream` of cell i
__device__ inline double unit_draw(uint64_t seed, int64_t i, int stream) {
  const uint64_t r = splitmix64(seed + (uint64_t)(4 * i + stream) * 0x9E3779B97F4A7C15ull);
  return (double)(r >> 11) * 0x1.0p-53;
}

__device__ inline uint32_t morton_axis(uint32_t id, int axis) {
  uint32_t v = 0;
  for (int t = 0; t < 11; ++t) v |= ((id >> (3 * t + axis)) & 1u) << t;
  return v;
}

__global__ void sample_cells_kernel(int64_t n, uint64_t seed, double lo0, double lo1, double lo2, double hi0,
                                    double hi1, double hi2, int level_lo, int level_hi,
                                    const uint32_t* __restrict__ vis_ids, const int64_t* __restrict__ vis_off,
                                    int vis_levels, int64_t vis_total, float* __restrict__ centres,
                                    float* __restrict__ halves, int32_t* __restrict__ levels) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lo[3] = {lo0, lo1, lo2}, ext[3] = {hi0 - lo0, hi1 - lo1, hi2 - lo2};
  int L;
  uint32_t ijk[3];
  if (vis_total > 0 && unit_draw(seed, i, 0) < 0.5) {
    int64_t pick = (int64_t)(unit_draw(seed, i, 1) * (double)vis_total);
    if (pick >= vis_total) pick = vis_total - 1;
    L = 0;
    while (L + 1 < vis_levels && vis_off[L + 1] <= pick) ++L;
    const uint32_t id = vis_ids[pick];
    for (int a = 0; a < 3; ++a) ijk[a] = morton_axis(id, a);
  } else {
    const int nl = level_hi - level_lo + 1;
    L = level_lo + (int)(unit_draw(seed, i, 1) * nl);
    if (L > level_hi) L = level_hi;
    const uint64_t side = 1ull << L;
    for (int a = 0; a < 3; ++a) {
      const uint64_t r = splitmix64(seed + (uint64_t)(4 * i + 2) * 0x9E3779B97F4A7C15ull + (uint64_t)a * 0x632BE59BD9B4E019ull);
      ijk[a] = (uint32_t)(((r >> 11) * side) >> 53);
    }
  }
  const double inv = 1.0 / (double)(2ull << L);  // 1 / 2^(L+1)
  for (int a = 0; a < 3; ++a) {
    const double step = ext[a] * inv;
    centres[i * 3 + a] = (float)(lo[a] + (2.0 * ijk[a] + 1.0) * step);
    halves[i * 3 + a] = (float)step;
  }
  levels[i] = L;
}

hipError_t launch_sample_cells(int64_t n, uint64_t seed, const float lo[3], const float hi[3], int level_lo,
                               int level_hi, const uint32_t* vis_ids, const int64_t* vis_off, int vis_levels,
                               int64_t vis_total, float* centres, float* halves, int32_t* levels, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sample_cells_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, seed, (double)lo[0],
                     (double)lo[1], (double)lo[2], (double)hi[0], (double)hi[1], (double)hi[2], level_lo, level_hi,
                     vis_ids, vis_off, vis_levels, vis_total, centres, halves, levels);
  return hipGetLastError();
}

constexpr int kCalBlock = 256;

// Per block: per level L < n_levels, (sum dmu^2, sum dls^2, count) over the
// block's cells, reduced in a fixed order; partial [block][n_levels][3].
__global__ void calib_err_kernel(int64_t n, int64_t per_block, const float* __restrict__ pred,
                                 const float* __restrict__ targ, const float* __restrict__ unit,
                                 const int32_t* __restrict__ levels, int n_levels, double* __restrict__ partial) {
  __shared__ double red[kCalBlock];
  const int t = threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * per_block;
  const int64_t b1 = b0 + per_block < n ? b0 + per_block : n;
  for (int L = 0; L < n_levels; ++L) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = b0 + t; i < b1; i += kCalBlock) {
      if (levels[i] != L) continue;
      double dmu = (double)pred[2 * i] - (double)targ[2 * i];
      if (unit) dmu /= (double)unit[i];
      const double ps = pred[2 * i + 1] > 1e-30f ? (double)pred[2 * i + 1] : 1e-30;
      const double ts = targ[2 * i + 1] > 1e-30f ? (double)targ[2 * i + 1] : 1e-30;
      const double dls = log(ps) - log(ts);
      s[0] += dmu * dmu;
      s[1] += dls * dls;
      s[2] += 1.0;
    }
    for (int q = 0; q < 3; ++q) {
      red[t] = s[q];
      __syncthreads();
      for (int w = kCalBlock / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
      }
      if (t == 0) partial[((int64_t)blockIdx.x * n_levels + L) * 3 + q] = red[0];
      __syncthreads();
    }
  }
}

// Counts per (level, ladder band): counts[(L * n_z + zi) * 2 + 0] misses of
// the prune rule at band zi, + 1 false accepts of the accept rule at band zi;
// kept[L] cells the plain test keeps.  Integer atomics (order-independent).
__global__ void calib_count_kernel(int64_t n, const float* __restrict__ pred, const float* __restrict__ targ,
                                   const float* __restrict__ unit, const int32_t* __restrict__ levels, int n_levels,
                                   float k, IsoList iso, const float* __restrict__ err_mu,
                                   const float* __restrict__ err_ls, const float* __restrict__ ladder, int n_z,
                                   unsigned long long* __restrict__ counts, unsigned long long* __restrict__ kept) {
  __shared__ uint32_t s_cnt[16 * 16 * 2];
  __shared__ uint32_t s_kept[16];
  const int t = threadIdx.x;
  for (int q = t; q < n_levels * n_z * 2; q += blockDim.x) s_cnt[q] = 0u;
  if (t < n_levels) s_kept[t] = 0u;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + t;
  if (i < n) {
    const int L = levels[i];
    const float mu = targ[2 * i], sg = targ[2 * i + 1];
    const float mh = pred[2 * i], sh = pred[2 * i + 1];
    if (L >= 0 && L < n_levels) {
      const float em = err_mu[L] * (unit ? unit[i] : 1.f), el = err_ls[L];
      uint32_t keep_bits = 0;
      for (int j = 0; j < iso.n; ++j)
        if (fabsf(mu - iso.c[j]) <= k * sg) keep_bits |= 1u << j;
      if (keep_bits) atomicAdd(&s_kept[L], 1u);
      for (int zi = 0; zi < n_z; ++zi) {
        const float z = ladder[zi];
        const float hi_s = k * sh * expf(z * el), lo_s = k * sh * expf(-z * el);
        bool miss = false, fa = false;
        for (int j = 0; j < iso.n; ++j) {
          const float d = fabsf(mh - iso.c[j]);
          const bool pk = (keep_bits >> j) & 1u;
          if (pk && d - z * em > hi_s) miss = true;
          if (!pk && d + z * em < lo_s) fa = true;
        }
        if (miss) atomicAdd(&s_cnt[(L * n_z + zi) * 2 + 0], 1u);
        if (fa) atomicAdd(&s_cnt[(L * n_z + zi) * 2 + 1], 1u);
      }
    }
  }
  __syncthreads();
  for (int q = t; q < n_levels * n_z * 2; q += blockDim.x)
    if (s_cnt[q]) atomicAdd(&counts[q], (unsigned long long)s_cnt[q]);
  if (t < n_levels && s_kept[t]) atomicAdd(&kept[t], (unsigned long long)s_kept[t]);
}

hipError_t launch_calib_err(int64_t n, const float* pred, const float* targ, const float* unit, const int32_t* levels,
                            int n_levels, double* partial, int64_t n_blocks, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t per_block = (n + n_blocks - 1) / n_blocks;
  hipLaunchKernelGGL(calib_err_kernel, dim3((unsigned)n_blocks), dim3(kCalBlock), 0, s, n, per_block, pred, targ, unit,
                     levels, n_levels, partial);
  return hipGetLastError();
}

hipError_t launch_calib_count(int64_t n, const float* pred, const float* targ, const float* unit, const int32_t* levels,
                              int n_levels, float k, const IsoList& iso, const float* err_mu, const float* err_ls,
                              const float* ladder, int n_z, unsigned long long* counts, unsigned long long* kept,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n_levels > 16 || n_z > 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(calib_count_kernel, dim3((unsigned)((n + kCalBlock - 1) / kCalBlock)), dim3(kCalBlock), 0, s, n,
                     pred, targ, unit, levels, n_levels, k, iso, err_mu, err_ls, ladder, n_z, counts, kept);
  return hipGetLastError();
}

// He-normal draws for the surrogate's initial weights: N(0, std^2) by the
// Box-Muller transform of two SplitMix64 uniforms (host side).
void host_normal_fill(uint64_t seed, float stddev, float* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t r1 = splitmix64(seed + (uint64_t)(2 * i) * 0x9E3779B97F4A7C15ull);
    const uint64_t r2 = splitmix64(seed + (uint64_t)(2 * i + 1) * 0x9E3779B97F4A7C15ull);
    const double u1 = ((double)(r1 >> 11) + 0.5) * 0x1.0p-53, u2 = (double)(r2 >> 11) * 0x1.0p-53;
    out[i] = (float)(stddev * std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * 3.14159265358979323846 * u2));
  }
}

}  // namespace isx
