// Ray casting of an INR's level set (App. A) and the reduced affine form it
// is compared with (RA-Fixed).
//
// RA-Fixed keeps an affine form's input symbols and folds every symbol a
// linearisation creates into one error magnitude per neuron: a neuron is
// (x0, a[3], e) = centre, input coefficients, error.  A linear layer maps
// x0 -> W x0 + b, a -> W a, e -> |W| e (the folded symbols are independent,
// so their bound is the weighted sum of magnitudes); an activation takes the
// affine rule of Eq. 4 on the range x0 -/+ (|a|_1 + e): x0 -> alpha x0 + beta,
// a -> alpha a, e -> |alpha| e + |gamma|.  The output range is
// x0 -/+ (|a|_1 + e).  Boxes start from a = diag(h), segments from
// a = (v, 0, 0) (one symbol along the segment).
//
// Ray casting (per ray, t from t_near to t_far, step dt):
//   segment [t, t + de], de = min(dt, t_far - t), as the centre
//   o + d (t + de / 2) and half-vector d de / 2 (float64, rounded to float32);
//   its bound (UP: mu -/+ k sigma; AA, RA-Fixed: the hard range) excludes
//   the iso-value -> t += de, dt = min(2 dt, dt_max), a miss once t >= t_far;
//   otherwise, if de <= dt_min, a hit at t + de / 2; otherwise dt = de / 2.
#include "isx_internal.h"
#include "rules.h"

#include <algorithm>
#include <cmath>

namespace isx {

namespace {

// one workgroup per PT cells; LDS: [2][5][n_max][PT] (centre, a0, a1, a2, e)
template <typename T, int PT>
__global__ void rafixed_kernel(int64_t n, NetView<T> net, int n_max, const float* __restrict__ centres,
                               const float* __restrict__ halves, int seg, float* __restrict__ out32,
                               double* __restrict__ out64) {
  extern __shared__ unsigned char smem_raw[];
  T* bin = reinterpret_cast<T*>(smem_raw);
  T* bout = bin + (size_t)5 * n_max * PT;
  const int64_t p0 = (int64_t)blockIdx.x * PT;
  const int t = threadIdx.x;
  const size_t plane = (size_t)n_max * PT;
  // the input as three pseudo-neurons k = 0, 1, 2 (the axes)
  for (int i = t; i < 3 * PT; i += blockDim.x) {
    const int p = i / 3, k = i - p * 3;
    const int64_t c = p0 + p < n ? p0 + p : n - 1;
    const size_t o = (size_t)k * PT + p;
    bin[o] = T(centres[c * 3 + k]);
    const T hk = T(halves[c * 3 + k]);
    bin[plane + o] = seg ? hk : (k == 0 ? hk : T(0));
    bin[2 * plane + o] = seg ? T(0) : (k == 1 ? hk : T(0));
    bin[3 * plane + o] = seg ? T(0) : (k == 2 ? hk : T(0));
    bin[4 * plane + o] = T(0);
  }
  __syncthreads();
  T* in = bin;
  T* out = bout;
  for (int l = 0; l < net.n_linear; ++l) {
    const int ni = net.n[l], no = net.n[l + 1];
    const T* W = net.W[l];
    const bool hidden = l + 1 < net.n_linear;
    for (int m = t; m < no; m += blockDim.x) {
      T x[PT], a0[PT], a1[PT], a2[PT], e[PT];
      const T bm = net.b[l][m];
#pragma unroll
      for (int p = 0; p < PT; ++p) {
        x[p] = bm;
        a0[p] = a1[p] = a2[p] = e[p] = T(0);
      }
      for (int k = 0; k < ni; ++k) {
        const T w = W[(int64_t)m * ni + k];
        const T aw = w < T(0) ? -w : w;
        const size_t o = (size_t)k * PT;
#pragma unroll
        for (int p = 0; p < PT; ++p) {
          x[p] += w * in[o + p];
          a0[p] += w * in[plane + o + p];
          a1[p] += w * in[2 * plane + o + p];
          a2[p] += w * in[3 * plane + o + p];
          e[p] += aw * in[4 * plane + o + p];
        }
      }
#pragma unroll
      for (int p = 0; p < PT; ++p) {
        const T r = RM<T>::abs_(a0[p]) + RM<T>::abs_(a1[p]) + RM<T>::abs_(a2[p]) + e[p];
        T al = T(1), be = T(0), ga = T(0);
        if (hidden) apply_rule<T, ISX_AA>(net.act, x[p], r, al, be, ga);
        const size_t o = (size_t)m * PT + p;
        out[o] = hidden ? al * x[p] + be : x[p];
        out[plane + o] = al * a0[p];
        out[2 * plane + o] = al * a1[p];
        out[3 * plane + o] = al * a2[p];
        out[4 * plane + o] = hidden ? RM<T>::abs_(al) * e[p] + RM<T>::abs_(ga) : r;  // output: the radius
      }
    }
    __syncthreads();
    T* tmp = in;
    in = out;
    out = tmp;
  }
  if (t < PT && p0 + t < n) {
    const int64_t c = p0 + t;
    const T x0 = in[t], r = in[4 * plane + t];
    out32[c * 2] = (float)x0;
    out32[c * 2 + 1] = (float)r;
    if (out64) {
      out64[c * 2] = (double)x0;
      out64[c * 2 + 1] = (double)r;
    }
  }
}

__global__ void ray_init_kernel(int64_t n, const float* __restrict__ tnear, const float* __restrict__ tfar,
                                double step0, double* __restrict__ t, double* __restrict__ dt,
                                float* __restrict__ thit, int32_t* __restrict__ iters, uint32_t* __restrict__ active) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  t[i] = (double)tnear[i];
  dt[i] = step0;
  thit[i] = NAN;
  iters[i] = 0;
  active[i] = tnear[i] < tfar[i] ? 1u : 0u;
}

__global__ void ray_segments_kernel(int64_t n_act, const uint32_t* __restrict__ idx, const float* __restrict__ org,
                                    const float* __restrict__ dir, const float* __restrict__ tfar,
                                    const double* __restrict__ t, const double* __restrict__ dt,
                                    float* __restrict__ centres, float* __restrict__ halfvec) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_act) return;
  const int64_t i = idx[j];
  const double te = t[i], rem = __dsub_rn((double)tfar[i], te);
  const double de = dt[i] < rem ? dt[i] : rem;
  const double h = de * 0.5;
  const double tm = __dadd_rn(te, h);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double d = (double)dir[i * 3 + a];
    centres[j * 3 + a] = (float)__dadd_rn((double)org[i * 3 + a], __dmul_rn(d, tm));
    halfvec[j * 3 + a] = (float)__dmul_rn(d, h);
  }
}

__global__ void ray_step_kernel(int64_t n_act, const uint32_t* __restrict__ idx, const float* __restrict__ out32,
                                const double* __restrict__ out64, double k, double iso, double step_min,
                                double step_max, const float* __restrict__ tfar, double* __restrict__ t,
                                double* __restrict__ dt, float* __restrict__ thit, int32_t* __restrict__ iters,
                                uint32_t* __restrict__ active) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_act) return;
  const int64_t i = idx[j];
  const double te = t[i], d = dt[i], rem = __dsub_rn((double)tfar[i], te);
  const double de = d < rem ? d : rem;
  const double c = out64 ? out64[2 * j] : (double)out32[2 * j];
  const double s = out64 ? out64[2 * j + 1] : (double)out32[2 * j + 1];
  const double ks = __dmul_rn(k, s);
  const double lo = __dsub_rn(c, ks), hi = __dadd_rn(c, ks);
  iters[i] += 1;
  if (lo > iso || hi < iso) {  // the segment's bound excludes the iso-value
    const double tn = __dadd_rn(te, de);
    t[i] = tn;
    dt[i] = 2.0 * d < step_max ? 2.0 * d : step_max;
    if (tn >= (double)tfar[i]) active[i] = 0u;
  } else if (de <= step_min) {
    thit[i] = (float)__dadd_rn(te, 0.5 * de);
    active[i] = 0u;
  } else {
    dt[i] = 0.5 * de;
  }
}

}  // namespace

template <typename T, int PT>
static hipError_t launch_rafixed_t(const Model& m, int64_t n, const float* centres, const float* halves, int seg,
                                   float* out32, double* out64, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int n_max = 3;
  for (int i = 0; i <= m.n_linear; ++i) n_max = std::max(n_max, m.pw[i]);
  const int bs = std::min(1024, std::max(64, (n_max + 63) / 64 * 64));
  const size_t lds = (size_t)2 * 5 * n_max * PT * sizeof(T);
  {
    hipError_t e = ensure_lds_limit(reinterpret_cast<const void*>(&rafixed_kernel<T, PT>), (int)lds);
    if (e != hipSuccess) return e;
  }
  NetView<T> view = net_view<T>(m);
  // a launch's work-items (blocks x bs) must stay below 2^32
  const int64_t per_launch = ((int64_t(1) << 31) / bs) * PT;
  for (int64_t o = 0; o < n; o += per_launch) {
    const int64_t c = std::min(per_launch, n - o);
    hipLaunchKernelGGL((rafixed_kernel<T, PT>), dim3((unsigned)((c + PT - 1) / PT)), dim3(bs), lds, s, c, view, n_max,
                       centres + 3 * o, halves + 3 * o, seg, out32 + 2 * o, out64 ? out64 + 2 * o : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// LDS per workgroup 2 * 5 * n_max * PT values: float64 takes 2 cells (1 above
// width 512), float32 4 (2 above 512), at most 80 KiB
hipError_t launch_rafixed(const Model& m, bool f64, int64_t n, const float* centres, const float* halves, int seg,
                          float* out32, double* out64, hipStream_t s) {
  int n_max = 3;
  for (int i = 0; i <= m.n_linear; ++i) n_max = std::max(n_max, m.pw[i]);
  const bool wide = n_max > 512;
  if (f64)
    return wide ? launch_rafixed_t<double, 1>(m, n, centres, halves, seg, out32, out64, s)
                : launch_rafixed_t<double, 2>(m, n, centres, halves, seg, out32, out64, s);
  return wide ? launch_rafixed_t<float, 2>(m, n, centres, halves, seg, out32, nullptr, s)
              : launch_rafixed_t<float, 4>(m, n, centres, halves, seg, out32, nullptr, s);
}

hipError_t launch_ray_init(int64_t n, const float* tnear, const float* tfar, double step0, double* t, double* dt,
                           float* thit, int32_t* iters, uint32_t* active, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ray_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, tnear, tfar, step0, t,
                     dt, thit, iters, active);
  return hipGetLastError();
}

hipError_t launch_ray_segments(int64_t n_act, const uint32_t* idx, const float* org, const float* dir,
                               const float* tfar, const double* t, const double* dt, float* centres, float* halfvec,
                               hipStream_t s) {
  if (n_act <= 0) return hipSuccess;
  hipLaunchKernelGGL(ray_segments_kernel, dim3((unsigned)((n_act + 255) / 256)), dim3(256), 0, s, n_act, idx, org,
                     dir, tfar, t, dt, centres, halfvec);
  return hipGetLastError();
}

hipError_t launch_ray_step(int64_t n_act, const uint32_t* idx, const float* out32, const double* out64, double k,
                           double iso, double step_min, double step_max, const float* tfar, double* t, double* dt,
                           float* thit, int32_t* iters, uint32_t* active, hipStream_t s) {
  if (n_act <= 0) return hipSuccess;
  hipLaunchKernelGGL(ray_step_kernel, dim3((unsigned)((n_act + 255) / 256)), dim3(256), 0, s, n_act, idx, out32,
                     out64, k, iso, step_min, step_max, tfar, t, dt, thit, iters, active);
  return hipGetLastError();
}

}  // namespace isx
