// Uncertainty propagation in covariance form on BF16 MFMA for hidden widths
// whose N x N covariance does not fit one CU's LDS: the per-cell matrices
// live in global memory (HBM, L2) between the steps of a layer.
//
// The form is the one of kernels_cov.hip (Eq. 8-9 through covariances):
//   X_1 = G G^T + diag(gamma_1^2),  G = D_1 W_1 diag(h / sqrt 3)  (N x 3),
//   per hidden layer h >= 2:
//     T = W_h X_{h-1}                      (computed as T^T = X W_h^T),
//     v_j = C_h[j][j] = sum_i T[j][i] W_h[j][i],  y = W_h z + b,
//     the rule gives (alpha, beta, gamma) from (y, v),
//     C_h = T W_h^T,  X_h = D C_h D + diag(gamma^2)  (not after the last).
// Steps per layer, each a launch over the cells of a chunk:
//   1. covg_gemm (T mode): per cell, 256 x 256 tiles of X W^T on
//      v_mfma_f32_32x32x16_bf16 (rows of X staged in LDS in K chunks, weight
//      fragments streamed from the L2-resident fragment-order copy, as in
//      the LDS kernel); the epilogue stores T (bfloat16, row-major) and each
//      row's partial variance sums and magnitude sums over the tile's rows
//      (fixed slots, no atomics);
//   2. covg_rule: per cell, the partial sums in a fixed order, the float32
//      centre y = W z + b, the rule, the layer's (y, alpha, beta, gamma);
//   3. covg_gemm (X mode): T W^T, the epilogue stores D C D + diag(gamma^2)
//      (bfloat16; C is symmetric, so the tile's columns are written as rows).
// The cancellation check is the LDS kernel's (variance <= 2^-9 of the
// magnitude sum where the rule depends on sigma marks the cell).
//
// MFMA 32x32x16 bf16 layout (lane l): A (row l%32, k 8(l/32)+e), B (k
// 8(l/32)+e, column l%32), e = 0..7; accumulator register r holds (row
// 8(r/4) + 4(l/32) + r%4, column l%32).
#include "isx_internal.h"
#include "rules.h"

#include <algorithm>

namespace isx {

namespace {

typedef __bf16 gbf16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(1))) const gbf16x8 ggbf16x8;  // in global memory
typedef float gv16f __attribute__((ext_vector_type(16)));

constexpr int kGThreads = 512;  // 8 waves: 2 row groups x 4 column groups
constexpr int kGTile = 256;     // output tile edge per workgroup
constexpr int kGK = 64;         // K chunk staged in LDS (4 k-steps)
constexpr int kGStr = kGK + 8;  // LDS row stride in bfloat16 (rows 144 bytes apart)
constexpr int kGRows = 128;     // rows of a wave (4 blocks of 32)
constexpr int kGCols = 64;      // columns of a wave (2 blocks of 32)
constexpr size_t kGLds = (size_t)2 * kGTile * kGStr * 2;  // two staged buffers

enum { COVG_T = 0, COVG_V = 1, COVG_X = 2 };

// four floats rounded to bfloat16, packed low to high
__device__ __forceinline__ uint2 pack_bf16x4(float a, float b, float c, float d) {
  union {
    __bf16 h[4];
    uint2 u;
  } p;
  p.h[0] = (__bf16)a;
  p.h[1] = (__bf16)b;
  p.h[2] = (__bf16)c;
  p.h[3] = (__bf16)d;
  return p.u;
}

// Out[r][c] = sum_k A[r][k] W[c][k] on the workgroup's 256 x 256 tile of one
// cell (A: the cell's N x N bfloat16 matrix, row-major; W: fragment order).
// MODE T: store T[c][r] = Out[r][c] to Tout and the partial sums
// sum_r Out[r][c] W[c][r] (and of magnitudes) over the wave's 128 rows into
// part[(cell * NP + p) * N + c], p = row tile * 2 + row group; V: only the
// partial sums; X: store X[c][r] = alpha_r alpha_c Out[r][c] (+ the rule's
// alpha_c^2 v_c + gamma_c^2 on the diagonal) to Xout.
template <int MODE>
__global__ __launch_bounds__(kGThreads) void covg_gemm_kernel(int64_t C, int N, const __bf16* __restrict__ Ain,
                                                               const __bf16* __restrict__ Wfr,
                                                               const float* __restrict__ Wf, __bf16* __restrict__ Out,
                                                               float* __restrict__ part, float* __restrict__ partm,
                                                               const float* __restrict__ alpha,
                                                               const float* __restrict__ gamma,
                                                               const float* __restrict__ var) {
  extern __shared__ uint4 covg_smem[];
  __bf16* lds = reinterpret_cast<__bf16*>(covg_smem);  // [2][kGTile][kGStr]
  const int tiles = N / kGTile;
  const int64_t blk = blockIdx.x;
  const int64_t cell = blk / (tiles * tiles);
  if (cell >= C) return;
  const int tt = (int)(blk - cell * tiles * tiles);
  const int tr = tt / tiles, tc = tt - tr * tiles;  // row tile (A rows), column tile (W rows)
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int l32 = lane & 31, hi = lane >> 5;
  const int wr = wave & 1, wc = wave >> 1;
  const int row0 = tr * kGTile + wr * kGRows;  // the wave's first A row
  const int col0 = tc * kGTile + wc * kGCols;  // the wave's first W row
  const int64_t NN = (int64_t)N * N;
  const __bf16* A = Ain + cell * NN + (int64_t)tr * kGTile * N;  // the tile's first row
  const int KS = N / 16;

  // staging: 256 rows x 64 k = 2048 chunks of 8 bf16, 4 per thread (rows
  // t / 8 + 64 u, chunk t % 8), held in named registers between load and store
  const int sr = t >> 3, sc8 = t & 7;
  const __bf16* ag = A + (int64_t)sr * N + 8 * sc8;
  const int64_t astep = (int64_t)64 * N;  // 64 rows further
  __bf16* ls = lds + (size_t)sr * kGStr + 8 * sc8;
  constexpr int lstep = 64 * kGStr;
  uint4 s0, s1, s2, s3;
#define COVG_LOAD(K0)                                                      \
  {                                                                        \
    s0 = *reinterpret_cast<const uint4*>(ag + (K0));                       \
    s1 = *reinterpret_cast<const uint4*>(ag + astep + (K0));               \
    s2 = *reinterpret_cast<const uint4*>(ag + 2 * astep + (K0));           \
    s3 = *reinterpret_cast<const uint4*>(ag + 3 * astep + (K0));           \
  }
#define COVG_STORE(BUF)                                                    \
  {                                                                        \
    __bf16* d_ = ls + (size_t)(BUF) * kGTile * kGStr;                      \
    *reinterpret_cast<uint4*>(d_) = s0;                                    \
    *reinterpret_cast<uint4*>(d_ + lstep) = s1;                            \
    *reinterpret_cast<uint4*>(d_ + 2 * lstep) = s2;                        \
    *reinterpret_cast<uint4*>(d_ + 3 * lstep) = s3;                        \
  }

  gv16f acc[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[r][c][e] = 0.f;

  // the wave's two weight blocks, this lane's fragment of k-step 0
  ggbf16x8* wfrag[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int wb = (col0 >> 5) + r;
    wfrag[r] = (ggbf16x8*)(Wfr + ((int64_t)wb * KS * 64 + lane) * 8);
  }

  COVG_LOAD(0);
  COVG_STORE(0);
  __syncthreads();
  const int nch = N / kGK;
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) COVG_LOAD((ch + 1) * kGK);
    gbf16x8 wf[4][2];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int r = 0; r < 2; ++r) wf[kk][r] = wfrag[r][64 * (ch * 4 + kk)];
    const __bf16* lb = lds + ((size_t)buf * kGTile + wr * kGRows + l32) * kGStr + 8 * hi;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      gbf16x8 lf[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) lf[c] = *reinterpret_cast<const gbf16x8*>(lb + (size_t)c * 32 * kGStr + 16 * kk);
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lf[c], wf[kk][r], acc[r][c], 0, 0, 0);
    }
    // the other buffer was last read before the previous barrier
    if (ch + 1 < nch) COVG_STORE(buf ^ 1);
    __syncthreads();
  }
#undef COVG_LOAD
#undef COVG_STORE

  // epilogue: block (r, c) holds Out[i][j], j = col0 + 32 r + l32 (the lane's
  // column), i = row0 + 32 c + 8 q4 + 4 hi + (0..3) (register quad q4)
  if (MODE == COVG_T || MODE == COVG_V) {
    const int NP = 2 * tiles;
    const int p = tr * 2 + wr;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int j = col0 + 32 * r + l32;
      const float* wrow = Wf + (int64_t)j * N;
      float pv = 0.f, pa = 0.f;
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int i0 = row0 + 32 * c + 8 * q4 + 4 * hi;
          const float4 w4 = *reinterpret_cast<const float4*>(wrow + i0);
          const float t0 = acc[r][c][4 * q4 + 0], t1 = acc[r][c][4 * q4 + 1];
          const float t2 = acc[r][c][4 * q4 + 2], t3 = acc[r][c][4 * q4 + 3];
          pv = fmaf(w4.x, t0, fmaf(w4.y, t1, fmaf(w4.z, t2, fmaf(w4.w, t3, pv))));
          pa = fmaf(fabsf(w4.x), fabsf(t0),
                    fmaf(fabsf(w4.y), fabsf(t1), fmaf(fabsf(w4.z), fabsf(t2), fmaf(fabsf(w4.w), fabsf(t3), pa))));
          if (MODE == COVG_T)
            *reinterpret_cast<uint2*>(Out + cell * NN + (int64_t)j * N + i0) = pack_bf16x4(t0, t1, t2, t3);
        }
      pv += __shfl_xor(pv, 32);
      pa += __shfl_xor(pa, 32);
      if (hi == 0) {
        part[(cell * NP + p) * N + j] = pv;
        partm[(cell * NP + p) * N + j] = pa;
      }
    }
  } else {
    const float* al = alpha + cell * N;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int j = col0 + 32 * r + l32;
      const float aj = al[j];
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int i0 = row0 + 32 * c + 8 * q4 + 4 * hi;
          const float4 ai = *reinterpret_cast<const float4*>(al + i0);
          float x0 = ai.x * aj * acc[r][c][4 * q4 + 0], x1 = ai.y * aj * acc[r][c][4 * q4 + 1];
          float x2 = ai.z * aj * acc[r][c][4 * q4 + 2], x3 = ai.w * aj * acc[r][c][4 * q4 + 3];
          if (j >= i0 && j < i0 + 4) {
            // the diagonal from the variance the rule used
            const float g = gamma[cell * N + j];
            const float d = aj * aj * var[cell * N + j] + g * g;
            const int e = j - i0;
            x0 = e == 0 ? d : x0;
            x1 = e == 1 ? d : x1;
            x2 = e == 2 ? d : x2;
            x3 = e == 3 ? d : x3;
          }
          *reinterpret_cast<uint2*>(Out + cell * NN + (int64_t)j * N + i0) = pack_bf16x4(x0, x1, x2, x3);
        }
    }
  }
}

// Layer 1 of each cell: the rule per neuron (y = W_1 c + b_1, variance
// |W_1[j] diag(h / sqrt 3)|^2), the layer's (y, alpha, beta, gamma), and
// X_1 = G G^T + diag(gamma^2) with G = D_1 W_1 diag(h / sqrt 3), bfloat16.
template <int ACT>
__global__ __launch_bounds__(kGThreads) void covg_layer1_kernel(int64_t C, int N, const float* __restrict__ W1,
                                                                 const float* __restrict__ b1,
                                                                 const float* __restrict__ centres,
                                                                 const float* __restrict__ halves,
                                                                 float* __restrict__ vec, __bf16* __restrict__ X,
                                                                 uint32_t* __restrict__ cancel) {
  extern __shared__ float4 covg_l1[];  // [N]: (G_j, gamma_j^2)
  const int64_t cell = blockIdx.x;
  if (cell >= C) return;
  const int t = threadIdx.x;
  const float sc = 0.57735026918962576451f;
  const float hx = halves[cell * 3 + 0] * sc, hy = halves[cell * 3 + 1] * sc, hz = halves[cell * 3 + 2] * sc;
  const int64_t NC = (int64_t)N * C;
  for (int j = t; j < N; j += kGThreads) {
    const float w0 = W1[j * 3 + 0], w1 = W1[j * 3 + 1], w2 = W1[j * 3 + 2];
    const float y = b1[j] + w0 * centres[cell * 3 + 0] + w1 * centres[cell * 3 + 1] + w2 * centres[cell * 3 + 2];
    const float f0 = w0 * hx, f1 = w1 * hy, f2 = w2 * hz;
    float a, b, g;
    apply_rule<float, ISX_UP>(ACT, y, f0 * f0 + f1 * f1 + f2 * f2, a, b, g);
    covg_l1[j] = make_float4(a * f0, a * f1, a * f2, g * g);
    const int64_t o = cell * N + j;
    vec[o] = y;
    vec[NC + o] = a;
    vec[2 * NC + o] = b;
    vec[3 * NC + o] = g;
  }
  if (t == 0 && cancel) cancel[cell] = 0u;
  __syncthreads();
  // X_1 rows: 8 consecutive entries per thread and step (one 16-byte store)
  const int per_row = N / 8;
  __bf16* Xc = X + cell * (int64_t)N * N;
  for (int idx = t; idx < N * per_row; idx += kGThreads) {
    const int i = idx / per_row, k0 = 8 * (idx - i * per_row);
    const float4 gi = covg_l1[i];
    gbf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float4 gk = covg_l1[k0 + e];
      float x = gi.x * gk.x + gi.y * gk.y + gi.z * gk.z;
      if (k0 + e == i) x += gi.w;
      v[e] = (__bf16)x;
    }
    *reinterpret_cast<gbf16x8*>(Xc + (int64_t)i * N + k0) = v;
  }
}

// A variance sum is flagged when it keeps at most this fraction of the
// summed magnitude of its terms (as in the LDS kernel).
constexpr float kGCancelRatio = 0x1p-9f;

// Layer h >= 2 of each cell: the variance from the partial sums (fixed
// order), the float32 centre y = W z + b with z = alpha . y_{h-1} + beta
// (one wave per row, lanes across k, a butterfly sum), the rule, and the
// layer's (y, alpha, beta, gamma) and variance.
template <int ACT>
__global__ __launch_bounds__(kGThreads) void covg_rule_kernel(int64_t C, int N, int NP, const float* __restrict__ W,
                                                               const float* __restrict__ bias,
                                                               const float* __restrict__ vprev,
                                                               float* __restrict__ vcur,
                                                               const float* __restrict__ part,
                                                               const float* __restrict__ partm,
                                                               float* __restrict__ var, uint32_t* __restrict__ cancel) {
  extern __shared__ float covg_z[];  // [N]
  const int64_t cell = blockIdx.x;
  if (cell >= C) return;
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int64_t NC = (int64_t)N * C;
  for (int k = t; k < N; k += kGThreads) {
    const int64_t o = cell * N + k;
    covg_z[k] = vprev[NC + o] * vprev[o] + vprev[2 * NC + o];
  }
  __syncthreads();
  for (int j = wave; j < N; j += kGThreads / 64) {
    const float* wrow = W + (int64_t)j * N;
    float s = 0.f;
    for (int k = lane; k < N; k += 64) s = fmaf(wrow[k], covg_z[k], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) {
      float v = 0.f, av = 0.f;
      for (int p = 0; p < NP; ++p) {
        v += part[(cell * NP + p) * N + j];
        av += partm[(cell * NP + p) * N + j];
      }
      const float y = s + bias[j];
      if (cancel && av > 0.f && !(v > kGCancelRatio * av)) {
        const float s6 = 6.f * sqrtf(fmaxf(v, 0.f) + 0x1p-7f * av);
        const bool dep = ACT == ISX_SINE ? (1.f + 2.f * fabsf(y)) * 0x1p-9f * av > 0x1p-20f
                                         : (ACT == ISX_ELU ? y < s6 : fabsf(y) < s6);
        if (dep) cancel[cell] = 1u;
      }
      float a, b, g;
      apply_rule<float, ISX_UP>(ACT, y, v, a, b, g);
      const int64_t o = cell * N + j;
      vcur[o] = y;
      vcur[NC + o] = a;
      vcur[2 * NC + o] = b;
      vcur[3 * NC + o] = g;
      var[o] = v;
    }
  }
}

}  // namespace

int covg_width(const Model& m) {
  if (m.n_linear < 3) return 0;
  const int n = m.pw[1];
  for (int h = 1; h < m.n_linear; ++h)
    if (m.pw[h] != n) return 0;
  for (int l = 1; l + 1 < m.n_linear; ++l)
    if (!m.L[l].Wfr) return 0;
  return (n % kGTile == 0 && n <= ISX_MAX_WIDTH) ? n : 0;
}

size_t covg_scratch_bytes(const Model& m, int64_t C) {
  const int N = covg_width(m);
  if (!N) return 0;
  const int NP = 2 * (N / kGTile);
  // X and T (bfloat16), the partial sums and magnitudes, the variances
  return (size_t)C * ((size_t)2 * N * N * 2 + (size_t)2 * NP * N * 4 + (size_t)N * 4);
}

int64_t covg_max_chunk(const Model& m) {
  const int N = covg_width(m);
  if (!N) return 0;
  const int64_t tiles = N / kGTile;
  return ((int64_t)1 << 22) / (tiles * tiles);
}

double covg_flops_per_cell(const Model& m) {
  const int N = covg_width(m);
  const int Lh = m.n_linear - 1;
  const double n3 = (double)N * N * N;
  // the T product of every layer >= 2, the C product of every layer but the
  // last, the centre (2 N^2 per layer)
  return 2.0 * n3 * (Lh - 1) + 2.0 * n3 * std::max(0, Lh - 2) + 2.0 * (double)N * N * Lh;
}

template <int ACT>
static hipError_t covg_run(const Model& m, int64_t C, const float* centres, const float* halves, float* vec,
                           uint32_t* cancel, void* scratch, hipStream_t s) {
  const int N = covg_width(m);
  const int tiles = N / kGTile, NP = 2 * tiles;
  const int64_t NN = (int64_t)N * N;
  const int Lh = m.n_linear - 1;
  __bf16* X = reinterpret_cast<__bf16*>(scratch);
  __bf16* T = X + C * NN;
  float* part = reinterpret_cast<float*>(T + C * NN);
  float* partm = part + C * NP * N;
  float* var = partm + C * NP * N;
  // the gemm's grid: C tiles^2 blocks of 512 threads, at most 2^31 work-items
  if (C > covg_max_chunk(m)) return hipErrorInvalidValue;
  {
    hipError_t e = ensure_lds_limit(reinterpret_cast<const void*>(&covg_gemm_kernel<COVG_T>), (int)kGLds);
    if (e == hipSuccess) e = ensure_lds_limit(reinterpret_cast<const void*>(&covg_gemm_kernel<COVG_V>), (int)kGLds);
    if (e == hipSuccess) e = ensure_lds_limit(reinterpret_cast<const void*>(&covg_gemm_kernel<COVG_X>), (int)kGLds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((covg_layer1_kernel<ACT>), dim3((unsigned)C), dim3(kGThreads), (size_t)N * sizeof(float4), s, C,
                     N, m.L[0].W, m.L[0].b, centres, halves, vec, X, cancel);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const float* vprev = vec;
  float* vcur = vec + 4 * NN / N * C;  // 4 N C floats per layer
  const dim3 grid((unsigned)(C * tiles * tiles));
  for (int h = 2; h <= Lh; ++h) {
    const Layer& L = m.L[h - 1];
    const __bf16* Wfr = reinterpret_cast<const __bf16*>(L.Wfr);
    const bool last = h == Lh;
    if (last)
      hipLaunchKernelGGL(covg_gemm_kernel<COVG_V>, grid, dim3(kGThreads), kGLds, s, C, N, X, Wfr, L.W, (__bf16*)nullptr,
                         part, partm, (const float*)nullptr, (const float*)nullptr, (const float*)nullptr);
    else
      hipLaunchKernelGGL(covg_gemm_kernel<COVG_T>, grid, dim3(kGThreads), kGLds, s, C, N, X, Wfr, L.W, T, part, partm,
                         (const float*)nullptr, (const float*)nullptr, (const float*)nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((covg_rule_kernel<ACT>), dim3((unsigned)C), dim3(kGThreads), (size_t)N * sizeof(float), s, C, N,
                       NP, L.W, L.b, vprev, vcur, part, partm, var, cancel);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!last) {
      const int64_t NC = (int64_t)N * C;
      hipLaunchKernelGGL(covg_gemm_kernel<COVG_X>, grid, dim3(kGThreads), kGLds, s, C, N, T, Wfr, L.W, X,
                         (float*)nullptr, (float*)nullptr, vcur + NC, vcur + 3 * NC, var);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    vprev = vcur;
    vcur += 4 * (int64_t)N * C;
  }
  return hipSuccess;
}

hipError_t launch_up_cov_global(const Model& m, int64_t C, const float* centres, const float* halves, float* vec,
                                uint32_t* cancel, void* scratch, hipStream_t s) {
  if (C <= 0) return hipSuccess;
  if (!covg_width(m) || !scratch) return hipErrorInvalidValue;
  switch (m.act) {
    case ISX_SINE: return covg_run<ISX_SINE>(m, C, centres, halves, vec, cancel, scratch, s);
    case ISX_ELU: return covg_run<ISX_ELU>(m, C, centres, halves, vec, cancel, scratch, s);
    default: return covg_run<ISX_RELU>(m, C, centres, halves, vec, cancel, scratch, s);
  }
}

}  // namespace isx
