// BF16 propagation: hidden-layer coefficient products on
// v_mfma_f32_32x32x16_bf16 with float32 accumulation.
//
// Storage: coefficient blocks are bfloat16, [cell][column][neuron] (a
// column's neurons contiguous); column 0 (the centre in the float32 layout)
// is kept zero and the centres travel in float32 vectors instead, computed on
// the vector ALUs: the centre is a plain point evaluation of the linearised
// network, and keeping it in float32 keeps the classification margin free of
// bfloat16 rounding.  Row statistics, the ReLU rule and all vectors are
// float32.  The newest symbol block of a layer, W_h diag(gamma_{h-1}), is not
// stored: the next layer multiplies by the constant W_h^T (bf16, shared by
// all cells) and scales the resulting columns by gamma_{h-1}, which halves
// the coefficient traffic to and from HBM.
//
// Per cell and block of BM neurons, each wave owns 32*RB neurons and keeps
// the operand A = bf16(W[rows, :] * alpha_{h-1}) for all K <= 256 in
// registers (alpha folded into the weights once per cell, rounded once from
// float32), so per k-step it only reads one B fragment (16 bytes per lane)
// from LDS per 32-column block.  Column tiles of BN columns are staged
// global -> registers -> LDS with the next tile's loads in flight while the
// current tile is multiplied (two LDS buffers); output tiles are staged in
// LDS too, so that global stores are whole 16-byte chunks of contiguous
// neurons.
//
// Operand layout of 32x32x16 bf16 (lane l): A elements (row l%32, k
// 8*(l/32)+e), B elements (k 8*(l/32)+e, column l%32), e = 0..7; accumulator
// register r holds (row 8*(r/4) + 4*(l/32) + r%4, column l%32).
#include "isx_internal.h"
#include "rules.h"

#include <algorithm>

namespace isx {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float v16f32 __attribute__((ext_vector_type(16)));

template <int METHOD>
__device__ __forceinline__ float bstat(float v) {
  return METHOD == ISX_UP ? v * v : fabsf(v);
}


// ------------------------------------------------------------- layer 1
template <int METHOD>
__global__ void layer1_bf16_kernel(int64_t C, int n, const float* __restrict__ centres,
                                   const float* __restrict__ halves, const float* __restrict__ W1,
                                   const float* __restrict__ b1, __bf16* __restrict__ Fout, float* __restrict__ Y,
                                   float* __restrict__ A, float* __restrict__ B, float* __restrict__ G,
                                   float* __restrict__ S, int act) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= C * n) return;
  const int64_t cell = idx / n;
  const int m = (int)(idx - cell * n);
  const float s = METHOD == ISX_UP ? 0.57735026918962576451f : 1.f;
  float f[3];
  float y = b1[m], stat = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float w = W1[m * 3 + i];
    y += w * centres[cell * 3 + i];
    f[i] = w * (halves[cell * 3 + i] * s);
    stat += bstat<METHOD>(f[i]);
  }
  float a, b, g;
  apply_rule<float, METHOD>(act, y, stat, a, b, g);
  Y[idx] = y;
  A[idx] = a;
  B[idx] = b;
  G[idx] = g;
  if (S) S[idx] = stat;
  if (Fout) {
    __bf16* col = Fout + cell * (int64_t)kHeadCols * n + m;
    col[0] = (__bf16)0.f;
    col[(int64_t)1 * n] = (__bf16)f[0];
    col[(int64_t)2 * n] = (__bf16)f[1];
    col[(int64_t)3 * n] = (__bf16)f[2];
#pragma unroll
    for (int c = 4; c < kHeadCols; ++c) col[(int64_t)c * n] = (__bf16)0.f;
  }
}

// -------------------------------------------------------- hidden layer
constexpr int kKMax = 512;  // largest n_in held in registers

// Hidden layer h.  Logical input block of the cell: F_{h-1} = [stored part
// (s_in columns, read from Fin) | W_{h-1} diag(gamma_{h-2}) (g_in columns)].
// The second part is never stored: its B operand is the constant bf16 matrix
// W_{h-1}^T (shared by all cells, L2-resident) and its output columns are
// scaled by gamma_{h-2} in the epilogue.  The output block written to Fout
// is the product over all s_in + g_in input columns; this layer's own new
// symbol block W_h diag(gamma_{h-1}) only contributes its statistic.
template <int METHOD, int NW, int RB, int NB, int KMAXT>
__global__ __launch_bounds__(64 * NW) void hidden_mfma_bf16_kernel(
    int64_t C, int n_in, int n_out, int64_t s_in, int g_in, int rb_count, const float* __restrict__ W,
    const float* __restrict__ bias, const __bf16* __restrict__ WtPrev, const float* __restrict__ Gprev2,
    const __bf16* __restrict__ Fin, const float* __restrict__ Yin, const float* __restrict__ Ain,
    const float* __restrict__ Bin, const float* __restrict__ Gin, __bf16* __restrict__ Fout, float* __restrict__ Y,
    float* __restrict__ A, float* __restrict__ B, float* __restrict__ G, float* __restrict__ S, int act) {
  constexpr int THREADS = 64 * NW;
  constexpr int BN = 32 * NB;                  // columns per tile
  constexpr int BM = 32 * RB * NW;             // output neurons per workgroup
  constexpr int KS = KMAXT / 16;               // k-steps (K zero-filled up to KMAXT)
  constexpr int CPC = KMAXT / 8;               // 16-byte chunks per staged column
  constexpr int PF = BN * CPC / THREADS;       // chunks per thread per tile
  constexpr int OSTR = BM + 8;                 // bf16 per column of the staged output tile
  constexpr int OCH = BN * BM / 8;             // 16-byte chunks of an output tile

  extern __shared__ uint4 lds4[];
  // LDS: two staged input tiles [BN][LSTR] then two output tiles [BN][OSTR]
  // (addresses are formed from the __shared__ base so they stay LDS accesses)
  constexpr int LSTR = KMAXT + 8;  // bf16 per staged input column (padded against bank conflicts)
  __bf16* const lds = reinterpret_cast<__bf16*>(lds4);
  __shared__ float s_z[KMAXT];
  __shared__ float s_alpha[KMAXT];
  __shared__ float s_gamma[KMAXT];
  __shared__ float s_gp[kKMax];  // indexed by the width of layer h-2, which may exceed KMAXT
  __shared__ float s_y[BM];
  __shared__ float s_row[BM];
  __shared__ float s_gen[BM];

  const int64_t blk = blockIdx.x;
  const int xcd = (int)(blk & 7);
  const int64_t q = blk >> 3;
  const int rb = (int)(q % rb_count);
  const int64_t cell = (q / rb_count) * 8 + xcd;
  if (cell >= C) return;
  const int m0 = rb * BM;
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform
  const int nch = n_in / 8;
  const int64_t cin = s_in + g_in;
  const __bf16* fin = Fin + cell * s_in * n_in;
  __bf16* fout = Fout ? Fout + cell * cin * n_out : nullptr;

  for (int k = t; k < n_in; k += THREADS) {
    const float a = Ain[cell * n_in + k];
    s_alpha[k] = a;
    s_z[k] = a * Yin[cell * n_in + k] + Bin[cell * n_in + k];
    s_gamma[k] = Gin[cell * n_in + k];
  }
  for (int j = t; j < g_in; j += THREADS) s_gp[j] = Gprev2[cell * g_in + j];
  __syncthreads();

  // One pass over the wave's float32 weight rows builds, per row: the A
  // fragments bf16(W[row, k] alpha[k]) (rounded once), the float32 centre
  // y = W z + b (z = alpha . y_{h-1} + beta), and the statistic of the new
  // symbol block W[row, k] gamma[k].  Lanes l and l+32 hold the two halves of
  // each row's k range.
  bf16x8 wa[RB][KS];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int rl = wave * 32 * RB + r * 32 + (lane & 31);
    const float* wrow = W + (int64_t)(m0 + rl) * n_in;
    float yc = 0.f, gs = 0.f;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      bf16x8 v;
      const int k = 16 * ks + 8 * (lane >> 5);
      if (k < n_in) {
        const float4 lo = *reinterpret_cast<const float4*>(wrow + k);
        const float4 hi = *reinterpret_cast<const float4*>(wrow + k + 4);
        const float wv[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          v[e] = (__bf16)(wv[e] * s_alpha[k + e]);
          yc += wv[e] * s_z[k + e];
          gs += bstat<METHOD>(wv[e] * s_gamma[k + e]);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (__bf16)0.f;
      }
      wa[r][ks] = v;
    }
    yc += __shfl_xor(yc, 32);
    gs += __shfl_xor(gs, 32);
    if (lane < 32) {
      s_y[rl] = yc + bias[m0 + rl];
      s_gen[rl] = gs;
    }
  }

  float st[RB][16];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int i = 0; i < 16; ++i) st[r][i] = 0.f;

  const int64_t ntiles = (cin + BN - 1) / BN;
  uint4 pf[PF];
  auto prefetch = [&](int64_t nt) {
    const int64_t c0 = nt * BN;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int idx = t + i * THREADS;
      const int col = idx / CPC, kc = idx - col * CPC;
      const int64_t gc = c0 + col;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (kc < nch) {
        if (gc > 0 && gc < s_in)
          v = *reinterpret_cast<const uint4*>(fin + gc * n_in + 8 * kc);
        else if (gc >= s_in && gc < cin)
          v = *reinterpret_cast<const uint4*>(WtPrev + (gc - s_in) * n_in + 8 * kc);
      }
      pf[i] = v;
    }
  };
  // chunks beyond n_in are written as zeros, so every k-step is valid
  auto stage = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int idx = t + i * THREADS;
      const int col = idx / CPC, kc = idx - col * CPC;
      *reinterpret_cast<uint4*>(lds + (size_t)buf * BN * LSTR + (size_t)col * LSTR + 8 * kc) = pf[i];
    }
  };
  auto write_out = [&](int64_t nt) {
    const int64_t c0 = nt * BN;
    const __bf16* ob = lds + (size_t)2 * BN * LSTR + (size_t)(nt & 1) * BN * OSTR;
    for (int i = t; i < OCH; i += THREADS) {
      const int col = i / (BM / 8), rc = i - col * (BM / 8);
      if (c0 + col < cin)
        *reinterpret_cast<uint4*>(fout + (c0 + col) * n_out + m0 + 8 * rc) =
            *reinterpret_cast<const uint4*>(ob + (size_t)col * OSTR + 8 * rc);
    }
  };

  if (ntiles > 0) {
    prefetch(0);
    stage(0);
  }
  __syncthreads();
  for (int64_t nt = 0; nt < ntiles; ++nt) {
    const int64_t c0 = nt * BN;
    if (nt + 1 < ntiles) prefetch(nt + 1);
    const __bf16* bt = lds + (size_t)(nt & 1) * BN * LSTR;
    v16f32 acc[RB][NB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[r][nb][i] = 0.f;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const bf16x8 bv =
            *reinterpret_cast<const bf16x8*>(bt + (size_t)(nb * 32 + (lane & 31)) * LSTR + 16 * ks + 8 * (lane >> 5));
#pragma unroll
        for (int r = 0; r < RB; ++r)
          acc[r][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[r][ks], bv, acc[r][nb], 0, 0, 0);
      }
    }
    // epilogue: gamma scaling of the regenerated columns, float32
    // statistics, bf16 output tile staged in LDS
    __bf16* ob = lds + (size_t)2 * BN * LSTR + (size_t)(nt & 1) * BN * OSTR;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int cl = nb * 32 + (lane & 31);
      const int64_t col = c0 + cl;
      if (col < cin) {
        const float sc = col == 0 ? 0.f : (col >= s_in ? s_gp[col - s_in] : 1.f);
#pragma unroll
        for (int r = 0; r < RB; ++r) {
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4) {
            const int rl = wave * 32 * RB + r * 32 + 8 * q4 + 4 * (lane >> 5);
            const float v0 = acc[r][nb][4 * q4 + 0] * sc, v1 = acc[r][nb][4 * q4 + 1] * sc;
            const float v2 = acc[r][nb][4 * q4 + 2] * sc, v3 = acc[r][nb][4 * q4 + 3] * sc;
            st[r][4 * q4 + 0] += bstat<METHOD>(v0);
            st[r][4 * q4 + 1] += bstat<METHOD>(v1);
            st[r][4 * q4 + 2] += bstat<METHOD>(v2);
            st[r][4 * q4 + 3] += bstat<METHOD>(v3);
            if (fout) {
              union {
                __bf16 h[4];
                uint2 u;
              } pk;
              pk.h[0] = (__bf16)v0;
              pk.h[1] = (__bf16)v1;
              pk.h[2] = (__bf16)v2;
              pk.h[3] = (__bf16)v3;
              *reinterpret_cast<uint2*>(ob + (size_t)cl * OSTR + rl) = pk.u;
            }
          }
        }
      }
    }
    if (nt + 1 < ntiles) stage((int)((nt + 1) & 1));
    __syncthreads();
    if (fout) write_out(nt);
  }
  // reduce each row's statistic over the 32 lanes holding its columns
#pragma unroll
  for (int r = 0; r < RB; ++r) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      float v = st[r][i];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 8);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 1);
      st[r][i] = v;
    }
    if ((lane & 31) == 0) {
#pragma unroll
      for (int i = 0; i < 16; ++i) s_row[wave * 32 * RB + r * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3)] = st[r][i];
    }
  }
  __syncthreads();
  for (int m = t; m < BM; m += THREADS) {
    const float tot = s_row[m] + s_gen[m];
    float a, b, gg;
    apply_rule<float, METHOD>(act, s_y[m], tot, a, b, gg);
    const int64_t o = cell * n_out + m0 + m;
    Y[o] = s_y[m];
    A[o] = a;
    B[o] = b;
    G[o] = gg;
    if (S) S[o] = tot;
  }
}

bool bf16_supported(const Model& m) {
  for (int h = 2; h < m.n_linear; ++h)
    if (m.pw[h - 1] > kKMax || m.pw[h - 1] % 16 != 0 || m.pw[h] % 32 != 0) return false;
  return true;
}

template <int METHOD, int NW, int RB, int NB, int KMAXT>
static hipError_t launch_bf16_k(int64_t C, int n_in, int n_out, int64_t s_in, int g_in, const float* W,
                                const float* bias, const __bf16* WtPrev, const float* Gprev2, const __bf16* Fin,
                                const float* Yin, const float* Ain, const float* Bin, const float* Gin, __bf16* Fout,
                                float* Y, float* A, float* B, float* G, float* S, int act, hipStream_t s) {
  constexpr int BM = 32 * RB * NW;
  constexpr int BN = 32 * NB;
  const int rb_count = n_out / BM;
  const int64_t blocks = ((C + 7) / 8) * 8 * rb_count;
  const size_t lds = (2 * (size_t)BN * (KMAXT + 8) + 2 * (size_t)BN * (BM + 8)) * sizeof(__bf16);
  {
    hipError_t e = ensure_lds_limit((const void*)hidden_mfma_bf16_kernel<METHOD, NW, RB, NB, KMAXT>, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((hidden_mfma_bf16_kernel<METHOD, NW, RB, NB, KMAXT>), dim3((unsigned)blocks), dim3(64 * NW), lds, s, C,
                     n_in, n_out, s_in, g_in, rb_count, W, bias, WtPrev, Gprev2, Fin, Yin, Ain, Bin, Gin, Fout, Y, A,
                     B, G, S, act);
  return hipGetLastError();
}

// Tile-shape variants (waves NW, 32-row blocks per wave RB, 32-column blocks
// per tile NB); `variant` 0 picks the default for the width, others force one
// (used by the tuner).
template <int METHOD, int NW, int RB, int NB>
static hipError_t launch_bf16_v(int64_t C, int n_in, int n_out, int64_t s_in, int g_in, const float* W,
                                const float* bias, const __bf16* WtPrev, const float* Gprev2, const __bf16* Fin,
                                const float* Yin, const float* Ain, const float* Bin, const float* Gin, __bf16* Fout,
                                float* Y, float* A, float* B, float* G, float* S, int act, hipStream_t s) {
#define ISX_BF16_KARGS C, n_in, n_out, s_in, g_in, W, bias, WtPrev, Gprev2, Fin, Yin, Ain, Bin, Gin, Fout, Y, A, B, G, S, act, s
  if (n_in <= 64) return launch_bf16_k<METHOD, NW, RB, NB, 64>(ISX_BF16_KARGS);
  if (n_in <= 128) return launch_bf16_k<METHOD, NW, RB, NB, 128>(ISX_BF16_KARGS);
  if (n_in <= 256) return launch_bf16_k<METHOD, NW, RB, NB, 256>(ISX_BF16_KARGS);
  // K = 512: the operand rows fill 128 registers per lane, and one 32-column
  // block per tile keeps the staged tiles within LDS (2 x 32 x 520 bf16 in,
  // 2 x 32 x (BM + 8) out)
  return launch_bf16_k<METHOD, NW, RB, 1, 512>(ISX_BF16_KARGS);
#undef ISX_BF16_KARGS
}

template <int METHOD>
static hipError_t launch_bf16_m(int variant, int64_t C, int n_in, int n_out, int64_t s_in, int g_in, const float* W,
                                const float* bias, const __bf16* WtPrev, const float* Gprev2, const __bf16* Fin,
                                const float* Yin, const float* Ain, const float* Bin, const float* Gin, __bf16* Fout,
                                float* Y, float* A, float* B, float* G, float* S, int act, hipStream_t s) {
#define ISX_BF16_ARGS C, n_in, n_out, s_in, g_in, W, bias, WtPrev, Gprev2, Fin, Yin, Ain, Bin, Gin, Fout, Y, A, B, G, S, act, s
  if (variant == 1 && n_out % 256 == 0) return launch_bf16_v<METHOD, 4, 2, 2>(ISX_BF16_ARGS);
  if (variant == 3 && n_out % 128 == 0) return launch_bf16_v<METHOD, 4, 1, 2>(ISX_BF16_ARGS);
  if (variant == 4 && n_out % 64 == 0) return launch_bf16_v<METHOD, 2, 1, 2>(ISX_BF16_ARGS);
  if (n_out % 256 == 0) return launch_bf16_v<METHOD, 8, 1, 2>(ISX_BF16_ARGS);
  if (n_out % 128 == 0) return launch_bf16_v<METHOD, 4, 1, 2>(ISX_BF16_ARGS);
  if (n_out % 64 == 0) return launch_bf16_v<METHOD, 2, 1, 2>(ISX_BF16_ARGS);
  return launch_bf16_v<METHOD, 1, 1, 1>(ISX_BF16_ARGS);
#undef ISX_BF16_ARGS
}

size_t prop_F_elems_bf16(const Model& m, int64_t C) {
  size_t best = 1;
  for (int h = 1; h < m.hidden(); ++h) best = std::max(best, (size_t)(m.stored_cols(h) * m.pw[h]));
  return best * (size_t)C;
}

// defined in kernels_prop.hip
hipError_t launch_output_f32(const Model& m, isx_method method, int64_t C, float* vec, const float* halves,
                             float* out32, hipStream_t s);

hipError_t propagate_bf16(const PropArgs& a, PropWork<float>& w, uint16_t* Fbf_raw[2], size_t) {
  const Model& m = *a.m;
  const int64_t C = a.C;
  if (C <= 0) return hipSuccess;
  if (!bf16_supported(m) && !a.covg) return hipErrorNotSupported;
  __bf16* Fbf[2] = {reinterpret_cast<__bf16*>(Fbf_raw[0]), reinterpret_cast<__bf16*>(Fbf_raw[1])};
  const int Lh = m.hidden();
  float *Y[ISX_MAX_LINEAR] = {}, *A[ISX_MAX_LINEAR] = {}, *B[ISX_MAX_LINEAR] = {}, *G[ISX_MAX_LINEAR] = {};
  {
    size_t off = 0;
    for (int h = 1; h <= Lh; ++h) {
      const size_t n = (size_t)m.pw[h] * C;
      Y[h] = w.vec + off;
      A[h] = w.vec + off + n;
      B[h] = w.vec + off + 2 * n;
      G[h] = w.vec + off + 3 * n;
      off += 4 * n;
    }
  }
  if (a.method == ISX_UP && a.covg) {
    // covariance form with the per-cell matrices in global memory
    Profiler::Rec rec{};
    double vec_bytes = 24.0;
    for (int h = 1; h <= Lh; ++h) vec_bytes += 16.0 * m.pw[h];
    const bool prof = a.prof && a.prof->begin(rec, ISX_KERNEL_HIDDEN_COV_BF16, covg_flops_per_cell(m) * (double)C,
                                              vec_bytes * (double)C, a.stream);
    hipError_t e = launch_up_cov_global(m, C, a.centres, a.halves, w.vec, a.cancel, Fbf_raw[0], a.stream);
    if (prof) a.prof->end(rec, a.stream);
    if (e != hipSuccess) return e;
    Profiler::Rec rec2{};
    const bool prof2 = a.prof && a.prof->begin(rec2, ISX_KERNEL_OUTPUT, output_flops_per_cell(m) * (double)C,
                                               4.0 * C * 4.0 * (double)m.pw[1] * Lh, a.stream);
    e = launch_output_mfma(m, a.method, C, Y, A, B, G, a.halves, a.out32, a.stream);
    if (prof2) a.prof->end(rec2, a.stream);
    return e;
  }
  if (a.method == ISX_UP && a.up_form == 0 && cov_supported(m)) {
    // covariance form: one fused launch for every hidden layer
    Profiler::Rec rec{};
    double vec_bytes = 24.0;
    for (int h = 1; h <= Lh; ++h) vec_bytes += 16.0 * m.pw[h];
    const bool prof = a.prof && a.prof->begin(rec, ISX_KERNEL_HIDDEN_COV_BF16, cov_flops_per_cell(m) * (double)C,
                                              vec_bytes * (double)C, a.stream);
    hipError_t e = launch_up_cov_bf16(m, C, a.centres, a.halves, w.vec, a.cancel, a.stream);
    if (prof) a.prof->end(rec, a.stream);
    if (e != hipSuccess) return e;
    Profiler::Rec rec2{};
    const bool prof2 = a.prof && a.prof->begin(rec2, ISX_KERNEL_OUTPUT, output_flops_per_cell(m) * (double)C,
                                               4.0 * C * 4.0 * (double)m.pw[1] * Lh, a.stream);
    // (the UP read-off on BF16 MFMA with hi/lo splits, float32 accuracy)
    e = output_bf16_supported(m) && !a.readoff_f32 ? launch_output_bf16(m, C, Y, A, B, G, a.halves, a.out32, a.stream)
                                 : launch_output_mfma(m, a.method, C, Y, A, B, G, a.halves, a.out32, a.stream);
    if (prof2) a.prof->end(rec2, a.stream);
    return e;
  }
  // AA rounding margin (kernels_margin.hip): bfloat16 operands from layer 2
  // on (u_b = 2^-8), float32 accumulation; the row statistics S and radii R
  // follow the four vectors of every layer in the vector buffer
  // (RA-UA runs the AA layers below and reads off with the uniform assumption)
  const bool marg = a.method == ISX_AA && a.aa_margin;
  float *S[ISX_MAX_LINEAR] = {}, *R[ISX_MAX_LINEAR] = {};
  if (marg) {
    size_t tot = 0;
    for (int h = 1; h <= Lh; ++h) tot += (size_t)m.pw[h] * C;
    size_t off = 4 * tot;
    for (int h = 1; h <= Lh; ++h) {
      S[h] = w.vec + off;
      R[h] = w.vec + off + tot;
      off += (size_t)m.pw[h] * C;
    }
  }
  int64_t D = 3;  // symbol columns summed by the row statistic of the layer
  int cur = 0;
  {
    const int n1 = m.pw[1];
    const int64_t threads = C * n1;
    if (a.method == ISX_UP)
      hipLaunchKernelGGL(layer1_bf16_kernel<ISX_UP>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, a.stream,
                         C, n1, a.centres, a.halves, m.L[0].W, m.L[0].b, Lh >= 2 ? Fbf[cur] : nullptr, Y[1], A[1], B[1],
                         G[1], (float*)nullptr, m.act);
    else
      hipLaunchKernelGGL(layer1_bf16_kernel<ISX_AA>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, a.stream,
                         C, n1, a.centres, a.halves, m.L[0].W, m.L[0].b, Lh >= 2 ? Fbf[cur] : nullptr, Y[1], A[1], B[1],
                         G[1], S[1], m.act);
    if (marg) {
      hipError_t e = launch_aa_margin_hidden<float>(C, 3, n1, m.L[0].Wt, m.L[0].b, nullptr, nullptr, nullptr, nullptr,
                                                    a.centres, a.halves, Y[1], S[1], A[1], B[1], G[1], R[1],
                                                    aa_margin_consts<float>(0x1p-24, 0.0, 3, D), a.stream);
      if (e != hipSuccess) return e;
    }
  }
  for (int h = 2; h <= Lh; ++h) {
    const int n_in = m.pw[h - 1], n_out = m.pw[h];
    const int64_t s_in = m.stored_cols(h - 1);
    const int g_in = h >= 3 ? m.pw[h - 2] : 0;
    __bf16* Fout = h < Lh ? Fbf[cur ^ 1] : nullptr;
    Profiler::Rec rec{};
    bool prof = false;
    if (a.prof && a.prof->on) {
      int64_t real_cols = 3;  // symbol columns (the centre is not part of the bf16 product)
      for (int i = 1; i <= h - 2; ++i) real_cols += m.widths[i];
      const double flops = 2.0 * m.widths[h] * m.widths[h - 1] * (double)real_cols * (double)C;
      // HBM: the stored part of the input block is read, the output block written
      const double stored_in = (double)(real_cols - (h >= 3 ? m.widths[h - 2] : 0));
      const double bytes = 2.0 * C * (stored_in * m.widths[h - 1] + (h < Lh ? (double)real_cols * m.widths[h] : 0.0));
      prof = a.prof->begin(rec, ISX_KERNEL_HIDDEN_BF16, flops, bytes, a.stream);
    }
    const Layer& L = m.L[h - 1];
    const __bf16* WtPrev = reinterpret_cast<const __bf16*>(m.L[h - 2].Wtbf);
    const float* Gp2 = h >= 3 ? G[h - 2] : nullptr;
    hipError_t e = a.method == ISX_UP
                       ? launch_bf16_m<ISX_UP>(a.bf16_variant, C, n_in, n_out, s_in, g_in, L.W, L.b, WtPrev, Gp2,
                                               Fbf[cur], Y[h - 1], A[h - 1], B[h - 1], G[h - 1], Fout, Y[h], A[h], B[h],
                                               G[h], (float*)nullptr, m.act, a.stream)
                       : launch_bf16_m<ISX_AA>(a.bf16_variant, C, n_in, n_out, s_in, g_in, L.W, L.b, WtPrev, Gp2,
                                               Fbf[cur], Y[h - 1], A[h - 1], B[h - 1], G[h - 1], Fout, Y[h], A[h], B[h],
                                               G[h], S[h], m.act, a.stream);
    if (e != hipSuccess) return e;
    if (prof) a.prof->end(rec, a.stream);
    D += n_in;
    if (marg) {
      e = launch_aa_margin_hidden<float>(C, n_in, n_out, L.Wt, L.b, Y[h - 1], A[h - 1], B[h - 1], R[h - 1], a.centres,
                                         a.halves, Y[h], S[h], A[h], B[h], G[h], R[h],
                                         aa_margin_consts<float>(0x1p-24, 0x1p-8, n_in, D), a.stream);
      if (e != hipSuccess) return e;
    }
    cur ^= 1;
  }
  Profiler::Rec rec{};
  const bool prof = a.prof && a.prof->begin(rec, ISX_KERNEL_OUTPUT, output_flops_per_cell(m) * (double)C,
                                            4.0 * C * 4.0 * (double)m.pw[1] * Lh, a.stream);
  // (UP: the read-off on BF16 MFMA with hi/lo splits where the widths allow;
  // AA keeps the float32 read-off, which the rounding margin assumes)
  hipError_t e = (a.kernel_choice == 1 || a.method == ISX_RAUA)
                     ? launch_output_f32(m, a.method, C, w.vec, a.halves, a.out32, a.stream)
                 : (a.method == ISX_UP && output_bf16_supported(m) && !a.readoff_f32)
                     ? launch_output_bf16(m, C, Y, A, B, G, a.halves, a.out32, a.stream)
                     : launch_output_mfma(m, a.method, C, Y, A, B, G, a.halves, a.out32, a.stream);
  if (prof) a.prof->end(rec, a.stream);
  if (e == hipSuccess && marg) {
    // the read-off runs on float32 vectors and weights (u_b = 0)
    int kmax = 3;
    for (int h = 1; h <= Lh; ++h) kmax = std::max(kmax, m.pw[h]);
    AaMargin<float> k = aa_margin_consts<float>(0x1p-24, 0.0, m.pw[Lh], D + m.pw[Lh]);
    const double u = 0x1p-24;
    k.c = (float)((m.n_linear + 1) * ((kmax + 1) * u / (1.0 - (kmax + 1) * u)));
    e = launch_aa_margin_output<float>(C, m.pw[Lh], m.L[Lh].Wt, m.L[Lh].b, Y[Lh], A[Lh], B[Lh], R[Lh], a.centres,
                                       a.halves, a.out32, nullptr, k, a.stream);
  }
  return e;
}

}  // namespace isx
