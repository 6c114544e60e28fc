// Hidden-layer coefficient products of the propagation on FP32 MFMA
// (v_mfma_f32_32x32x2f32), with the ReLU rule fused into the epilogue.
//
// For one cell and one block of BM output neurons, the workgroup computes
//   P = W[m0:m0+BM, :] * diag(alpha_{h-1}) * F_{h-1}   (all N = cols_in columns)
// tile by tile (BN columns at a time, K streamed in chunks of KT through LDS;
// alpha is applied, and beta added to the centre column, while the B tile is
// staged), writes P as the next coefficient block (unless this is the last
// hidden layer), accumulates each row's statistic (sum of squares for UP,
// of absolute values for AA) over all columns, appends the new symbol block
// W diag(gamma_{h-1}) with its statistic, and finally applies the ReLU rule
// to each of its BM neurons.  The statistic is reduced in a fixed order
// (lane butterflies, then waves in order), so results are deterministic.
//
// MFMA 32x32x2 f32 operand layout (lane l of a 64-wide wave): A element
// (row l%32, k l/32), B element (k l/32, col l%32); accumulator register r
// holds (row 8*(r/4) + 4*(l/32) + r%4, col l%32).
//
// Workgroups map to (cell, row block) so that the row blocks of one cell are
// consecutive on the same XCD (blocks are dealt to the 8 XCDs round-robin),
// letting the second row block find the cell's coefficients in that XCD's L2.
#include "isx_internal.h"
#include "rules.h"

namespace isx {

typedef float v16f __attribute__((ext_vector_type(16)));

template <int METHOD>
__device__ __forceinline__ float mstat(float v) {
  return METHOD == ISX_UP ? v * v : fabsf(v);
}


// SPLIT: the products as three BF16 MFMAs of float32 operands split into
// bfloat16 parts, x = hi + lo (hi = bf16(x), lo = bf16(x - hi)):
//   a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi,
// each of v_mfma_f32_32x32x16_bf16, accumulated in float32.  The dropped
// a_lo b_lo and the rounding of the lo parts leave about 3 2^-18 of |a b| per
// term, against 2^-24 for float32 products; one k-step of 16 costs three
// 32-cycle products instead of eight 64-cycle float32 ones.  Operands are
// staged in LDS as [row][k] bfloat16 (hi block, then lo block), 8 + 32
// elements per row.  The accumulator layout is the float32 product's.
typedef __bf16 sbf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split_bf16x4(float4 v, uint2& hi, uint2& lo) {
  union {
    __bf16 h[4];
    uint2 u;
  } ph, pl;
  ph.h[0] = (__bf16)v.x;
  ph.h[1] = (__bf16)v.y;
  ph.h[2] = (__bf16)v.z;
  ph.h[3] = (__bf16)v.w;
  pl.h[0] = (__bf16)(v.x - (float)ph.h[0]);
  pl.h[1] = (__bf16)(v.y - (float)ph.h[1]);
  pl.h[2] = (__bf16)(v.z - (float)ph.h[2]);
  pl.h[3] = (__bf16)(v.w - (float)ph.h[3]);
  hi = ph.u;
  lo = pl.u;
}

template <int BM>
struct Cfg {
  static constexpr int NWAVES = 8;
  static constexpr int THREADS = 64 * NWAVES;
  static constexpr int WR = BM / 32;           // wave rows (32 neurons each)
  static constexpr int WC = NWAVES / WR;       // wave columns
  static constexpr int NB = BM == 128 ? 2 : 1; // 32-column MFMA blocks per wave
  static constexpr int BN = 32 * NB * WC;      // columns per tile
  static constexpr int KT = 32;                // K chunk
  static constexpr int ASTR = BM;
  static constexpr int BSTR = BN + 1;
  static constexpr int G = THREADS / BM;       // thread groups in the generated-block pass
  static constexpr int SSTR = KT + 8;          // SPLIT: bfloat16 row stride of the staged operands
};

// At most 128 VGPRs (four waves per SIMD): two workgroups share a CU, so one
// workgroup's barriers and chunk stores overlap the other's products.
template <int METHOD, int BM, bool SPLIT>
__global__ __launch_bounds__(512, 4) void hidden_mfma_f32_kernel(
    int64_t C, int n_in, int n_out, int64_t cols_in, int rb_count, const float* __restrict__ Wt,
    const float* __restrict__ Wrow, const float* __restrict__ bias, const float* __restrict__ Fin,
    const float* __restrict__ Ain, const float* __restrict__ Bin, const float* __restrict__ Gin,
    float* __restrict__ Fout, float* __restrict__ Y, float* __restrict__ A, float* __restrict__ B,
    float* __restrict__ G, float* __restrict__ S, int act) {
  using K = Cfg<BM>;
  // float32 tiles [k][row] / [k][column], or (SPLIT) bfloat16 hi | lo blocks
  // of [row][k] / [column][k]
  __shared__ float As[SPLIT ? BM * K::SSTR : K::KT * K::ASTR];
  __shared__ float Bs[SPLIT ? K::BN * K::SSTR : K::KT * K::BSTR];
  __shared__ float s_alpha[ISX_MAX_WIDTH];
  __shared__ float s_beta[ISX_MAX_WIDTH];
  __shared__ float s_gamma[ISX_MAX_WIDTH];
  __shared__ float s_y[BM];
  __shared__ float s_stat[K::WC][BM];
  __shared__ float s_gen[K::G][BM];

  const int64_t blk = blockIdx.x;
  const int xcd = (int)(blk & 7);
  const int64_t q = blk >> 3;
  const int rb = (int)(q % rb_count);
  const int64_t cell = (q / rb_count) * 8 + xcd;
  if (cell >= C) return;  // uniform for the whole workgroup
  const int m0 = rb * BM;
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform
  const int wr = wave % K::WR, wc = wave / K::WR;
  const int64_t cols_out = cols_in + n_in;
  const float* fin = Fin + cell * cols_in * n_in;
  float* fout = Fout ? Fout + cell * cols_out * n_out : nullptr;
  for (int k = t; k < n_in; k += K::THREADS) {
    s_alpha[k] = Ain[cell * n_in + k];
    s_beta[k] = Bin[cell * n_in + k];
    s_gamma[k] = Gin[cell * n_in + k];
  }
  __syncthreads();

  // each row's statistic, summed over the tiles in order by the wave that
  // owns the row block (s_stat[wc] is written by wave (wr, wc) only)
  for (int i = t; i < K::WC * BM; i += K::THREADS) (&s_stat[0][0])[i] = 0.f;

  // SPLIT: the centre column (a point evaluation of the linearised net,
  // y_j = sum_k W[j][k] (alpha_k y_k + beta_k) + b_j) in float32 on the vector
  // ALUs: its dot products cancel, and the split products' error relative to
  // the summed magnitudes would show in the classification margin
  __shared__ float s_yx[SPLIT ? BM : 1];
  if constexpr (SPLIT) {
    constexpr int TPR = K::THREADS / BM;  // threads per row (consecutive lanes)
    const int row = t / TPR, part = t % TPR;
    const float* wrow = Wrow + (int64_t)(m0 + row) * n_in;
    float yv = 0.f;
    for (int k = part; k < n_in; k += TPR) yv = fmaf(wrow[k], fmaf(s_alpha[k], fin[k], s_beta[k]), yv);
#pragma unroll
    for (int off = TPR / 2; off > 0; off >>= 1) yv += __shfl_xor(yv, off);
    if (part == 0) s_yx[row] = yv + bias[m0 + row];
  }

  const int64_t ntiles = (cols_in + K::BN - 1) / K::BN;
  for (int64_t nt = 0; nt < ntiles; ++nt) {
    const int64_t c0 = nt * K::BN;
    const bool wave_active = c0 + wc * 32 * K::NB < cols_in;
    // 32-column blocks of this wave that hold real columns (wave-uniform):
    // the last tile of a layer is mostly padding (the centre and the three
    // input symbols make every layer's column count 4 above a multiple of 32)
    const int nb_real = (int)min((int64_t)K::NB, (cols_in - c0 - wc * 32 * K::NB + 31) / 32);
    v16f acc[K::NB];
#pragma unroll
    for (int nb = 0; nb < K::NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;

    // K chunks: the next chunk's operands are loaded into registers while
    // the current one is multiplied, then stored to LDS
    constexpr int TA = K::KT * BM / 4, TB = K::KT * K::BN / 4;  // float4 per chunk
    constexpr int NA = (TA + K::THREADS - 1) / K::THREADS;      // per thread
    constexpr int NBL = (TB + K::THREADS - 1) / K::THREADS;
    static_assert(NA <= 2 && NBL <= 4, "prefetch registers");
    // named registers (not arrays) keep the prefetch out of memory
    float4 ra0 = make_float4(0.f, 0.f, 0.f, 0.f), ra1 = ra0, rb0 = ra0, rb1 = ra0, rb2 = ra0, rb3 = ra0;
// loads are unconditional (indices clamped to valid addresses, values
// masked afterwards), so they stay in flight while the products run
#define ISX_F32_LOAD_A(U, DST, K0)                                                                 \
  {                                                                                                \
    const int idx = min(t + (U) * K::THREADS, TA - 1);                                             \
    if constexpr (SPLIT) {                                                                         \
      const int mm = idx / (K::KT / 4), kq = idx - mm * (K::KT / 4);                               \
      DST = *reinterpret_cast<const float4*>(Wrow + (int64_t)(m0 + mm) * n_in + (K0) + 4 * kq);    \
    } else {                                                                                       \
      const int kk = idx / (BM / 4), mq = idx - kk * (BM / 4);                                     \
      DST = *reinterpret_cast<const float4*>(Wt + (int64_t)((K0) + kk) * n_out + m0 + 4 * mq);     \
    }                                                                                              \
  }
#define ISX_F32_LOAD_B(U, DST, K0)                                                                 \
  {                                                                                                \
    const int idx = min(t + (U) * K::THREADS, TB - 1);                                             \
    const int col = idx / (K::KT / 4), kq = idx - col * (K::KT / 4);                               \
    const int64_t gc = c0 + col;                                                                   \
    const int64_t gcc = gc < cols_in ? gc : cols_in - 1;                                           \
    const float4 v = *reinterpret_cast<const float4*>(fin + gcc * n_in + (K0) + 4 * kq);           \
    DST = gc < cols_in ? v : make_float4(0.f, 0.f, 0.f, 0.f);                                      \
  }
#define ISX_F32_LOAD_CHUNK(K0)                         \
  {                                                    \
    ISX_F32_LOAD_A(0, ra0, K0);                        \
    if constexpr (NA > 1) ISX_F32_LOAD_A(1, ra1, K0);  \
    ISX_F32_LOAD_B(0, rb0, K0);                        \
    if constexpr (NBL > 1) ISX_F32_LOAD_B(1, rb1, K0); \
    if constexpr (NBL > 2) ISX_F32_LOAD_B(2, rb2, K0); \
    if constexpr (NBL > 3) ISX_F32_LOAD_B(3, rb3, K0); \
  }
#define ISX_F32_STORE_A(U, SRC)                                                              \
  {                                                                                          \
    const int idx = t + (U) * K::THREADS;                                                    \
    if constexpr (SPLIT) {                                                                   \
      const int mm = idx / (K::KT / 4), kq = idx - mm * (K::KT / 4);                         \
      if (idx < TA) {                                                                        \
        __bf16* ah = reinterpret_cast<__bf16*>(As) + mm * K::SSTR + 4 * kq;                  \
        uint2 h_, l_;                                                                        \
        split_bf16x4(SRC, h_, l_);                                                           \
        *reinterpret_cast<uint2*>(ah) = h_;                                                  \
        *reinterpret_cast<uint2*>(ah + BM * K::SSTR) = l_;                                   \
      }                                                                                      \
    } else {                                                                                 \
      const int kk = idx / (BM / 4), mq = idx - kk * (BM / 4);                               \
      if (idx < TA) *reinterpret_cast<float4*>(As + kk * K::ASTR + 4 * mq) = SRC;            \
    }                                                                                        \
  }
#define ISX_F32_STORE_B(U, SRC)                                    \
  {                                                                \
    const int idx = t + (U) * K::THREADS;                          \
    const int col = idx / (K::KT / 4), kq = idx - col * (K::KT / 4); \
    if (idx < TB) {                                                \
      const int k = k0 + 4 * kq;                                   \
      float4 v = SRC;                                              \
      v.x *= s_alpha[k];                                           \
      v.y *= s_alpha[k + 1];                                       \
      v.z *= s_alpha[k + 2];                                       \
      v.w *= s_alpha[k + 3];                                       \
      if (c0 + col == 0) {                                         \
        v.x += s_beta[k];                                          \
        v.y += s_beta[k + 1];                                      \
        v.z += s_beta[k + 2];                                      \
        v.w += s_beta[k + 3];                                      \
      }                                                            \
      if constexpr (SPLIT) {                                       \
        __bf16* bh = reinterpret_cast<__bf16*>(Bs) + col * K::SSTR + 4 * kq; \
        uint2 h_, l_;                                              \
        split_bf16x4(v, h_, l_);                                   \
        *reinterpret_cast<uint2*>(bh) = h_;                        \
        *reinterpret_cast<uint2*>(bh + K::BN * K::SSTR) = l_;      \
      } else {                                                     \
        Bs[(4 * kq + 0) * K::BSTR + col] = v.x;                    \
        Bs[(4 * kq + 1) * K::BSTR + col] = v.y;                    \
        Bs[(4 * kq + 2) * K::BSTR + col] = v.z;                    \
        Bs[(4 * kq + 3) * K::BSTR + col] = v.w;                    \
      }                                                            \
    }                                                              \
  }
    ISX_F32_LOAD_CHUNK(0);
    for (int k0 = 0; k0 < n_in; k0 += K::KT) {
      __syncthreads();  // the previous chunk's products are done with LDS
      ISX_F32_STORE_A(0, ra0);
      if constexpr (NA > 1) ISX_F32_STORE_A(1, ra1);
      // B = alpha . F (+ beta on the centre column)
      ISX_F32_STORE_B(0, rb0);
      if constexpr (NBL > 1) ISX_F32_STORE_B(1, rb1);
      if constexpr (NBL > 2) ISX_F32_STORE_B(2, rb2);
      if constexpr (NBL > 3) ISX_F32_STORE_B(3, rb3);
      __syncthreads();
      if (k0 + K::KT < n_in) ISX_F32_LOAD_CHUNK(k0 + K::KT);
      if (wave_active) {
        if constexpr (SPLIT) {
          const __bf16* a0 = reinterpret_cast<const __bf16*>(As) + (wr * 32 + (lane & 31)) * K::SSTR + 8 * (lane >> 5);
          const __bf16* b0 = reinterpret_cast<const __bf16*>(Bs) + (wc * 32 * K::NB + (lane & 31)) * K::SSTR +
                             8 * (lane >> 5);
#pragma unroll
          for (int kk = 0; kk < K::KT / 16; ++kk) {
            const sbf16x8 ah = *reinterpret_cast<const sbf16x8*>(a0 + 16 * kk);
            const sbf16x8 al = *reinterpret_cast<const sbf16x8*>(a0 + BM * K::SSTR + 16 * kk);
#pragma unroll
            for (int nb = 0; nb < K::NB; ++nb) {
              if (nb > 0 && nb >= nb_real) break;
              const __bf16* bp = b0 + nb * 32 * K::SSTR + 16 * kk;
              const sbf16x8 bh = *reinterpret_cast<const sbf16x8*>(bp);
              const sbf16x8 bl = *reinterpret_cast<const sbf16x8*>(bp + K::BN * K::SSTR);
              acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[nb], 0, 0, 0);
              acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[nb], 0, 0, 0);
              acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[nb], 0, 0, 0);
            }
          }
        } else {
#pragma unroll
          for (int ks = 0; ks < K::KT / 2; ++ks) {
            const int kr = 2 * ks + (lane >> 5);
            const float a = As[kr * K::ASTR + wr * 32 + (lane & 31)];
#pragma unroll
            for (int nb = 0; nb < K::NB; ++nb) {
              if (nb > 0 && nb >= nb_real) break;
              const float bv = Bs[kr * K::BSTR + wc * 32 * K::NB + nb * 32 + (lane & 31)];
              acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv, acc[nb], 0, 0, 0);
            }
          }
        }
      }
    }
#undef ISX_F32_LOAD_CHUNK
#undef ISX_F32_LOAD_A
#undef ISX_F32_LOAD_B
#undef ISX_F32_STORE_A
#undef ISX_F32_STORE_B
    __syncthreads();
    if (wave_active) {
      float stat[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) stat[r] = 0.f;
#pragma unroll
      for (int nb = 0; nb < K::NB; ++nb) {
        const int64_t col = c0 + wc * 32 * K::NB + nb * 32 + (lane & 31);
        if (col < cols_in) {
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4) {
            const int rl = wr * 32 + 8 * q4 + 4 * (lane >> 5);
            float v0 = acc[nb][4 * q4 + 0], v1 = acc[nb][4 * q4 + 1];
            float v2 = acc[nb][4 * q4 + 2], v3 = acc[nb][4 * q4 + 3];
            if (col == 0) {
              if constexpr (SPLIT) {
                v0 = s_yx[rl + 0];
                v1 = s_yx[rl + 1];
                v2 = s_yx[rl + 2];
                v3 = s_yx[rl + 3];
              } else {
                v0 += bias[m0 + rl + 0];
                v1 += bias[m0 + rl + 1];
                v2 += bias[m0 + rl + 2];
                v3 += bias[m0 + rl + 3];
              }
              s_y[rl + 0] = v0;
              s_y[rl + 1] = v1;
              s_y[rl + 2] = v2;
              s_y[rl + 3] = v3;
            } else {
              stat[4 * q4 + 0] += mstat<METHOD>(v0);
              stat[4 * q4 + 1] += mstat<METHOD>(v1);
              stat[4 * q4 + 2] += mstat<METHOD>(v2);
              stat[4 * q4 + 3] += mstat<METHOD>(v3);
            }
            if (fout) *reinterpret_cast<float4*>(fout + col * n_out + m0 + rl) = make_float4(v0, v1, v2, v3);
          }
        }
      }
      // reduce each row's statistic over the 32 lanes holding the tile's
      // columns and add it to the row's running sum
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        float v = stat[r];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 8);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 1);
        stat[r] = v;
      }
      if ((lane & 31) == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) s_stat[wc][wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)] += stat[r];
      }
    }
  }
  // new symbol block W diag(gamma_{h-1}) and its statistic
  {
    // eight independent weight loads in flight per thread
    constexpr int U = 8;
    const int m = t % BM, g = t / BM;
    float gs = 0.f;
    for (int j0 = g; j0 < n_in; j0 += U * K::G) {
      float wv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * K::G;
        wv[u] = j < n_in ? Wt[(int64_t)j * n_out + m0 + m] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * K::G;
        if (j < n_in) {
          const float v = wv[u] * s_gamma[j];
          gs += mstat<METHOD>(v);
          if (fout) fout[(cols_in + j) * n_out + m0 + m] = v;
        }
      }
    }
    s_gen[g][m] = gs;
  }
  __syncthreads();
  if (t < BM) {
    float tot = 0.f;
#pragma unroll
    for (int w = 0; w < K::WC; ++w) tot += s_stat[w][t];
#pragma unroll
    for (int g = 0; g < K::G; ++g) tot += s_gen[g][t];
    float a, b, gg;
    apply_rule<float, METHOD>(act, s_y[t], tot, a, b, gg);
    const int64_t o = cell * n_out + m0 + t;
    Y[o] = s_y[t];
    A[o] = a;
    B[o] = b;
    G[o] = gg;
    if (S) S[o] = tot;
  }
}

bool mfma_supported(const Model& m) {
  for (int h = 1; h < m.hidden(); ++h)
    if (m.pw[h] % 32 != 0 || m.pw[h + 1] % 32 != 0 || m.pw[h] > ISX_MAX_WIDTH) return false;
  return true;
}

template <int METHOD, int BM, bool SPLIT>
static void launch_bm(int64_t C, int n_in, int n_out, int64_t cols_in, const float* Wt, const float* Wrow,
                      const float* bias, const float* Fin, const float* Ain, const float* Bin, const float* Gin,
                      float* Fout, float* Y, float* A, float* B, float* G, float* S, int act, hipStream_t s) {
  const int rb_count = n_out / BM;
  const int64_t blocks = ((C + 7) / 8) * 8 * rb_count;
  hipLaunchKernelGGL((hidden_mfma_f32_kernel<METHOD, BM, SPLIT>), dim3((unsigned)blocks), dim3(Cfg<BM>::THREADS), 0,
                     s, C, n_in, n_out, cols_in, rb_count, Wt, Wrow, bias, Fin, Ain, Bin, Gin, Fout, Y, A, B, G, S,
                     act);
}

template <int METHOD, bool SPLIT>
static void launch_m(int bm, int64_t C, int n_in, int n_out, int64_t cols_in, const float* Wt, const float* Wrow,
                     const float* bias, const float* Fin, const float* Ain, const float* Bin, const float* Gin,
                     float* Fout, float* Y, float* A, float* B, float* G, float* S, int act, hipStream_t s) {
  if (bm == 128)
    launch_bm<METHOD, 128, SPLIT>(C, n_in, n_out, cols_in, Wt, Wrow, bias, Fin, Ain, Bin, Gin, Fout, Y, A, B, G, S,
                                  act, s);
  else if (bm == 64)
    launch_bm<METHOD, 64, SPLIT>(C, n_in, n_out, cols_in, Wt, Wrow, bias, Fin, Ain, Bin, Gin, Fout, Y, A, B, G, S,
                                 act, s);
  else
    launch_bm<METHOD, 32, SPLIT>(C, n_in, n_out, cols_in, Wt, Wrow, bias, Fin, Ain, Bin, Gin, Fout, Y, A, B, G, S,
                                 act, s);
}

hipError_t launch_hidden_mfma_f32(int method, int64_t C, int n_in, int n_out, int64_t cols_in, const float* Wt,
                                  const float* Wrow, const float* bias, const float* Fin, const float* Ain,
                                  const float* Bin, const float* Gin, float* Fout, float* Y, float* A, float* B,
                                  float* G, float* S, hipStream_t s) {
  if (C <= 0) return hipSuccess;
  if (n_out % 32 != 0 || n_in % 32 != 0 || n_in > ISX_MAX_WIDTH) return hipErrorInvalidValue;
  // method: the propagation method in bits 0-3, the activation in bits 4-7,
  // bit 8 the split bf16 products (SPLIT)
  const int act = (method >> 4) & 15;
  const bool split = (method >> 8) & 1;
  method &= 15;
  if (split && !Wrow) return hipErrorInvalidValue;
  const int bm = n_out % 128 == 0 ? 128 : (n_out % 64 == 0 ? 64 : 32);
  if (method == ISX_UP) {
    if (split)
      launch_m<ISX_UP, true>(bm, C, n_in, n_out, cols_in, Wt, Wrow, bias, Fin, Ain, Bin, Gin, Fout, Y, A, B, G, S, act, s);
    else
      launch_m<ISX_UP, false>(bm, C, n_in, n_out, cols_in, Wt, Wrow, bias, Fin, Ain, Bin, Gin, Fout, Y, A, B, G, S, act, s);
  } else {
    if (split)
      launch_m<ISX_AA, true>(bm, C, n_in, n_out, cols_in, Wt, Wrow, bias, Fin, Ain, Bin, Gin, Fout, Y, A, B, G, S, act, s);
    else
      launch_m<ISX_AA, false>(bm, C, n_in, n_out, cols_in, Wt, Wrow, bias, Fin, Ain, Bin, Gin, Fout, Y, A, B, G, S, act, s);
  }
  return hipGetLastError();
}

}  // namespace isx
