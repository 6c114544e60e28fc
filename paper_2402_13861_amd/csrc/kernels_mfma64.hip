// Hidden-layer coefficient products of the float64 propagation on FP64 MFMA
// (v_mfma_f64_16x16x4f64), with the ReLU rule fused into the epilogue.  This
// is the arithmetic of the float64 re-check band and of ISX_FP64.
//
// Same decomposition as the FP32 MFMA kernel: a workgroup computes, for one
// cell and one block of BM output neurons,
//   P = W[m0:m0+BM, :] * diag(alpha_{h-1}) * F_{h-1}   (all columns)
// tile by tile (BN columns, K streamed through LDS in chunks of KT; alpha is
// applied and beta added to the centre column while the B tile is staged),
// writes P as the next coefficient block (unless this is the last hidden
// layer), accumulates each row's statistic over all columns in a fixed order,
// appends the new symbol block W diag(gamma_{h-1}) with its statistic, and
// applies the ReLU rule to its BM neurons.
//
// MFMA 16x16x4 f64 operand layout (lane l): A element (row l%16, k l/16),
// B element (k l/16, column l%16); accumulator register i holds
// (row l/16 + 4i, column l%16).  Each wave owns 32 rows x 32*NB columns as
// 2 x 2NB tiles of 16 x 16.
#include "isx_internal.h"
#include "rules.h"

#include <algorithm>

namespace isx {

typedef double v4d_t __attribute__((ext_vector_type(4)));

template <int METHOD>
__device__ __forceinline__ double dstat(double v) {
  return METHOD == ISX_UP ? v * v : fabs(v);
}


template <int BM>
struct Cfg64 {
  static constexpr int NWAVES = 8;
  static constexpr int THREADS = 64 * NWAVES;
  static constexpr int WR = BM / 32;            // wave rows (32 neurons each)
  static constexpr int WC = NWAVES / WR;        // wave columns
  static constexpr int NB = BM == 128 ? 2 : 1;  // 32-column blocks per wave
  static constexpr int BN = 32 * NB * WC;       // columns per tile
  static constexpr int KT = 16;                 // K chunk
  static constexpr int ASTR = BM;
  static constexpr int BSTR = BN + 1;
  static constexpr int G = THREADS / BM;        // thread groups in the new-block pass
};

template <int METHOD, int BM>
__global__ __launch_bounds__(512) void hidden_mfma_f64_kernel(
    int64_t C, int n_in, int n_out, int64_t cols_in, int rb_count, const double* __restrict__ Wt,
    const double* __restrict__ bias, const double* __restrict__ Fin, const double* __restrict__ Ain,
    const double* __restrict__ Bin, const double* __restrict__ Gin, double* __restrict__ Fout,
    double* __restrict__ Y, double* __restrict__ A, double* __restrict__ B, double* __restrict__ G,
    double* __restrict__ S, int act) {
  using K = Cfg64<BM>;
  __shared__ double As[K::KT * K::ASTR];
  __shared__ double Bs[K::KT * K::BSTR];
  __shared__ double s_alpha[ISX_MAX_WIDTH];
  __shared__ double s_beta[ISX_MAX_WIDTH];
  __shared__ double s_gamma[ISX_MAX_WIDTH];
  __shared__ double s_y[BM];
  __shared__ double s_stat[K::WC][BM];
  __shared__ double s_gen[K::G][BM];

  // workgroups are dealt to the 8 XCDs round-robin: keep a cell's row
  // blocks on one XCD
  const int64_t blk = blockIdx.x;
  const int xcd = (int)(blk & 7);
  const int64_t qq = blk >> 3;
  const int rb = (int)(qq % rb_count);
  const int64_t cell = (qq / rb_count) * 8 + xcd;
  if (cell >= C) return;  // uniform for the whole workgroup
  const int m0 = rb * BM;
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform
  const int wr = wave % K::WR, wc = wave / K::WR;
  const int l16 = lane & 15, q4 = lane >> 4;
  const int64_t cols_out = cols_in + n_in;
  const double* fin = Fin + cell * cols_in * n_in;
  double* fout = Fout ? Fout + cell * cols_out * n_out : nullptr;
  for (int k = t; k < n_in; k += K::THREADS) {
    s_alpha[k] = Ain[cell * n_in + k];
    s_beta[k] = Bin[cell * n_in + k];
    s_gamma[k] = Gin[cell * n_in + k];
  }
  __syncthreads();

  double stat[2][4];
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int i = 0; i < 4; ++i) stat[rs][i] = 0.0;

  const int64_t ntiles = (cols_in + K::BN - 1) / K::BN;
  for (int64_t nt = 0; nt < ntiles; ++nt) {
    const int64_t c0 = nt * K::BN;
    const bool wave_active = c0 + wc * 32 * K::NB < cols_in;
    v4d_t acc[2][2 * K::NB];
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
      for (int cs = 0; cs < 2 * K::NB; ++cs)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[rs][cs][i] = 0.0;

    // K chunks: the next chunk's operands are loaded into registers while
    // the current one is multiplied, then stored to LDS
    constexpr int TA = K::KT * BM / 2, TB = K::KT * K::BN / 2;  // double2 per chunk
    constexpr int NA = (TA + K::THREADS - 1) / K::THREADS;      // per thread
    constexpr int NBL = (TB + K::THREADS - 1) / K::THREADS;
    static_assert(NA <= 2 && NBL <= 4, "prefetch registers");
    // named registers (not arrays) keep the prefetch out of memory
    double2 ra0 = make_double2(0.0, 0.0), ra1 = ra0, rb0 = ra0, rb1 = ra0, rb2 = ra0, rb3 = ra0;
// loads are unconditional (indices clamped to valid addresses, values
// masked afterwards), so they stay in flight while the products run
#define ISX_F64_LOAD_A(U, DST, K0)                                                                   \
  {                                                                                                  \
    const int idx = min(t + (U) * K::THREADS, TA - 1);                                               \
    const int kk = idx / (BM / 2), mp = idx - kk * (BM / 2);                                         \
    DST = *reinterpret_cast<const double2*>(Wt + (int64_t)((K0) + kk) * n_out + m0 + 2 * mp);        \
  }
#define ISX_F64_LOAD_B(U, DST, K0)                                                                   \
  {                                                                                                  \
    const int idx = min(t + (U) * K::THREADS, TB - 1);                                               \
    const int col = idx / (K::KT / 2), kp = idx - col * (K::KT / 2);                                 \
    const int64_t gc = c0 + col;                                                                     \
    const int64_t gcc = gc < cols_in ? gc : cols_in - 1;                                             \
    const double2 v = *reinterpret_cast<const double2*>(fin + gcc * n_in + (K0) + 2 * kp);           \
    DST = gc < cols_in ? v : make_double2(0.0, 0.0);                                                 \
  }
#define ISX_F64_LOAD_CHUNK(K0)                                  \
  {                                                             \
    ISX_F64_LOAD_A(0, ra0, K0);                                 \
    if constexpr (NA > 1) ISX_F64_LOAD_A(1, ra1, K0);           \
    ISX_F64_LOAD_B(0, rb0, K0);                                 \
    if constexpr (NBL > 1) ISX_F64_LOAD_B(1, rb1, K0);          \
    if constexpr (NBL > 2) ISX_F64_LOAD_B(2, rb2, K0);          \
    if constexpr (NBL > 3) ISX_F64_LOAD_B(3, rb3, K0);          \
  }
#define ISX_F64_STORE_A(U, SRC)                                                     \
  {                                                                                 \
    const int idx = t + (U) * K::THREADS;                                           \
    const int kk = idx / (BM / 2), mp = idx - kk * (BM / 2);                        \
    if (idx < TA) *reinterpret_cast<double2*>(As + kk * K::ASTR + 2 * mp) = SRC;    \
  }
#define ISX_F64_STORE_B(U, SRC)                                                     \
  {                                                                                 \
    const int idx = t + (U) * K::THREADS;                                           \
    const int col = idx / (K::KT / 2), kp = idx - col * (K::KT / 2);                \
    if (idx < TB) {                                                                 \
      const int k = k0 + 2 * kp;                                                    \
      double2 v = SRC;                                                              \
      v.x *= s_alpha[k];                                                            \
      v.y *= s_alpha[k + 1];                                                        \
      if (c0 + col == 0) {                                                          \
        v.x += s_beta[k];                                                           \
        v.y += s_beta[k + 1];                                                       \
      }                                                                             \
      Bs[(2 * kp + 0) * K::BSTR + col] = v.x;                                       \
      Bs[(2 * kp + 1) * K::BSTR + col] = v.y;                                       \
    }                                                                               \
  }
    ISX_F64_LOAD_CHUNK(0);
    for (int k0 = 0; k0 < n_in; k0 += K::KT) {
      __syncthreads();  // the previous chunk's products are done with LDS
      ISX_F64_STORE_A(0, ra0);
      if constexpr (NA > 1) ISX_F64_STORE_A(1, ra1);
      // B = alpha . F (+ beta on the centre column)
      ISX_F64_STORE_B(0, rb0);
      if constexpr (NBL > 1) ISX_F64_STORE_B(1, rb1);
      if constexpr (NBL > 2) ISX_F64_STORE_B(2, rb2);
      if constexpr (NBL > 3) ISX_F64_STORE_B(3, rb3);
      __syncthreads();
      if (k0 + K::KT < n_in) ISX_F64_LOAD_CHUNK(k0 + K::KT);
      if (wave_active) {
#pragma unroll
        for (int ks = 0; ks < K::KT / 4; ++ks) {
          const int kr = 4 * ks + q4;
          double a[2];
#pragma unroll
          for (int rs = 0; rs < 2; ++rs) a[rs] = As[kr * K::ASTR + wr * 32 + rs * 16 + l16];
#pragma unroll
          for (int cs = 0; cs < 2 * K::NB; ++cs) {
            // 16-column sub-tiles past the last real column are skipped
            if (c0 + wc * 32 * K::NB + cs * 16 >= cols_in) continue;
            const double bv = Bs[kr * K::BSTR + wc * 32 * K::NB + cs * 16 + l16];
#pragma unroll
            for (int rs = 0; rs < 2; ++rs)
              acc[rs][cs] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rs], bv, acc[rs][cs], 0, 0, 0);
          }
        }
      }
    }
#undef ISX_F64_LOAD_CHUNK
#undef ISX_F64_LOAD_A
#undef ISX_F64_LOAD_B
#undef ISX_F64_STORE_A
#undef ISX_F64_STORE_B
    __syncthreads();
    if (wave_active) {
#pragma unroll
      for (int cs = 0; cs < 2 * K::NB; ++cs) {
        const int64_t col = c0 + wc * 32 * K::NB + cs * 16 + l16;
        if (col < cols_in) {
#pragma unroll
          for (int rs = 0; rs < 2; ++rs) {
            const int rl = wr * 32 + rs * 16 + q4;  // rows rl + 4i
            double v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = acc[rs][cs][i];
            if (col == 0) {
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                v[i] += bias[m0 + rl + 4 * i];
                s_y[rl + 4 * i] = v[i];
              }
            } else {
#pragma unroll
              for (int i = 0; i < 4; ++i) stat[rs][i] += dstat<METHOD>(v[i]);
            }
            if (fout) {
              double* dst = fout + col * n_out + m0 + rl;
#pragma unroll
              for (int i = 0; i < 4; ++i) dst[4 * i] = v[i];
            }
          }
        }
      }
    }
  }
  // reduce each row's statistic over the 16 lanes holding its columns
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double v = stat[rs][i];
      v += __shfl_xor(v, 8);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 1);
      stat[rs][i] = v;
    }
  if (l16 == 0) {
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
      for (int i = 0; i < 4; ++i) s_stat[wc][wr * 32 + rs * 16 + q4 + 4 * i] = stat[rs][i];
  }
  // new symbol block W diag(gamma_{h-1}) and its statistic
  {
    constexpr int U = 8;
    const int m = t % BM, g = t / BM;
    double gs = 0.0;
    for (int j0 = g; j0 < n_in; j0 += U * K::G) {
      double wv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * K::G;
        wv[u] = j < n_in ? Wt[(int64_t)j * n_out + m0 + m] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * K::G;
        if (j < n_in) {
          const double v = wv[u] * s_gamma[j];
          gs += dstat<METHOD>(v);
          if (fout) fout[(cols_in + j) * n_out + m0 + m] = v;
        }
      }
    }
    s_gen[g][m] = gs;
  }
  __syncthreads();
  if (t < BM) {
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < K::WC; ++w) tot += s_stat[w][t];
#pragma unroll
    for (int g = 0; g < K::G; ++g) tot += s_gen[g][t];
    double a, b, gg;
    apply_rule<double, METHOD>(act, s_y[t], tot, a, b, gg);
    const int64_t o = cell * n_out + m0 + t;
    Y[o] = s_y[t];
    A[o] = a;
    B[o] = b;
    G[o] = gg;
    if (S) S[o] = tot;
  }
}

template <int METHOD, int BM>
static void launch64_bm(int64_t C, int n_in, int n_out, int64_t cols_in, const double* Wt, const double* bias,
                        const double* Fin, const double* Ain, const double* Bin, const double* Gin, double* Fout,
                        double* Y, double* A, double* B, double* G, double* S, int act, hipStream_t s) {
  const int rb_count = n_out / BM;
  const int64_t blocks = ((C + 7) / 8) * 8 * rb_count;
  hipLaunchKernelGGL((hidden_mfma_f64_kernel<METHOD, BM>), dim3((unsigned)blocks), dim3(Cfg64<BM>::THREADS), 0, s,
                     C, n_in, n_out, cols_in, rb_count, Wt, bias, Fin, Ain, Bin, Gin, Fout, Y, A, B, G, S, act);
}

hipError_t launch_hidden_mfma_f64(int method, int64_t C, int n_in, int n_out, int64_t cols_in, const double* Wt,
                                  const double* bias, const double* Fin, const double* Ain, const double* Bin,
                                  const double* Gin, double* Fout, double* Y, double* A, double* B, double* G,
                                  double* S, hipStream_t s) {
  if (C <= 0) return hipSuccess;
  if (n_out % 32 != 0 || n_in % 32 != 0 || n_in > ISX_MAX_WIDTH) return hipErrorInvalidValue;
  // method: the propagation method in the low 4 bits, the activation above
  const int act = method >> 4;
  method &= 15;
  // 64-row blocks run two workgroups per CU (the 128-row tile needs more
  // registers than that allows); wider layers keep 128 so that each cell's
  // coefficient block is streamed fewer times
  const int bm = (n_out % 64 == 0 && n_out <= 256) ? 64 : (n_out % 128 == 0 ? 128 : (n_out % 64 == 0 ? 64 : 32));
#define ISX_F64_ARGS C, n_in, n_out, cols_in, Wt, bias, Fin, Ain, Bin, Gin, Fout, Y, A, B, G, S, act, s
  if (method == ISX_UP) {
    if (bm == 128) launch64_bm<ISX_UP, 128>(ISX_F64_ARGS);
    else if (bm == 64) launch64_bm<ISX_UP, 64>(ISX_F64_ARGS);
    else launch64_bm<ISX_UP, 32>(ISX_F64_ARGS);
  } else {
    if (bm == 128) launch64_bm<ISX_AA, 128>(ISX_F64_ARGS);
    else if (bm == 64) launch64_bm<ISX_AA, 64>(ISX_F64_ARGS);
    else launch64_bm<ISX_AA, 32>(ISX_F64_ARGS);
  }
#undef ISX_F64_ARGS
  return hipGetLastError();
}

}  // namespace isx
