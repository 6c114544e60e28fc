// Dense forward passes of the MLP on FP32 MFMA (v_mfma_f32_32x32x2f32):
//
//   * point evaluation f(x) (Sec. III-B), used for the corners of the active
//     leaves before marching cubes;
//   * the centre linearisation of a cell: f(c) together with the directional
//     derivatives of f at c along the three input symbols of the uncertainty
//     propagation's input form (columns h_a e_a / sqrt(3), Sec. IV-C), i.e.
//     what the propagation reduces to when no neuron's sign changes inside
//     the cell.  It returns (f(c), s) with s = |J(c) diag(h)| / sqrt(3).  A
//     ReLU's derivative at exactly 0 is taken as 0.
//
// A workgroup owns BN columns (points, or 4 columns per cell: the centre and
// three tangents).  Their activations stay in LDS for the whole network as
// X[col][k] (a column's neurons contiguous, row stride KMAX + 4 floats), so
// the only global traffic is the inputs, the weights (shared by every
// workgroup, L2 resident) and one value per column.
//
// Hidden layer n_in -> n_out as MFMA tiles of 32 output neurons x 32
// columns; K runs in groups of 8, and inside a group lane half q = l / 32
// takes k = 8g + 4q + s in step s = 0..3.  That permutation of K lets every
// lane fetch its 4 weights and its 4 activations of a group as one 16-byte
// load each (A from global memory, B from LDS).  Accumulator register r of
// lane l holds (neuron 8(r/4) + 4q + r%4, column l%32); four consecutive
// registers are four consecutive neurons of one column, written back to LDS
// as one 16-byte store after every wave has finished reading the layer input.
#include "isx_internal.h"
#include "rules.h"

#include <algorithm>

namespace isx {

typedef float v16f_d __attribute__((ext_vector_type(16)));

constexpr int kDenseThreads = 512;  // 8 waves
constexpr int kDenseBlocksPerWave = 4;

enum { DENSE_EVAL = 0, DENSE_LIN = 1 };

struct DenseNet {
  int n_linear;
  int n[ISX_MAX_LINEAR + 1];
  const float* W[ISX_MAX_LINEAR];
  const float* b[ISX_MAX_LINEAR];
};

// BN columns per workgroup for a maximum padded hidden width KMAX: the LDS
// tile BN x (KMAX + 4) floats stays near 130 KB.
template <int KMAX>
struct DenseShape {
  static constexpr int BN = KMAX <= 256 ? 128 : (KMAX <= 512 ? 64 : 32);
  static constexpr int STRIDE = KMAX + 4;
  static constexpr size_t LDS = (size_t)BN * STRIDE * sizeof(float);
};

// acc[j] += A[rows of tile t0+j, :] * X[:, columns of tile t0+j] for the
// wave's tiles t0 .. t0+bpw-1 (< nblk) of 32 rows x 32 columns; A row-major
// [M][K] in global memory, X in LDS as [column][k] with row stride STRIDE; K a
// multiple of 8 (groups of 8 with the permuted K order described above).
template <int CB, int STRIDE>
__device__ __forceinline__ void dense_tile_gemm(const float* __restrict__ A, int K, const float* X, int t0, int bpw,
                                                int nblk, int l32, int q, v16f_d (&acc)[kDenseBlocksPerWave]) {
  const int groups = K / 8;
  if (CB == kDenseBlocksPerWave && bpw == kDenseBlocksPerWave && t0 + kDenseBlocksPerWave <= nblk) {
    // the wave's four tiles are the four column tiles of one row block: one
    // A fragment serves all of them
    const int rb = t0 / CB;
    const float* arow = A + (int64_t)(rb * 32 + l32) * K + 4 * q;
    const float* xcol = X + l32 * STRIDE + 4 * q;
    float4 a_next = *reinterpret_cast<const float4*>(arow);
    for (int g = 0; g < groups; ++g) {
      const float4 a = a_next;
      if (g + 1 < groups) a_next = *reinterpret_cast<const float4*>(arow + 8 * (g + 1));
#pragma unroll
      for (int j = 0; j < kDenseBlocksPerWave; ++j) {
        const float4 bv = *reinterpret_cast<const float4*>(xcol + j * 32 * STRIDE + 8 * g);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, bv.x, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, bv.y, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, bv.z, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, bv.w, acc[j], 0, 0, 0);
      }
    }
  } else {
    for (int g = 0; g < groups; ++g) {
#pragma unroll
      for (int j = 0; j < kDenseBlocksPerWave; ++j) {
        const int t = t0 + j;
        if (j < bpw && t < nblk) {
          const int rb = t / CB, cb = t - rb * CB;
          const float4 a = *reinterpret_cast<const float4*>(A + (int64_t)(rb * 32 + l32) * K + 4 * q + 8 * g);
          const float4 bv = *reinterpret_cast<const float4*>(X + (cb * 32 + l32) * STRIDE + 4 * q + 8 * g);
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, bv.x, acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, bv.y, acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, bv.z, acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, bv.w, acc[j], 0, 0, 0);
        }
      }
    }
  }
}

// The activation (evaluation mode) is a compile-time constant, so ReLU keeps
// the register budget of a kernel without the sine and ELU branches.
template <int MODE, int KMAX, int ACT>
__global__ __launch_bounds__(kDenseThreads) void dense_mfma_kernel(int64_t n_items, DenseNet net,
                                                                   const float* __restrict__ in0,
                                                                   const float* __restrict__ in1,
                                                                   float* __restrict__ out) {
  constexpr int BN = DenseShape<KMAX>::BN;
  constexpr int STRIDE = DenseShape<KMAX>::STRIDE;
  constexpr int CB = BN / 32;
  constexpr int PER = MODE == DENSE_LIN ? 4 : 1;  // columns per item
  extern __shared__ float4 dense_smem4[];
  float* X = reinterpret_cast<float*>(dense_smem4);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int q = lane >> 5;
  const int l32 = lane & 31;
  const int64_t item0 = (int64_t)blockIdx.x * (BN / PER);

  // ---- layer 1 (3 -> n1) on the vector ALUs
  {
    const int n1 = net.n[1];
    const float* W1 = net.W[0];
    const float* b1 = net.b[0];
    for (int e = tid; e < BN * n1; e += kDenseThreads) {
      const int col = e / n1, j = e - col * n1;
      const int64_t item = item0 + col / PER;
      float v = 0.f;
      if (item < n_items) {
        const float w0 = W1[j * 3 + 0], w1 = W1[j * 3 + 1], w2 = W1[j * 3 + 2];
        const float* x = in0 + item * 3;
        const float pre = b1[j] + w0 * x[0] + w1 * x[1] + w2 * x[2];
        if (MODE == DENSE_EVAL) {
          v = activate<float>(ACT, pre);
        } else {
          const int a = col % 4;  // 0: centre, 1..3: tangent along axis a-1
          if (a == 0) {
            v = pre > 0.f ? pre : 0.f;
          } else if (pre > 0.f) {
            const float wa = a == 1 ? w0 : (a == 2 ? w1 : w2);
            v = wa * in1[item * 3 + (a - 1)] * 0.57735026918962576451f;
          }
        }
      }
      X[col * STRIDE + j] = v;
    }
  }
  __syncthreads();

  // ---- hidden layers 2 .. n_linear-1 on MFMA
  const int L = net.n_linear;
  for (int l = 1; l + 1 < L; ++l) {
    const int n_in = net.n[l], n_out = net.n[l + 1];
    const float* __restrict__ W = net.W[l];
    const float* __restrict__ bias = net.b[l];
    const int RB = n_out / 32;
    const int nblk = RB * CB;
    const int bpw = (nblk + 7) / 8;  // <= kDenseBlocksPerWave
    const int t0 = wave * bpw;
    v16f_d acc[kDenseBlocksPerWave];
#pragma unroll
    for (int j = 0; j < kDenseBlocksPerWave; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;
    dense_tile_gemm<CB, STRIDE>(W, n_in, X, t0, bpw, nblk, l32, q, acc);
    __syncthreads();  // every wave has read the layer input
#pragma unroll
    for (int j = 0; j < kDenseBlocksPerWave; ++j) {
      const int t = t0 + j;
      if (j < bpw && t < nblk) {
        const int rb = t / CB, cb = t - rb * CB;
        const int col = cb * 32 + l32;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int row = rb * 32 + 8 * qq + 4 * q;
          float v[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float y = acc[j][4 * qq + i];
            if (MODE == DENSE_EVAL) {
              v[i] = activate<float>(ACT, y + bias[row + i]);
            } else {
              // the centre column of this lane's cell is lane (l & ~3): its
              // pre-activation decides the sign for the whole quad
              const bool centre = (l32 & 3) == 0;
              const float pre = y + (centre ? bias[row + i] : 0.f);
              const float pc =
                  __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(pre), 0x00, 0xf, 0xf, false));
              v[i] = pc > 0.f ? pre : 0.f;
            }
          }
          *reinterpret_cast<float4*>(X + col * STRIDE + row) = make_float4(v[0], v[1], v[2], v[3]);
        }
      }
    }
    __syncthreads();
  }

  // ---- output layer (n_last -> 1): 4 threads per column, fixed order
  {
    const int nl = net.n[L - 1];
    const float* w = net.W[L - 1];
    const float bo = net.b[L - 1][0];
    for (int c0 = 0; c0 < BN; c0 += kDenseThreads / 4) {
      const int col = c0 + tid / 4, part = tid & 3;
      float s = 0.f;
      if (col < BN) {
        const float* x = X + col * STRIDE;
        for (int k = part; k < nl; k += 4) s += w[k] * x[k];
      }
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      if (MODE == DENSE_EVAL) {
        const int64_t item = item0 + col;
        if (col < BN && part == 0 && item < n_items) out[item] = s + bo;
      } else {
        // gather the quad's four column sums (columns 4i..4i+3 of one cell)
        // (4 consecutive columns = 16 consecutive lanes)
        const int base = lane & ~15;
        const float f = __shfl(s, base);
        const float d1 = __shfl(s, base + 4), d2 = __shfl(s, base + 8), d3 = __shfl(s, base + 12);
        const int64_t item = item0 + col / 4;
        if (col < BN && (tid & 15) == 0 && item < n_items) {
          out[item * 2 + 0] = f + bo;
          out[item * 2 + 1] = sqrtf(d1 * d1 + d2 * d2 + d3 * d3);
        }
      }
    }
  }
}

static DenseNet dense_net(const Model& m) {
  DenseNet d{};
  d.n_linear = m.n_linear;
  for (int i = 0; i <= m.n_linear; ++i) d.n[i] = m.pw[i];
  for (int l = 0; l < m.n_linear; ++l) {
    d.W[l] = m.L[l].W;
    d.b[l] = m.L[l].b;
  }
  return d;
}

static int dense_kmax(const Model& m) {
  int w = 0;
  for (int h = 1; h < m.n_linear; ++h) w = std::max(w, m.pw[h]);
  return w;
}

template <int MODE, int KMAX, int ACT>
static hipError_t launch_dense_k(const Model& m, int64_t n, const float* in0, const float* in1, float* out,
                                 hipStream_t s) {
  using Sh = DenseShape<KMAX>;
  constexpr int per = MODE == DENSE_LIN ? 4 : 1;
  constexpr int items = Sh::BN / per;
  {
    hipError_t e = ensure_lds_limit(reinterpret_cast<const void*>(&dense_mfma_kernel<MODE, KMAX, ACT>), (int)Sh::LDS);
    if (e != hipSuccess) return e;
  }
  // a launch's work-items must stay below 2^32: at most 2^31 / kDenseThreads
  // blocks per launch (in0 holds 3 floats per item, in1 3 or none, out 1 or 2)
  const int64_t per_launch = ((int64_t(1) << 31) / kDenseThreads) * items;
  constexpr int outw = MODE == DENSE_LIN ? 2 : 1;
  for (int64_t o = 0; o < n; o += per_launch) {
    const int64_t c = std::min(per_launch, n - o);
    hipLaunchKernelGGL((dense_mfma_kernel<MODE, KMAX, ACT>), dim3((unsigned)((c + items - 1) / items)), dim3(kDenseThreads),
                       Sh::LDS, s, c, dense_net(m), in0 + 3 * o, in1 ? in1 + 3 * o : nullptr, out + outw * o);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int MODE, int ACT>
static hipError_t launch_dense(const Model& m, int64_t n, const float* in0, const float* in1, float* out,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int kmax = dense_kmax(m);
  if (m.n_linear < 2 || kmax < 32) return hipErrorNotSupported;
  if (kmax <= 256) return launch_dense_k<MODE, 256, ACT>(m, n, in0, in1, out, s);
  if (kmax <= 512) return launch_dense_k<MODE, 512, ACT>(m, n, in0, in1, out, s);
  return launch_dense_k<MODE, 1024, ACT>(m, n, in0, in1, out, s);
}

hipError_t eval_points_mfma(const Model& m, int64_t n, const float* pts, float* vals, hipStream_t s) {
  switch (m.act) {
    case ISX_SINE: return launch_dense<DENSE_EVAL, ISX_SINE>(m, n, pts, nullptr, vals, s);
    case ISX_ELU: return launch_dense<DENSE_EVAL, ISX_ELU>(m, n, pts, nullptr, vals, s);
    default: return launch_dense<DENSE_EVAL, ISX_RELU>(m, n, pts, nullptr, vals, s);
  }
}

// (ReLU only: the tangent columns take the centre's ReLU mask)
hipError_t linearize_mfma(const Model& m, int64_t n, const float* centres, const float* halves, float* out,
                          hipStream_t s) {
  if (m.act != ISX_RELU) return hipErrorNotSupported;
  return launch_dense<DENSE_LIN, ISX_RELU>(m, n, centres, halves, out, s);
}

// ------------------------------------------------------- output read-off
// Mean and spread of the output (Eq. 2 / Eq. 7) from the per-neuron vectors
// the hidden layers left (pre-activation centre Y, ReLU slope A, shift B and
// new-symbol coefficient G of every hidden layer), without the coefficient
// blocks: with the row vector v_L = w_out and v_{h-1} = (v_h . A_h) W_h, the
// output's coefficient on the symbols created at hidden layer h is
// v_h[j] G_h[j] and on input symbol a it is ((v_1 . A_1) W_1)[a] times the
// input scale, so the spread sums those (squares for UP, magnitudes for AA).
// The chain of row vectors of BN cells is a sequence of GEMMs
// U_{h-1} = (W_h^T U_h) . A_{h-1} on MFMA, with U in LDS as [cell][neuron].
struct OutNet {
  int n_linear;
  int n[ISX_MAX_LINEAR + 1];
  const float* Wt[ISX_MAX_LINEAR];  // W^T of each linear layer, [n_in][n_out]
  const float* W0;                  // first layer [n_1][3]
  const float* wout;                // last layer [n_last]
  const float* bout;
  const float* Y[ISX_MAX_LINEAR];   // per hidden layer h: [C][n_h]
  const float* A[ISX_MAX_LINEAR];
  const float* B[ISX_MAX_LINEAR];
  const float* G[ISX_MAX_LINEAR];
};

template <int METHOD>
__device__ __forceinline__ float out_stat(float v) {
  return METHOD == ISX_UP ? v * v : fabsf(v);
}

template <int METHOD, int KMAX>
__global__ __launch_bounds__(kDenseThreads) void output_mfma_kernel(int64_t C, OutNet net,
                                                                    const float* __restrict__ halves,
                                                                    float* __restrict__ out) {
  constexpr int BN = DenseShape<KMAX>::BN;
  constexpr int STRIDE = DenseShape<KMAX>::STRIDE;
  constexpr int CB = BN / 32;
  constexpr int RBMAX = KMAX / 32;
  extern __shared__ float4 out_smem4[];
  float* X = reinterpret_cast<float*>(out_smem4);  // [BN][STRIDE]
  float* slots = X + BN * STRIDE;                  // [BN][RBMAX] spread partials per 32-row block
  float* cmu = slots + BN * RBMAX;                 // [BN]
  float* cacc = cmu + BN;                          // [BN]

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int q = lane >> 5;
  const int l32 = lane & 31;
  const int64_t cell0 = (int64_t)blockIdx.x * BN;
  const int Lh = net.n_linear - 1;

  for (int i = tid; i < BN * RBMAX; i += kDenseThreads) slots[i] = 0.f;
  // last hidden layer: mean, its new symbols, and U_L = w_out . A_L
  {
    const int nL = net.n[Lh];
    const float* Yh = net.Y[Lh];
    const float* Ah = net.A[Lh];
    const float* Bh = net.B[Lh];
    const float* Gh = net.G[Lh];
    for (int c0 = 0; c0 < BN; c0 += kDenseThreads / 4) {
      const int col = c0 + tid / 4, part = tid & 3;
      const int64_t cell = cell0 + col;
      float mu_p = 0.f, acc_p = 0.f;
      if (col < BN) {
        for (int j = part; j < nL; j += 4) {
          float u = 0.f;
          if (cell < C) {
            const float w = net.wout[j];
            const int64_t e = cell * nL + j;
            mu_p += w * (Ah[e] * Yh[e] + Bh[e]);
            acc_p += out_stat<METHOD>(w * Gh[e]);
            u = w * Ah[e];
          }
          X[col * STRIDE + j] = u;
        }
      }
      mu_p += __shfl_xor(mu_p, 1);
      mu_p += __shfl_xor(mu_p, 2);
      acc_p += __shfl_xor(acc_p, 1);
      acc_p += __shfl_xor(acc_p, 2);
      if (col < BN && part == 0) {
        cmu[col] = mu_p;
        cacc[col] = acc_p;
      }
    }
  }
  __syncthreads();

  for (int h = Lh; h >= 2; --h) {
    const int nh = net.n[h], np = net.n[h - 1];
    const int RB = np / 32;
    const int nblk = RB * CB;
    const int bpw = (nblk + 7) / 8;
    const int t0 = wave * bpw;
    v16f_d acc[kDenseBlocksPerWave];
#pragma unroll
    for (int j = 0; j < kDenseBlocksPerWave; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;
    dense_tile_gemm<CB, STRIDE>(net.Wt[h - 1], nh, X, t0, bpw, nblk, l32, q, acc);
    __syncthreads();  // every wave has read U_h
    const float* Gp = net.G[h - 1];
    const float* Ap = net.A[h - 1];
#pragma unroll
    for (int j = 0; j < kDenseBlocksPerWave; ++j) {
      const int t = t0 + j;
      if (j < bpw && t < nblk) {
        const int rb = t / CB, cb = t - rb * CB;
        const int col = cb * 32 + l32;
        const int64_t cell = cell0 + col;
        float sp = 0.f;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int row = rb * 32 + 8 * qq + 4 * q;
          float4 g4 = make_float4(0.f, 0.f, 0.f, 0.f), a4 = g4;
          if (cell < C) {
            g4 = *reinterpret_cast<const float4*>(Gp + cell * np + row);
            a4 = *reinterpret_cast<const float4*>(Ap + cell * np + row);
          }
          const float v0 = acc[j][4 * qq + 0], v1 = acc[j][4 * qq + 1];
          const float v2 = acc[j][4 * qq + 2], v3 = acc[j][4 * qq + 3];
          sp += out_stat<METHOD>(v0 * g4.x) + out_stat<METHOD>(v1 * g4.y) + out_stat<METHOD>(v2 * g4.z) +
                out_stat<METHOD>(v3 * g4.w);
          *reinterpret_cast<float4*>(X + col * STRIDE + row) = make_float4(v0 * a4.x, v1 * a4.y, v2 * a4.z, v3 * a4.w);
        }
        sp += __shfl_xor(sp, 32);
        if (q == 0) slots[col * RBMAX + rb] += sp;
      }
    }
    __syncthreads();
  }

  // input symbols: ((v_1 . A_1) W_1)[a] times the input scale
  {
    const int n1 = net.n[1];
    const float sc = METHOD == ISX_UP ? 0.57735026918962576451f : 1.f;
    for (int c0 = 0; c0 < BN; c0 += kDenseThreads / 4) {
      const int col = c0 + tid / 4, part = tid & 3;
      const int64_t cell = cell0 + col;
      float t = 0.f;
      if (col < BN && part < 3 && cell < C) {
        float sa = 0.f;
        for (int j = 0; j < n1; ++j) sa += X[col * STRIDE + j] * net.W0[j * 3 + part];
        t = out_stat<METHOD>(sa * (halves[cell * 3 + part] * sc));
      }
      t += __shfl_xor(t, 1);
      t += __shfl_xor(t, 2);
      if (col < BN && part == 0 && cell < C) {
        float a = cacc[col] + t;
        for (int r = 0; r < RBMAX; ++r) a += slots[col * RBMAX + r];
        out[cell * 2 + 0] = cmu[col] + net.bout[0];
        out[cell * 2 + 1] = METHOD == ISX_UP ? sqrtf(a) : a;
      }
    }
  }
}

template <int METHOD, int KMAX>
static hipError_t launch_output_k(int64_t C, const OutNet& net, const float* halves, float* out, hipStream_t s) {
  using Sh = DenseShape<KMAX>;
  const size_t lds = Sh::LDS + (size_t)(Sh::BN * (KMAX / 32) + 2 * Sh::BN) * sizeof(float);
  {
    hipError_t e = ensure_lds_limit(reinterpret_cast<const void*>(&output_mfma_kernel<METHOD, KMAX>), (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t blocks = (C + Sh::BN - 1) / Sh::BN;
  hipLaunchKernelGGL((output_mfma_kernel<METHOD, KMAX>), dim3((unsigned)blocks), dim3(kDenseThreads), lds, s, C, net,
                     halves, out);
  return hipGetLastError();
}

double output_flops_per_cell(const Model& m) {
  double f = 6.0 * m.widths[m.n_linear - 1] + 6.0 * m.widths[1];
  for (int h = 2; h < m.n_linear; ++h) f += 2.0 * m.widths[h] * m.widths[h - 1] + 4.0 * m.widths[h - 1];
  return f;
}

hipError_t launch_output_mfma(const Model& m, isx_method method, int64_t C, float* const* Y, float* const* A,
                              float* const* B, float* const* G, const float* halves, float* out, hipStream_t s) {
  if (C <= 0) return hipSuccess;
  OutNet net{};
  net.n_linear = m.n_linear;
  for (int i = 0; i <= m.n_linear; ++i) net.n[i] = m.pw[i];
  for (int l = 0; l < m.n_linear; ++l) net.Wt[l] = m.L[l].Wt;
  net.W0 = m.L[0].W;
  net.wout = m.L[m.n_linear - 1].W;
  net.bout = m.L[m.n_linear - 1].b;
  for (int h = 1; h < m.n_linear; ++h) {
    net.Y[h] = Y[h];
    net.A[h] = A[h];
    net.B[h] = B[h];
    net.G[h] = G[h];
  }
  const int kmax = dense_kmax(m);
  if (m.n_linear < 2 || kmax < 32) return hipErrorNotSupported;
  const bool up = method == ISX_UP;
  if (kmax <= 256) return up ? launch_output_k<ISX_UP, 256>(C, net, halves, out, s)
                             : launch_output_k<ISX_AA, 256>(C, net, halves, out, s);
  if (kmax <= 512) return up ? launch_output_k<ISX_UP, 512>(C, net, halves, out, s)
                             : launch_output_k<ISX_AA, 512>(C, net, halves, out, s);
  return up ? launch_output_k<ISX_UP, 1024>(C, net, halves, out, s)
            : launch_output_k<ISX_AA, 1024>(C, net, halves, out, s);
}

// ------------------------------------------ centre linearisation in BF16
// The same (f(c), s) as DENSE_LIN for nets whose hidden layers all have one
// padded width N <= kCovNMax, on BF16 MFMA (v_mfma_f32_32x32x16_bf16):
//   * every column (the centre and the three tangents) is carried as two
//     bfloat16 parts, x = xh + xl (xl = bf16(x - xh)), and each layer's
//     product is Wh xh + Wh xl + Wl xh with W = Wh + Wl (both bfloat16); the
//     dropped term Wl xl and the splits leave a relative error near 2^-16 per
//     layer, the level of a float32 dot product of this length (three
//     bfloat16 products cost about a fifth of one float32 product).
// A workgroup owns 32 cells.  In LDS: X[col][cell][2N] = (xh | xl) for
// col = 0 (centre) and 1..3 (tangents), rows padded by 8 bfloat16 (16 bytes).
// Wave w owns weight row block w (32 neurons) and its four column tiles, so
// each pair of weight fragments (Wh, Wl) serves twelve products.
namespace {
typedef __bf16 lbf16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(1))) const lbf16x8 glbf16x8;
typedef float lv16f __attribute__((ext_vector_type(16)));
constexpr int kLinCells = 32;

template <int N>
struct LinShape {
  static constexpr int STR = 2 * N + 8;  // row stride (bfloat16): xh | xl | pad
  static constexpr int KS = N / 16;
  static constexpr int RB = N / 32;
  static constexpr size_t LDS = (size_t)4 * kLinCells * STR * 2;
};
}  // namespace

template <int N>
__global__ __launch_bounds__(kDenseThreads) void lin_bf16_kernel(int64_t n_items, int n_linear,
                                                                 const DevLayer* __restrict__ layers,
                                                                 const float* __restrict__ centres,
                                                                 const float* __restrict__ halves,
                                                                 float* __restrict__ out) {
  using S = LinShape<N>;
  constexpr int STR = S::STR, KS = S::KS;
  extern __shared__ float4 lin_smem4[];
  __bf16* X = reinterpret_cast<__bf16*>(lin_smem4);  // [4][kLinCells][STR]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, hi = lane >> 5;
  const int64_t item0 = (int64_t)blockIdx.x * kLinCells;
  auto row = [&](int col, int cell) { return X + (size_t)(col * kLinCells + cell) * STR; };

  // ---- layer 1 (3 -> N) on the vector ALUs
  {
    const DevLayer L1 = layers[0];
    for (int e = tid; e < kLinCells * N; e += kDenseThreads) {
      const int cell = e / N, j = e - cell * N;
      const int64_t item = item0 + cell;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (item < n_items) {
        const float w0 = L1.W[j * 3 + 0], w1 = L1.W[j * 3 + 1], w2 = L1.W[j * 3 + 2];
        const float* c = centres + item * 3;
        const float pre = L1.b[j] + w0 * c[0] + w1 * c[1] + w2 * c[2];
        if (pre > 0.f) {
          const float* h = halves + item * 3;
          v[0] = pre;
          v[1] = w0 * h[0] * 0.57735026918962576451f;
          v[2] = w1 * h[1] * 0.57735026918962576451f;
          v[3] = w2 * h[2] * 0.57735026918962576451f;
        }
      }
#pragma unroll
      for (int col = 0; col < 4; ++col) {
        const __bf16 xh = (__bf16)v[col];
        row(col, cell)[j] = xh;
        row(col, cell)[N + j] = (__bf16)(v[col] - (float)xh);
      }
    }
  }
  __syncthreads();

  // ---- hidden layers 2 .. n_linear-1
  for (int l = 1; l + 1 < n_linear; ++l) {
    const DevLayer Lw = layers[l];
    const bool active = wave < S::RB;  // wave-uniform
    const int rb = active ? wave : 0;
    glbf16x8* ah = (glbf16x8*)(reinterpret_cast<const __bf16*>(Lw.Wfr) + ((int64_t)rb * KS * 64 + lane) * 8);
    glbf16x8* al = (glbf16x8*)(reinterpret_cast<const __bf16*>(Lw.Wfrl) + ((int64_t)rb * KS * 64 + lane) * 8);
    lv16f acc[4];
#pragma unroll
    for (int col = 0; col < 4; ++col)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[col][r] = 0.f;
    if (active) {
      lbf16x8 a_next = ah[0], l_next = al[0];
      for (int ks = 0; ks < KS; ++ks) {
        const lbf16x8 a = a_next, lo = l_next;
        if (ks + 1 < KS) {
          a_next = ah[64 * (ks + 1)];
          l_next = al[64 * (ks + 1)];
        }
#pragma unroll
        for (int col = 0; col < 4; ++col) {
          const __bf16* b = row(col, l32) + 8 * hi + 16 * ks;  // this lane's cell, k = 8 hi
          const lbf16x8 xh = *reinterpret_cast<const lbf16x8*>(b);
          const lbf16x8 xl = *reinterpret_cast<const lbf16x8*>(b + N);
          acc[col] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, xh, acc[col], 0, 0, 0);
          acc[col] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, xl, acc[col], 0, 0, 0);
          acc[col] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo, xh, acc[col], 0, 0, 0);
        }
      }
    }
    __syncthreads();  // every wave has read the layer input
    // register r of acc[col] holds (neuron 32 rb + 8(r/4) + 4 hi + r%4, cell
    // l32); the tangents take the ReLU mask of the centre's pre-activation
    if (active) {
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        const int i0 = rb * 32 + 8 * q4 + 4 * hi;
        bool on[4];
#pragma unroll
        for (int col = 0; col < 4; ++col) {
          __bf16 vh[4], vl[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            float x = acc[col][4 * q4 + u];
            if (col == 0) {
              x += Lw.b[i0 + u];
              on[u] = x > 0.f;
            }
            x = on[u] ? x : 0.f;
            vh[u] = (__bf16)x;
            vl[u] = (__bf16)(x - (float)vh[u]);
          }
          *reinterpret_cast<uint2*>(row(col, l32) + i0) = *reinterpret_cast<const uint2*>(vh);
          *reinterpret_cast<uint2*>(row(col, l32) + N + i0) = *reinterpret_cast<const uint2*>(vl);
        }
      }
    }
    __syncthreads();
  }

  // ---- output layer (N -> 1): per cell the value and the three directional
  // derivatives, each a float32 dot product by 4 threads in a fixed order
  {
    const DevLayer Lo = layers[n_linear - 1];
    const int dot = tid >> 2, part = tid & 3;  // 128 dots: (cell, column)
    const int cell = dot >> 2, col = dot & 3;
    const __bf16* x = row(col, cell);
    float s = 0.f;
    for (int k = part; k < N; k += 4) s += Lo.W[k] * ((float)x[k] + (float)x[N + k]);
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    // the cell's four sums sit in lanes 16c', 16c'+4, 16c'+8, 16c'+12 of the wave
    const int base = lane & ~15;
    const float f = __shfl(s, base), d1 = __shfl(s, base + 4), d2 = __shfl(s, base + 8),
                d3 = __shfl(s, base + 12);
    const int64_t item = item0 + cell;
    if ((tid & 15) == 0 && item < n_items) {
      out[item * 2 + 0] = f + Lo.b[0];
      out[item * 2 + 1] = sqrtf(d1 * d1 + d2 * d2 + d3 * d3);
    }
  }
}

template <int N>
static hipError_t launch_lin_n(const Model& m, int64_t n, const float* centres, const float* halves, float* out,
                               hipStream_t s) {
  {
    hipError_t e = ensure_lds_limit(reinterpret_cast<const void*>(&lin_bf16_kernel<N>), (int)LinShape<N>::LDS);
    if (e != hipSuccess) return e;
  }
  // a launch's work-items must stay below 2^32
  const int64_t per_launch = ((int64_t(1) << 31) / kDenseThreads) * kLinCells;
  for (int64_t o = 0; o < n; o += per_launch) {
    const int64_t c = std::min(per_launch, n - o);
    hipLaunchKernelGGL((lin_bf16_kernel<N>), dim3((unsigned)((c + kLinCells - 1) / kLinCells)), dim3(kDenseThreads),
                       LinShape<N>::LDS, s, c, m.n_linear, m.dev_layers, centres + 3 * o, halves + 3 * o, out + 2 * o);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

bool lin_bf16_supported(const Model& m) {
  if (m.n_linear < 3 || !cov_supported(m)) return false;
  for (int l = 1; l + 1 < m.n_linear; ++l)
    if (!m.L[l].Wfr || !m.L[l].Wfrl) return false;
  return true;
}

hipError_t linearize_bf16(const Model& m, int64_t n, const float* centres, const float* halves, float* out,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (!lin_bf16_supported(m)) return hipErrorNotSupported;
  switch (m.pw[1]) {
    case 32: return launch_lin_n<32>(m, n, centres, halves, out, s);
    case 64: return launch_lin_n<64>(m, n, centres, halves, out, s);
    case 96: return launch_lin_n<96>(m, n, centres, halves, out, s);
    case 128: return launch_lin_n<128>(m, n, centres, halves, out, s);
    case 160: return launch_lin_n<160>(m, n, centres, halves, out, s);
    case 192: return launch_lin_n<192>(m, n, centres, halves, out, s);
    case 224: return launch_lin_n<224>(m, n, centres, halves, out, s);
    case 256: return launch_lin_n<256>(m, n, centres, halves, out, s);
    default: return hipErrorNotSupported;
  }
}


// ------------------------------------------ output read-off in BF16 (UP)
// The read-off's downward chain U_{h-1} = (U_h W_h) . A_{h-1} (rows: cells)
// for the BF16 path's nets with one padded hidden width N <= kCovNMax, on
// BF16 MFMA: U in LDS as bfloat16 hi/lo parts ([cell][neuron], rows padded
// by 8), W_h^T in fragment order as hi/lo copies, and each product
// Wh Uh + Wh Ul + Wl Uh in float32 (the dropped Wl Ul and the splits leave a
// relative error near 2^-16 per layer; the spread is a sum of squares, so it
// does not cancel).  Only for UP: the AA rounding margin assumes a float32
// read-off.  A workgroup owns 64 cells; wave w owns neuron block w of
// U_{h-1} and both cell blocks.
namespace {
constexpr int kOutCells = 64;

template <int N>
struct OutShape {
  static constexpr int STR = N + 8;
  static constexpr int KS = N / 16;
  static constexpr int RB = N / 32;
  static constexpr int CB = kOutCells / 32;
  static constexpr size_t LDS = (size_t)2 * kOutCells * STR * 2 + (size_t)kOutCells * (RB + 2) * sizeof(float);
};

__device__ __forceinline__ void split_store4(__bf16* h, __bf16* l, float v0, float v1, float v2, float v3) {
  __bf16 a[4], b[4];
  const float v[4] = {v0, v1, v2, v3};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    a[e] = (__bf16)v[e];
    b[e] = (__bf16)(v[e] - (float)a[e]);
  }
  *reinterpret_cast<uint2*>(h) = *reinterpret_cast<const uint2*>(a);
  *reinterpret_cast<uint2*>(l) = *reinterpret_cast<const uint2*>(b);
}
}  // namespace

template <int N>
__global__ __launch_bounds__(kDenseThreads) void output_bf16_kernel(int64_t C, OutNet net,
                                                                    const DevLayer* __restrict__ layers,
                                                                    const float* __restrict__ halves,
                                                                    float* __restrict__ out) {
  using S = OutShape<N>;
  constexpr int STR = S::STR, KS = S::KS, RB = S::RB, CB = S::CB;
  extern __shared__ float4 ob_smem4[];
  __bf16* Uh = reinterpret_cast<__bf16*>(ob_smem4);  // [kOutCells][STR]
  __bf16* Ul = Uh + kOutCells * STR;
  float* slots = reinterpret_cast<float*>(Ul + kOutCells * STR);  // [kOutCells][RB] spread partials
  float* cmu = slots + kOutCells * RB;                            // [kOutCells]
  float* cacc = cmu + kOutCells;                                  // [kOutCells]
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l32 = lane & 31, hi = lane >> 5;
  const int64_t cell0 = (int64_t)blockIdx.x * kOutCells;
  const int Lh = net.n_linear - 1;

  for (int i = tid; i < kOutCells * RB; i += kDenseThreads) slots[i] = 0.f;
  // last hidden layer: 8 lanes per cell, 4 neurons each per step (one
  // 128-byte line per cell and array): the mean, the layer's own symbols and
  // U_L = w_out . A_L
  {
    const int cl = tid >> 3, part = tid & 7;
    const int64_t cell = cell0 + cl;
    const float* Yh = net.Y[Lh];
    const float* Ah = net.A[Lh];
    const float* Bh = net.B[Lh];
    const float* Gh = net.G[Lh];
    float mu = 0.f, ac = 0.f;
    for (int j = 4 * part; j < N; j += 32) {
      float4 y4 = make_float4(0.f, 0.f, 0.f, 0.f), a4 = y4, b4 = y4, g4 = y4;
      if (cell < C) {
        const int64_t e = cell * N + j;
        y4 = *reinterpret_cast<const float4*>(Yh + e);
        a4 = *reinterpret_cast<const float4*>(Ah + e);
        b4 = *reinterpret_cast<const float4*>(Bh + e);
        g4 = *reinterpret_cast<const float4*>(Gh + e);
      }
      const float4 w4 = *reinterpret_cast<const float4*>(net.wout + j);
      mu += w4.x * (a4.x * y4.x + b4.x) + w4.y * (a4.y * y4.y + b4.y) + w4.z * (a4.z * y4.z + b4.z) +
            w4.w * (a4.w * y4.w + b4.w);
      const float q0 = w4.x * g4.x, q1 = w4.y * g4.y, q2 = w4.z * g4.z, q3 = w4.w * g4.w;
      ac += q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
      split_store4(Uh + cl * STR + j, Ul + cl * STR + j, w4.x * a4.x, w4.y * a4.y, w4.z * a4.z, w4.w * a4.w);
    }
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
      mu += __shfl_xor(mu, o);
      ac += __shfl_xor(ac, o);
    }
    if (part == 0) {
      cmu[cl] = mu;
      cacc[cl] = ac;
    }
  }
  __syncthreads();

  for (int h = Lh; h >= 2; --h) {
    const DevLayer Lw = layers[h - 1];  // W_h, [N][N]
    lv16f acc[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[cb][e] = 0.f;
    // the epilogue's G and A of layer h-1 are loaded before the products
    // (they do not depend on them), so their latency overlaps the MFMAs
    float4 gpre[CB][4], apre[CB][4];
    if (wave < RB) {
      const float* Gp = net.G[h - 1];
      const float* Ap = net.A[h - 1];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int64_t cell = cell0 + cb * 32 + l32;
        const int64_t cc = cell < C ? cell : C - 1;  // (rows past the end read a valid cell, unused)
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int i0 = wave * 32 + 8 * q4 + 4 * hi;
          gpre[cb][q4] = *reinterpret_cast<const float4*>(Gp + cc * N + i0);
          apre[cb][q4] = *reinterpret_cast<const float4*>(Ap + cc * N + i0);
        }
      }
    }
    if (wave < RB) {
      const int64_t fo = ((int64_t)wave * KS * 64 + lane) * 8;
      glbf16x8* ah_p = (glbf16x8*)(reinterpret_cast<const __bf16*>(Lw.WTfr) + fo);
      glbf16x8* al_p = (glbf16x8*)(reinterpret_cast<const __bf16*>(Lw.WTfrl) + fo);
#pragma unroll 4
      for (int ks = 0; ks < KS; ++ks) {
        const lbf16x8 ah = ah_p[64 * ks], al = al_p[64 * ks];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const size_t o = (size_t)(cb * 32 + l32) * STR + 16 * ks + 8 * hi;
          const lbf16x8 bh = *reinterpret_cast<const lbf16x8*>(Uh + o);
          const lbf16x8 bl = *reinterpret_cast<const lbf16x8*>(Ul + o);
          acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[cb], 0, 0, 0);
          acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[cb], 0, 0, 0);
          acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[cb], 0, 0, 0);
        }
      }
    }
    __syncthreads();  // every wave has read U_h
    if (wave < RB) {
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int col = cb * 32 + l32;
        float sp = 0.f;
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int i0 = wave * 32 + 8 * q4 + 4 * hi;  // accumulator rows i0..i0+3
          const float4 g4 = gpre[cb][q4], a4 = apre[cb][q4];
          const float v0 = acc[cb][4 * q4 + 0], v1 = acc[cb][4 * q4 + 1];
          const float v2 = acc[cb][4 * q4 + 2], v3 = acc[cb][4 * q4 + 3];
          const float r0 = v0 * g4.x, r1 = v1 * g4.y, r2 = v2 * g4.z, r3 = v3 * g4.w;
          sp += r0 * r0 + r1 * r1 + r2 * r2 + r3 * r3;
          split_store4(Uh + col * STR + i0, Ul + col * STR + i0, v0 * a4.x, v1 * a4.y, v2 * a4.z, v3 * a4.w);
        }
        sp += __shfl_xor(sp, 32);
        if (hi == 0) slots[col * RB + wave] += sp;
      }
    }
    __syncthreads();
  }

  // input symbols: ((v_1 . A_1) W_1)[a] times the input scale h_a / sqrt 3
  {
    const int cl = tid >> 3, part = tid & 7;
    const int64_t cell = cell0 + cl;
    float t = 0.f;
    if (part < 3 && cell < C) {
      float sa = 0.f;
      for (int j = 0; j < N; ++j)
        sa += ((float)Uh[cl * STR + j] + (float)Ul[cl * STR + j]) * net.W0[j * 3 + part];
      const float v = sa * (halves[cell * 3 + part] * 0.57735026918962576451f);
      t = v * v;
    }
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) t += __shfl_xor(t, o);
    if (part == 0 && cell < C) {
      float a = cacc[cl] + t;
      for (int r = 0; r < RB; ++r) a += slots[cl * RB + r];
      out[cell * 2 + 0] = cmu[cl] + net.bout[0];
      out[cell * 2 + 1] = sqrtf(a);
    }
  }
}

template <int N>
static hipError_t launch_out_bf16_n(int64_t C, const OutNet& net, const Model& m, const float* halves, float* out,
                                    hipStream_t s) {
  {
    hipError_t e = ensure_lds_limit(reinterpret_cast<const void*>(&output_bf16_kernel<N>), (int)OutShape<N>::LDS);
    if (e != hipSuccess) return e;
  }
  const int64_t blocks = (C + kOutCells - 1) / kOutCells;
  hipLaunchKernelGGL((output_bf16_kernel<N>), dim3((unsigned)blocks), dim3(kDenseThreads), OutShape<N>::LDS, s, C,
                     net, m.dev_layers, halves, out);
  return hipGetLastError();
}

bool output_bf16_supported(const Model& m) {
  if (m.n_linear < 2 || !cov_supported(m)) return false;
  for (int l = 1; l + 1 < m.n_linear; ++l)
    if (!m.L[l].WTfr || !m.L[l].WTfrl) return false;
  return true;
}

hipError_t launch_output_bf16(const Model& m, int64_t C, float* const* Y, float* const* A, float* const* B,
                              float* const* G, const float* halves, float* out, hipStream_t s) {
  if (C <= 0) return hipSuccess;
  if (!output_bf16_supported(m)) return hipErrorNotSupported;
  OutNet net{};
  net.n_linear = m.n_linear;
  for (int i = 0; i <= m.n_linear; ++i) net.n[i] = m.pw[i];
  for (int l = 0; l < m.n_linear; ++l) net.Wt[l] = m.L[l].Wt;
  net.W0 = m.L[0].W;
  net.wout = m.L[m.n_linear - 1].W;
  net.bout = m.L[m.n_linear - 1].b;
  for (int h = 1; h < m.n_linear; ++h) {
    net.Y[h] = Y[h];
    net.A[h] = A[h];
    net.B[h] = B[h];
    net.G[h] = G[h];
  }
  switch (m.pw[1]) {
    case 32: return launch_out_bf16_n<32>(C, net, m, halves, out, s);
    case 64: return launch_out_bf16_n<64>(C, net, m, halves, out, s);
    case 96: return launch_out_bf16_n<96>(C, net, m, halves, out, s);
    case 128: return launch_out_bf16_n<128>(C, net, m, halves, out, s);
    case 160: return launch_out_bf16_n<160>(C, net, m, halves, out, s);
    case 192: return launch_out_bf16_n<192>(C, net, m, halves, out, s);
    case 224: return launch_out_bf16_n<224>(C, net, m, halves, out, s);
    case 256: return launch_out_bf16_n<256>(C, net, m, halves, out, s);
    default: return hipErrorNotSupported;
  }
}

}  // namespace isx
