// Uncertainty propagation in covariance form on BF16 MFMA for hidden widths
// whose N x N covariance does not fit one CU's LDS: between layers the
// per-cell matrices live in device memory, and each layer is one launch.
//
// The form is the one of kernels_cov.hip (Eq. 8-9 through covariances):
//   C_1 = F F^T,  F = W_1 diag(h / sqrt 3)  (N x 3),
//   per hidden layer h >= 2, with X_{h-1} = D C_{h-1} D + diag(gamma^2)
//   (D = diag(alpha) and gamma of layer h-1):
//     T = W_h X_{h-1},  v_j = C_h[j][j] = sum_i T[j][i] W_h[j][i],
//     y = W_h z + b (z = alpha . y_{h-1} + beta),
//     the rule gives (alpha, beta, gamma) from (y, v),
//     C_h = T W_h^T  (not after the last hidden layer).
// Stored between layers: Chat[i][k] = alpha_k C[i][k] (bfloat16, one factor
// of D applied along the second index), with the diagonal alpha_i v_i from
// the variance the rule used, in 32 x 8 blocks (chat_index): the 16 bytes of
// 8 consecutive k of a row, for 32 consecutive rows, are one 512-byte run.
// Then X[i][k] = alpha_i Chat[i][k] + [i = k] gamma_i^2, so that
//   T[j][i] = alpha_i (Chat W_h^T)[i][j] + gamma_i^2 W_h[j][i]
// needs no per-element scaling of an MFMA operand: a workgroup that owns
// neurons R can store its block of the next Chat (columns R, scaled by its
// own alpha_R) without the other workgroups' alphas.
// Layer 2 at widths 256 and 512 runs in rank-3 form: with X_1 = D_1 F F^T
// D_1 + diag(gamma_1^2), step 1's product is F_i . P_j, P_j = sum_k
// W_2[j][k] alpha_k F_k, formed on the vector ALUs, and Chat_1 is never
// stored (at 1024 its extra LDS does not fit and layer 1 writes Chat_1).
// One launch per layer h >= 2; a workgroup owns RB = 65536 / N neurons j of
// one cell (N / RB workgroups per cell, 8 blocks apart so that they run on
// the same XCD and share the cell's Chat through its L2):
//   1. Out = Chat W_R^T (N x RB) on v_mfma_f32_32x32x16_bf16, rows of Chat
//      staged through LDS in K chunks (double buffer, each chunk's loads two
//      chunks ahead), weight fragments of rows R streamed from the
//      L2-resident fragment-order copy of W_h one chunk ahead; the epilogue
//      forms T[j][i] (float32), sums each neuron's variance, its magnitude
//      and its centre W z over the lane's rows (float32 weights from the
//      accumulator-quad copy), and keeps T_R in LDS as bfloat16 (row-major,
//      rows R);
//   2. per neuron j in R: the partial sums in a fixed order, the rule, the
//      layer's (y, alpha, beta, gamma);
//   3. C_R = T_R W_h^T (RB x N), A = rows of T_R from LDS, B = weight
//      fragments in a ring four k-steps ahead; the epilogue stores
//      Chat[m][j] = alpha_j C[j][m] (C is symmetric), the diagonal
//      alpha_j v_j, one 512-byte run per store instruction.  The last hidden
//      layer stops after step 2.
// The cancellation check is the LDS kernel's (a variance sum that keeps at
// most 2^-9 of its terms' magnitude, where the rule depends on sigma, marks
// the cell for the host's float64 re-propagation).
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

constexpr int kGThreads = 512;  // 8 waves

template <int N>
struct CovgShape {
  static constexpr int RB = 65536 / N;  // neurons per workgroup (256, 128, 64)
  static constexpr int NR = N / RB;     // workgroups per cell (1, 4, 16)
  static constexpr int KC = N <= 512 ? 32 : 16;  // K chunk of the staged Chat rows
  static constexpr int SSTR = KC + 8;            // staged row stride (bfloat16; 16-byte multiple)
  static constexpr int SPT = N * KC / 8 / 512;   // 16-byte pieces per thread and chunk (2, 4, 4)
  static constexpr int D = 2;                    // chunks in flight (register sets)
  static constexpr int TSTR = N + 8;    // row stride of T_R in LDS
  // step 1: Out (N x RB) on WI1 x WJ1 waves of PI x PJ blocks of 32 x 32
  static constexpr int PI = 4, PJ = 2;
  static constexpr int WI1 = N / 32 / PI;  // 2, 4, 8
  static constexpr int WJ1 = 8 / WI1;      // 4, 2, 1
  // step 3: C_R (RB x N) on WJ3 x WM3 waves of QJ x QM blocks
  static constexpr int WJ3 = N == 256 ? 2 : 1;
  static constexpr int WM3 = 8 / WJ3;
  static constexpr int QJ = RB / 32 / WJ3;  // 4, 4, 2
  static constexpr int QM = N / 32 / WM3;   // 2, 2, 4
  static constexpr size_t STAGE = (size_t)2 * N * SSTR * 2;
  static constexpr size_t TBYTES = (size_t)RB * TSTR * 2;
  static constexpr size_t REGION = STAGE > TBYTES ? STAGE : TBYTES;  // staging, then T_R
  static constexpr size_t PART = (size_t)3 * WI1 * RB * 4;          // partial sums
  static constexpr size_t VECS = (size_t)(3 * N + 2 * RB) * 4;
  static constexpr size_t LDS = REGION + PART + VECS;
  // layer 2 in rank-3 form: F and alpha of layer 1 and P after the vectors
  static constexpr size_t LDS_FIRST = LDS + (size_t)(N + RB) * 16;
  static constexpr bool RANK3 = LDS_FIRST <= 160 * 1024;  // widths 256 and 512
  static_assert(PI * WI1 * 32 == N && PJ * WJ1 * 32 == RB, "step-1 tiling");
  static_assert(QJ * WJ3 * 32 == RB && QM * WM3 * 32 == N, "step-3 tiling");
  static_assert(LDS <= 160 * 1024, "LDS");
};

// Element offset of Chat[i][k] within a cell's N x N matrix: blocks of 32
// rows x 8 columns (512 bytes), row blocks outermost, then column groups.
template <int N>
__device__ __forceinline__ int64_t chat_index(int i, int k) {
  return ((int64_t)(i >> 5) * (N / 8) + (k >> 3)) * 256 + (i & 31) * 8 + (k & 7);
}

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

// A variance sum is flagged when it keeps at most this fraction of the
// summed magnitude of its terms (as in the LDS kernel).
constexpr float kGCancelRatio = 0x1p-9f;

// Layer h >= 2: steps 1-3 above for the RB neurons of one workgroup.
// vprev / vcur: the (y, alpha, beta, gamma) blocks of layers h-1 and h
// ([4][C][N] floats each); Cin / Cout: Chat of layers h-1 and h ([C][N][N]).
// FIRST (layer 2, where X_1 = D_1 F F^T D_1 + diag(gamma_1^2) has rank 3
// plus a diagonal): step 1's product is Out[i][j] = F_i . P_j with
// P_j = sum_k W[j][k] alpha_k F_k, formed on the vector ALUs from the cell's
// box and W_1 (Chat_1 is never stored).
template <int N, int ACT, bool LAST, bool FIRST>
__global__ __launch_bounds__(kGThreads) void covg_layer_kernel(int64_t C, const __bf16* __restrict__ Cin,
                                                                __bf16* __restrict__ Cout,
                                                                const __bf16* __restrict__ Wfr,
                                                                const float4* __restrict__ Wq,
                                                                const float* __restrict__ W1,
                                                                const float* __restrict__ halves,
                                                                const float* __restrict__ bias,
                                                                const float* __restrict__ vprev,
                                                                float* __restrict__ vcur,
                                                                uint32_t* __restrict__ cancel) {
  using S = CovgShape<N>;
  constexpr int RB = S::RB, NR = S::NR, KC = S::KC, SSTR = S::SSTR, TSTR = S::TSTR;
  constexpr int PI = S::PI, PJ = S::PJ, WI1 = S::WI1, QJ = S::QJ, QM = S::QM, WM3 = S::WM3;
  constexpr int KS = N / 16;
  extern __shared__ uint4 covg_smem[];
  unsigned char* base = reinterpret_cast<unsigned char*>(covg_smem);
  __bf16* stage = reinterpret_cast<__bf16*>(base);  // [2][N][SSTR] (step 1)
  __bf16* Tl = reinterpret_cast<__bf16*>(base);     // [RB][TSTR] (steps 1-3)
  float* pv = reinterpret_cast<float*>(base + S::REGION);  // [WI1][RB] variance
  float* pm = pv + WI1 * RB;                               // [WI1][RB] magnitude
  float* py = pm + WI1 * RB;                               // [WI1][RB] centre
  float* s_alpha = py + WI1 * RB;  // [N] alpha of layer h-1
  float* s_g2 = s_alpha + N;       // [N] gamma^2 of layer h-1
  float* s_z = s_g2 + N;           // [N] mean of layer h-1's output
  float* s_ac = s_z + N;           // [RB] alpha of the workgroup's neurons
  float* s_vc = s_ac + RB;         // [RB] their variances

  // block -> (cell, neuron block): the NR blocks of a cell lie 8 apart
  const int64_t blk = blockIdx.x;
  const int64_t grp = blk / (8 * NR);
  const int w8 = (int)(blk - grp * 8 * NR);
  const int64_t cell = grp * 8 + (w8 & 7);
  if (cell >= C) return;
  const int R0 = (w8 >> 3) * RB;
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int l32 = lane & 31, hi = lane >> 5;
  const int64_t NC = (int64_t)N * C;
  const int64_t NN = (int64_t)N * N;

  for (int k = t; k < N; k += kGThreads) {
    const int64_t o = cell * N + k;
    const float a = vprev[NC + o], g = vprev[3 * NC + o];
    s_alpha[k] = a;
    s_g2[k] = g * g;
    s_z[k] = a * vprev[o] + vprev[2 * NC + o];
  }

  // ---- step 1: Out[i][j] = sum_k Chat[i][k] W[j][k], i < N, j in R
  const int wi = wave % WI1, wj = wave / WI1;
  const int i0w = wi * (PI * 32);        // the wave's first row i
  const int j0w = R0 + wj * (PJ * 32);   // the wave's first neuron j
  gv16f acc[PI][PJ];
#pragma unroll
  for (int c = 0; c < PI; ++c)
#pragma unroll
    for (int p = 0; p < PJ; ++p)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[c][p][e] = 0.f;
  if constexpr (FIRST) {
    // F_k (three arrays) and alpha_k of layer 1 and P_j for the workgroup's
    // neurons, after the vectors (the staging region becomes T_R)
    float* s_Fx = s_vc + RB;  // [N] each
    float* s_Fy = s_Fx + N;
    float* s_Fz = s_Fy + N;
    float* s_Fa = s_Fz + N;
    float4* s_P = reinterpret_cast<float4*>(s_Fa + N);  // [RB]
    const float sc = 0.57735026918962576451f;
    const float hx = halves[cell * 3 + 0] * sc, hy = halves[cell * 3 + 1] * sc, hz = halves[cell * 3 + 2] * sc;
    for (int k = t; k < N; k += kGThreads) {
      s_Fx[k] = W1[k * 3 + 0] * hx;
      s_Fy[k] = W1[k * 3 + 1] * hy;
      s_Fz[k] = W1[k * 3 + 2] * hz;
      s_Fa[k] = vprev[NC + cell * N + k];
    }
    __syncthreads();
    // P_j over the epilogue's lane layout (W[j][i..i+3] from the
    // accumulator-quad copy, all loads of a lane in flight at once): partial
    // sums over the lane's rows i, then over hi and the i-waves in a fixed
    // order through the partial-sum area
#pragma unroll
    for (int p = 0; p < PJ; ++p) {
      const int j = j0w + 32 * p + l32;
      const float4* wq = Wq + ((int64_t)((j0w >> 5) + p) * (N / 32) + (i0w >> 5)) * 4 * 64 + lane;
      float px = 0.f, py2 = 0.f, pz = 0.f;
#pragma unroll
      for (int c = 0; c < PI; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = i0w + 32 * c + 8 * q + 4 * hi;
          const float4 w4 = wq[(c * 4 + q) * 64];
          const float4 a4 = *reinterpret_cast<const float4*>(s_Fa + i);
          const float4 fx = *reinterpret_cast<const float4*>(s_Fx + i);
          const float4 fy = *reinterpret_cast<const float4*>(s_Fy + i);
          const float4 fz = *reinterpret_cast<const float4*>(s_Fz + i);
          const float w0 = w4.x * a4.x, w1 = w4.y * a4.y, w2 = w4.z * a4.z, w3 = w4.w * a4.w;
          px = fmaf(w0, fx.x, fmaf(w1, fx.y, fmaf(w2, fx.z, fmaf(w3, fx.w, px))));
          py2 = fmaf(w0, fy.x, fmaf(w1, fy.y, fmaf(w2, fy.z, fmaf(w3, fy.w, py2))));
          pz = fmaf(w0, fz.x, fmaf(w1, fz.y, fmaf(w2, fz.z, fmaf(w3, fz.w, pz))));
        }
      px += __shfl_xor(px, 32);
      py2 += __shfl_xor(py2, 32);
      pz += __shfl_xor(pz, 32);
      if (hi == 0) {
        pv[wi * RB + (j - R0)] = px;
        pm[wi * RB + (j - R0)] = py2;
        py[wi * RB + (j - R0)] = pz;
      }
    }
    __syncthreads();
    if (t < RB) {
      float px = 0.f, py2 = 0.f, pz = 0.f;
#pragma unroll
      for (int w = 0; w < WI1; ++w) {
        px += pv[w * RB + t];
        py2 += pm[w * RB + t];
        pz += py[w * RB + t];
      }
      s_P[t] = make_float4(px, py2, pz, 0.f);
    }
    __syncthreads();
    // the epilogue forms Out[i][j] = F_i . P_j itself, and its T_R stores
    // overwrite the region no wave reads any more
  } else {
  ggbf16x8* wfrag[PJ];
#pragma unroll
  for (int p = 0; p < PJ; ++p) wfrag[p] = (ggbf16x8*)(Wfr + ((int64_t)((j0w >> 5) + p) * KS * 64 + lane) * 8);

  // staging: N rows x KC in pieces of 8 bfloat16 (a row and 8 columns), SPT
  // per thread: lanes run over the 32 rows of a block, then the chunk's P8
  // column groups, so that a wave reads whole 512-byte runs of the blocked
  // layout (rows 32 (t / (32 P8)) + t % 32 + u RSTEP, group (t / 32) % P8).
  // A chunk's pieces are loaded D chunks before the end of the chunk that
  // stores them to LDS (one register set per chunk in flight), so that a load
  // has D chunks of products to arrive.
  constexpr int P8 = KC / 8, RSTEP = kGThreads / P8, SPT = S::SPT, D = S::D;
  constexpr int NCH = N / KC, KK = KC / 16;
  static_assert(NCH % D == 0 && D % 2 == 0, "staging ring");
  const int srow = 32 * (t / (32 * P8)) + (t & 31), sgrp = (t >> 5) % P8;
  const __bf16* ag = Cin + cell * NN + chat_index<N>(srow, 8 * sgrp);
  __bf16* ls = stage + srow * SSTR + 8 * sgrp;
  static_assert(SPT == 2 || SPT == 4, "pieces per thread");
  uint4 a0, a1, a2, a3, b0, b1, b2, b3;  // register sets 0 (a) and 1 (b)
  // (RSTEP rows further: RSTEP / 32 row blocks of 32 N elements; K0 columns
  // further: K0 / 8 groups of 256 elements)
#define COVG_LD1(R, U, K0) R = *reinterpret_cast<const uint4*>(ag + (int64_t)(U) * RSTEP * N + (int64_t)(K0) * 32);
#define COVG_ST1(R, U, BUF) *reinterpret_cast<uint4*>(ls + (BUF) * N * SSTR + (U) * RSTEP * SSTR) = R;
#define COVG_LOAD(R, K0)              \
  {                                   \
    COVG_LD1(R##0, 0, K0)             \
    COVG_LD1(R##1, 1, K0)             \
    if constexpr (SPT > 2) {          \
      COVG_LD1(R##2, 2, K0)           \
      COVG_LD1(R##3, 3, K0)           \
    }                                 \
  }
#define COVG_STORE(R, BUF)            \
  {                                   \
    COVG_ST1(R##0, 0, BUF)            \
    COVG_ST1(R##1, 1, BUF)            \
    if constexpr (SPT > 2) {          \
      COVG_ST1(R##2, 2, BUF)          \
      COVG_ST1(R##3, 3, BUF)          \
    }                                 \
  }
  // weight fragments of the chunk being multiplied (set u & 1); the next
  // chunk's are loaded one chunk ahead
  gbf16x8 wf[2][KK][PJ];
#pragma unroll
  for (int kk = 0; kk < KK; ++kk)
#pragma unroll
    for (int p = 0; p < PJ; ++p) wf[0][kk][p] = wfrag[p][64 * kk];
  // chunk 0 to buffer 0; chunks 1 and 2 in flight in sets b and a
  COVG_LOAD(a, 0);
  COVG_STORE(a, 0);
  COVG_LOAD(b, KC);
  COVG_LOAD(a, 2 * KC);
  __syncthreads();
  // one chunk: ch = ch0 + U is in LDS buffer U & 1; NXT is the register
  // set that holds chunk ch + 1 (D = 2: the two instances cover a period)
#define COVG_CHUNK(U, NXT)                                                                            \
  {                                                                                              \
    const int ch = ch0 + (U);                                                                    \
    if (ch + 1 < NCH) {                                                                          \
      _Pragma("unroll") for (int kk = 0; kk < KK; ++kk)                                          \
          _Pragma("unroll") for (int p = 0; p < PJ; ++p) wf[((U) + 1) & 1][kk][p] =              \
              wfrag[p][64 * ((ch + 1) * KK + kk)];                                               \
    }                                                                                            \
    __builtin_amdgcn_sched_barrier(0); /* the loads stay ahead of this chunk's products */       \
    const __bf16* lb = stage + ((size_t)((U) & 1) * N + i0w + l32) * SSTR + 8 * hi;              \
    _Pragma("unroll") for (int kk = 0; kk < KK; ++kk) {                                          \
      gbf16x8 lf[PI];                                                                            \
      _Pragma("unroll") for (int c = 0; c < PI; ++c) lf[c] =                                     \
          *reinterpret_cast<const gbf16x8*>(lb + (size_t)c * 32 * SSTR + 16 * kk);               \
      _Pragma("unroll") for (int p = 0; p < PJ; ++p) _Pragma("unroll") for (int c = 0; c < PI; ++c) \
          acc[c][p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lf[c], wf[(U) & 1][kk][p], acc[c][p], 0, 0, 0); \
    }                                                                                            \
    /* chunk ch + 1 to the other buffer (last read before the previous                           \
       barrier), then its register set takes chunk ch + 1 + D */                                 \
    if (ch + 1 < NCH) {                                                                          \
      COVG_STORE(NXT, ((U) + 1) & 1);                                                            \
    }                                                                                            \
    if (ch + 1 + D < NCH) {                                                                      \
      COVG_LOAD(NXT, (ch + 1 + D) * KC);                                                         \
    }                                                                                            \
    __builtin_amdgcn_sched_barrier(0);                                                           \
    __syncthreads();                                                                             \
  }
  static_assert(D == 2, "two chunk instances per period");
  for (int ch0 = 0; ch0 < NCH; ch0 += D) {
    COVG_CHUNK(0, b);
    COVG_CHUNK(1, a);
  }
#undef COVG_CHUNK
#undef COVG_LD1
#undef COVG_ST1
#undef COVG_LOAD
#undef COVG_STORE
  }

  // step-1 epilogue: block (c, p) holds Out[i][j], j = j0w + 32 p + l32 (the
  // lane's neuron), i = i0w + 32 c + 8 q + 4 hi + (0..3) (register quad q);
  // T[j][i] = alpha_i Out[i][j] + gamma_i^2 W[j][i] replaces the staging
  // buffers (every wave passed the loop's last barrier)
#pragma unroll
  for (int p = 0; p < PJ; ++p) {
    const int j = j0w + 32 * p + l32;
    // W[j][i..i+3] from the accumulator-quad copy: one 1 KiB run per wave
    const float4* wq = Wq + ((int64_t)((j0w >> 5) + p) * (N / 32) + (i0w >> 5)) * 4 * 64 + lane;
    float4 pj = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (FIRST) pj = reinterpret_cast<const float4*>(s_vc + RB + 4 * N)[j - R0];
    float v = 0.f, mg = 0.f, y = 0.f;
#pragma unroll
    for (int c = 0; c < PI; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0w + 32 * c + 8 * q + 4 * hi;
        const float4 w4 = wq[(c * 4 + q) * 64];
        const float4 a4 = *reinterpret_cast<const float4*>(s_alpha + i);
        const float4 g4 = *reinterpret_cast<const float4*>(s_g2 + i);
        const float4 z4 = *reinterpret_cast<const float4*>(s_z + i);
        float o0, o1, o2, o3;
        if constexpr (FIRST) {
          // Out[i][j] = F_i . P_j (F in three arrays after the vectors)
          const float* fb = s_vc + RB;
          const float4 fx = *reinterpret_cast<const float4*>(fb + i);
          const float4 fy = *reinterpret_cast<const float4*>(fb + N + i);
          const float4 fz = *reinterpret_cast<const float4*>(fb + 2 * N + i);
          o0 = fmaf(pj.x, fx.x, fmaf(pj.y, fy.x, pj.z * fz.x));
          o1 = fmaf(pj.x, fx.y, fmaf(pj.y, fy.y, pj.z * fz.y));
          o2 = fmaf(pj.x, fx.z, fmaf(pj.y, fy.z, pj.z * fz.z));
          o3 = fmaf(pj.x, fx.w, fmaf(pj.y, fy.w, pj.z * fz.w));
        } else {
          o0 = acc[c][p][4 * q + 0];
          o1 = acc[c][p][4 * q + 1];
          o2 = acc[c][p][4 * q + 2];
          o3 = acc[c][p][4 * q + 3];
        }
        const float t0 = fmaf(a4.x, o0, g4.x * w4.x);
        const float t1 = fmaf(a4.y, o1, g4.y * w4.y);
        const float t2 = fmaf(a4.z, o2, g4.z * w4.z);
        const float t3 = fmaf(a4.w, o3, g4.w * w4.w);
        v = fmaf(w4.x, t0, fmaf(w4.y, t1, fmaf(w4.z, t2, fmaf(w4.w, t3, v))));
        mg = fmaf(fabsf(w4.x), fabsf(t0),
                  fmaf(fabsf(w4.y), fabsf(t1), fmaf(fabsf(w4.z), fabsf(t2), fmaf(fabsf(w4.w), fabsf(t3), mg))));
        y = fmaf(w4.x, z4.x, fmaf(w4.y, z4.y, fmaf(w4.z, z4.z, fmaf(w4.w, z4.w, y))));
        if (!LAST) *reinterpret_cast<uint2*>(Tl + (size_t)(j - R0) * TSTR + i) = pack_bf16x4(t0, t1, t2, t3);
      }
    v += __shfl_xor(v, 32);
    mg += __shfl_xor(mg, 32);
    y += __shfl_xor(y, 32);
    if (hi == 0) {
      pv[wi * RB + (j - R0)] = v;
      pm[wi * RB + (j - R0)] = mg;
      py[wi * RB + (j - R0)] = y;
    }
  }
  __syncthreads();

  // ---- step 2: the rule for the workgroup's neurons
  if (t < RB) {
    const int j = R0 + t;
    float v = 0.f, av = 0.f, y = 0.f;
#pragma unroll
    for (int w = 0; w < WI1; ++w) {
      v += pv[w * RB + t];
      av += pm[w * RB + t];
      y += py[w * RB + t];
    }
    y += bias[j];
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
    s_ac[t] = a;
    s_vc[t] = v;
  }
  if (LAST) return;
  __syncthreads();

  // ---- step 3: C[j][m] = sum_i T[j][i] W[m][i], j in R, m < N
  const int wj3 = wave / WM3, wm = wave % WM3;
  const int jl0 = wj3 * (QJ * 32);  // the wave's first local neuron
  const int m0 = wm * (QM * 32);    // its first column m
  gv16f acc3[QJ][QM];
#pragma unroll
  for (int c = 0; c < QJ; ++c)
#pragma unroll
    for (int q = 0; q < QM; ++q)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc3[c][q][e] = 0.f;
  ggbf16x8* bfr[QM];
#pragma unroll
  for (int q = 0; q < QM; ++q) bfr[q] = (ggbf16x8*)(Wfr + ((int64_t)((m0 >> 5) + q) * KS * 64 + lane) * 8);
  const __bf16* ta = Tl + (size_t)(jl0 + l32) * TSTR + 8 * hi;
  // weight fragments in a ring of PD k-steps, each slot reloaded PD k-steps
  // ahead of its use
  constexpr int PD = QM > 2 ? 2 : 4;
  static_assert(KS % PD == 0, "ring");
  gbf16x8 ring[PD][QM];
#pragma unroll
  for (int d = 0; d < PD; ++d)
#pragma unroll
    for (int q = 0; q < QM; ++q) ring[d][q] = bfr[q][64 * d];
  for (int k0 = 0; k0 < KS; k0 += PD) {
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      const int ks = k0 + d;
      gbf16x8 af[QJ], bq[QM];
#pragma unroll
      for (int c = 0; c < QJ; ++c) af[c] = *reinterpret_cast<const gbf16x8*>(ta + (size_t)c * 32 * TSTR + 16 * ks);
#pragma unroll
      for (int q = 0; q < QM; ++q) bq[q] = ring[d][q];
      if (ks + PD < KS) {
#pragma unroll
        for (int q = 0; q < QM; ++q) ring[d][q] = bfr[q][64 * (ks + PD)];
      }
      // keep the reloads here: the scheduler would otherwise sink them to
      // their use PD k-steps later and expose the L2 latency
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < QM; ++q)
#pragma unroll
        for (int c = 0; c < QJ; ++c) acc3[c][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[c], bq[q], acc3[c][q], 0, 0, 0);
    }
  }

  // step-3 epilogue: block (c, q) holds C[j][m], m = m0 + 32 q + l32, local
  // j = jl0 + 32 c + 8 r + 4 hi + (0..3) (quad r); stored as row m of Chat
  // (C is symmetric), scaled by alpha_j, the diagonal alpha_j v_j.  In the
  // blocked layout a wave's store of (c, q, r) is one 512-byte run.
  __bf16* Co = Cout + cell * NN;
#pragma unroll
  for (int c = 0; c < QJ; ++c)
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      const int m = m0 + 32 * q + l32;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jl = jl0 + 32 * c + 8 * r + 4 * hi;
        const float4 a4 = *reinterpret_cast<const float4*>(s_ac + jl);
        float x0 = a4.x * acc3[c][q][4 * r + 0], x1 = a4.y * acc3[c][q][4 * r + 1];
        float x2 = a4.z * acc3[c][q][4 * r + 2], x3 = a4.w * acc3[c][q][4 * r + 3];
        const int d = m - (R0 + jl);
        if (d >= 0 && d < 4) {
          const float dv = s_ac[jl + d] * s_vc[jl + d];
          x0 = d == 0 ? dv : x0;
          x1 = d == 1 ? dv : x1;
          x2 = d == 2 ? dv : x2;
          x3 = d == 3 ? dv : x3;
        }
        *reinterpret_cast<uint2*>(Co + chat_index<N>(m, R0 + jl)) = pack_bf16x4(x0, x1, x2, x3);
      }
    }
}

// Layer 1 of each cell: the rule per neuron (y = W_1 c + b_1, v = |F_j|^2
// with F = W_1 diag(h / sqrt 3)), the layer's (y, alpha, beta, gamma), and,
// unless layer 2 runs in rank-3 form (Cout null), Chat_1[i][k] =
// alpha_k F_i . F_k (bfloat16).
template <int ACT>
__global__ __launch_bounds__(kGThreads) void covg_layer1_kernel(int64_t C, int N, const float* __restrict__ W1,
                                                                 const float* __restrict__ b1,
                                                                 const float* __restrict__ centres,
                                                                 const float* __restrict__ halves,
                                                                 float* __restrict__ vec, __bf16* __restrict__ Cout,
                                                                 uint32_t* __restrict__ cancel) {
  extern __shared__ float4 covg_l1[];  // [N]: (F_j, alpha_j)
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
    covg_l1[j] = make_float4(f0, f1, f2, a);
    const int64_t o = cell * N + j;
    vec[o] = y;
    vec[NC + o] = a;
    vec[2 * NC + o] = b;
    vec[3 * NC + o] = g;
  }
  if (t == 0 && cancel) cancel[cell] = 0u;
  if (!Cout) return;
  __syncthreads();
  // Chat_1 in the blocked layout: 8 consecutive entries of a row per thread
  // and step (one 16-byte store), lanes over the 32 rows of a block
  const int per_blk = 32 * (N / 8);
  __bf16* Cc = Cout + cell * (int64_t)N * N;
  for (int idx = t; idx < N * (N / 8); idx += kGThreads) {
    const int blk = idx / per_blk, rem = idx - blk * per_blk;
    const int i = 32 * blk + (rem & 31), k0 = 8 * (rem >> 5);
    const float4 fi = covg_l1[i];
    gbf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float4 fk = covg_l1[k0 + e];
      v[e] = (__bf16)(fk.w * (fi.x * fk.x + fi.y * fk.y + fi.z * fk.z));
    }
    *reinterpret_cast<gbf16x8*>(Cc + ((int64_t)blk * (N / 8) + (rem >> 5)) * 256 + (rem & 31) * 8) = v;
  }
}

}  // namespace

int covg_width(const Model& m) {
  if (m.n_linear < 3) return 0;
  const int n = m.pw[1];
  for (int h = 1; h < m.n_linear; ++h)
    if (m.pw[h] != n) return 0;
  for (int l = 1; l + 1 < m.n_linear; ++l)
    if (!m.L[l].Wfr || !m.L[l].Wq) return 0;
  return (n == 256 || n == 512 || n == 1024) ? n : 0;
}

size_t covg_scratch_bytes(const Model& m, int64_t C) {
  const int N = covg_width(m);
  if (!N) return 0;
  // Chat of two consecutive layers (bfloat16)
  return (size_t)C * 2 * N * N * 2;
}

int64_t covg_max_chunk(const Model& m) {
  const int N = covg_width(m);
  if (!N) return 0;
  // (C + 7) N / RB blocks of 512 threads stay below 2^22 blocks
  const int64_t nr = (int64_t)N * N / 65536;
  return (((int64_t)1 << 22) / nr) - 8;
}

double covg_flops_per_cell(const Model& m) {
  const int N = covg_width(m);
  const int Lh = m.n_linear - 1;
  const double n3 = (double)N * N * N, n2 = (double)N * N;
  // the T product of every layer >= 2 (layer 2 at widths <= 512 in rank-3
  // form: 6 N^2 for P and for F_i . P_j), the C product of every layer but
  // the last, the centre (2 N^2 per layer)
  const double t2 = N <= 512 ? 12.0 * n2 : 2.0 * n3;
  return t2 + 2.0 * n3 * (Lh - 2) + 2.0 * n3 * std::max(0, Lh - 2) + 2.0 * n2 * Lh;
}

template <int N, int ACT>
static hipError_t covg_run(const Model& m, int64_t C, const float* centres, const float* halves, float* vec,
                           uint32_t* cancel, void* scratch, hipStream_t s) {
  using S = CovgShape<N>;
  const int64_t NN = (int64_t)N * N;
  const int Lh = m.n_linear - 1;
  if (C > covg_max_chunk(m)) return hipErrorInvalidValue;
  __bf16* Cb[2] = {reinterpret_cast<__bf16*>(scratch), reinterpret_cast<__bf16*>(scratch) + C * NN};
  constexpr bool R3 = S::RANK3;
  {
    hipError_t e = ensure_lds_limit(reinterpret_cast<const void*>(&covg_layer_kernel<N, ACT, false, false>), (int)S::LDS);
    if (e == hipSuccess)
      e = ensure_lds_limit(reinterpret_cast<const void*>(&covg_layer_kernel<N, ACT, true, false>), (int)S::LDS);
    if (R3 && e == hipSuccess)
      e = ensure_lds_limit(reinterpret_cast<const void*>(&covg_layer_kernel<N, ACT, false, R3>), (int)S::LDS_FIRST);
    if (R3 && e == hipSuccess)
      e = ensure_lds_limit(reinterpret_cast<const void*>(&covg_layer_kernel<N, ACT, true, R3>), (int)S::LDS_FIRST);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((covg_layer1_kernel<ACT>), dim3((unsigned)C), dim3(kGThreads), (size_t)N * sizeof(float4), s, C,
                     N, m.L[0].W, m.L[0].b, centres, halves, vec, R3 ? (__bf16*)nullptr : Cb[0], cancel);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)(((C + 7) / 8) * 8 * S::NR));
  const int64_t layer = 4 * (int64_t)N * C;  // floats of one layer's vectors
  for (int h = 2; h <= Lh; ++h) {
    const Layer& L = m.L[h - 1];
    const __bf16* Wfr = reinterpret_cast<const __bf16*>(L.Wfr);
    const float4* Wq = reinterpret_cast<const float4*>(L.Wq);
    const __bf16* cin = Cb[(h - 2) & 1];
    __bf16* cout = Cb[(h - 1) & 1];
    const float* vprev = vec + (h - 2) * layer;
    float* vcur = vec + (h - 1) * layer;
    const bool last = h == Lh, first = R3 && h == 2;
#define COVG_LAUNCH(LASTV, FIRSTV)                                                                             \
  hipLaunchKernelGGL((covg_layer_kernel<N, ACT, LASTV, FIRSTV>), grid, dim3(kGThreads),                        \
                     (FIRSTV) ? S::LDS_FIRST : S::LDS, s, C, cin, cout, Wfr, Wq, m.L[0].W, halves, L.b, vprev,      \
                     vcur, cancel)
    if (first) {
      if (last)
        COVG_LAUNCH(true, R3);
      else
        COVG_LAUNCH(false, R3);
    } else {
      if (last)
        COVG_LAUNCH(true, false);
      else
        COVG_LAUNCH(false, false);
    }
#undef COVG_LAUNCH
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int N>
static hipError_t covg_run_n(const Model& m, int64_t C, const float* centres, const float* halves, float* vec,
                             uint32_t* cancel, void* scratch, hipStream_t s) {
  switch (m.act) {
    case ISX_SINE: return covg_run<N, ISX_SINE>(m, C, centres, halves, vec, cancel, scratch, s);
    case ISX_ELU: return covg_run<N, ISX_ELU>(m, C, centres, halves, vec, cancel, scratch, s);
    default: return covg_run<N, ISX_RELU>(m, C, centres, halves, vec, cancel, scratch, s);
  }
}

hipError_t launch_up_cov_global(const Model& m, int64_t C, const float* centres, const float* halves, float* vec,
                                uint32_t* cancel, void* scratch, hipStream_t s) {
  if (C <= 0) return hipSuccess;
  if (!scratch) return hipErrorInvalidValue;
  switch (covg_width(m)) {
    case 256: return covg_run_n<256>(m, C, centres, halves, vec, cancel, scratch, s);
    case 512: return covg_run_n<512>(m, C, centres, halves, vec, cancel, scratch, s);
    case 1024: return covg_run_n<1024>(m, C, centres, halves, vec, cancel, scratch, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace isx
