// Uncertainty propagation in covariance form on BF16 MFMA
// (v_mfma_f32_32x32x16_bf16, float32 accumulation).
//
// The Gaussian rule of a hidden layer only needs each neuron's variance, the
// diagonal of C_h = P_h P_h^T, where P_h is the layer's coefficient matrix
// (Eq. 8).  Since P_h = W_h [D_{h-1} P_{h-1} | diag(gamma_{h-1})] (Eq. 9, the
// rule scales the rows of the previous form and appends one new symbol per
// neuron), the covariances follow exactly from
//   C_1 = W_1 diag(h^2 / 3) W_1^T,
//   C_h = W_h X_{h-1} W_h^T,  X_{h-1} = D_{h-1} C_{h-1} D_{h-1} + diag(gamma_{h-1}^2),
// with D = diag(alpha): the same result as tracking the coefficients, without
// the growing symbol blocks.  For hidden widths up to 256 a cell's X fits in
// one CU's LDS as bfloat16, so one workgroup carries a cell through every
// hidden layer without touching HBM between layers; the only global traffic
// is the weights (L2-resident) and each layer's (y, alpha, beta, gamma)
// vectors for the output read-off.  Affine arithmetic has no such form (its
// statistic is a sum of magnitudes) and keeps the coefficient kernel.
//
// Layer 1: X_1 = G G^T + diag(gamma_1^2) with G = D_1 W_1 diag(h / sqrt 3)
// (N x 3) has rank 3, so with P = W_2 G (N x 3),
//   C_2 = W_2 X_1 W_2^T = P P^T + T' W_2^T,  T' = W_2 diag(gamma_1^2):
// layer 2 writes T' element by element in its per-neuron pass (which also
// gives P and the variances |P_j|^2 + sum_k W_2[j][k]^2 gamma_1k^2) and makes
// one product, whose accumulators start from P_i . P_j.
// Per layer h >= 3 (8 waves, 512 threads):
//   2. T = W_h X_{h-1}, computed as T^T = X W_h^T: each wave computes a tile
//      of RPW x CPW blocks of 32 x 32, with A = rows of X from LDS and B =
//      bfloat16 fragments of its weight rows streamed from the L2-resident
//      fragment-order copy of W a few k-steps ahead (a wave's fragment load
//      is one 1 KiB run).  A weight fragment serves CPW products and an LDS
//      fragment RPW.
//   3. From the float32 accumulators (a lane's register quad holds four
//      consecutive entries of one row j of T): T replaces X in LDS
//      (row-major), and each lane sums its columns' share of the variance
//      C_h[j][j] = sum_i T[j][i] W[j][i] and of the centre W[j] z, with z =
//      alpha . y_{h-1} + beta, from a float32 copy of W in the accumulators'
//      order (one 1 KiB run per wave and register quad).
//   4. Per neuron, the column groups' partial sums, y = W z + b, and the
//      activation's rule (ReLU, sine or ELU), which gives (alpha, beta, gamma).
//   5. C_h = T W_h^T on the wave's tile (A = rows of T from LDS, B = weight
//      fragments, whose lane layout is the B layout of the transposed
//      product).  The last hidden layer stops after step 4 (and keeps no T).
//   6. X_h = D C_h D + diag(gamma^2) goes to LDS as bfloat16 for layer h+1
//      (C_h is symmetric, so the tile's columns are written as rows).
// Cancellation check: the variance sums of step 3 are signed (X carries
// bfloat16 rounding of about 2^-8 per entry, so a sum that keeps only a
// small part of its terms' magnitude can lose every digit or turn negative).
// Step 3 also sums |T[j][i] W[j][i]|; a neuron whose variance is not above
// kCancelRatio times that magnitude, and whose pre-activation lies within 6
// of its largest plausible sigma (so that its rule depends on sigma), marks
// its cell, and the host re-propagates marked cells in float64.  Layers 1
// and 2 sum squares and cannot cancel.
// MFMA 32x32x16 bf16 layout (lane l): A (row l%32, k 8(l/32)+e), B (k
// 8(l/32)+e, column l%32), e = 0..7; accumulator register r holds (row
// 8(r/4) + 4(l/32) + r%4, column l%32).
#include "isx_internal.h"
#include "rules.h"

#include <algorithm>

namespace isx {

typedef __bf16 cbf16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(1))) const cbf16x8 gbf16x8;  // in global memory
typedef __attribute__((address_space(1))) const float gfloat;
typedef float cv4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const cv4f gfloat4;
typedef float cv16f __attribute__((ext_vector_type(16)));

constexpr int kCovThreads = 512;  // 8 waves

// A variance sum is flagged when it keeps at most this fraction of the
// summed magnitude of its terms (the exact sums of the 3->256x5->1 benchmark
// INR keep at least 5e-3 over cells of levels 2-9, so ordinary cells are not
// flagged; at 2^-9 the bfloat16 operand rounding alone, 2^-8 per term, can
// exceed the result).
constexpr float kCancelRatio = 0x1p-9f;

template <int N>
struct CovShape {
  static constexpr int STR = N + 8;  // LDS row stride in bfloat16 (16-byte shifted rows)
  static constexpr int KS = N / 16;  // k-steps of one product
  static constexpr int NB = N / 32;  // 32-row (and 32-column) blocks
  // Each wave computes RPW x CPW blocks of 32 x 32: RPW blocks whose operand
  // is weight rows (global memory) and CPW blocks whose operand comes from
  // LDS; a weight fragment serves CPW products and an LDS fragment RPW.
  static constexpr int RPW = NB >= 5 ? 2 : 1;
  static constexpr int CPW = NB <= 2 ? 1 : (NB <= 4 ? 2 : (NB <= 6 ? 3 : 4));
  static constexpr int RG = (NB + RPW - 1) / RPW;  // wave groups along the weight rows
  static constexpr int CG = (NB + CPW - 1) / CPW;  // wave groups along the LDS operand
  static constexpr int PF = 4;                     // weight fragments loaded this many k-steps ahead
  static constexpr size_t LDS = (size_t)N * STR * 2 + 14 * N * sizeof(float);
  static_assert(RG * CG <= 8, "more tiles than waves");
};

// acc[r][c] += W[wrow[r] rows] * L[lrow[c] rows]^T over all N k values, as
// MFMA products D[i][j] = sum_k A[i][k] B[k][j]: with WA the weight rows are
// the A operand (rows of D) and the LDS rows the B operand (columns of D);
// otherwise the roles swap.  wfrag[r] points at this lane's A fragment of
// k-step 0 of weight block r in the fragment-order copy (the next k-step's
// fragment lies 64 fragments on), lfrag[c] at its 8-element chunk of LDS row
// lrow[c].
template <int N, bool WA>
__device__ __forceinline__ void cov_tile_gemm(gbf16x8* const (&wfrag)[CovShape<N>::RPW],
                                              const __bf16* const (&lfrag)[CovShape<N>::CPW], bool tile_ok,
                                              cv16f (&acc)[CovShape<N>::RPW][CovShape<N>::CPW]) {
  using S = CovShape<N>;
  constexpr int KS = S::KS, RPW = S::RPW, CPW = S::CPW, PF = S::PF < S::KS ? S::PF : S::KS;
  // fragments are loaded unconditionally (invalid blocks point at block 0)
  cbf16x8 wf[KS][RPW];
#pragma unroll
  for (int ks = 0; ks < PF; ++ks)
#pragma unroll
    for (int r = 0; r < RPW; ++r) wf[ks][r] = wfrag[r][64 * ks];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    if (ks + PF < KS) {
#pragma unroll
      for (int r = 0; r < RPW; ++r) wf[ks + PF][r] = wfrag[r][64 * (ks + PF)];
    }
    cbf16x8 lf[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) lf[c] = *reinterpret_cast<const cbf16x8*>(lfrag[c] + 16 * ks);
    // keep the loads above the products: without this the scheduler sinks
    // the weight loads next to their use and every step waits on L2
    __builtin_amdgcn_sched_barrier(0);
    if (tile_ok) {
#pragma unroll
      for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int c = 0; c < CPW; ++c)
          acc[r][c] = WA ? __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[ks][r], lf[c], acc[r][c], 0, 0, 0)
                         : __builtin_amdgcn_mfma_f32_32x32x16_bf16(lf[c], wf[ks][r], acc[r][c], 0, 0, 0);
    }
  }
}

// Y, A, B, G of one hidden layer (n neurons) inside the vector buffer, which
// holds them for layers 1..L-1 in order, each [C][n]
__device__ __forceinline__ void cov_store_vec(float* v, int64_t C, int n, int64_t cell, int j, float y, float a,
                                              float b, float g) {
  const int64_t NC = (int64_t)n * C;
  const int64_t o = cell * n + j;
  v[o] = y;
  v[NC + o] = a;
  v[2 * NC + o] = b;
  v[3 * NC + o] = g;
}


// Sum over the 4 lanes of a quad (all four active), via DPP quad permutes.
__device__ __forceinline__ float quad_sum(float x) {
  x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));  // lane ^ 1
  x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x4E, 0xF, 0xF, false));  // lane ^ 2
  return x;
}

// All hidden layers have padded width N (the input layer is 3 wide).  The
// activation is a compile-time constant: its rule is inlined, and ReLU keeps
// the register budget of a kernel without the float64 sine and ELU rules.
template <int N, int ACT>
__global__ __launch_bounds__(kCovThreads) void up_cov_bf16_kernel(int64_t C, int n_linear,
                                                                  const DevLayer* __restrict__ layers,
                                                                  float* __restrict__ vec,
                                                                  const float* __restrict__ centres,
                                                                  const float* __restrict__ halves,
                                                                  uint32_t* __restrict__ cancel) {
  constexpr int act = ACT;
  using S = CovShape<N>;
  constexpr int STR = S::STR, KS = S::KS, NB = S::NB;
  extern __shared__ float4 cov_smem4[];
  __shared__ uint32_t s_cancel;
  __bf16* X = reinterpret_cast<__bf16*>(cov_smem4);  // [N][STR]: X, then T
  float* s_alpha = reinterpret_cast<float*>(X + (size_t)N * STR);
  float* s_zbuf = s_alpha + N;  // two buffers of z = alpha . y + beta (previous layer, this layer)
  float* s_gamma = s_zbuf + 2 * N;
  float* s_var = s_gamma + N;
  float4* s_G = reinterpret_cast<float4*>(s_var + N);  // layer 1: (G_j, gamma_1j^2), G = D_1 W_1 diag(h / sqrt 3)
  float4* s_P = s_G + N;                               // layer 2: (P_j, 0), P = W_2 G

  const int64_t cell = blockIdx.x;
  if (cell >= C) return;
  // the wave index is uniform across a wave: kept in a scalar register,
  // everything derived from it (tile, row groups) is too
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int l32 = lane & 31, hi = lane >> 5;
  constexpr int RPW = S::RPW, CPW = S::CPW, RG = S::RG, CG = S::CG;
  static_assert(CG <= 2, "the column groups' partial sums (float4 [CG][N]) reuse the G and P area");
  if (t == 0) s_cancel = 0u;
  // row passes: 16-row groups, a quad of lanes per row (lane q of row rq)
  constexpr int NG = N / 16, GPW = (NG + 7) / 8;
  static_assert(GPW <= 4, "one rule lane per group");
  const int q = lane & 3, rq = lane >> 2;
  // this wave's tile: weight-row blocks rg*RPW.., LDS-row blocks cg*CPW..
  const int rg = wave % RG, cg = wave / RG;
  const bool tile = cg < CG;
  const int Lh = n_linear - 1;
  float* vh = vec;  // this hidden layer's Y, A, B, G

  // ---- layer 1: centre, variances, rule, G
  {
    const DevLayer L1 = layers[0];
    gfloat* W1 = (gfloat*)L1.W;
    gfloat* b1 = (gfloat*)L1.b;
    const float sc = 0.57735026918962576451f;
    const float hx = halves[cell * 3 + 0] * sc, hy = halves[cell * 3 + 1] * sc, hz = halves[cell * 3 + 2] * sc;
    float* s_z = s_zbuf + N;  // read by layer 2
    for (int j = t; j < N; j += kCovThreads) {
      const float w0 = W1[j * 3 + 0], w1 = W1[j * 3 + 1], w2 = W1[j * 3 + 2];
      const float y = b1[j] + w0 * centres[cell * 3 + 0] + w1 * centres[cell * 3 + 1] + w2 * centres[cell * 3 + 2];
      const float f0 = w0 * hx, f1 = w1 * hy, f2 = w2 * hz;
      float a, b, g;
      apply_rule<float, ISX_UP>(act, y, f0 * f0 + f1 * f1 + f2 * f2, a, b, g);
      s_alpha[j] = a;
      s_z[j] = a * y + b;
      s_gamma[j] = g;
      s_G[j] = make_float4(a * f0, a * f1, a * f2, g * g);
      cov_store_vec(vh, C, N, cell, j, y, a, b, g);
    }
    __syncthreads();
    vh += 4 * (int64_t)N * C;
  }

  for (int h = 2; h <= Lh; ++h) {
    const DevLayer Lw = layers[h - 1];
    const bool last = h == Lh;
    const __bf16* Wb = reinterpret_cast<const __bf16*>(Lw.Wfr);
    gbf16x8* wfrag[RPW];
    bool wok[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int blk = rg * RPW + r;
      wok[r] = tile && blk < NB;
      wfrag[r] = (gbf16x8*)(Wb + ((int64_t)(wok[r] ? blk : 0) * KS * 64 + lane) * 8);
    }
    const __bf16* lfrag[CPW];
    bool lok[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int blk = cg * CPW + c;
      lok[c] = tile && blk < NB;
      lfrag[c] = X + (size_t)((lok[c] ? blk : 0) * 32 + l32) * STR + 8 * hi;
    }

    const float* s_zin = s_zbuf + (h - 1 & 1) * N;  // z of layer h-1
    float* s_zout = s_zbuf + (h & 1) * N;           // z of layer h
    if (h == 2) {
      // 3./4. per neuron j (a lane quad), one pass over the row-pass copy of
      //    its weight row, both row groups of the wave together (G and z
      //    are read once for both): y_j = W[j] z + b_j, P_j = W[j] G, the
      //    variance |P_j|^2 + sum_k W[j][k]^2 gamma_1k^2 and the rule,
      //    and row j of T' = W diag(gamma_1^2) into LDS
      {
        float r5[GPW][5];
        gfloat* wv[GPW];
        bool gok[GPW];
#pragma unroll
        for (int gi = 0; gi < GPW; ++gi) {
#pragma unroll
          for (int u = 0; u < 5; ++u) r5[gi][u] = 0.f;
          gok[gi] = wave + 8 * gi < NG;  // wave-uniform
          const int j = 16 * (gok[gi] ? wave + 8 * gi : 0) + rq;
          wv[gi] = (gfloat*)Lw.Wv + (int64_t)j * N + 8 * q;
        }
#pragma unroll 2
        for (int m = 0; m < N / 32; ++m) {
          const int k = 8 * cov_row_chunk(N, q, m);
          cv4f w0[GPW], w1[GPW];
#pragma unroll
          for (int gi = 0; gi < GPW; ++gi) {
            w0[gi] = *reinterpret_cast<gfloat4*>(wv[gi] + 32 * m);
            w1[gi] = *reinterpret_cast<gfloat4*>(wv[gi] + 32 * m + 4);
          }
          const float4 z0 = *reinterpret_cast<const float4*>(s_zin + k);
          const float4 z1 = *reinterpret_cast<const float4*>(s_zin + k + 4);
          float4 g4[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) g4[u] = s_G[k + u];
#pragma unroll
          for (int gi = 0; gi < GPW; ++gi) {
            if (!gok[gi]) continue;
            const float wk[8] = {w0[gi].x, w0[gi].y, w0[gi].z, w0[gi].w, w1[gi].x, w1[gi].y, w1[gi].z, w1[gi].w};
            r5[gi][0] += wk[0] * z0.x + wk[1] * z0.y + wk[2] * z0.z + wk[3] * z0.w + wk[4] * z1.x + wk[5] * z1.y +
                         wk[6] * z1.z + wk[7] * z1.w;
            cbf16x8 t8;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              r5[gi][1] += wk[u] * g4[u].x;
              r5[gi][2] += wk[u] * g4[u].y;
              r5[gi][3] += wk[u] * g4[u].z;
              const float wg = wk[u] * g4[u].w;
              r5[gi][4] += wk[u] * wg;
              t8[u] = (__bf16)wg;
            }
            *reinterpret_cast<cbf16x8*>(X + (size_t)(16 * (wave + 8 * gi) + rq) * STR + k) = t8;
          }
        }
#pragma unroll
        for (int gi = 0; gi < GPW; ++gi)
#pragma unroll
          for (int u = 0; u < 5; ++u) r5[gi][u] = quad_sum(r5[gi][u]);
        // lane q of the quad applies the rule to the row of group q
        int j = -1;
        float sel[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int gi = 0; gi < GPW; ++gi)
          if (q == gi && gok[gi]) {
            j = 16 * (wave + 8 * gi) + rq;
#pragma unroll
            for (int u = 0; u < 5; ++u) sel[u] = r5[gi][u];
          }
        if (j >= 0) {
          float a, b, g;
          const float y = sel[0] + ((gfloat*)Lw.b)[j];
          const float v = sel[1] * sel[1] + sel[2] * sel[2] + sel[3] * sel[3] + sel[4];
          apply_rule<float, ISX_UP>(act, y, v, a, b, g);
          s_var[j] = v;
          s_alpha[j] = a;
          s_zout[j] = a * y + b;
          s_gamma[j] = g;
          s_P[j] = make_float4(sel[1], sel[2], sel[3], 0.f);
          cov_store_vec(vh, C, N, cell, j, y, a, b, g);
        }
      }
      if (last) break;
      __syncthreads();
    } else {
      // 2. T^T = X W^T on the wave's tile (X symmetric)
      cv16f acc[RPW][CPW];
#pragma unroll
      for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int c = 0; c < CPW; ++c)
#pragma unroll
          for (int e = 0; e < 16; ++e) acc[r][c][e] = 0.f;
      cov_tile_gemm<N, false>(wfrag, lfrag, tile, acc);
      // 3. from the float32 accumulators: T -> LDS row-major (not needed
      //    after the last hidden layer), and per weight row j the partial
      //    sums of the variance C_h[j][j] = sum_i T[j][i] W[j][i] and of the
      //    centre W[j] z over the tile's columns i, with the float32 weights
      //    in accumulator order (one 1 KiB run per wave and register quad).
      //    A lane's register quad holds four consecutive entries of row j;
      //    the other half of the wave holds the next four.  The column
      //    groups' partial sums meet in LDS that is free from layer 3 on
      //    (G, P).  Blocks go in the order bi = r CPW + c; their weights
      //    are loaded two blocks ahead, the first two before the barrier
      //    (blocks outside the matrix read block 0 and are not used).
      gfloat4* wq = (gfloat4*)Lw.Wq;
      constexpr int NBL = RPW * CPW;
      auto wq_at = [&](int bi, int q4) -> cv4f {
        const int r = bi / CPW, c = bi % CPW;
        const int rb = wok[r] ? rg * RPW + r : 0, cb = lok[c] ? cg * CPW + c : 0;
        return wq[((int64_t)(rb * NB + cb) * 4 + q4) * 64 + lane];
      };
      cv4f wb[3][4];
#pragma unroll
      for (int bi = 0; bi < 2 && bi < NBL; ++bi)
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) wb[bi][q4] = wq_at(bi, q4);
      __syncthreads();  // every wave has read X
      {
        float4* s_part = s_G;  // [CG][N]: (variance, centre, |terms|, -)
        float pv[RPW], py[RPW], pa[RPW];
#pragma unroll
        for (int r = 0; r < RPW; ++r) pv[r] = py[r] = pa[r] = 0.f;
#pragma unroll
        for (int bi = 0; bi < NBL; ++bi) {
          const int r = bi / CPW, c = bi % CPW;
          if (bi + 2 < NBL) {
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) wb[(bi + 2) % 3][q4] = wq_at(bi + 2, q4);
          }
          // keeps later blocks' loads from being hoisted here (registers)
          __asm__ volatile("" ::: "memory");
          if (wok[r] && lok[c]) {
            const int j = (rg * RPW + r) * 32 + l32;
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
              const int i0 = (cg * CPW + c) * 32 + 8 * q4 + 4 * hi;
              const cv4f w4 = wb[bi % 3][q4];
              const float4 z4 = *reinterpret_cast<const float4*>(s_zin + i0);
              const float t0 = acc[r][c][4 * q4 + 0], t1 = acc[r][c][4 * q4 + 1];
              const float t2 = acc[r][c][4 * q4 + 2], t3 = acc[r][c][4 * q4 + 3];
              pv[r] = fmaf(w4.x, t0, fmaf(w4.y, t1, fmaf(w4.z, t2, fmaf(w4.w, t3, pv[r]))));
              pa[r] = fmaf(fabsf(w4.x), fabsf(t0),
                           fmaf(fabsf(w4.y), fabsf(t1), fmaf(fabsf(w4.z), fabsf(t2), fmaf(fabsf(w4.w), fabsf(t3), pa[r]))));
              py[r] = fmaf(w4.x, z4.x, fmaf(w4.y, z4.y, fmaf(w4.z, z4.z, fmaf(w4.w, z4.w, py[r]))));
              if (!last) {
                __bf16 v4[4] = {(__bf16)t0, (__bf16)t1, (__bf16)t2, (__bf16)t3};
                *reinterpret_cast<uint2*>(X + (size_t)j * STR + i0) = *reinterpret_cast<const uint2*>(v4);
              }
            }
          }
        }
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          const float v = pv[r] + __shfl_xor(pv[r], 32);
          const float y = py[r] + __shfl_xor(py[r], 32);
          const float av = pa[r] + __shfl_xor(pa[r], 32);
          if (wok[r] && hi == 0) s_part[cg * N + (rg * RPW + r) * 32 + l32] = make_float4(v, y, av, 0.f);
        }
      }
      __syncthreads();
      // 4. per neuron: the column groups' sums in a fixed order, the centre
      //    y = W z + b with z = alpha . y_{h-1} + beta, and the rule
      {
        const float4* s_part = s_G;
        for (int j = t; j < N; j += kCovThreads) {
          float v = 0.f, yc = 0.f, av = 0.f;
#pragma unroll
          for (int g = 0; g < CG; ++g) {
            const float4 p = s_part[g * N + j];
            v += p.x;
            yc += p.y;
            av += p.z;
          }
          float a, b, g;
          const float y = yc + ((gfloat*)Lw.b)[j];
          // a cancelled sum matters only where the rule depends on sigma:
          // for ReLU, beyond 6 sigma (taken at its largest with the terms'
          // rounding, sqrt(v + 2^-7 sum |terms|)) alpha is 0 or 1 and beta,
          // gamma vanish to float32 accuracy whatever sigma is; for ELU that
          // holds 6 sigma above 0 only.  The sine rule depends on the
          // variance smoothly (alpha = cos(y) e^{-v/2}, |d beta / dv| <=
          // (1 + |y|) / 2, gamma^2 of order v^2), so a variance error of at
          // most 2^-8 sum |terms| moves the centre by at most
          // (1 + 2|y|) 2^-9 sum |terms|: flagged only above 2^-20, below
          // which it stays under the float32 rounding of the centre's sums
          if (av > 0.f && !(v > kCancelRatio * av)) {
            const float s6 = 6.f * sqrtf(fmaxf(v, 0.f) + 0x1p-7f * av);
            const bool dep = act == ISX_SINE ? (1.f + 2.f * fabsf(y)) * 0x1p-9f * av > 0x1p-20f
                                             : (act == ISX_ELU ? y < s6 : fabsf(y) < s6);
            if (dep) s_cancel = 1u;
          }
          apply_rule<float, ISX_UP>(act, y, v, a, b, g);
          s_var[j] = v;
          s_alpha[j] = a;
          s_zout[j] = a * y + b;
          s_gamma[j] = g;
          cov_store_vec(vh, C, N, cell, j, y, a, b, g);
        }
      }
      if (last) break;
    }
    vh += 4 * (int64_t)N * C;
    // 5. C_h on the wave's tile, C[i][j] = sum_k T[i][k] W[j][k] (rows i:
    //    T blocks from LDS, columns j: weight blocks)
    //    (at layer 2 the accumulators start from the rank-3 part P_i . P_j:
    //    two float32 products with k = 2, over P's components (0, 1) and
    //    (2, 3), the fourth being zero)
    cv16f cacc[RPW][CPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
      for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int e = 0; e < 16; ++e) cacc[r][c][e] = 0.f;
    if (h == 2) {
      float pa[CPW][2], pb[RPW][2];
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const float4 p = s_P[(lok[c] ? cg * CPW + c : 0) * 32 + l32];
        pa[c][0] = hi ? p.y : p.x;
        pa[c][1] = hi ? p.w : p.z;
      }
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const float4 p = s_P[(wok[r] ? rg * RPW + r : 0) * 32 + l32];
        pb[r][0] = hi ? p.y : p.x;
        pb[r][1] = hi ? p.w : p.z;
      }
      if (tile) {
#pragma unroll
        for (int r = 0; r < RPW; ++r)
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            cacc[r][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(pa[c][0], pb[r][0], cacc[r][c], 0, 0, 0);
            cacc[r][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(pa[c][1], pb[r][1], cacc[r][c], 0, 0, 0);
          }
      }
    }
    cov_tile_gemm<N, false>(wfrag, lfrag, tile, cacc);
    __syncthreads();  // every wave has read T; the new slopes are in LDS
    // 6. X_h = D C D + diag(gamma^2); C is symmetric, so the tile's columns j
    //    are written as rows of X.  The lane that wrote a diagonal entry
    //    rewrites it from the variance the rule used.
    //    Column blocks outermost: a block's 16 column slopes are read once
    //    for the RPW row blocks.
    float aj[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) aj[r] = s_alpha[(wok[r] ? rg * RPW + r : 0) * 32 + l32];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      if (!lok[c]) continue;
      // (kept next to their use: hoisting every block's slopes would cost
      // registers)
      __asm__ volatile("" ::: "memory");
      float4 ab[4];
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4)
        ab[q4] = *reinterpret_cast<const float4*>(s_alpha + (cg * CPW + c) * 32 + 8 * q4 + 4 * hi);
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        if (!wok[r]) continue;
        const int j = (rg * RPW + r) * 32 + l32;
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int i0 = (cg * CPW + c) * 32 + 8 * q4 + 4 * hi;
          const float4 ai = ab[q4];
          __bf16 v4[4];
          v4[0] = (__bf16)(ai.x * aj[r] * cacc[r][c][4 * q4 + 0]);
          v4[1] = (__bf16)(ai.y * aj[r] * cacc[r][c][4 * q4 + 1]);
          v4[2] = (__bf16)(ai.z * aj[r] * cacc[r][c][4 * q4 + 2]);
          v4[3] = (__bf16)(ai.w * aj[r] * cacc[r][c][4 * q4 + 3]);
          *reinterpret_cast<uint2*>(X + (size_t)j * STR + i0) = *reinterpret_cast<const uint2*>(v4);
        }
        if (cg * CPW + c == rg * RPW + r && ((l32 >> 2) & 1) == hi)
          X[(size_t)j * STR + j] = (__bf16)(aj[r] * aj[r] * s_var[j] + s_gamma[j] * s_gamma[j]);
      }
    }
    __syncthreads();
  }
  __syncthreads();  // every rule has been applied
  if (t == 0 && cancel) cancel[cell] = s_cancel;
}

// Padded width shared by every hidden layer, or 0 if they differ or exceed
// the LDS tile.
static int cov_width(const Model& m) {
  if (m.n_linear < 2) return 0;
  const int n = m.pw[1];
  for (int h = 1; h < m.n_linear; ++h)
    if (m.pw[h] != n) return 0;
  return (n % 32 == 0 && n <= kCovNMax) ? n : 0;
}

bool cov_supported(const Model& m) { return cov_width(m) != 0; }

template <int N, int ACT>
static hipError_t launch_cov_na(const Model& m, int64_t C, const float* centres, const float* halves, float* vec,
                               uint32_t* cancel, hipStream_t s) {
  {
    hipError_t e = ensure_lds_limit(reinterpret_cast<const void*>(&up_cov_bf16_kernel<N, ACT>), (int)CovShape<N>::LDS);
    if (e != hipSuccess) return e;
  }
  // one workgroup per cell: a launch's work-items must stay below 2^32
  if (C > (int64_t(1) << 22)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((up_cov_bf16_kernel<N, ACT>), dim3((unsigned)C), dim3(kCovThreads), CovShape<N>::LDS, s, C,
                     m.n_linear, m.dev_layers, vec, centres, halves, cancel);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_cov_n(const Model& m, int64_t C, const float* centres, const float* halves, float* vec,
                               uint32_t* cancel, hipStream_t s) {
  switch (m.act) {
    case ISX_SINE: return launch_cov_na<N, ISX_SINE>(m, C, centres, halves, vec, cancel, s);
    case ISX_ELU: return launch_cov_na<N, ISX_ELU>(m, C, centres, halves, vec, cancel, s);
    default: return launch_cov_na<N, ISX_RELU>(m, C, centres, halves, vec, cancel, s);
  }
}

hipError_t launch_up_cov_bf16(const Model& m, int64_t C, const float* centres, const float* halves, float* vec,
                              uint32_t* cancel, hipStream_t s) {
  if (C <= 0) return hipSuccess;
  switch (cov_width(m)) {
    case 32: return launch_cov_n<32>(m, C, centres, halves, vec, cancel, s);
    case 64: return launch_cov_n<64>(m, C, centres, halves, vec, cancel, s);
    case 96: return launch_cov_n<96>(m, C, centres, halves, vec, cancel, s);
    case 128: return launch_cov_n<128>(m, C, centres, halves, vec, cancel, s);
    case 160: return launch_cov_n<160>(m, C, centres, halves, vec, cancel, s);
    case 192: return launch_cov_n<192>(m, C, centres, halves, vec, cancel, s);
    case 224: return launch_cov_n<224>(m, C, centres, halves, vec, cancel, s);
    case 256: return launch_cov_n<256>(m, C, centres, halves, vec, cancel, s);
    default: return hipErrorNotSupported;
  }
}

// Algorithmic flops per cell of the covariance form (true widths): layer 2
// builds T from the rank-3 factor (P = W G, T = P G^T + W diag(gamma^2) and
// the variances: 14 n_2 n_1) and multiplies C = T W^T (2 n_2^2 n_1); every
// later layer h multiplies T = W X (2 n_h n_{h-1}^2) and C = T W^T
// (2 n_h^2 n_{h-1}); the last hidden layer needs only the diagonal of C
// (2 n_h n_{h-1}).
double cov_flops_per_cell(const Model& m) {
  double f = 0.0;
  const int Lh = m.n_linear - 1;
  for (int h = 2; h <= Lh; ++h) {
    const double a = m.widths[h], b = m.widths[h - 1];
    f += h == 2 ? 14.0 * a * b : 2.0 * a * b * b;
    f += h < Lh ? 2.0 * a * a * b : (h == 2 ? 0.0 : 2.0 * a * b);
  }
  return f;
}

}  // namespace isx
