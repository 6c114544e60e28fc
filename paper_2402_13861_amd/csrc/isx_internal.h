// Internal declarations of libisx (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "isx.h"

namespace isx {

// Raise a kernel's dynamic LDS limit to `bytes` on the current device, once
// per (device, kernel, size).  Safe when several host threads launch at once
// (batched extraction drives one context per thread).
inline hipError_t ensure_lds_limit(const void* fn, int bytes) {
  static std::mutex mu;
  static std::vector<std::tuple<int, const void*, int>> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> g(mu);
  for (const auto& t : done)
    if (std::get<0>(t) == dev && std::get<1>(t) == fn && std::get<2>(t) >= bytes) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) done.emplace_back(dev, fn, bytes);
  return e;
}

// Column layout of a cell's coefficient block at hidden layer h (1-based):
// column 0 holds the centre, columns 1..3 the coefficients of the three input
// symbols, columns 4..15 are zero, then one block of n_{i} columns for the
// symbols introduced by the ReLUs of hidden layers i = 1..h-1.  Inside a
// cell, a column's n_h coefficients are contiguous (column-major block).
constexpr int kHeadCols = 16;

// A loaded MLP.  Hidden widths are zero-padded to a multiple of 32: a padded
// neuron has zero weights and bias, its pre-activation form is identically 0,
// and the zero columns of the next layer's weights remove it from every
// later value, so all results are unchanged.
struct Layer {
  int n_in = 0, n_out = 0;  // padded widths
  float* W = nullptr;       // [n_out][n_in] row-major
  float* Wt = nullptr;      // [n_in][n_out]
  float* b = nullptr;       // [n_out]
  double* Wd = nullptr;
  double* Wtd = nullptr;
  double* bd = nullptr;
  uint16_t* Wtbf = nullptr; // bfloat16 bits of W^T, [n_in][n_out]
  uint16_t* Wbf = nullptr;  // bfloat16 bits of W, [n_out][n_in]
  // square hidden layers only (Wfr and Wq at every width, the others at
  // widths <= kCovNMax; else null):
  uint16_t* Wfr = nullptr;  // bfloat16 bits of W in MFMA fragment order (cov_frag_index)
  uint16_t* Wfrl = nullptr; // bfloat16 bits of W - bf16(W), same order
  float* Wv = nullptr;      // W with each row's chunks in row-pass order (cov_row_pos)
  float* Wq = nullptr;      // W in accumulator-quad order (cov_quad_pos)
  uint16_t* WTfr = nullptr;  // bfloat16 bits of W^T in fragment order (rows: W's columns)
  uint16_t* WTfrl = nullptr; // bfloat16 bits of W^T - bf16(W^T), same order
};

// Covariance-form layouts of a square N x N layer (N a multiple of 32, at
// most kCovNMax).
constexpr int kCovNMax = 256;

// Position of W[row][k] in the fragment-order copy: for each 32-row block and
// each 16-wide k-step, the 64 lanes' 8-element A fragments of the
// 32x32x16 bf16 product (lane 32 (k%16 >= 8) + row%32) lie in one 1 KiB run.
__host__ __device__ inline int64_t cov_frag_index(int N, int row, int k) {
  const int blk = row >> 5, l32 = row & 31, ks = k >> 4, hi = (k >> 3) & 1, e = k & 7;
  return ((int64_t)(blk * (N >> 4) + ks) * 64 + hi * 32 + l32) * 8 + e;
}

// The row passes give each row 4 lanes (q = 0..3); at step m (m < N/32)
// lane q reads the row's 8-element chunk cov_row_chunk(N, q, m).  For N a
// multiple of 128 the four chunks of a step lie 32 elements apart, so the
// bfloat16 rows of 4 neighbouring rows (LDS row stride = 4 dwords mod 16)
// fall in distinct LDS banks.
__host__ __device__ inline int cov_row_chunk(int N, int q, int m) {
  return N % 128 == 0 ? 4 * q + (m & 3) + 16 * (m >> 2) : q * (N >> 5) + m;
}

// Position of W[row][8 c + e] in the row-pass copy, c = cov_row_chunk(N, q, m):
// the four lanes' chunks of one step are adjacent (32 floats, one 128-byte
// line).
__host__ __device__ inline int64_t cov_row_pos(int N, int row, int q, int m, int e) {
  return (int64_t)row * N + (4 * m + q) * 8 + e;
}

// Position of W[row][k] in the accumulator-quad copy.  In the transposed
// product T^T = X W^T a lane (l32, hi) of the wave that owns row block rb and
// column block cb holds, in register quad q4, T[rb 32 + l32][cb 32 + 8 q4 +
// 4 hi + e], e = 0..3; the matching four weights are one float4, and the 64
// lanes' float4s of one (rb, cb, q4) are adjacent (1 KiB).
__host__ __device__ inline int64_t cov_quad_pos(int N, int row, int k) {
  const int rb = row >> 5, l32 = row & 31, cb = k >> 5, q4 = (k >> 3) & 3, hi = (k >> 2) & 1, e = k & 3;
  return ((((int64_t)(rb * (N >> 5) + cb) * 4 + q4) * 64) + hi * 32 + l32) * 4 + e;
}

// Per-layer pointers in device memory, for kernels that walk the layers with a
// runtime index (one scalar load per layer instead of whole pointer arrays in
// kernel arguments).
struct DevLayer {
  const float* W;         // [n_out][n_in]
  const uint16_t* Wbf;    // bfloat16 bits of W, [n_out][n_in]
  const uint16_t* Wfr;    // fragment order (square layers <= kCovNMax, else null)
  const uint16_t* Wfrl;   // W - bf16(W) in fragment order (same layers)
  const float* Wv;        // row-pass order (square layers <= kCovNMax, else null)
  const float* Wq;        // accumulator-quad order (same layers)
  const uint16_t* WTfr;   // W^T hi / lo in fragment order (same layers)
  const uint16_t* WTfrl;
  const float* b;         // [n_out]
  int n_in, n_out;        // padded widths
};

struct Model {
  bool live = false;
  int n_linear = 0;
  int widths[ISX_MAX_LINEAR + 1] = {};  // as loaded
  int pw[ISX_MAX_LINEAR + 1] = {};      // padded (pw[0] = 3, pw[L] = 1)
  Layer L[ISX_MAX_LINEAR];
  DevLayer* dev_layers = nullptr;  // device copy of the per-layer pointers
  float lo[3] = {-1.f, -1.f, -1.f}, hi[3] = {1.f, 1.f, 1.f};
  int n_iso = 0;
  float iso[ISX_MAX_ISO] = {};
  int act = ISX_RELU;  // hidden activation (isx_activation)
  // surrogate attached for extraction (-1 = none)
  int sur_id = -1;
  int sur_levels = 0;
  float sur_err_mu[16] = {}, sur_err_ls[16] = {};
  float sur_z[16] = {}, sur_z_acc[16] = {};  // per-level prune / accept bands
  int sur_accept_leaves = 0;
  // bf16 coefficient-form tile shape picked by timing (-1 = not yet timed)
  mutable int bf16_tuned = -1;
  mutable float bf16_tune_ms[5] = {};
  int hidden() const { return n_linear - 1; }
  // columns of hidden layer h's coefficient block (h = 1..hidden())
  int64_t cols(int h) const {
    int64_t c = kHeadCols;
    for (int i = 1; i < h; ++i) c += pw[i];
    return c;
  }
  // bf16 path: columns of hidden layer h's block that are stored (the last
  // symbol block, W_h diag(gamma_{h-1}), is never stored: the next layer
  // multiplies by W_h^T directly and scales those columns by gamma_{h-1})
  int64_t stored_cols(int h) const {
    int64_t c = kHeadCols;
    for (int i = 1; i + 1 < h; ++i) c += pw[i];
    return c;
  }
};

// Per-chunk working memory of the propagation (element type T).
template <typename T>
struct PropWork {
  T* F[2] = {nullptr, nullptr};        // ping-pong coefficient blocks
  size_t F_elems = 0;                  // capacity of each, in elements
  T* vec = nullptr;                    // Y, A, B, G of every hidden layer
  size_t vec_elems = 0;
};

// Device-side views passed by value to kernels.
template <typename T>
struct NetView {
  int n_linear;
  int act;  // hidden activation (isx_activation)
  int n[ISX_MAX_LINEAR + 1];  // padded widths
  const T* W[ISX_MAX_LINEAR];
  const T* b[ISX_MAX_LINEAR];
  // per hidden layer h = 1..n_linear-1, chunk-local [C][n_h]
  const T* Y[ISX_MAX_LINEAR];
  const T* A[ISX_MAX_LINEAR];
  const T* B[ISX_MAX_LINEAR];
  const T* G[ISX_MAX_LINEAR];
};

struct IsoList {
  int n;
  float c[ISX_MAX_ISO];
};

// Optional timing of kernel launches (HIP events on the stream), kept per
// kernel kind (isx_kernel_kind).
struct Profiler {
  static constexpr int kKinds = 8;
  bool on = false;
  struct Rec {
    hipEvent_t a, b;
    double flops, bytes;
    int kind;
  };
  struct Tot {
    int64_t launches = 0;
    double ms = 0, flops = 0, bytes = 0;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  Tot tot[kKinds];
  hipEvent_t take() {
    hipEvent_t e = nullptr;
    if (!pool.empty()) {
      e = pool.back();
      pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  // start a record of `kind` (returns false when off or out of events)
  bool begin(Rec& r, int kind, double flops, double bytes, hipStream_t s) {
    if (!on) return false;
    r.a = take();
    r.b = take();
    r.kind = kind;
    r.flops = flops;
    r.bytes = bytes;
    if (!r.a || !r.b) return false;
    (void)hipEventRecord(r.a, s);
    return true;
  }
  void end(Rec& r, hipStream_t s) {
    (void)hipEventRecord(r.b, s);
    pending.push_back(r);
    if (pending.size() > 4096) harvest();
  }
  // fold completed records into the totals (blocks on the last one)
  void harvest() {
    for (Rec& r : pending) {
      float t = 0.f;
      if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess &&
          r.kind >= 0 && r.kind < kKinds) {
        Tot& T = tot[r.kind];
        T.ms += t;
        T.flops += r.flops;
        T.bytes += r.bytes;
        ++T.launches;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  ~Profiler() {
    for (Rec& r : pending) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// ---- propagation launchers (kernels_prop.hip) ----
// Propagate C boxes; writes (centre, spread) to out32 [C][2] and, if given,
// out64 [C][2].  `work` must be sized by prop_work_need().
struct PropArgs {
  const Model* m;
  isx_method method;
  int64_t C;
  const float* centres;
  const float* halves;
  float* out32;
  double* out64;
  int kernel_choice;  // 0 auto, 1 SIMT, 2 MFMA
  hipStream_t stream;
  Profiler* prof;     // may be null
  int bf16_variant;   // 0 = default tile shape for the width
  int up_form = 0;    // bf16 UP: 0 = covariance form when supported, 1 = coefficient form
  int aa_margin = 0;  // AA: widen by the rounding margin (kernels_margin.hip)
  uint32_t* cancel = nullptr;  // bf16 UP covariance form: per-cell cancellation flags [C] (may be null)
  int seg = 0;                 // 1: inputs are segments (centre, half-vector) with one input symbol
  int readoff_f32 = 0;         // bf16 UP: 1 = the float32 MFMA read-off instead of the bf16 hi/lo one
  bool covg = false;           // bf16 UP: the covariance form with the matrices in global memory (scratch: Fbf[0])
  bool f32_split = false;      // float32 MFMA path: products as three bf16 MFMAs of hi/lo splits
};

// Constants of the affine-arithmetic rounding margin of one layer
// (kernels_margin.hip): c for the coefficient term, c_z for the centre term
// (no operand rounding: the centre is computed from float32 / float64
// weights), the inflation of the margin's own sums, of the row statistic, and
// the rule's slack.
template <typename T>
struct AaMargin {
  T c, c_z, infl_m, infl_s, slack;
};
template <typename T>
AaMargin<T> aa_margin_consts(double u, double u_b, int K, int64_t D);
template <typename T>
hipError_t launch_aa_margin_hidden(int64_t C, int n_in, int n_out, const T* Wt, const T* bias, const T* Yp,
                                   const T* Ap, const T* Bp, const T* Rp, const float* centres, const float* halves,
                                   const T* Y, const T* S, T* A, T* B, T* G, T* R, const AaMargin<T>& k,
                                   hipStream_t s);
template <typename T>
hipError_t launch_aa_margin_output(int64_t C, int n_in, const T* Wt, const T* bias, const T* Yp, const T* Ap,
                                   const T* Bp, const T* Rp, const float* centres, const float* halves, float* out32,
                                   double* out64, const AaMargin<T>& k, hipStream_t s);
size_t prop_F_elems(const Model& m, int64_t C);
size_t prop_vec_elems(const Model& m, int64_t C, bool with_margin = false);
hipError_t propagate_f32(const PropArgs& a, PropWork<float>& w);
hipError_t propagate_f64(const PropArgs& a, PropWork<double>& w);
hipError_t propagate_bf16(const PropArgs& a, PropWork<float>& w, uint16_t* Fbf[2], size_t Fbf_elems);
bool bf16_supported(const Model& m);
// covariance-form UP on BF16 MFMA (kernels_cov.hip)
bool cov_supported(const Model& m);
double cov_flops_per_cell(const Model& m);
// Covariance form with the per-cell matrices in global memory
// (kernels_covg.hip): uniform padded hidden width N, a multiple of 256 up to
// ISX_MAX_WIDTH, with fragment-order weight copies (0 if not supported);
// scratch bytes for C cells; executed flops per cell.
int covg_width(const Model& m);
size_t covg_scratch_bytes(const Model& m, int64_t C);
int64_t covg_max_chunk(const Model& m);  // cells per launch (the gemm grid stays below 2^31 work-items)
double covg_flops_per_cell(const Model& m);
hipError_t launch_up_cov_global(const Model& m, int64_t C, const float* centres, const float* halves, float* vec,
                                uint32_t* cancel, void* scratch, hipStream_t s);
// vec: the Y, A, B, G vectors of hidden layers 1..L-1, each [C][padded width], in that order per layer
// cancel [C] (may be null): 1 where a variance sum cancelled (kernels_cov.hip)
hipError_t launch_up_cov_bf16(const Model& m, int64_t C, const float* centres, const float* halves, float* vec,
                              uint32_t* cancel, hipStream_t s);
size_t prop_F_elems_bf16(const Model& m, int64_t C);
hipError_t eval_points_f32(const Model& m, int64_t n, const float* pts, float* vals, hipStream_t s);
hipError_t eval_points_f64(const Model& m, int64_t n, const float* pts, float* vals, hipStream_t s);
// ---- dense FP32-MFMA forward passes (kernels_dense.hip) ----
hipError_t eval_points_mfma(const Model& m, int64_t n, const float* pts, float* vals, hipStream_t s);
// (f(c), |J(c) diag(h)| / sqrt(3)) per cell, out [n][2]
bool lin_bf16_supported(const Model& m);
hipError_t linearize_bf16(const Model& m, int64_t n, const float* centres, const float* halves, float* out,
                          hipStream_t s);
hipError_t linearize_mfma(const Model& m, int64_t n, const float* centres, const float* halves, float* out,
                          hipStream_t s);
// output read-off of C cells from the hidden layers' Y, A, B, G vectors
// (indexed by hidden layer 1..n_linear-1, each [C][padded width])
// UP read-off on BF16 MFMA with hi/lo splits (nets with one padded hidden
// width <= kCovNMax; kernels_dense.hip)
bool output_bf16_supported(const Model& m);
hipError_t launch_output_bf16(const Model& m, int64_t C, float* const* Y, float* const* A, float* const* B,
                              float* const* G, const float* halves, float* out, hipStream_t s);
hipError_t launch_output_mfma(const Model& m, isx_method method, int64_t C, float* const* Y, float* const* A,
                              float* const* B, float* const* G, const float* halves, float* out, hipStream_t s);
// algorithmic flops of the output read-off per cell
double output_flops_per_cell(const Model& m);

// ---- hierarchy / scan / marching cubes launchers (kernels_hier.hip) ----
hipError_t launch_root(const Model& m, uint32_t full_mask, uint32_t* ids, uint32_t* pmask, float* centres,
                       float* halves, hipStream_t s);
hipError_t launch_children(const Model& m, int level, int64_t n_par, const uint32_t* par_ids,
                           const uint32_t* par_masks, uint32_t* ids, uint32_t* pmask, float* centres,
                           float* halves, hipStream_t s);
// k-d tree of Alg. 1 on a cube domain (split axes x, y, z in turn): the 2
// children of each parent at node depth `depth`, and the conversion of depth
// 3 D node ids to octree Morton ids of level D
hipError_t launch_children_kd(const Model& m, int depth, int64_t n_par, const uint32_t* par_ids,
                              const uint32_t* par_masks, uint32_t* ids, uint32_t* pmask, float* centres,
                              float* halves, hipStream_t s);
hipError_t launch_kd_to_morton(int64_t n, int levels, uint32_t* ids, hipStream_t s);
// ids[i] = i, masks[i] = full for i < n (every cell of a level)
hipError_t launch_dense_leaves(int64_t n, uint32_t full, uint32_t* ids, uint32_t* masks, hipStream_t s);
// the 8^levels descendants of each of n_par cells, levels further down, in
// Morton order (parents in order): ids (par << 3 levels) | j, the parent's mask
hipError_t launch_subtree_leaves(int64_t n_par, int levels, const uint32_t* par_ids, const uint32_t* par_masks,
                                 uint32_t* ids, uint32_t* masks, hipStream_t s);
hipError_t launch_classify(int64_t n, const float* out, float k, const IsoList& iso, const uint32_t* pmask,
                           uint32_t* mask, hipStream_t s);
// Stable compaction of the entries with mask != 0: writes (ids ? ids[i] : i)
// and mask[i] in order, and the count to *d_count.  `tmp` needs
// compact_tmp_bytes(n) bytes.
size_t compact_tmp_bytes(int64_t n);
hipError_t launch_compact(int64_t n, const uint32_t* mask, const uint32_t* ids, uint32_t* out_idx,
                          uint32_t* out_mask, int64_t* d_count, void* tmp, hipStream_t s);
// Corner set of the leaves: bitmap over the (2^D+1)^3 grid, its word prefix
// sums, and the sorted list of corner grid indices.
size_t corner_bitmap_words(int depth);
hipError_t launch_corner_mark(int depth, int64_t n_leaves, const uint32_t* leaf_ids, uint32_t* bitmap,
                              uint64_t words, hipStream_t s);
hipError_t launch_corner_list(int depth, uint64_t words, const uint32_t* bitmap, uint32_t* word_prefix,
                              int64_t* d_count, void* tmp, size_t tmp_bytes, uint32_t* corner_g,
                              hipStream_t s);
size_t scan_tmp_bytes(int64_t n);
hipError_t launch_corner_points(const Model& m, int depth, int64_t n, const uint32_t* corner_g, float* pts,
                                hipStream_t s);
// Marching cubes on (leaf, iso) pairs.
hipError_t upload_mc_table();
hipError_t launch_mc_count(const Model& m, int depth, int64_t n_leaves, const uint32_t* leaf_ids,
                           const uint32_t* leaf_masks, const uint32_t* bitmap, const uint32_t* word_prefix,
                           const float* corner_vals, uint32_t* tri_offsets, int64_t* d_total, void* tmp,
                           size_t tmp_bytes, hipStream_t s);
hipError_t launch_mc_emit(const Model& m, int depth, int64_t n_leaves, const uint32_t* leaf_ids,
                          const uint32_t* leaf_masks, const uint32_t* bitmap, const uint32_t* word_prefix,
                          const float* corner_vals, const uint32_t* tri_offsets, float* tri_pos,
                          uint64_t* tri_keys, int32_t* tri_iso, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
// float64 re-check of the band (kernels_hier.hip): flag cells with a bound
// endpoint within `band` of a carried iso-value, gather boxes by index, and
// overwrite the classification of re-checked cells from their float64 bounds.
hipError_t launch_band_flags(int64_t n, const float* out, float k, const IsoList& iso, const uint32_t* mask_pre,
                             float band, float band_rel, uint32_t* flags, hipStream_t s);
hipError_t launch_widen_pairs(int64_t n, const float* src, double* dst, hipStream_t s);
hipError_t launch_scatter_pairs(int64_t n, const uint32_t* idx, const double* src, double* dst, hipStream_t s);
hipError_t launch_gather_boxes(int64_t n, const uint32_t* idx, const float* centres, const float* halves,
                               float* c_out, float* h_out, hipStream_t s);
hipError_t launch_recheck_apply(int64_t n, const uint32_t* idx, const double* out64, double k, const IsoList& iso,
                                const uint32_t* pmask, float* out, uint32_t* mask, hipStream_t s);

// ---- surrogate kernels (kernels_sur.hip) ----
hipError_t sur_gemm(int M, int N, int K, const float* A, int lda, bool ta, const float* B, int ldb, bool tb, float* C,
                    int ldc, const float* bias, bool relu, const float* mask, int ldm, hipStream_t s);
// C = A B without epilogue, K split over workgroups when the M x N tiles are
// too few to fill the chip (partials in `work`, which needs
// sur_gemm_splits(M, N, K) * M * N floats, else no split)
int sur_gemm_splits(int M, int N, int K);
hipError_t sur_gemm_splitk(int M, int N, int K, const float* A, int lda, bool ta, const float* B, int ldb, bool tb,
                           float* C, int ldc, float* work, size_t work_elems, hipStream_t s);
hipError_t sur_features(int64_t n, int64_t r0, int B, const float* centres, const float* halves, float a, float b,
                        float* X, const float* mu_sigma, float mu_bar, float scale, const float* base,
                        float s_floor, float* T, hipStream_t s);
hipError_t sur_loss(int B, const float* out, const float* T, float* dout, float* loss_out, hipStream_t s);
hipError_t sur_colsum(int M, int N, const float* dY, float* db, hipStream_t s);
hipError_t sur_adam(int n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t s);
hipError_t sur_unstd(int64_t n, const float* o, float mu_bar, float scale, const float* base, float s_floor,
                     float* out, float* sb_out, hipStream_t s);
hipError_t sur_partition(int64_t n, const float* pred, const float* mu_unit, float k, const IsoList& iso,
                         const uint32_t* pmask, float err_mu, float err_ls, float z, float z_acc, int leaf,
                         int accept_leaves, uint32_t* mask, uint32_t* fallback, hipStream_t s);
hipError_t gather_u32(int64_t n, const uint32_t* idx, const uint32_t* src, uint32_t* dst, hipStream_t s);
hipError_t scatter_u32(int64_t n, const uint32_t* idx, const uint32_t* src, uint32_t* dst, hipStream_t s);
hipError_t scatter_u64(int64_t n, const uint32_t* idx, const uint64_t* src, uint64_t* dst, hipStream_t s);

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the output for state x,
// so that output n of the stream with seed s is splitmix64(s + n * golden).
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// ---- surrogate training set and band calibration (kernels_calib.hip) ----
hipError_t launch_sample_cells(int64_t n, uint64_t seed, const float lo[3], const float hi[3], int level_lo,
                               int level_hi, const uint32_t* vis_ids, const int64_t* vis_off, int vis_levels,
                               int64_t vis_total, float* centres, float* halves, int32_t* levels, hipStream_t s);
hipError_t launch_calib_err(int64_t n, const float* pred, const float* targ, const float* unit, const int32_t* levels,
                            int n_levels, double* partial, int64_t n_blocks, hipStream_t s);
hipError_t launch_calib_count(int64_t n, const float* pred, const float* targ, const float* unit, const int32_t* levels,
                              int n_levels, float k, const IsoList& iso, const float* err_mu, const float* err_ls,
                              const float* ladder, int n_z, unsigned long long* counts, unsigned long long* kept,
                              hipStream_t s);
void host_normal_fill(uint64_t seed, float stddev, float* out, int64_t n);

// ---- distribution-quality report (kernels_dist.hip) ----
// Sample points of blocks b0 .. b0 + nb - 1 (SplitMix64 counters), their
// statistics, and the histogram with the KL divergences of Eq. 11.
hipError_t launch_dist_points(int64_t nb, int64_t b0, int64_t ns, uint64_t seed, const float* centres,
                              const float* halves, float* pts, hipStream_t s);
hipError_t launch_dist_stats(int64_t nb, int64_t ns, int n_fit, const float* vals, double* stats, hipStream_t s);
hipError_t launch_dist_hist_kl(int64_t nb, int64_t ns, int n_bins, const float* vals, const double* stats,
                               const double* up64, const double* raua64, double* out, uint32_t* hist, hipStream_t s);

// The row-major weights and biases of a model as kernels read them
// (kernels_prop.hip; float and double).
template <typename T>
NetView<T> net_view(const Model& m);

// ---- ray casting and RA-Fixed (kernels_ray.hip) ----
hipError_t launch_rafixed(const Model& m, bool f64, int64_t n, const float* centres, const float* halves, int seg,
                          float* out32, double* out64, hipStream_t s);
hipError_t launch_ray_init(int64_t n, const float* tnear, const float* tfar, double step0, double* t, double* dt,
                           float* thit, int32_t* iters, uint32_t* active, hipStream_t s);
hipError_t launch_ray_segments(int64_t n_act, const uint32_t* idx, const float* org, const float* dir,
                               const float* tfar, const double* t, const double* dt, float* centres, float* halfvec,
                               hipStream_t s);
hipError_t launch_ray_step(int64_t n_act, const uint32_t* idx, const float* out32, const double* out64, double k,
                           double iso, double step_min, double step_max, const float* tfar, double* t, double* dt,
                           float* thit, int32_t* iters, uint32_t* active, hipStream_t s);

// ---- marching-cubes case table (mc_table.cpp) ----
struct McTable {
  uint8_t count[256];       // triangles per case
  int8_t edges[256][15];    // edge indices, 3 per triangle
};
const McTable& mc_table();

}  // namespace isx
