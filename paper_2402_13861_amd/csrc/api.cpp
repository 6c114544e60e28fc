// C ABI of libisx (declared in include/isx.h): context, weights, batched
// propagation, classification/compaction, and the full hierarchical
// extraction of Alg. 1 followed by corner evaluation and marching cubes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "isx_internal.h"

using namespace isx;

namespace {

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

std::string g_create_error;

// ---- fixed working memory of the allocation-free classify/compact entry
// point: per-cell masks, then the scan's block partials (one uint64 per
// 2048 cells, plus one).  Each device holds its own copy of this array; host
// code never uses its name as an address, only the per-device pointer that
// hipGetSymbolAddress returns at context creation.
constexpr size_t kNoAllocMaskBytes = size_t(ISX_NOALLOC_MAX_CELLS) * sizeof(uint32_t);
constexpr size_t kNoAllocBytes = kNoAllocMaskBytes + (size_t(ISX_NOALLOC_MAX_CELLS) / 2048 + 2) * sizeof(uint64_t);
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Looks up the device address of `scratch` on the current device `dev` once.
hipError_t init_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void* ptr = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
    g_scratch_done[dev] = true;
  }
  return g_scratch_err[dev];
}

void* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch_ptr[dev];
}

}  // namespace

// Surrogate state: float32 master weights, Adam moments, gradients.
struct Sur {
  bool live = false;
  int L = 0;
  int w[ISX_MAX_LINEAR + 1] = {};
  float *W[ISX_MAX_LINEAR] = {}, *b[ISX_MAX_LINEAR] = {};
  float *mW[ISX_MAX_LINEAR] = {}, *vW[ISX_MAX_LINEAR] = {}, *mb[ISX_MAX_LINEAR] = {}, *vb[ISX_MAX_LINEAR] = {};
  float *gW[ISX_MAX_LINEAR] = {}, *gb[ISX_MAX_LINEAR] = {};
  int64_t t = 0;
  float mu_bar = 0.f, scale = 1.f, size_a = 1.f, size_b = 0.f;
  // outputs are corrections to this MLP's centre linearisation (-1: plain)
  int32_t base_mlp = -1;
  float s_floor = 0.f;
};

struct isx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<Model> models;
  bool keep_levels = false;
  bool verbose = false;
  int kernel_choice = 0;
  int bf16_variant = 0;
  int autotune = 0;   // ISX_AUTOTUNE
  int readoff_f32 = 0;  // ISX_BF16_READOFF
  bool tuning = false;
  Buf tune_c, tune_h, tune_out;
  int up_form = 0;
  int lin_prec = 1;  // centre linearisation: 1 = bf16 split where supported, 0 = float32
  int aa_margin = 0; // AA: widen by the rounding margin
  int cancel_check = 1;  // bf16 UP covariance form: re-propagate cells whose variance sums cancel, in float64
  int64_t n_cancel_last = 0;  // cells re-propagated for cancellation by the last run_propagate
  size_t prop_budget = size_t(16) << 30;  // bytes of propagation scratch per chunk
  // propagation scratch
  Buf F32[2], vec32, F64[2], vec64, Fbf[2];
  // level scratch
  Buf ids, pmask, centres, halves, out, mask, act_ids[2], act_mask[2], scan_tmp, count;
  Buf rc_idx, rc_centres, rc_halves, rc_out32, rc_out64, rc_count;
  // corner / mc scratch
  Buf bitmap, word_prefix, corner_g, corner_pts, corner_vals, tri_off;
  Buf cls_mask;
  // surrogate: models, training/inference activations, extraction scratch
  std::vector<Sur> surs;
  Buf sur_act[ISX_MAX_LINEAR + 1], sur_out, sur_T, sur_d[2], sur_base, sp_base, sp_scale, sur_work;
  Buf sp_pred, sp_fb, sp_idx, sp_pm, sp_c, sp_h, sp_out, sp_mask, sp_cnt, sp_tmp;
  Buf rc_flags, rc_fidx, rc_fmask;
  Buf rc_pm, rc_flags2, rc_idx2, rc2_c, rc2_h, rc2_out32, rc2_out64;  // two-stage re-check
  int recheck_cascade = 0;                                          // ISX_RECHECK_CASCADE
  int dense_from = 0;                                               // ISX_DENSE_FROM_LEVEL
  int recheck_split = 0;                                            // ISX_RECHECK_SPLIT
  bool f32_split_now = false;  // the float32 propagation running is the cascade's first stage (split products)
  int64_t n_rc64_last = 0;  // cells propagated in float64 by the re-checks since the level began
  Buf cx_flags, cx_idx, cx_c, cx_h, cx_out, cx_out64, cx_cnt;
  // surrogate training set and band calibration
  Buf sp_vis, sp_vis_off, cal_pred, cal_unit, cal_part, cal_cnt, cal_vec, fit_c, fit_h, fit_t, fit_l, fit_loss;
  // distribution-quality report
  Buf ds_pts, ds_vals, ds_stats, ds_o32, ds_up64, ds_ra64;
  // ray casting
  Buf ray_t, ray_dt, ray_act, ray_idx, ray_c, ray_v, ray_o32, ray_o64, ray_cnt;
  int64_t* h_count = nullptr;  // pinned
  Profiler prof;
  // batched extraction: worker contexts with their own stream and scratch;
  // a worker borrows its parent's models and surrogates (never frees them)
  std::vector<isx_ctx*> workers;
  bool borrowed = false;
  bool own_stream = false;
  int batch_workers = 4;
};

struct isx_mesh {
  int depth = 0;
  int64_t n_tris = 0, n_leaves = 0, n_corners = 0;
  uint32_t* leaf_ids = nullptr;
  uint32_t* leaf_masks = nullptr;
  float* tri_pos = nullptr;
  uint64_t* tri_keys = nullptr;
  int32_t* tri_iso = nullptr;
  std::vector<int64_t> lvl_cells, lvl_active, lvl_recheck, lvl_prop, lvl_cancel, lvl_recheck64;
  std::vector<std::vector<uint32_t>> lvl_ids, lvl_masks;
  std::vector<std::vector<float>> lvl_out;
  bool kept = false;
  float ms_acp = 0, ms_inr = 0, ms_mc = 0, ms_total = 0;
};

namespace {

isx_status fail(isx_ctx* c, isx_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

isx_status hip_fail(isx_ctx* c, hipError_t e, const char* where) {
  return fail(c, e == hipErrorOutOfMemory ? ISX_ENOMEM : ISX_EHIP,
              std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr)                                    \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
  } while (0)

hipError_t ensure(Buf& b, size_t bytes) {
  if (bytes == 0) bytes = 1;
  if (b.bytes >= bytes) return hipSuccess;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    if (e != hipSuccess) return e;
  }
  b.p = nullptr;
  b.bytes = 0;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return e;
  }
  b.bytes = bytes;
  return hipSuccess;
}

void release(Buf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

void free_model_table(Model& m) {
  if (m.dev_layers) (void)hipFree(m.dev_layers);
  m.dev_layers = nullptr;
}

void free_layer(Layer& l) {
  void* ps[] = {l.W, l.Wt, l.b, l.Wd, l.Wtd, l.bd, l.Wtbf, l.Wbf, l.Wfr, l.Wfrl, l.Wv, l.Wq, l.WTfr, l.WTfrl};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  l = Layer{};
}

Model* get_model(isx_ctx* ctx, int32_t id) {
  if (!ctx || id < 0 || id >= (int32_t)ctx->models.size() || !ctx->models[id].live) return nullptr;
  return &ctx->models[id];
}

uint16_t f32_to_bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  // round to nearest even
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

template <typename T>
hipError_t upload(T** dst, const std::vector<T>& src) {
  hipError_t e = hipMalloc((void**)dst, src.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

// Scratch bytes per cell of the propagation at precision T.
template <typename T>
size_t per_cell_bytes(const Model& m) {
  return (2 * prop_F_elems(m, 1) + prop_vec_elems(m, 1, true)) * sizeof(T);
}

// Cells per propagation chunk at most: kernels that give a cell a whole
// workgroup keep a launch's work-items below 2^32 with it.
constexpr int64_t kMaxPropChunk = int64_t(1) << 22;

template <typename T>
int64_t chunk_for(isx_ctx* ctx, const Model& m, int64_t n, int64_t req) {
  int64_t c = req > 0 ? req : (int64_t)(ctx->prop_budget / per_cell_bytes<T>(m));
  c = std::max<int64_t>(1, std::min<int64_t>({c, n, kMaxPropChunk}));
  return c;
}

isx_status run_propagate(isx_ctx* ctx, const Model& m, isx_method method, isx_precision prec, int64_t n,
                         const float* centres, const float* halves, float* out, double* out64, int64_t chunk_req,
                         int seg = 0);

// Cells whose covariance-form variance sums cancelled (flags[i] != 0) are
// propagated again in float64 and their (mu, sigma) replaced.  Synchronises
// the stream once to read the count.
isx_status recheck_cancelled(isx_ctx* ctx, const Model& m, int64_t n, const float* centres, const float* halves,
                             float* out, const uint32_t* flags, int64_t chunk_req) {
  hipStream_t s = ctx->stream;
  HIPCHK(ensure(ctx->cx_idx, n * 4));
  HIPCHK(ensure(ctx->cx_cnt, sizeof(int64_t)));
  HIPCHK(ensure(ctx->scan_tmp, compact_tmp_bytes(n)));
  HIPCHK(launch_compact(n, flags, nullptr, (uint32_t*)ctx->cx_idx.p, nullptr, (int64_t*)ctx->cx_cnt.p,
                        ctx->scan_tmp.p, s));
  HIPCHK(hipMemcpyAsync(ctx->h_count, ctx->cx_cnt.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int64_t nc = ctx->h_count[0];
  ctx->n_cancel_last = nc;
  if (nc <= 0) return ISX_OK;
  HIPCHK(ensure(ctx->cx_c, nc * 12));
  HIPCHK(ensure(ctx->cx_h, nc * 12));
  HIPCHK(ensure(ctx->cx_out, nc * 8));
  HIPCHK(ensure(ctx->cx_out64, nc * 16));
  const uint32_t* idx = (const uint32_t*)ctx->cx_idx.p;
  HIPCHK(launch_gather_boxes(nc, idx, centres, halves, (float*)ctx->cx_c.p, (float*)ctx->cx_h.p, s));
  isx_status st = run_propagate(ctx, m, ISX_UP, ISX_FP64, nc, (const float*)ctx->cx_c.p, (const float*)ctx->cx_h.p,
                                (float*)ctx->cx_out.p, (double*)ctx->cx_out64.p, chunk_req);
  if (st != ISX_OK) return st;
  HIPCHK(scatter_u64(nc, idx, (const uint64_t*)ctx->cx_out.p, (uint64_t*)out, s));
  return ISX_OK;
}

// Tile shape of the bf16 coefficient-form hidden-layer kernel for this MLP:
// each candidate propagates the same 4096 cells (octree levels 3..6 of the
// domain, SplitMix64 positions) once untimed and twice timed with HIP
// events; the fastest is kept in the model.  The shapes only split the same
// products differently, so they give identical results.
static isx_status tune_bf16(isx_ctx* ctx, const Model& m) {
  if (m.bf16_tuned >= 0) return ISX_OK;
  constexpr int kN = 4096;
  std::vector<float> hc(3 * kN), hh(3 * kN);
  for (int i = 0; i < kN; ++i) {
    const int L = 3 + (int)(splitmix64(0x5eedull + 4ull * i) % 4ull);
    const int64_t res = (int64_t)1 << L;
    for (int a = 0; a < 3; ++a) {
      const int64_t q = (int64_t)(splitmix64(0x5eedull + 4ull * i + 1ull + (uint64_t)a) % (uint64_t)res);
      const double ext = (double)m.hi[a] - m.lo[a];
      hh[3 * i + a] = (float)(0.5 * ext / (double)res);
      hc[3 * i + a] = (float)((double)m.lo[a] + ext * ((double)q + 0.5) / (double)res);
    }
  }
  HIPCHK(ensure(ctx->tune_c, sizeof(float) * 3 * kN));
  HIPCHK(ensure(ctx->tune_h, sizeof(float) * 3 * kN));
  HIPCHK(ensure(ctx->tune_out, sizeof(float) * 2 * kN));
  hipStream_t s = ctx->stream;
  HIPCHK(hipMemcpyAsync(ctx->tune_c.p, hc.data(), sizeof(float) * 3 * kN, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ctx->tune_h.p, hh.data(), sizeof(float) * 3 * kN, hipMemcpyHostToDevice, s));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int saved = ctx->bf16_variant, saved_form = ctx->up_form;
  const bool saved_prof = ctx->prof.on;
  ctx->tuning = true;
  ctx->prof.on = false;
  ctx->up_form = 1;  // the coefficient form, whose kernel the shapes belong to
  int best = 0;
  float best_ms = 0.f;
  isx_status st = ISX_OK;
  for (int v : {0, 1, 3, 4}) {
    ctx->bf16_variant = v;
    float ms = 0.f;
    for (int rep = 0; rep < 3 && st == ISX_OK; ++rep) {
      if (rep == 1) (void)hipEventRecord(e0, s);
      st = run_propagate(ctx, m, ISX_UP, ISX_BF16, kN, (const float*)ctx->tune_c.p, (const float*)ctx->tune_h.p,
                         (float*)ctx->tune_out.p, nullptr, 0);
    }
    if (st != ISX_OK) break;
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(&ms, e0, e1);
    m.bf16_tune_ms[v] = ms / 2.f;
    if (v == 0 || ms < best_ms) {
      best = v;
      best_ms = ms;
    }
  }
  ctx->bf16_variant = saved;
  ctx->up_form = saved_form;
  ctx->tuning = false;
  ctx->prof.on = saved_prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != ISX_OK) return st;
  m.bf16_tuned = best;
  if (ctx->verbose) {
    std::fprintf(stderr, "isx: bf16 tile shape %d picked (ms per 4096 cells: default %.3f, 1 %.3f, 3 %.3f, 4 %.3f)\n",
                 best, m.bf16_tune_ms[0], m.bf16_tune_ms[1], m.bf16_tune_ms[3], m.bf16_tune_ms[4]);
    std::fflush(stderr);
  }
  return ISX_OK;
}

isx_status run_propagate(isx_ctx* ctx, const Model& m, isx_method method, isx_precision prec, int64_t n,
                         const float* centres, const float* halves, float* out, double* out64, int64_t chunk_req,
                         int seg) {
  if (n <= 0) return ISX_OK;
  const bool marg = method == ISX_AA && ctx->aa_margin != 0;
  if (marg && m.act != ISX_RELU) return fail(ctx, ISX_EUNSUPPORTED, "the AA rounding margin needs a ReLU net");
  if (seg && (marg || prec == ISX_BF16))
    return fail(ctx, ISX_EUNSUPPORTED, "segments take float32 or float64 without the AA rounding margin");
  if (method == ISX_RAFIXED) {
    // one SIMT pass per cell: the form is the input symbols and one error term
    if (prec == ISX_BF16) return fail(ctx, ISX_EUNSUPPORTED, "RA-Fixed runs in float32 or float64");
    HIPCHK(launch_rafixed(m, prec == ISX_FP64, n, centres, halves, seg, out, prec == ISX_FP64 ? out64 : nullptr,
                          ctx->stream));
    return ISX_OK;
  }
  if (prec == ISX_FP64) {
    const int64_t chunk = chunk_for<double>(ctx, m, n, chunk_req);
    PropWork<double> w;
    HIPCHK(ensure(ctx->F64[0], prop_F_elems(m, chunk) * sizeof(double)));
    HIPCHK(ensure(ctx->F64[1], prop_F_elems(m, chunk) * sizeof(double)));
    HIPCHK(ensure(ctx->vec64, prop_vec_elems(m, chunk, marg) * sizeof(double)));
    w.F[0] = (double*)ctx->F64[0].p;
    w.F[1] = (double*)ctx->F64[1].p;
    w.vec = (double*)ctx->vec64.p;
    for (int64_t s = 0; s < n; s += chunk) {
      PropArgs a{&m, method, std::min(chunk, n - s), centres + 3 * s, halves + 3 * s, out + 2 * s,
                 out64 ? out64 + 2 * s : nullptr, ctx->kernel_choice, ctx->stream, &ctx->prof, ctx->bf16_variant};
      a.aa_margin = marg;
      a.seg = seg;
      HIPCHK(propagate_f64(a, w));
    }
    return ISX_OK;
  }
  if (prec == ISX_BF16) {
    // UP in covariance form: on chip (hidden widths <= 256), or with the
    // per-cell matrices in device memory (one hidden width of 512 or 1024 by
    // default; ISX_UP_FORM = 2 also at 256)
    const bool cov = method == ISX_UP && ctx->up_form == 0 && cov_supported(m);
    const bool covg = method == ISX_UP && !marg && covg_width(m) &&
                      ((ctx->up_form == 0 && !cov_supported(m)) || ctx->up_form == 2);
    if (method == ISX_UP && ctx->up_form == 2 && !covg)
      return fail(ctx, ISX_EUNSUPPORTED,
                  "ISX_UP_FORM 2 needs hidden layers of one width, a multiple of 256 up to 1024");
    if (!bf16_supported(m) && !covg)
      return fail(ctx, ISX_EUNSUPPORTED, "bf16 propagation needs every hidden layer's input width <= 512");
    const size_t per_cell = (cov ? 0 : (covg ? covg_scratch_bytes(m, 1) : 2 * prop_F_elems_bf16(m, 1) * 2)) +
                            prop_vec_elems(m, 1, marg) * 4;
    int64_t chunk = chunk_req > 0 ? chunk_req : (int64_t)(ctx->prop_budget / per_cell);
    chunk = std::max<int64_t>(1, std::min<int64_t>({chunk, n, kMaxPropChunk}));
    if (covg) chunk = std::min(chunk, covg_max_chunk(m));
    PropWork<float> w;
    if (covg) {
      HIPCHK(ensure(ctx->Fbf[0], covg_scratch_bytes(m, chunk)));
    } else if (!cov) {
      HIPCHK(ensure(ctx->Fbf[0], prop_F_elems_bf16(m, chunk) * 2));
      HIPCHK(ensure(ctx->Fbf[1], prop_F_elems_bf16(m, chunk) * 2));
    }
    HIPCHK(ensure(ctx->vec32, prop_vec_elems(m, chunk, marg) * sizeof(float)));
    w.vec = (float*)ctx->vec32.p;
    const bool check = (cov || covg) && ctx->cancel_check != 0;
    if (check) HIPCHK(ensure(ctx->cx_flags, n * 4));
    int variant = ctx->bf16_variant;
    if (variant == 0 && !cov && !covg && ctx->autotune && !ctx->tuning) {
      const isx_status st = tune_bf16(ctx, m);
      if (st != ISX_OK) return st;
      variant = m.bf16_tuned;
    }
    uint16_t* Fbf[2] = {(uint16_t*)ctx->Fbf[0].p, (uint16_t*)ctx->Fbf[1].p};
    for (int64_t s = 0; s < n; s += chunk) {
      PropArgs a{&m, method, std::min(chunk, n - s), centres + 3 * s, halves + 3 * s, out + 2 * s, nullptr,
                 ctx->kernel_choice, ctx->stream, &ctx->prof, variant, ctx->up_form};
      a.aa_margin = marg;
      if (check) a.cancel = (uint32_t*)ctx->cx_flags.p + s;
      a.readoff_f32 = ctx->readoff_f32;
      a.covg = covg;
      HIPCHK(propagate_bf16(a, w, Fbf, 0));
    }
    ctx->n_cancel_last = 0;
    if (check) return recheck_cancelled(ctx, m, n, centres, halves, out, (const uint32_t*)ctx->cx_flags.p, chunk_req);
    return ISX_OK;
  }
  const int64_t chunk = chunk_for<float>(ctx, m, n, chunk_req);
  PropWork<float> w;
  HIPCHK(ensure(ctx->F32[0], prop_F_elems(m, chunk) * sizeof(float)));
  HIPCHK(ensure(ctx->F32[1], prop_F_elems(m, chunk) * sizeof(float)));
  HIPCHK(ensure(ctx->vec32, prop_vec_elems(m, chunk, marg) * sizeof(float)));
  w.F[0] = (float*)ctx->F32[0].p;
  w.F[1] = (float*)ctx->F32[1].p;
  w.vec = (float*)ctx->vec32.p;
  for (int64_t s = 0; s < n; s += chunk) {
    PropArgs a{&m, method, std::min(chunk, n - s), centres + 3 * s, halves + 3 * s, out + 2 * s, nullptr,
               ctx->kernel_choice, ctx->stream, &ctx->prof, ctx->bf16_variant};
    a.aa_margin = marg;
    a.seg = seg;
    // (UP only: AA's rounding margin assumes float32 products)
    a.f32_split = (ctx->f32_split_now || ctx->kernel_choice == 3) && method == ISX_UP;
    HIPCHK(propagate_f32(a, w));
  }
  return ISX_OK;
}

IsoList iso_list(const Model& m) {
  IsoList l;
  l.n = m.n_iso;
  for (int j = 0; j < ISX_MAX_ISO; ++j) l.c[j] = j < m.n_iso ? m.iso[j] : 0.f;
  return l;
}

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

}  // namespace


extern "C" {

isx_status isx_create(int device, void* hip_stream, isx_ctx** out) {
  if (!out) return ISX_EINVAL;
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || device < 0 || device >= n) {
    g_create_error = "isx_create: no such HIP device";
    return ISX_EINVAL;
  }
  e = hipSetDevice(device);
  if (e != hipSuccess) {
    g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
    return ISX_EHIP;
  }
  e = upload_mc_table();
  if (e != hipSuccess) {
    g_create_error = std::string("upload_mc_table: ") + hipGetErrorString(e);
    return ISX_EHIP;
  }
  e = init_scratch(device);
  if (e != hipSuccess) {
    g_create_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return ISX_EHIP;
  }
  isx_ctx* c = new isx_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  e = hipHostMalloc((void**)&c->h_count, 4 * sizeof(int64_t), hipHostMallocDefault);
  if (e != hipSuccess) {
    delete c;
    g_create_error = std::string("hipHostMalloc: ") + hipGetErrorString(e);
    return ISX_EHIP;
  }
  *out = c;
  return ISX_OK;
}

isx_status isx_destroy(isx_ctx* ctx) {
  if (!ctx) return ISX_EINVAL;
  (void)hipSetDevice(ctx->device);
  for (isx_ctx* w : ctx->workers) (void)isx_destroy(w);
  ctx->workers.clear();
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->borrowed) {
    ctx->models.clear();
    ctx->surs.clear();
  }
  for (Model& m : ctx->models) {
    for (int l = 0; l < ISX_MAX_LINEAR; ++l) free_layer(m.L[l]);
    free_model_table(m);
  }
  Buf* bufs[] = {&ctx->F32[0], &ctx->F32[1], &ctx->vec32, &ctx->F64[0], &ctx->F64[1], &ctx->vec64, &ctx->Fbf[0],
                 &ctx->Fbf[1],
                 &ctx->ids, &ctx->pmask, &ctx->centres, &ctx->halves, &ctx->out, &ctx->mask,
                 &ctx->act_ids[0], &ctx->act_ids[1], &ctx->act_mask[0], &ctx->act_mask[1], &ctx->scan_tmp,
                 &ctx->count, &ctx->rc_idx, &ctx->rc_centres, &ctx->rc_halves, &ctx->rc_out32, &ctx->rc_out64,
                 &ctx->rc_count, &ctx->bitmap, &ctx->word_prefix, &ctx->corner_g, &ctx->corner_pts,
                 &ctx->corner_vals, &ctx->tri_off, &ctx->cls_mask};
  for (Buf* b : bufs) release(*b);
  Buf* sbufs[] = {&ctx->sur_out, &ctx->sur_T, &ctx->sur_d[0], &ctx->sur_d[1], &ctx->sur_base, &ctx->sp_base,
                  &ctx->sp_scale, &ctx->sp_pred, &ctx->sp_fb,
                  &ctx->sp_idx, &ctx->sp_pm, &ctx->sp_c, &ctx->sp_h, &ctx->sp_out, &ctx->sp_mask, &ctx->sp_cnt,
                  &ctx->sp_tmp, &ctx->rc_flags, &ctx->rc_fidx, &ctx->rc_fmask, &ctx->sur_work};
  for (Buf* b : sbufs) release(*b);
  for (Buf& b : ctx->sur_act) release(b);
  Buf* cbufs[] = {&ctx->cx_flags, &ctx->cx_idx, &ctx->cx_c,     &ctx->cx_h,     &ctx->cx_out,   &ctx->cx_out64,
                  &ctx->cx_cnt,   &ctx->sp_vis, &ctx->sp_vis_off, &ctx->cal_pred, &ctx->cal_unit, &ctx->cal_part,
                  &ctx->cal_cnt,  &ctx->cal_vec, &ctx->fit_c,     &ctx->fit_h,    &ctx->fit_t,    &ctx->fit_l,
                  &ctx->fit_loss, &ctx->ds_pts,  &ctx->ds_vals, &ctx->ds_stats, &ctx->ds_o32, &ctx->ds_up64,
                  &ctx->ds_ra64,  &ctx->ray_t,   &ctx->ray_dt,  &ctx->ray_act,  &ctx->ray_idx, &ctx->ray_c,
                  &ctx->ray_v,    &ctx->ray_o32, &ctx->ray_o64, &ctx->ray_cnt, &ctx->rc_pm,   &ctx->rc_flags2,
                  &ctx->rc_idx2,  &ctx->rc2_c,   &ctx->rc2_h,   &ctx->rc2_out32, &ctx->rc2_out64};
  for (Buf* b : cbufs) release(*b);
  for (int i = 0; i < (int)ctx->surs.size(); ++i) isx_surrogate_free(ctx, i);
  if (ctx->h_count) (void)hipHostFree(ctx->h_count);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return ISX_OK;
}

const char* isx_last_error(const isx_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

isx_status isx_set_option(isx_ctx* ctx, isx_option option, int64_t value) {
  if (!ctx) return ISX_EINVAL;
  switch (option) {
    case ISX_KEEP_LEVELS:
      ctx->keep_levels = value != 0;
      return ISX_OK;
    case ISX_HIDDEN_KERNEL:
      if (value < 0 || value > 3) return fail(ctx, ISX_EINVAL, "ISX_HIDDEN_KERNEL must be 0, 1, 2 or 3");
      ctx->kernel_choice = (int)value;
      return ISX_OK;
    case ISX_PROFILE:
      ctx->prof.on = value != 0;
      return ISX_OK;
    case ISX_VERBOSE:
      ctx->verbose = value != 0;
      return ISX_OK;
    case ISX_UP_FORM:
      if (value < 0 || value > 2) return fail(ctx, ISX_EINVAL, "ISX_UP_FORM must be 0, 1 or 2");
      ctx->up_form = (int)value;
      return ISX_OK;
    case ISX_BATCH_WORKERS:
      if (value < 1 || value > 16) return fail(ctx, ISX_EINVAL, "ISX_BATCH_WORKERS must be in [1, 16]");
      ctx->batch_workers = (int)value;
      return ISX_OK;
    case ISX_AA_MARGIN:
      if (value < 0 || value > 1) return fail(ctx, ISX_EINVAL, "ISX_AA_MARGIN must be 0 or 1");
      ctx->aa_margin = (int)value;
      return ISX_OK;
    case ISX_LIN_PRECISION:
      if (value < 0 || value > 1) return fail(ctx, ISX_EINVAL, "ISX_LIN_PRECISION must be 0 or 1");
      ctx->lin_prec = (int)value;
      return ISX_OK;
    case ISX_BF16_VARIANT:
      if (value < 0 || value > 4) return fail(ctx, ISX_EINVAL, "ISX_BF16_VARIANT must be in [0, 4]");
      if (value != 0)
        return fail(ctx, ISX_EUNSUPPORTED,
                    "tile shapes other than the default are switched off (a device fault surfaced while they ran; "
                    "its cause is not established)");
      ctx->bf16_variant = (int)value;
      return ISX_OK;
    case ISX_CANCEL_CHECK:
      if (value < 0 || value > 1) return fail(ctx, ISX_EINVAL, "ISX_CANCEL_CHECK must be 0 or 1");
      ctx->cancel_check = (int)value;
      return ISX_OK;
    case ISX_AUTOTUNE:
      if (value < 0 || value > 1) return fail(ctx, ISX_EINVAL, "ISX_AUTOTUNE must be 0 or 1");
      if (value != 0)
        return fail(ctx, ISX_EUNSUPPORTED,
                    "tile-shape timing is switched off with the non-default shapes (a device fault surfaced while "
                    "they ran; its cause is not established)");
      ctx->autotune = (int)value;
      return ISX_OK;
    case ISX_RECHECK_CASCADE:
      if (value < 0 || value > 1) return fail(ctx, ISX_EINVAL, "ISX_RECHECK_CASCADE must be 0 or 1");
      ctx->recheck_cascade = (int)value;
      return ISX_OK;
    case ISX_RECHECK_SPLIT:
      if (value < 0 || value > 1) return fail(ctx, ISX_EINVAL, "ISX_RECHECK_SPLIT must be 0 or 1");
      ctx->recheck_split = (int)value;
      return ISX_OK;
    case ISX_DENSE_FROM_LEVEL:
      if (value < 0 || value > 10) return fail(ctx, ISX_EINVAL, "ISX_DENSE_FROM_LEVEL must be in [0, 10]");
      ctx->dense_from = (int)value;
      return ISX_OK;
    case ISX_BF16_READOFF:
      if (value < 0 || value > 1) return fail(ctx, ISX_EINVAL, "ISX_BF16_READOFF must be 0 or 1");
      ctx->readoff_f32 = (int)value;
      return ISX_OK;
    case ISX_SCRATCH_BYTES:
      if (value < (int64_t)(1 << 20)) return fail(ctx, ISX_EINVAL, "ISX_SCRATCH_BYTES must be >= 1 MiB");
      ctx->prop_budget = (size_t)value;
      return ISX_OK;
  }
  return fail(ctx, ISX_EINVAL, "unknown option");
}

isx_status isx_get_profile(isx_ctx* ctx, int32_t kernel, int64_t* launches, double* ms, double* flops,
                           double* bytes, int32_t reset) {
  if (!ctx) return ISX_EINVAL;
  if (kernel < 0 || kernel >= Profiler::kKinds) return fail(ctx, ISX_EINVAL, "unknown kernel kind");
  (void)hipSetDevice(ctx->device);
  ctx->prof.harvest();
  const Profiler::Tot& T = ctx->prof.tot[kernel];
  if (launches) *launches = T.launches;
  if (ms) *ms = T.ms;
  if (flops) *flops = T.flops;
  if (bytes) *bytes = T.bytes;
  if (reset)
    for (Profiler::Tot& t : ctx->prof.tot) t = Profiler::Tot{};
  return ISX_OK;
}

isx_status isx_mc_case_table(uint8_t* h_count, int8_t* h_edges) {
  const McTable& t = mc_table();
  if (h_count) std::memcpy(h_count, t.count, sizeof(t.count));
  if (h_edges) std::memcpy(h_edges, t.edges, sizeof(t.edges));
  return ISX_OK;
}

isx_status isx_load_mlp(isx_ctx* ctx, int32_t n_linear, const int32_t* widths, const float* const* h_W,
                        const float* const* h_b, int32_t* mlp_id) {
  if (!ctx || !widths || !h_W || !h_b || !mlp_id) return fail(ctx, ISX_EINVAL, "null argument");
  if (n_linear < 2 || n_linear > ISX_MAX_LINEAR)
    return fail(ctx, ISX_ESHAPE, "n_linear must be in [2, " + std::to_string(ISX_MAX_LINEAR) + "]");
  if (widths[0] != 3 || widths[n_linear] != 1) return fail(ctx, ISX_ESHAPE, "widths[0] must be 3 and widths[L] 1");
  for (int l = 1; l < n_linear; ++l)
    if (widths[l] < 1 || widths[l] > ISX_MAX_WIDTH)
      return fail(ctx, ISX_ESHAPE, "hidden width out of range at layer " + std::to_string(l));
  for (int l = 0; l < n_linear; ++l) {
    if (!h_W[l] || !h_b[l]) return fail(ctx, ISX_EINVAL, "null weight pointer");
    const int64_t nw = (int64_t)widths[l] * widths[l + 1];
    for (int64_t i = 0; i < nw; ++i)
      if (!std::isfinite(h_W[l][i])) return fail(ctx, ISX_ENAN, "non-finite weight in layer " + std::to_string(l));
    for (int i = 0; i < widths[l + 1]; ++i)
      if (!std::isfinite(h_b[l][i])) return fail(ctx, ISX_ENAN, "non-finite bias in layer " + std::to_string(l));
  }
  (void)hipSetDevice(ctx->device);
  Model m;
  m.n_linear = n_linear;
  for (int l = 0; l <= n_linear; ++l) {
    m.widths[l] = widths[l];
    m.pw[l] = (l == 0 || l == n_linear) ? widths[l] : (widths[l] + 31) / 32 * 32;
  }
  for (int l = 0; l < n_linear; ++l) {
    const int ni = m.pw[l], no = m.pw[l + 1];
    const int wi = widths[l], wo = widths[l + 1];
    std::vector<float> W((size_t)no * ni, 0.f), Wt((size_t)ni * no, 0.f), b((size_t)no, 0.f);
    std::vector<double> Wd((size_t)no * ni, 0.0), Wtd((size_t)ni * no, 0.0), bd((size_t)no, 0.0);
    std::vector<uint16_t> Wtbf((size_t)ni * no, 0), Wbf((size_t)no * ni, 0);
    for (int o = 0; o < wo; ++o) {
      for (int i = 0; i < wi; ++i) {
        const float w = h_W[l][(size_t)o * wi + i];
        W[(size_t)o * ni + i] = w;
        Wt[(size_t)i * no + o] = w;
        Wd[(size_t)o * ni + i] = w;
        Wtd[(size_t)i * no + o] = w;
        Wtbf[(size_t)i * no + o] = f32_to_bf16_bits(w);
        Wbf[(size_t)o * ni + i] = f32_to_bf16_bits(w);
      }
      b[o] = h_b[l][o];
      bd[o] = h_b[l][o];
    }
    Layer& L = m.L[l];
    L.n_in = ni;
    L.n_out = no;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = upload(&L.W, W);
    if (e == hipSuccess) e = upload(&L.Wt, Wt);
    if (e == hipSuccess) e = upload(&L.b, b);
    if (e == hipSuccess) e = upload(&L.Wd, Wd);
    if (e == hipSuccess) e = upload(&L.Wtd, Wtd);
    if (e == hipSuccess) e = upload(&L.bd, bd);
    if (e == hipSuccess) e = upload(&L.Wtbf, Wtbf);
    if (e == hipSuccess) e = upload(&L.Wbf, Wbf);
    if (e == hipSuccess && l >= 1 && l + 1 < n_linear && ni == no && no > kCovNMax) {
      // the fragment-order and accumulator-quad copies that the device-memory
      // covariance form reads
      const int N = no;
      std::vector<uint16_t> Wfr((size_t)N * N);
      std::vector<float> Wq((size_t)N * N);
      for (int r = 0; r < N; ++r)
        for (int k = 0; k < N; ++k) {
          Wfr[cov_frag_index(N, r, k)] = Wbf[(size_t)r * N + k];
          Wq[cov_quad_pos(N, r, k)] = W[(size_t)r * N + k];
        }
      e = upload(&L.Wfr, Wfr);
      if (e == hipSuccess) e = upload(&L.Wq, Wq);
    }
    if (e == hipSuccess && l >= 1 && l + 1 < n_linear && ni == no && no <= kCovNMax) {
      // copies in the covariance kernel's access orders
      const int N = no;
      std::vector<uint16_t> Wfr((size_t)N * N), Wfrl((size_t)N * N), WTfr((size_t)N * N), WTfrl((size_t)N * N);
      std::vector<float> Wv((size_t)N * N), Wq((size_t)N * N);
      for (int r = 0; r < N; ++r)
        for (int k = 0; k < N; ++k) {
          const uint16_t hb = Wbf[(size_t)r * N + k];
          uint32_t hu = (uint32_t)hb << 16;
          float hf;
          std::memcpy(&hf, &hu, 4);
          Wfr[cov_frag_index(N, r, k)] = hb;
          Wfrl[cov_frag_index(N, r, k)] = f32_to_bf16_bits(W[(size_t)r * N + k] - hf);
          // W^T: row k of W^T is column k of W
          WTfr[cov_frag_index(N, k, r)] = hb;
          WTfrl[cov_frag_index(N, k, r)] = f32_to_bf16_bits(W[(size_t)r * N + k] - hf);
        }
      for (int r = 0; r < N; ++r)
        for (int m = 0; m < N / 32; ++m)
          for (int q = 0; q < 4; ++q)
            for (int x = 0; x < 8; ++x)
              Wv[cov_row_pos(N, r, q, m, x)] = W[(size_t)r * N + 8 * cov_row_chunk(N, q, m) + x];
      for (int r = 0; r < N; ++r)
        for (int k = 0; k < N; ++k) Wq[cov_quad_pos(N, r, k)] = W[(size_t)r * N + k];
      e = upload(&L.Wfr, Wfr);
      if (e == hipSuccess) e = upload(&L.Wfrl, Wfrl);
      if (e == hipSuccess) e = upload(&L.Wv, Wv);
      if (e == hipSuccess) e = upload(&L.Wq, Wq);
      if (e == hipSuccess) e = upload(&L.WTfr, WTfr);
      if (e == hipSuccess) e = upload(&L.WTfrl, WTfrl);
    }
    if (e != hipSuccess) {
      for (int k = 0; k <= l; ++k) free_layer(m.L[k]);
      return hip_fail(ctx, e, "isx_load_mlp upload");
    }
  }
  {
    std::vector<DevLayer> table(n_linear);
    for (int l = 0; l < n_linear; ++l)
      table[l] = DevLayer{m.L[l].W,   m.L[l].Wbf, m.L[l].Wfr,  m.L[l].Wfrl,
                          m.L[l].Wv,  m.L[l].Wq,  m.L[l].WTfr, m.L[l].WTfrl,
                          m.L[l].b,   m.L[l].n_in, m.L[l].n_out};
    hipError_t e = upload(&m.dev_layers, table);
    if (e != hipSuccess) {
      for (int k = 0; k < n_linear; ++k) free_layer(m.L[k]);
      free_model_table(m);
      return hip_fail(ctx, e, "isx_load_mlp upload");
    }
  }
  m.live = true;
  for (size_t i = 0; i < ctx->models.size(); ++i) {
    if (!ctx->models[i].live) {
      ctx->models[i] = m;
      *mlp_id = (int32_t)i;
      return ISX_OK;
    }
  }
  ctx->models.push_back(m);
  *mlp_id = (int32_t)ctx->models.size() - 1;
  return ISX_OK;
}

isx_status isx_unload_mlp(isx_ctx* ctx, int32_t mlp_id) {
  Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "no such mlp");
  (void)hipStreamSynchronize(ctx->stream);
  for (int l = 0; l < ISX_MAX_LINEAR; ++l) free_layer(m->L[l]);
  free_model_table(*m);
  m->live = false;
  return ISX_OK;
}

isx_status isx_set_activation(isx_ctx* ctx, int32_t mlp_id, isx_activation act) {
  Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "bad mlp id");
  if (act != ISX_RELU && act != ISX_SINE && act != ISX_ELU) return fail(ctx, ISX_EINVAL, "unknown activation");
  if (act != ISX_RELU)
    for (const Sur& S : ctx->surs)
      if (S.live && S.base_mlp == mlp_id)
        return fail(ctx, ISX_EUNSUPPORTED, "a surrogate uses this MLP's centre linearisation, which needs ReLU");
  m->act = act;
  return ISX_OK;
}

isx_status isx_set_domain(isx_ctx* ctx, int32_t mlp_id, const float h_lo[3], const float h_hi[3]) {
  Model* m = get_model(ctx, mlp_id);
  if (!m || !h_lo || !h_hi) return fail(ctx, ISX_EINVAL, "bad mlp id or null domain");
  if (!finite3(h_lo) || !finite3(h_hi)) return fail(ctx, ISX_ENAN, "non-finite domain");
  for (int a = 0; a < 3; ++a)
    if (!(h_hi[a] > h_lo[a])) return fail(ctx, ISX_EINVAL, "domain hi must exceed lo on every axis");
  for (int a = 0; a < 3; ++a) {
    m->lo[a] = h_lo[a];
    m->hi[a] = h_hi[a];
  }
  return ISX_OK;
}

isx_status isx_set_isovalues(isx_ctx* ctx, int32_t mlp_id, int32_t n_iso, const float* h_iso) {
  Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "bad mlp id");
  if (n_iso < 0 || n_iso > ISX_MAX_ISO || (n_iso > 0 && !h_iso))
    return fail(ctx, ISX_EINVAL, "n_iso must be in [0, " + std::to_string(ISX_MAX_ISO) + "]");
  for (int j = 0; j < n_iso; ++j)
    if (!std::isfinite(h_iso[j])) return fail(ctx, ISX_ENAN, "non-finite iso-value");
  m->n_iso = n_iso;
  for (int j = 0; j < ISX_MAX_ISO; ++j) m->iso[j] = j < n_iso ? h_iso[j] : 0.f;
  return ISX_OK;
}

isx_status isx_propagate(isx_ctx* ctx, int32_t mlp_id, isx_method method, isx_precision precision, int64_t n_cells,
                         const float* d_centres, const float* d_halves, float* d_out, double* d_out64) {
  Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "bad mlp id");
  if (method != ISX_AA && method != ISX_UP && method != ISX_RAUA && method != ISX_RAFIXED)
    return fail(ctx, ISX_EINVAL, "unknown method");
  if (precision != ISX_FP32 && precision != ISX_BF16 && precision != ISX_FP64)
    return fail(ctx, ISX_EINVAL, "unknown precision");
  if (n_cells < 0) return fail(ctx, ISX_EINVAL, "n_cells < 0");
  if (n_cells == 0) return ISX_OK;
  if (!d_centres || !d_halves || !d_out) return fail(ctx, ISX_EINVAL, "null buffer");
  if (d_out64 && precision != ISX_FP64) return fail(ctx, ISX_EINVAL, "d_out64 is only written with ISX_FP64");
  (void)hipSetDevice(ctx->device);
  return run_propagate(ctx, *m, method, precision, n_cells, d_centres, d_halves, d_out, d_out64, 0);
}

static isx_status read_count(isx_ctx* ctx, const int64_t* d, int64_t* h);

isx_status isx_propagate_segments(isx_ctx* ctx, int32_t mlp_id, isx_method method, isx_precision precision,
                                  int64_t n, const float* d_centres, const float* d_halfvec, float* d_out,
                                  double* d_out64) {
  Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "bad mlp id");
  if (method != ISX_AA && method != ISX_UP && method != ISX_RAUA && method != ISX_RAFIXED)
    return fail(ctx, ISX_EINVAL, "unknown method");
  if (precision != ISX_FP32 && precision != ISX_BF16 && precision != ISX_FP64)
    return fail(ctx, ISX_EINVAL, "unknown precision");
  if (n < 0) return fail(ctx, ISX_EINVAL, "n < 0");
  if (n == 0) return ISX_OK;
  if (!d_centres || !d_halfvec || !d_out) return fail(ctx, ISX_EINVAL, "null buffer");
  if (d_out64 && precision != ISX_FP64) return fail(ctx, ISX_EINVAL, "d_out64 is only written with ISX_FP64");
  (void)hipSetDevice(ctx->device);
  return run_propagate(ctx, *m, method, precision, n, d_centres, d_halfvec, d_out, d_out64, 0, 1);
}

// Ray casting (App. A): per step, the active rays are compacted, their
// segments formed and bounded, and the rays advanced, refined or finished.
isx_status isx_raycast(isx_ctx* ctx, int32_t mlp_id, const isx_ray_params* p, int64_t n, const float* d_org,
                       const float* d_dir, const float* d_tnear, const float* d_tfar, float* d_thit,
                       int32_t* d_iters, int64_t* h_stats) {
  Model* m = get_model(ctx, mlp_id);
  if (!m || !p) return fail(ctx, ISX_EINVAL, "bad arguments");
  if (p->method != ISX_AA && p->method != ISX_UP && p->method != ISX_RAUA && p->method != ISX_RAFIXED)
    return fail(ctx, ISX_EINVAL, "unknown method");
  if (p->precision == ISX_BF16) return fail(ctx, ISX_EUNSUPPORTED, "ray casting runs in float32 or float64");
  if (p->precision != ISX_FP32 && p->precision != ISX_FP64) return fail(ctx, ISX_EINVAL, "unknown precision");
  if (!(p->step0 > 0.f) || !(p->step_min > 0.f) || !(p->step_max >= p->step0) || !(p->k >= 0.f) ||
      !std::isfinite(p->k) || !std::isfinite(p->iso) || !std::isfinite(p->step_max) || p->max_iter < 1)
    return fail(ctx, ISX_EINVAL, "ray parameters: need step0, step_min > 0, step_max >= step0, k >= 0, max_iter >= 1");
  if (n < 0) return fail(ctx, ISX_EINVAL, "n_rays < 0");
  if (h_stats) h_stats[0] = h_stats[1] = 0;
  if (n == 0) return ISX_OK;
  if (!d_org || !d_dir || !d_tnear || !d_tfar || !d_thit || !d_iters) return fail(ctx, ISX_EINVAL, "null buffer");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = ctx->stream;
  const bool f64 = p->precision == ISX_FP64;
  const double k = (p->method == ISX_AA || p->method == ISX_RAFIXED) ? 1.0 : (double)p->k;
  HIPCHK(ensure(ctx->ray_t, n * 8));
  HIPCHK(ensure(ctx->ray_dt, n * 8));
  HIPCHK(ensure(ctx->ray_act, n * 4));
  HIPCHK(ensure(ctx->ray_idx, n * 4));
  HIPCHK(ensure(ctx->ray_c, n * 12));
  HIPCHK(ensure(ctx->ray_v, n * 12));
  HIPCHK(ensure(ctx->ray_o32, n * 8));
  if (f64) HIPCHK(ensure(ctx->ray_o64, n * 16));
  HIPCHK(ensure(ctx->ray_cnt, sizeof(int64_t)));
  HIPCHK(ensure(ctx->scan_tmp, compact_tmp_bytes(n)));
  double* t = (double*)ctx->ray_t.p;
  double* dt = (double*)ctx->ray_dt.p;
  uint32_t* act = (uint32_t*)ctx->ray_act.p;
  uint32_t* idx = (uint32_t*)ctx->ray_idx.p;
  HIPCHK(launch_ray_init(n, d_tnear, d_tfar, (double)p->step0, t, dt, d_thit, d_iters, act, s));
  int64_t segments = 0, steps = 0;
  for (int it = 0; it < p->max_iter; ++it) {
    HIPCHK(launch_compact(n, act, nullptr, idx, nullptr, (int64_t*)ctx->ray_cnt.p, ctx->scan_tmp.p, s));
    int64_t n_act = 0;
    isx_status st = read_count(ctx, (const int64_t*)ctx->ray_cnt.p, &n_act);
    if (st != ISX_OK) return st;
    if (n_act == 0) break;
    HIPCHK(launch_ray_segments(n_act, idx, d_org, d_dir, d_tfar, t, dt, (float*)ctx->ray_c.p, (float*)ctx->ray_v.p, s));
    st = run_propagate(ctx, *m, p->method, p->precision, n_act, (const float*)ctx->ray_c.p,
                       (const float*)ctx->ray_v.p, (float*)ctx->ray_o32.p, f64 ? (double*)ctx->ray_o64.p : nullptr,
                       0, 1);
    if (st != ISX_OK) return st;
    HIPCHK(launch_ray_step(n_act, idx, (const float*)ctx->ray_o32.p, f64 ? (const double*)ctx->ray_o64.p : nullptr,
                           k, (double)p->iso, (double)p->step_min, (double)p->step_max, d_tfar, t, dt, d_thit,
                           d_iters, act, s));
    segments += n_act;
    steps = it + 1;
  }
  if (h_stats) {
    h_stats[0] = segments;
    h_stats[1] = steps;
  }
  return ISX_OK;
}

isx_status isx_classify_compact(isx_ctx* ctx, int32_t mlp_id, float k, int64_t n_cells, const float* d_out,
                                const uint32_t* d_parent_mask, uint32_t* d_active_idx, uint32_t* d_active_mask,
                                int64_t* d_n_active) {
  Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "bad mlp id");
  if (!(k >= 0.f) || !std::isfinite(k)) return fail(ctx, ISX_EINVAL, "k must be finite and >= 0");
  if (n_cells < 0 || !d_n_active || (n_cells > 0 && (!d_out || !d_active_idx || !d_active_mask)))
    return fail(ctx, ISX_EINVAL, "bad arguments");
  if (n_cells > (int64_t)UINT32_MAX) return fail(ctx, ISX_ECAPACITY, "n_cells exceeds 2^32-1");
  (void)hipSetDevice(ctx->device);
  HIPCHK(ensure(ctx->cls_mask, (size_t)n_cells * sizeof(uint32_t)));
  HIPCHK(ensure(ctx->scan_tmp, compact_tmp_bytes(n_cells)));
  HIPCHK(launch_classify(n_cells, d_out, k, iso_list(*m), d_parent_mask, (uint32_t*)ctx->cls_mask.p, ctx->stream));
  HIPCHK(launch_compact(n_cells, (const uint32_t*)ctx->cls_mask.p, nullptr, d_active_idx, d_active_mask, d_n_active,
                        ctx->scan_tmp.p, ctx->stream));
  return ISX_OK;
}

isx_status isx_classify_compact_noalloc(isx_ctx* ctx, int32_t mlp_id, float k, int64_t n_cells, const float* d_out,
                                        const uint32_t* d_parent_mask, uint32_t* d_active_idx,
                                        uint32_t* d_active_mask, int64_t* d_n_active) {
  Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "bad mlp id");
  if (!(k >= 0.f) || !std::isfinite(k)) return fail(ctx, ISX_EINVAL, "k must be finite and >= 0");
  if (n_cells < 0 || !d_n_active || (n_cells > 0 && (!d_out || !d_active_idx || !d_active_mask)))
    return fail(ctx, ISX_EINVAL, "bad arguments");
  if (n_cells > (int64_t)ISX_NOALLOC_MAX_CELLS)
    return fail(ctx, ISX_ECAPACITY, "n_cells " + std::to_string(n_cells) + " exceeds ISX_NOALLOC_MAX_CELLS (" +
                                        std::to_string((int64_t)ISX_NOALLOC_MAX_CELLS) + ")");
  (void)hipSetDevice(ctx->device);
  uint8_t* base = static_cast<uint8_t*>(scratch_ptr(ctx->device));
  if (!base) return fail(ctx, ISX_EHIP, "the fixed working memory of this device is not available");
  // every mask entry is written by the classification and every scan
  // partial by the scan before it is read: nothing needs clearing
  uint32_t* cls = reinterpret_cast<uint32_t*>(base);
  void* tmp = base + kNoAllocMaskBytes;
  HIPCHK(launch_classify(n_cells, d_out, k, iso_list(*m), d_parent_mask, cls, ctx->stream));
  HIPCHK(launch_compact(n_cells, cls, nullptr, d_active_idx, d_active_mask, d_n_active, tmp, ctx->stream));
  return ISX_OK;
}

// float32 point evaluation: FP32 MFMA, or the SIMT kernel when forced
static hipError_t eval_f32(isx_ctx* ctx, const Model& m, int64_t n, const float* pts, float* vals, hipStream_t s) {
  if (ctx->kernel_choice == 1) return eval_points_f32(m, n, pts, vals, s);
  double flops = 6.0 * m.widths[1] + 2.0 * m.widths[m.n_linear - 1];
  for (int h = 2; h < m.n_linear; ++h) flops += 2.0 * m.widths[h] * m.widths[h - 1];
  Profiler::Rec rec{};
  const bool prof = ctx->prof.begin(rec, ISX_KERNEL_DENSE, flops * (double)n, 16.0 * n, s);
  hipError_t e = eval_points_mfma(m, n, pts, vals, s);
  if (prof) ctx->prof.end(rec, s);
  return e;
}

isx_status isx_eval_points(isx_ctx* ctx, int32_t mlp_id, isx_precision precision, int64_t n, const float* d_points,
                           float* d_values) {
  Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "bad mlp id");
  if (n < 0 || (n > 0 && (!d_points || !d_values))) return fail(ctx, ISX_EINVAL, "bad arguments");
  (void)hipSetDevice(ctx->device);
  if (precision == ISX_FP64) {
    HIPCHK(eval_points_f64(*m, n, d_points, d_values, ctx->stream));
  } else if (precision == ISX_FP32 || precision == ISX_BF16) {
    HIPCHK(eval_f32(ctx, *m, n, d_points, d_values, ctx->stream));
  } else {
    return fail(ctx, ISX_EINVAL, "unknown precision");
  }
  return ISX_OK;
}

// Distribution-quality report (Sec. V-E, Eq. 11): float64 UP and RA-UA of
// the blocks, then per chunk of blocks the sample points, their float32
// evaluation, statistics, histogram and KL divergences.
isx_status isx_distribution_kl(isx_ctx* ctx, int32_t mlp_id, int64_t n_blocks, const float* d_centres,
                               const float* d_halves, int64_t n_samples, int32_t n_bins, int32_t n_fit,
                               uint64_t seed, double* d_out, uint32_t* d_hist) {
  Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "bad mlp id");
  if (n_blocks < 0 || n_samples < 1 || n_samples >= ((int64_t)1 << 31) || n_bins < 1 || n_bins > 8192 ||
      n_fit < 1 || n_fit > n_samples)
    return fail(ctx, ISX_EINVAL, "distribution report: bad sizes");
  if (n_blocks == 0) return ISX_OK;
  if (!d_centres || !d_halves || !d_out) return fail(ctx, ISX_EINVAL, "distribution report: null buffer");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = ctx->stream;
  HIPCHK(ensure(ctx->ds_o32, (size_t)n_blocks * 8));
  HIPCHK(ensure(ctx->ds_up64, (size_t)n_blocks * 16));
  HIPCHK(ensure(ctx->ds_ra64, (size_t)n_blocks * 16));
  HIPCHK(ensure(ctx->ds_stats, (size_t)n_blocks * 48));
  isx_status st = run_propagate(ctx, *m, ISX_UP, ISX_FP64, n_blocks, d_centres, d_halves, (float*)ctx->ds_o32.p,
                                (double*)ctx->ds_up64.p, 0);
  if (st != ISX_OK) return st;
  st = run_propagate(ctx, *m, ISX_RAUA, ISX_FP64, n_blocks, d_centres, d_halves, (float*)ctx->ds_o32.p,
                     (double*)ctx->ds_ra64.p, 0);
  if (st != ISX_OK) return st;
  const int64_t max_samples = (int64_t)1 << 26;
  const int64_t per = std::max<int64_t>(1, std::min<int64_t>(n_blocks, max_samples / n_samples));
  HIPCHK(ensure(ctx->ds_pts, (size_t)per * n_samples * 12));
  HIPCHK(ensure(ctx->ds_vals, (size_t)per * n_samples * 4));
  for (int64_t b0 = 0; b0 < n_blocks; b0 += per) {
    const int64_t nb = std::min(per, n_blocks - b0);
    HIPCHK(launch_dist_points(nb, b0, n_samples, seed, d_centres, d_halves, (float*)ctx->ds_pts.p, s));
    HIPCHK(eval_f32(ctx, *m, nb * n_samples, (const float*)ctx->ds_pts.p, (float*)ctx->ds_vals.p, s));
    double* stats = (double*)ctx->ds_stats.p + b0 * 6;
    HIPCHK(launch_dist_stats(nb, n_samples, n_fit, (const float*)ctx->ds_vals.p, stats, s));
    HIPCHK(launch_dist_hist_kl(nb, n_samples, n_bins, (const float*)ctx->ds_vals.p, stats,
                               (const double*)ctx->ds_up64.p + b0 * 2, (const double*)ctx->ds_ra64.p + b0 * 2,
                               d_out + b0 * ISX_DIST_FIELDS, d_hist ? d_hist + b0 * n_bins : nullptr, s));
  }
  return ISX_OK;
}

// Centre linearisation of n cells: bf16 split where the option and the
// widths allow, else float32; timed as ISX_KERNEL_LINEARIZE.
static hipError_t linearize_cells(isx_ctx* ctx, const Model& m, int64_t n, const float* centres,
                                  const float* halves, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const bool bf = ctx->lin_prec == 1 && lin_bf16_supported(m);
  double f = 0.0;
  for (int h = 2; h < m.n_linear; ++h) f += 2.0 * m.widths[h] * m.widths[h - 1];
  f *= bf ? 6.0 : 4.0;  // bf16: three centre products and three tangents; float32: four columns
  Profiler::Rec rec{};
  const bool prof = ctx->prof.begin(rec, ISX_KERNEL_LINEARIZE, f * (double)n, 32.0 * n, s);
  hipError_t e = bf ? linearize_bf16(m, n, centres, halves, out, s) : linearize_mfma(m, n, centres, halves, out, s);
  if (prof) ctx->prof.end(rec, s);
  return e;
}

isx_status isx_linearize(isx_ctx* ctx, int32_t mlp_id, int64_t n, const float* d_centres, const float* d_halves,
                         float* d_out) {
  Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "bad mlp id");
  if (m->act != ISX_RELU) return fail(ctx, ISX_EUNSUPPORTED, "the centre linearisation needs a ReLU net");
  if (n < 0 || (n > 0 && (!d_centres || !d_halves || !d_out))) return fail(ctx, ISX_EINVAL, "bad arguments");
  if (n == 0) return ISX_OK;
  (void)hipSetDevice(ctx->device);
  HIPCHK(linearize_cells(ctx, *m, n, d_centres, d_halves, d_out, ctx->stream));
  return ISX_OK;
}

// ---------------------------------------------------------------- extract
static isx_status read_count(isx_ctx* ctx, const int64_t* d, int64_t* h) {
  HIPCHK(hipMemcpyAsync(ctx->h_count, d, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *h = ctx->h_count[0];
  return ISX_OK;
}

// Propagate n cells, classify them (closed soft/hard bound, parent masks) and
// re-check in float64 the cells within the band.  Writes out[n][2], mask[n].
static isx_status prop_classify(isx_ctx* ctx, const Model& m, const isx_params* p, float k, const IsoList& iso,
                                int64_t n, const float* centres, const float* halves, const uint32_t* pmask,
                                float* out, uint32_t* mask, int64_t* n_rc_out, int64_t* n_cancel_out) {
  hipStream_t s = ctx->stream;
  *n_rc_out = 0;
  *n_cancel_out = 0;
  if (n <= 0) return ISX_OK;
  isx_status st = run_propagate(ctx, m, p->method, p->precision, n, centres, halves, out, nullptr, p->chunk_cells);
  if (st != ISX_OK) return st;
  *n_cancel_out = p->precision == ISX_BF16 ? ctx->n_cancel_last : 0;
  HIPCHK(launch_classify(n, out, k, iso, pmask, mask, s));
  if (!(p->fp64_band > 0.f || p->fp64_band_rel > 0.f) || p->precision == ISX_FP64) return ISX_OK;
  HIPCHK(ensure(ctx->rc_flags, n * 4));
  HIPCHK(ensure(ctx->rc_fidx, n * 4));
  HIPCHK(ensure(ctx->rc_count, sizeof(int64_t)));
  HIPCHK(ensure(ctx->scan_tmp, compact_tmp_bytes(n)));
  HIPCHK(launch_band_flags(n, out, k, iso, pmask, p->fp64_band, p->fp64_band_rel, (uint32_t*)ctx->rc_flags.p, s));
  HIPCHK(launch_compact(n, (const uint32_t*)ctx->rc_flags.p, nullptr, (uint32_t*)ctx->rc_fidx.p, nullptr,
                        (int64_t*)ctx->rc_count.p, ctx->scan_tmp.p, s));
  int64_t n_rc = 0;
  st = read_count(ctx, (const int64_t*)ctx->rc_count.p, &n_rc);
  if (st != ISX_OK) return st;
  if (n_rc > 0) {
    HIPCHK(ensure(ctx->rc_centres, n_rc * 12));
    HIPCHK(ensure(ctx->rc_halves, n_rc * 12));
    HIPCHK(ensure(ctx->rc_out32, n_rc * 8));
    HIPCHK(ensure(ctx->rc_out64, n_rc * 16));
    HIPCHK(launch_gather_boxes(n_rc, (const uint32_t*)ctx->rc_fidx.p, centres, halves, (float*)ctx->rc_centres.p,
                               (float*)ctx->rc_halves.p, s));
    int64_t n64 = n_rc;
    if (ctx->recheck_cascade && p->precision == ISX_BF16) {
      // float32 first; float64 only where the float32 bound still lies within
      // an eighth of the band of a carried iso-value (the float32 endpoint
      // error is far below that, so elsewhere both decide alike)
      ctx->f32_split_now = ctx->recheck_split != 0;
      st = run_propagate(ctx, m, p->method, ISX_FP32, n_rc, (const float*)ctx->rc_centres.p,
                         (const float*)ctx->rc_halves.p, (float*)ctx->rc_out32.p, nullptr, p->chunk_cells);
      ctx->f32_split_now = false;
      if (st != ISX_OK) return st;
      HIPCHK(launch_widen_pairs(n_rc, (const float*)ctx->rc_out32.p, (double*)ctx->rc_out64.p, s));
      HIPCHK(ensure(ctx->rc_pm, n_rc * 4));
      HIPCHK(ensure(ctx->rc_flags2, n_rc * 4));
      HIPCHK(ensure(ctx->rc_idx2, n_rc * 4));
      HIPCHK(ensure(ctx->scan_tmp, compact_tmp_bytes(n_rc)));
      const uint32_t* rc_pm = nullptr;
      if (pmask) {
        HIPCHK(gather_u32(n_rc, (const uint32_t*)ctx->rc_fidx.p, pmask, (uint32_t*)ctx->rc_pm.p, s));
        rc_pm = (const uint32_t*)ctx->rc_pm.p;
      }
      HIPCHK(launch_band_flags(n_rc, (const float*)ctx->rc_out32.p, k, iso, rc_pm, 0.125f * p->fp64_band,
                               0.125f * p->fp64_band_rel, (uint32_t*)ctx->rc_flags2.p, s));
      HIPCHK(launch_compact(n_rc, (const uint32_t*)ctx->rc_flags2.p, nullptr, (uint32_t*)ctx->rc_idx2.p, nullptr,
                            (int64_t*)ctx->rc_count.p, ctx->scan_tmp.p, s));
      st = read_count(ctx, (const int64_t*)ctx->rc_count.p, &n64);
      if (st != ISX_OK) return st;
      if (n64 > 0) {
        HIPCHK(ensure(ctx->rc2_c, n64 * 12));
        HIPCHK(ensure(ctx->rc2_h, n64 * 12));
        HIPCHK(ensure(ctx->rc2_out32, n64 * 8));
        HIPCHK(ensure(ctx->rc2_out64, n64 * 16));
        const uint32_t* idx2 = (const uint32_t*)ctx->rc_idx2.p;
        HIPCHK(launch_gather_boxes(n64, idx2, (const float*)ctx->rc_centres.p, (const float*)ctx->rc_halves.p,
                                   (float*)ctx->rc2_c.p, (float*)ctx->rc2_h.p, s));
        st = run_propagate(ctx, m, p->method, ISX_FP64, n64, (const float*)ctx->rc2_c.p, (const float*)ctx->rc2_h.p,
                           (float*)ctx->rc2_out32.p, (double*)ctx->rc2_out64.p, p->chunk_cells);
        if (st != ISX_OK) return st;
        HIPCHK(launch_scatter_pairs(n64, idx2, (const double*)ctx->rc2_out64.p, (double*)ctx->rc_out64.p, s));
      }
    } else {
      st = run_propagate(ctx, m, p->method, ISX_FP64, n_rc, (const float*)ctx->rc_centres.p,
                         (const float*)ctx->rc_halves.p, (float*)ctx->rc_out32.p, (double*)ctx->rc_out64.p,
                         p->chunk_cells);
      if (st != ISX_OK) return st;
    }
    ctx->n_rc64_last += n64;
    HIPCHK(launch_recheck_apply(n_rc, (const uint32_t*)ctx->rc_fidx.p, (const double*)ctx->rc_out64.p, (double)k, iso,
                                pmask, out, mask, s));
  }
  *n_rc_out = n_rc;
  return ISX_OK;
}

static Sur* get_sur(isx_ctx* ctx, int32_t id) {
  if (!ctx || id < 0 || id >= (int32_t)ctx->surs.size() || !ctx->surs[id].live) return nullptr;
  return &ctx->surs[id];
}

// Surrogate forward pass over n cells, (mu_hat, sigma_hat) in field units;
// with a base MLP also the per-cell base scale s_b into sb_out (if given).
static isx_status sur_predict_n(isx_ctx* ctx, Sur& S, int64_t n, const float* centres, const float* halves,
                                float* out, float* sb_out) {
  hipStream_t s = ctx->stream;
  const Model* base = nullptr;
  if (S.base_mlp >= 0) {
    base = get_model(ctx, S.base_mlp);
    if (!base) return fail(ctx, ISX_EINVAL, "the surrogate's base MLP was unloaded");
  }
  const int64_t chunk = std::min<int64_t>(n, (int64_t)1 << 20);
  for (int l = 0; l < S.L; ++l) HIPCHK(ensure(ctx->sur_act[l], (size_t)chunk * S.w[l] * 4));
  HIPCHK(ensure(ctx->sur_out, (size_t)chunk * 8));
  if (base) HIPCHK(ensure(ctx->sp_base, (size_t)chunk * 8));
  for (int64_t r0 = 0; r0 < n; r0 += chunk) {
    const int B = (int)std::min<int64_t>(chunk, n - r0);
    HIPCHK(sur_features(n, r0, B, centres, halves, S.size_a, S.size_b, (float*)ctx->sur_act[0].p, nullptr, 0.f, 1.f,
                        nullptr, 0.f, nullptr, s));
    for (int l = 0; l < S.L; ++l) {
      float* C = l + 1 < S.L ? (float*)ctx->sur_act[l + 1].p : (float*)ctx->sur_out.p;
      HIPCHK(sur_gemm(B, S.w[l + 1], S.w[l], (const float*)ctx->sur_act[l].p, S.w[l], false, S.W[l], S.w[l], true, C,
                      S.w[l + 1], S.b[l], l + 1 < S.L, nullptr, 0, s));
    }
    if (base) HIPCHK(linearize_cells(ctx, *base, B, centres + 3 * r0, halves + 3 * r0, (float*)ctx->sp_base.p, s));
    HIPCHK(sur_unstd(B, (const float*)ctx->sur_out.p, S.mu_bar, S.scale, base ? (const float*)ctx->sp_base.p : nullptr,
                     S.s_floor, out + 2 * r0, sb_out ? sb_out + r0 : nullptr, s));
  }
  return ISX_OK;
}

// Leaf phase shared by the extractions: the leaves (ids, masks on the
// device) are copied into the mesh, their distinct corners evaluated (float64
// for ISX_FP64, else float32) and marching cubes run on every (leaf, iso)
// pair of the masks.  Records ev_inr after the corner values and ev_mc after
// the triangles; on an error the caller frees the mesh.
static isx_status leaf_phase(isx_ctx* ctx, const Model& m, int D, isx_precision prec, int64_t n_leaves,
                             const uint32_t* ids, const uint32_t* masks, isx_mesh* mesh, hipEvent_t ev_inr,
                             hipEvent_t ev_mc) {
  hipStream_t s = ctx->stream;
  mesh->n_leaves = n_leaves;
  HIPCHK(hipMalloc((void**)&mesh->leaf_ids, std::max<int64_t>(1, n_leaves) * 4));
  HIPCHK(hipMalloc((void**)&mesh->leaf_masks, std::max<int64_t>(1, n_leaves) * 4));
  if (n_leaves > 0) {
    HIPCHK(hipMemcpyAsync(mesh->leaf_ids, ids, n_leaves * 4, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(mesh->leaf_masks, masks, n_leaves * 4, hipMemcpyDeviceToDevice, s));
  }
  // corners: bitmap, prefix, list, points, values
  const uint64_t words = corner_bitmap_words(D);
  HIPCHK(ensure(ctx->bitmap, words * 4));
  HIPCHK(ensure(ctx->word_prefix, words * 4));
  HIPCHK(ensure(ctx->scan_tmp, std::max(scan_tmp_bytes((int64_t)words), scan_tmp_bytes(n_leaves * m.n_iso))));
  HIPCHK(launch_corner_mark(D, n_leaves, mesh->leaf_ids, (uint32_t*)ctx->bitmap.p, words, s));
  HIPCHK(launch_corner_list(D, words, (const uint32_t*)ctx->bitmap.p, (uint32_t*)ctx->word_prefix.p,
                          (int64_t*)ctx->count.p, ctx->scan_tmp.p, ctx->scan_tmp.bytes, nullptr, s));
  int64_t n_corners = 0;
  {
    isx_status st = read_count(ctx, (const int64_t*)ctx->count.p, &n_corners);
    if (st != ISX_OK) return st;
  }
  mesh->n_corners = n_corners;
  HIPCHK(ensure(ctx->corner_g, n_corners * 4));
  HIPCHK(ensure(ctx->corner_pts, n_corners * 12));
  HIPCHK(ensure(ctx->corner_vals, n_corners * 4));
  HIPCHK(launch_corner_list(D, words, (const uint32_t*)ctx->bitmap.p, (uint32_t*)ctx->word_prefix.p,
                          (int64_t*)ctx->count.p, ctx->scan_tmp.p, ctx->scan_tmp.bytes, (uint32_t*)ctx->corner_g.p,
                          s));
  HIPCHK(launch_corner_points(m, D, n_corners, (const uint32_t*)ctx->corner_g.p, (float*)ctx->corner_pts.p, s));
  if (prec == ISX_FP64) {
    HIPCHK(eval_points_f64(m, n_corners, (const float*)ctx->corner_pts.p, (float*)ctx->corner_vals.p, s));
  } else {
    HIPCHK(eval_f32(ctx, m, n_corners, (const float*)ctx->corner_pts.p, (float*)ctx->corner_vals.p, s));
  }
  HIPCHK(hipEventRecord(ev_inr, s));
  // marching cubes
  const int64_t pairs = n_leaves * m.n_iso;
  HIPCHK(ensure(ctx->tri_off, std::max<int64_t>(1, pairs) * 4));
  HIPCHK(launch_mc_count(m, D, n_leaves, mesh->leaf_ids, mesh->leaf_masks, (const uint32_t*)ctx->bitmap.p,
                       (const uint32_t*)ctx->word_prefix.p, (const float*)ctx->corner_vals.p, (uint32_t*)ctx->tri_off.p,
                       (int64_t*)ctx->count.p, ctx->scan_tmp.p, ctx->scan_tmp.bytes, s));
  int64_t n_tris = 0;
  {
    isx_status st = read_count(ctx, (const int64_t*)ctx->count.p, &n_tris);
    if (st != ISX_OK) return st;
  }
  mesh->n_tris = n_tris;
  HIPCHK(hipMalloc((void**)&mesh->tri_pos, std::max<int64_t>(1, n_tris) * 36));
  HIPCHK(hipMalloc((void**)&mesh->tri_keys, std::max<int64_t>(1, n_tris) * 24));
  HIPCHK(hipMalloc((void**)&mesh->tri_iso, std::max<int64_t>(1, n_tris) * 4));
  HIPCHK(launch_mc_emit(m, D, n_leaves, mesh->leaf_ids, mesh->leaf_masks, (const uint32_t*)ctx->bitmap.p,
                      (const uint32_t*)ctx->word_prefix.p, (const float*)ctx->corner_vals.p,
                      (const uint32_t*)ctx->tri_off.p, mesh->tri_pos, mesh->tri_keys, mesh->tri_iso, s));
  HIPCHK(hipEventRecord(ev_mc, s));
  return ISX_OK;
}

isx_status isx_extract(isx_ctx* ctx, int32_t mlp_id, const isx_params* p, isx_mesh** out) {
  Model* mp = get_model(ctx, mlp_id);
  if (!mp || !p || !out) return fail(ctx, ISX_EINVAL, "bad arguments");
  *out = nullptr;
  const Model& m = *mp;
  if (p->method != ISX_AA && p->method != ISX_UP && p->method != ISX_RAUA && p->method != ISX_RAFIXED)
    return fail(ctx, ISX_EINVAL, "unknown method");
  if (p->precision != ISX_FP32 && p->precision != ISX_BF16 && p->precision != ISX_FP64)
    return fail(ctx, ISX_EINVAL, "unknown precision");
  if (p->max_depth < 0 || p->max_depth > 10) return fail(ctx, ISX_EINVAL, "max_depth must be in [0, 10]");
  if (!(p->k >= 0.f) || !std::isfinite(p->k)) return fail(ctx, ISX_EINVAL, "k must be finite and >= 0");
  if (!(p->fp64_band >= 0.f) || !(p->fp64_band_rel >= 0.f) || !std::isfinite(p->fp64_band_rel))
    return fail(ctx, ISX_EINVAL, "fp64_band and fp64_band_rel must be >= 0");
  if (m.n_iso < 1) return fail(ctx, ISX_EINVAL, "no iso-values set");
  if (p->tree != 0 && p->tree != 1) return fail(ctx, ISX_EINVAL, "tree must be 0 (octree) or 1 (k-d tree)");
  const bool kd = p->tree == 1;
  // dense subtrees below level dense_from (0: the full refinement)
  const int dense_from = ctx->dense_from > 0 && ctx->dense_from < p->max_depth ? ctx->dense_from : 0;
  if (kd && dense_from) return fail(ctx, ISX_EUNSUPPORTED, "ISX_DENSE_FROM_LEVEL takes the octree");
  if (kd) {
    if (p->use_surrogate) return fail(ctx, ISX_EUNSUPPORTED, "the k-d tree does not take the surrogate");
    const double e0 = (double)m.hi[0] - m.lo[0];
    if ((double)m.hi[1] - m.lo[1] != e0 || (double)m.hi[2] - m.lo[2] != e0)
      return fail(ctx, ISX_EUNSUPPORTED, "the k-d tree needs a cube domain");
  }
  (void)hipSetDevice(ctx->device);
  hipStream_t s = ctx->stream;
  const float k = (p->method == ISX_AA || p->method == ISX_RAFIXED) ? 1.f : p->k;
  const int64_t cap = p->max_cells > 0 ? p->max_cells : (int64_t)1 << 28;
  const IsoList iso = iso_list(m);
  const uint32_t full = m.n_iso >= 32 ? 0xffffffffu : ((1u << m.n_iso) - 1u);

  hipEvent_t ev[4];
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  HIPCHK(hipEventRecord(ev[0], s));

  isx_mesh* mesh = new isx_mesh();
  mesh->depth = p->max_depth;
  mesh->kept = ctx->keep_levels;
  auto bail = [&](isx_status st) {
    isx_mesh_free(mesh);
    for (auto& e : ev) (void)hipEventDestroy(e);
    return st;
  };
#define XCHK(expr)                                   \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return bail(hip_fail(ctx, _e, #expr)); \
  } while (0)

  int64_t n_par = 0;
  int cur = 0;  // parents in act_*[cur]
  const int last_level = kd ? 3 * p->max_depth : (dense_from ? dense_from : p->max_depth);
  for (int L = 0; L <= last_level; ++L) {
    const int64_t n = L == 0 ? 1 : (kd ? 2 : 8) * n_par;
    if (n > cap)
      return bail(fail(ctx, ISX_ECAPACITY, "level " + std::to_string(L) + " has " + std::to_string(n) +
                                               " cells, above max_cells=" + std::to_string(cap)));
    XCHK(ensure(ctx->ids, n * 4));
    XCHK(ensure(ctx->pmask, n * 4));
    XCHK(ensure(ctx->centres, n * 12));
    XCHK(ensure(ctx->halves, n * 12));
    XCHK(ensure(ctx->out, n * 8));
    XCHK(ensure(ctx->mask, n * 4));
    XCHK(ensure(ctx->act_ids[cur ^ 1], n * 4));
    XCHK(ensure(ctx->act_mask[cur ^ 1], n * 4));
    XCHK(ensure(ctx->scan_tmp, compact_tmp_bytes(n)));
    XCHK(ensure(ctx->count, 2 * sizeof(int64_t)));
    uint32_t* ids = (uint32_t*)ctx->ids.p;
    uint32_t* pmask = (uint32_t*)ctx->pmask.p;
    float* centres = (float*)ctx->centres.p;
    float* halves = (float*)ctx->halves.p;
    float* outb = (float*)ctx->out.p;
    uint32_t* mask = (uint32_t*)ctx->mask.p;
    if (L == 0) {
      XCHK(launch_root(m, full, ids, pmask, centres, halves, s));
    } else if (kd) {
      XCHK(launch_children_kd(m, L, n_par, (const uint32_t*)ctx->act_ids[cur].p,
                              (const uint32_t*)ctx->act_mask[cur].p, ids, pmask, centres, halves, s));
    } else {
      XCHK(launch_children(m, L, n_par, (const uint32_t*)ctx->act_ids[cur].p, (const uint32_t*)ctx->act_mask[cur].p,
                           ids, pmask, centres, halves, s));
    }
    int64_t n_rc = 0, n_prop = n, n_cx = 0;
    ctx->n_rc64_last = 0;
    isx_status st = ISX_OK;
    Sur* S = p->use_surrogate ? get_sur(ctx, m.sur_id) : nullptr;
    if (p->use_surrogate && !S) return bail(fail(ctx, ISX_EINVAL, "use_surrogate set but no surrogate attached"));
    if (!S) {
      st = prop_classify(ctx, m, p, k, iso, n, centres, halves, pmask, outb, mask, &n_rc, &n_cx);
      if (st != ISX_OK) return bail(st);
    } else {
      // surrogate decides the confident cells, the others are propagated
      XCHK(ensure(ctx->sp_pred, n * 8));
      XCHK(ensure(ctx->sp_fb, n * 4));
      XCHK(ensure(ctx->sp_idx, n * 4));
      XCHK(ensure(ctx->sp_cnt, sizeof(int64_t)));
      const bool based = S->base_mlp >= 0;
      if (based) XCHK(ensure(ctx->sp_scale, n * 4));
      float* unit = based ? (float*)ctx->sp_scale.p : nullptr;
      st = sur_predict_n(ctx, *S, n, centres, halves, (float*)ctx->sp_pred.p, unit);
      if (st != ISX_OK) return bail(st);
      const int Ls = std::min(L, std::max(0, m.sur_levels - 1));
      XCHK(sur_partition(n, (const float*)ctx->sp_pred.p, unit, k, iso, pmask, m.sur_err_mu[Ls], m.sur_err_ls[Ls], m.sur_z[Ls], m.sur_z_acc[Ls],
                         L == p->max_depth ? 1 : 0, m.sur_accept_leaves, mask, (uint32_t*)ctx->sp_fb.p, s));
      XCHK(hipMemcpyAsync(outb, ctx->sp_pred.p, n * 8, hipMemcpyDeviceToDevice, s));
      XCHK(launch_compact(n, (const uint32_t*)ctx->sp_fb.p, nullptr, (uint32_t*)ctx->sp_idx.p, nullptr,
                          (int64_t*)ctx->sp_cnt.p, ctx->scan_tmp.p, s));
      int64_t n_fb = 0;
      st = read_count(ctx, (const int64_t*)ctx->sp_cnt.p, &n_fb);
      if (st != ISX_OK) return bail(st);
      if (n_fb > 0) {
        XCHK(ensure(ctx->sp_c, n_fb * 12));
        XCHK(ensure(ctx->sp_h, n_fb * 12));
        XCHK(ensure(ctx->sp_pm, n_fb * 4));
        XCHK(ensure(ctx->sp_out, n_fb * 8));
        XCHK(ensure(ctx->sp_mask, n_fb * 4));
        const uint32_t* fidx = (const uint32_t*)ctx->sp_idx.p;
        XCHK(launch_gather_boxes(n_fb, fidx, centres, halves, (float*)ctx->sp_c.p, (float*)ctx->sp_h.p, s));
        XCHK(gather_u32(n_fb, fidx, pmask, (uint32_t*)ctx->sp_pm.p, s));
        st = prop_classify(ctx, m, p, k, iso, n_fb, (const float*)ctx->sp_c.p, (const float*)ctx->sp_h.p,
                           (const uint32_t*)ctx->sp_pm.p, (float*)ctx->sp_out.p, (uint32_t*)ctx->sp_mask.p, &n_rc,
                           &n_cx);
        if (st != ISX_OK) return bail(st);
        XCHK(scatter_u32(n_fb, fidx, (const uint32_t*)ctx->sp_mask.p, mask, s));
        XCHK(scatter_u64(n_fb, fidx, (const uint64_t*)ctx->sp_out.p, (uint64_t*)outb, s));
      }
      n_prop = n_fb;
    }
    XCHK(launch_compact(n, mask, ids, (uint32_t*)ctx->act_ids[cur ^ 1].p, (uint32_t*)ctx->act_mask[cur ^ 1].p,
                        (int64_t*)ctx->count.p, ctx->scan_tmp.p, s));
    int64_t n_act = 0;
    st = read_count(ctx, (const int64_t*)ctx->count.p, &n_act);
    if (st != ISX_OK) return bail(st);
    mesh->lvl_cells.push_back(n);
    mesh->lvl_active.push_back(n_act);
    mesh->lvl_recheck.push_back(n_rc);
    mesh->lvl_prop.push_back(n_prop);
    mesh->lvl_cancel.push_back(n_cx);
    mesh->lvl_recheck64.push_back(ctx->n_rc64_last);
    if (ctx->verbose) {
      std::fprintf(stderr, "isx: level %d: %lld cells, %lld active, %lld propagated, %lld re-checked, %lld cancelled\n",
                   L, (long long)n, (long long)n_act, (long long)n_prop, (long long)n_rc, (long long)n_cx);
      std::fflush(stderr);
    }
    if (ctx->keep_levels) {
      std::vector<uint32_t> hi(n), hm(n);
      std::vector<float> ho(2 * n);
      XCHK(hipMemcpyAsync(hi.data(), ids, n * 4, hipMemcpyDeviceToHost, s));
      XCHK(hipMemcpyAsync(hm.data(), mask, n * 4, hipMemcpyDeviceToHost, s));
      XCHK(hipMemcpyAsync(ho.data(), outb, n * 8, hipMemcpyDeviceToHost, s));
      XCHK(hipStreamSynchronize(s));
      mesh->lvl_ids.push_back(std::move(hi));
      mesh->lvl_masks.push_back(std::move(hm));
      mesh->lvl_out.push_back(std::move(ho));
    }
    cur ^= 1;
    n_par = n_act;
  }
  // k-d leaves (node depth 3 D) are octree cells of level D: Morton ids
  if (kd) XCHK(launch_kd_to_morton(n_par, p->max_depth, (uint32_t*)ctx->act_ids[cur].p, s));
  XCHK(hipEventRecord(ev[1], s));

  if (dense_from) {
    // every max_depth cell below an active level-dense_from cell is a leaf
    const int sub = p->max_depth - dense_from;
    const int64_t n_leaves = n_par << (3 * sub);
    if (n_leaves > ((int64_t)1 << 28) || n_leaves * m.n_iso > ((int64_t)1 << 31))
      return bail(fail(ctx, ISX_ECAPACITY, "the subtrees below level " + std::to_string(dense_from) + " hold " +
                                               std::to_string(n_leaves) + " leaves, above 2^28 (or 2^31 pairs)"));
    XCHK(ensure(ctx->ids, n_leaves * 4));
    XCHK(ensure(ctx->mask, n_leaves * 4));
    XCHK(launch_subtree_leaves(n_par, sub, (const uint32_t*)ctx->act_ids[cur].p, (const uint32_t*)ctx->act_mask[cur].p,
                               (uint32_t*)ctx->ids.p, (uint32_t*)ctx->mask.p, s));
    isx_status st = leaf_phase(ctx, m, p->max_depth, p->precision, n_leaves, (const uint32_t*)ctx->ids.p,
                               (const uint32_t*)ctx->mask.p, mesh, ev[2], ev[3]);
    if (st != ISX_OK) return bail(st);
  } else {
    isx_status st = leaf_phase(ctx, m, p->max_depth, p->precision, n_par, (const uint32_t*)ctx->act_ids[cur].p,
                               (const uint32_t*)ctx->act_mask[cur].p, mesh, ev[2], ev[3]);
    if (st != ISX_OK) return bail(st);
  }
  XCHK(hipEventSynchronize(ev[3]));
  float t01 = 0, t12 = 0, t23 = 0, t03 = 0;
  XCHK(hipEventElapsedTime(&t01, ev[0], ev[1]));
  XCHK(hipEventElapsedTime(&t12, ev[1], ev[2]));
  XCHK(hipEventElapsedTime(&t23, ev[2], ev[3]));
  XCHK(hipEventElapsedTime(&t03, ev[0], ev[3]));
  mesh->ms_acp = t01;
  mesh->ms_inr = t12;
  mesh->ms_mc = t23;
  mesh->ms_total = t03;
  for (auto& e : ev) (void)hipEventDestroy(e);
#undef XCHK
  *out = mesh;
  return ISX_OK;
}

isx_status isx_extract_dense(isx_ctx* ctx, int32_t mlp_id, int32_t depth, isx_precision precision,
                             isx_mesh** out) {
  Model* mp = get_model(ctx, mlp_id);
  if (!mp || !out) return fail(ctx, ISX_EINVAL, "bad arguments");
  *out = nullptr;
  const Model& m = *mp;
  if (precision != ISX_FP32 && precision != ISX_BF16 && precision != ISX_FP64)
    return fail(ctx, ISX_EINVAL, "unknown precision");
  if (depth < 0 || depth > 10) return fail(ctx, ISX_EINVAL, "depth must be in [0, 10]");
  if (m.n_iso < 1) return fail(ctx, ISX_EINVAL, "no iso-values set");
  const int64_t n = (int64_t)1 << (3 * depth);
  if (n > ((int64_t)1 << 28) || n * m.n_iso > ((int64_t)1 << 31))
    return fail(ctx, ISX_ECAPACITY, "the dense grid of depth " + std::to_string(depth) + " with " +
                                        std::to_string(m.n_iso) + " iso-values exceeds 2^28 cells or 2^31 pairs");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = ctx->stream;
  const uint32_t full = m.n_iso >= 32 ? 0xffffffffu : ((1u << m.n_iso) - 1u);
  hipEvent_t ev[4];
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  isx_mesh* mesh = new isx_mesh();
  mesh->depth = depth;
  auto bail = [&](isx_status st) {
    isx_mesh_free(mesh);
    for (auto& e : ev) (void)hipEventDestroy(e);
    return st;
  };
#define XCHK(expr)                                               \
  do {                                                           \
    hipError_t _e = (expr);                                      \
    if (_e != hipSuccess) return bail(hip_fail(ctx, _e, #expr)); \
  } while (0)
  XCHK(hipEventRecord(ev[0], s));
  XCHK(ensure(ctx->act_ids[0], n * 4));
  XCHK(ensure(ctx->act_mask[0], n * 4));
  XCHK(ensure(ctx->count, 2 * sizeof(int64_t)));
  XCHK(launch_dense_leaves(n, full, (uint32_t*)ctx->act_ids[0].p, (uint32_t*)ctx->act_mask[0].p, s));
  XCHK(hipEventRecord(ev[1], s));
  {
    isx_status st = leaf_phase(ctx, m, depth, precision, n, (const uint32_t*)ctx->act_ids[0].p,
                               (const uint32_t*)ctx->act_mask[0].p, mesh, ev[2], ev[3]);
    if (st != ISX_OK) return bail(st);
  }
  XCHK(hipEventSynchronize(ev[3]));
  float t01 = 0, t12 = 0, t23 = 0, t03 = 0;
  XCHK(hipEventElapsedTime(&t01, ev[0], ev[1]));
  XCHK(hipEventElapsedTime(&t12, ev[1], ev[2]));
  XCHK(hipEventElapsedTime(&t23, ev[2], ev[3]));
  XCHK(hipEventElapsedTime(&t03, ev[0], ev[3]));
  mesh->ms_acp = t01;
  mesh->ms_inr = t12;
  mesh->ms_mc = t23;
  mesh->ms_total = t03;
  for (auto& e : ev) (void)hipEventDestroy(e);
#undef XCHK
  *out = mesh;
  return ISX_OK;
}

// Batched extraction: the INRs are dealt to up to ISX_BATCH_WORKERS worker
// contexts, each with its own stream and level scratch, driven by one host
// thread each, so that the level loops of different INRs (small launches and
// host reads of level counts) overlap on the device.
static isx_status make_worker(isx_ctx* ctx, isx_ctx** out) {
  isx_ctx* w = new isx_ctx();
  w->device = ctx->device;
  w->borrowed = true;
  w->own_stream = true;
  hipError_t e = hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipHostMalloc((void**)&w->h_count, 4 * sizeof(int64_t), hipHostMallocDefault);
  if (e != hipSuccess) {
    if (w->stream) (void)hipStreamDestroy(w->stream);
    delete w;
    return hip_fail(ctx, e, "batch worker");
  }
  *out = w;
  return ISX_OK;
}

isx_status isx_extract_batch(isx_ctx* ctx, int32_t n, const int32_t* mlp_ids, const isx_params* p,
                             isx_mesh** out) {
  if (!ctx || n < 0 || (n > 0 && (!mlp_ids || !p || !out))) return fail(ctx, ISX_EINVAL, "bad arguments");
  for (int32_t i = 0; i < n; ++i) {
    out[i] = nullptr;
    if (!get_model(ctx, mlp_ids[i])) return fail(ctx, ISX_EINVAL, "bad mlp id at " + std::to_string(i));
  }
  if (n == 0) return ISX_OK;
  (void)hipSetDevice(ctx->device);
  // the caller's stream may hold work the INRs depend on
  HIPCHK(hipStreamSynchronize(ctx->stream));
  // tile shapes are timed here, one model at a time, so that the timing
  // runs alone on the device
  if (ctx->autotune && p->precision == ISX_BF16 && ctx->bf16_variant == 0) {
    for (int32_t i = 0; i < n; ++i) {
      const Model& mi = *get_model(ctx, mlp_ids[i]);
      if (mi.act != ISX_RELU || !bf16_supported(mi)) continue;
      if ((p->method == ISX_UP && ctx->up_form == 0 && cov_supported(mi))) continue;
      const isx_status st = tune_bf16(ctx, mi);
      if (st != ISX_OK) return st;
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  const int nw = std::min<int>(ctx->batch_workers, n);
  while ((int)ctx->workers.size() < nw) {
    isx_ctx* w = nullptr;
    const isx_status st = make_worker(ctx, &w);
    if (st != ISX_OK) return st;
    ctx->workers.push_back(w);
  }
  for (int i = 0; i < nw; ++i) {
    isx_ctx* w = ctx->workers[i];
    w->models = ctx->models;
    w->surs = ctx->surs;
    w->kernel_choice = ctx->kernel_choice;
    w->bf16_variant = ctx->bf16_variant;
    w->autotune = ctx->autotune;
    w->readoff_f32 = ctx->readoff_f32;
    w->recheck_cascade = ctx->recheck_cascade;
    w->recheck_split = ctx->recheck_split;
    w->dense_from = ctx->dense_from;
    w->up_form = ctx->up_form;
    w->lin_prec = ctx->lin_prec;
    w->aa_margin = ctx->aa_margin;
    w->cancel_check = ctx->cancel_check;
    w->keep_levels = ctx->keep_levels;
    w->verbose = false;
    w->prop_budget = std::max<size_t>(size_t(1) << 28, ctx->prop_budget / nw);
  }
  std::atomic<int32_t> next{0};
  std::vector<isx_status> st(nw, ISX_OK);
  std::vector<std::string> err(nw);
  auto run = [&](int wi) {
    isx_ctx* w = ctx->workers[wi];
    (void)hipSetDevice(w->device);
    for (int32_t i = next.fetch_add(1); i < n; i = next.fetch_add(1)) {
      const isx_status s = isx_extract(w, mlp_ids[i], p, &out[i]);
      if (s != ISX_OK) {
        st[wi] = s;
        err[wi] = "INR " + std::to_string(i) + ": " + w->err;
        next.store(n);
        return;
      }
    }
  };
  std::vector<std::thread> threads;
  for (int wi = 1; wi < nw; ++wi) threads.emplace_back(run, wi);
  run(0);
  for (std::thread& t : threads) t.join();
  for (int wi = 0; wi < nw; ++wi) {
    if (st[wi] != ISX_OK) {
      for (int32_t i = 0; i < n; ++i) {
        if (out[i]) isx_mesh_free(out[i]);
        out[i] = nullptr;
      }
      return fail(ctx, st[wi], err[wi]);
    }
  }
  return ISX_OK;
}

isx_status isx_mesh_info(const isx_mesh* mesh, int64_t* n_tris, int64_t* n_leaves, int64_t* n_corners,
                         int32_t* n_levels) {
  if (!mesh) return ISX_EINVAL;
  if (n_tris) *n_tris = mesh->n_tris;
  if (n_leaves) *n_leaves = mesh->n_leaves;
  if (n_corners) *n_corners = mesh->n_corners;
  if (n_levels) *n_levels = (int32_t)mesh->lvl_cells.size();
  return ISX_OK;
}

isx_status isx_mesh_level(const isx_mesh* mesh, int32_t level, int64_t* n_cells, int64_t* n_active,
                          int64_t* n_rechecked, int64_t* n_propagated) {
  if (!mesh || level < 0 || level >= (int32_t)mesh->lvl_cells.size()) return ISX_EINVAL;
  if (n_cells) *n_cells = mesh->lvl_cells[level];
  if (n_active) *n_active = mesh->lvl_active[level];
  if (n_rechecked) *n_rechecked = mesh->lvl_recheck[level];
  if (n_propagated) *n_propagated = mesh->lvl_prop[level];
  return ISX_OK;
}

isx_status isx_mesh_level_cancelled(const isx_mesh* mesh, int32_t level, int64_t* n_cancelled) {
  if (!mesh || !n_cancelled || level < 0 || level >= (int32_t)mesh->lvl_cancel.size()) return ISX_EINVAL;
  *n_cancelled = mesh->lvl_cancel[level];
  return ISX_OK;
}

isx_status isx_mesh_level_rechecked_fp64(const isx_mesh* mesh, int32_t level, int64_t* n_fp64) {
  if (!mesh || !n_fp64 || level < 0 || level >= (int32_t)mesh->lvl_recheck64.size()) return ISX_EINVAL;
  *n_fp64 = mesh->lvl_recheck64[level];
  return ISX_OK;
}

isx_status isx_mesh_times(const isx_mesh* mesh, float* ms_acp, float* ms_inr, float* ms_mc, float* ms_total) {
  if (!mesh) return ISX_EINVAL;
  if (ms_acp) *ms_acp = mesh->ms_acp;
  if (ms_inr) *ms_inr = mesh->ms_inr;
  if (ms_mc) *ms_mc = mesh->ms_mc;
  if (ms_total) *ms_total = mesh->ms_total;
  return ISX_OK;
}

isx_status isx_mesh_copy_tris(const isx_mesh* mesh, float* h_pos, uint64_t* h_keys, int32_t* h_iso) {
  if (!mesh) return ISX_EINVAL;
  if (mesh->n_tris == 0) return ISX_OK;
  if (h_pos && hipMemcpy(h_pos, mesh->tri_pos, mesh->n_tris * 36, hipMemcpyDeviceToHost) != hipSuccess) return ISX_EHIP;
  if (h_keys && hipMemcpy(h_keys, mesh->tri_keys, mesh->n_tris * 24, hipMemcpyDeviceToHost) != hipSuccess)
    return ISX_EHIP;
  if (h_iso && hipMemcpy(h_iso, mesh->tri_iso, mesh->n_tris * 4, hipMemcpyDeviceToHost) != hipSuccess) return ISX_EHIP;
  return ISX_OK;
}

isx_status isx_mesh_copy_leaves(const isx_mesh* mesh, uint32_t* h_ids, uint32_t* h_masks) {
  if (!mesh) return ISX_EINVAL;
  if (mesh->n_leaves == 0) return ISX_OK;
  if (h_ids && hipMemcpy(h_ids, mesh->leaf_ids, mesh->n_leaves * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return ISX_EHIP;
  if (h_masks && hipMemcpy(h_masks, mesh->leaf_masks, mesh->n_leaves * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return ISX_EHIP;
  return ISX_OK;
}

isx_status isx_mesh_copy_level(const isx_mesh* mesh, int32_t level, uint32_t* h_ids, float* h_out,
                               uint32_t* h_masks) {
  if (!mesh || level < 0 || level >= (int32_t)mesh->lvl_cells.size()) return ISX_EINVAL;
  if (!mesh->kept) return ISX_EUNSUPPORTED;
  const size_t n = mesh->lvl_ids[level].size();
  if (h_ids) std::memcpy(h_ids, mesh->lvl_ids[level].data(), n * 4);
  if (h_masks) std::memcpy(h_masks, mesh->lvl_masks[level].data(), n * 4);
  if (h_out) std::memcpy(h_out, mesh->lvl_out[level].data(), n * 8);
  return ISX_OK;
}

isx_status isx_mesh_free(isx_mesh* mesh) {
  if (!mesh) return ISX_EINVAL;
  void* ps[] = {mesh->leaf_ids, mesh->leaf_masks, mesh->tri_pos, mesh->tri_keys, mesh->tri_iso};
  for (void* q : ps)
    if (q) (void)hipFree(q);
  delete mesh;
  return ISX_OK;
}

isx_status isx_surrogate_load(isx_ctx* ctx, int32_t n_linear, const int32_t* widths, const float* const* h_W,
                              const float* const* h_b, int32_t* sur_id) {
  if (!ctx || !widths || !h_W || !h_b || !sur_id) return fail(ctx, ISX_EINVAL, "null argument");
  if (n_linear < 1 || n_linear > ISX_MAX_LINEAR) return fail(ctx, ISX_ESHAPE, "bad surrogate depth");
  if (widths[0] != 4 || widths[n_linear] != 2) return fail(ctx, ISX_ESHAPE, "surrogate widths must be 4 -> ... -> 2");
  for (int l = 1; l < n_linear; ++l)
    if (widths[l] < 1 || widths[l] > ISX_MAX_WIDTH) return fail(ctx, ISX_ESHAPE, "bad surrogate hidden width");
  for (int l = 0; l < n_linear; ++l) {
    if (!h_W[l] || !h_b[l]) return fail(ctx, ISX_EINVAL, "null weight pointer");
    for (int64_t i = 0; i < (int64_t)widths[l] * widths[l + 1]; ++i)
      if (!std::isfinite(h_W[l][i])) return fail(ctx, ISX_ENAN, "non-finite surrogate weight");
    for (int i = 0; i < widths[l + 1]; ++i)
      if (!std::isfinite(h_b[l][i])) return fail(ctx, ISX_ENAN, "non-finite surrogate bias");
  }
  (void)hipSetDevice(ctx->device);
  Sur S;
  S.L = n_linear;
  for (int l = 0; l <= n_linear; ++l) S.w[l] = widths[l];
  for (int l = 0; l < n_linear; ++l) {
    const size_t nw = (size_t)widths[l] * widths[l + 1], nb = (size_t)widths[l + 1];
    std::vector<float> W(h_W[l], h_W[l] + nw), b(h_b[l], h_b[l] + nb), zw(nw, 0.f), zb(nb, 0.f);
    hipError_t e = upload(&S.W[l], W);
    if (e == hipSuccess) e = upload(&S.b[l], b);
    if (e == hipSuccess) e = upload(&S.mW[l], zw);
    if (e == hipSuccess) e = upload(&S.vW[l], zw);
    if (e == hipSuccess) e = upload(&S.gW[l], zw);
    if (e == hipSuccess) e = upload(&S.mb[l], zb);
    if (e == hipSuccess) e = upload(&S.vb[l], zb);
    if (e == hipSuccess) e = upload(&S.gb[l], zb);
    if (e != hipSuccess) return hip_fail(ctx, e, "isx_surrogate_load upload");
  }
  S.live = true;
  ctx->surs.push_back(S);
  *sur_id = (int32_t)ctx->surs.size() - 1;
  return ISX_OK;
}

isx_status isx_surrogate_free(isx_ctx* ctx, int32_t sur_id) {
  Sur* S = get_sur(ctx, sur_id);
  if (!S) return fail(ctx, ISX_EINVAL, "no such surrogate");
  (void)hipStreamSynchronize(ctx->stream);
  for (int l = 0; l < S->L; ++l) {
    float* ps[] = {S->W[l], S->b[l], S->mW[l], S->vW[l], S->mb[l], S->vb[l], S->gW[l], S->gb[l]};
    for (float* q : ps)
      if (q) (void)hipFree(q);
  }
  *S = Sur{};
  for (Model& m : ctx->models)
    if (m.sur_id == sur_id) m.sur_id = -1;
  return ISX_OK;
}

isx_status isx_surrogate_save_file(isx_ctx* ctx, int32_t sur_id, const char* path) {
  Sur* S = get_sur(ctx, sur_id);
  if (!S || !path) return fail(ctx, ISX_EINVAL, "bad surrogate id or path");
  std::vector<std::vector<float>> W(S->L), b(S->L);
  std::vector<float*> pw(S->L), pb(S->L);
  for (int l = 0; l < S->L; ++l) {
    W[l].resize((size_t)S->w[l + 1] * S->w[l]);
    b[l].resize(S->w[l + 1]);
    pw[l] = W[l].data();
    pb[l] = b[l].data();
  }
  const isx_status st = isx_surrogate_get(ctx, sur_id, pw.data(), pb.data());
  if (st != ISX_OK) return st;
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(ctx, ISX_EINVAL, std::string("cannot write ") + path);
  bool ok = std::fwrite("ISXSUR01", 1, 8, f) == 8;
  const int32_t L = S->L, has_base = S->base_mlp >= 0 ? 1 : 0;
  const float norm[5] = {S->mu_bar, S->scale, S->size_a, S->size_b, S->s_floor};
  ok = ok && std::fwrite(&L, 4, 1, f) == 1 && std::fwrite(S->w, 4, L + 1, f) == (size_t)(L + 1) &&
       std::fwrite(norm, 4, 5, f) == 5 && std::fwrite(&has_base, 4, 1, f) == 1;
  for (int l = 0; ok && l < L; ++l)
    ok = std::fwrite(W[l].data(), 4, W[l].size(), f) == W[l].size() &&
         std::fwrite(b[l].data(), 4, b[l].size(), f) == b[l].size();
  ok = (std::fclose(f) == 0) && ok;
  return ok ? ISX_OK : fail(ctx, ISX_EINVAL, std::string("write failed: ") + path);
}

isx_status isx_surrogate_load_file(isx_ctx* ctx, const char* path, int32_t base_mlp_id, int32_t* sur_id) {
  if (!ctx || !path || !sur_id) return fail(ctx, ISX_EINVAL, "bad arguments");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(ctx, ISX_EINVAL, std::string("cannot read ") + path);
  char magic[8];
  int32_t L = 0, has_base = 0;
  int32_t w[ISX_MAX_LINEAR + 1] = {};
  float norm[5] = {};
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "ISXSUR01", 8) == 0 &&
            std::fread(&L, 4, 1, f) == 1 && L >= 1 && L <= ISX_MAX_LINEAR &&
            std::fread(w, 4, L + 1, f) == (size_t)(L + 1) && std::fread(norm, 4, 5, f) == 5 &&
            std::fread(&has_base, 4, 1, f) == 1;
  for (int l = 0; ok && l <= L; ++l) ok = w[l] >= 1 && w[l] <= 4096;
  std::vector<std::vector<float>> W, b;
  if (ok) {
    W.resize(L);
    b.resize(L);
    for (int l = 0; ok && l < L; ++l) {
      W[l].resize((size_t)w[l + 1] * w[l]);
      b[l].resize(w[l + 1]);
      ok = std::fread(W[l].data(), 4, W[l].size(), f) == W[l].size() &&
           std::fread(b[l].data(), 4, b[l].size(), f) == b[l].size();
    }
  }
  std::fclose(f);
  if (!ok) return fail(ctx, ISX_EINVAL, std::string("malformed surrogate file ") + path);
  if ((has_base != 0) != (base_mlp_id >= 0))
    return fail(ctx, ISX_EINVAL, has_base ? "the file's surrogate needs a base MLP" : "the file has no base");
  std::vector<const float*> pw(L), pb(L);
  for (int l = 0; l < L; ++l) {
    pw[l] = W[l].data();
    pb[l] = b[l].data();
  }
  int32_t id = -1;
  isx_status st = isx_surrogate_load(ctx, L, w, pw.data(), pb.data(), &id);
  if (st == ISX_OK) st = isx_surrogate_set_norm(ctx, id, norm[0], norm[1], norm[2], norm[3]);
  if (st == ISX_OK && has_base) st = isx_surrogate_set_base(ctx, id, base_mlp_id, norm[4]);
  if (st != ISX_OK) {
    if (id >= 0) (void)isx_surrogate_free(ctx, id);
    return st;
  }
  *sur_id = id;
  return ISX_OK;
}

isx_status isx_surrogate_get(isx_ctx* ctx, int32_t sur_id, float* const* h_W, float* const* h_b) {
  Sur* S = get_sur(ctx, sur_id);
  if (!S || !h_W || !h_b) return fail(ctx, ISX_EINVAL, "bad arguments");
  (void)hipSetDevice(ctx->device);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int l = 0; l < S->L; ++l) {
    HIPCHK(hipMemcpy(h_W[l], S->W[l], (size_t)S->w[l] * S->w[l + 1] * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(h_b[l], S->b[l], (size_t)S->w[l + 1] * 4, hipMemcpyDeviceToHost));
  }
  return ISX_OK;
}

isx_status isx_surrogate_set_norm(isx_ctx* ctx, int32_t sur_id, float mu_bar, float scale, float size_a,
                                  float size_b) {
  Sur* S = get_sur(ctx, sur_id);
  if (!S) return fail(ctx, ISX_EINVAL, "no such surrogate");
  if (!std::isfinite(mu_bar) || !(scale > 0.f) || !std::isfinite(scale) || !std::isfinite(size_a) ||
      !std::isfinite(size_b))
    return fail(ctx, ISX_EINVAL, "bad normalisation");
  S->mu_bar = mu_bar;
  S->scale = scale;
  S->size_a = size_a;
  S->size_b = size_b;
  return ISX_OK;
}

// One forward and backward pass on rows [r0, r0 + batch) (wrapping) of the
// training set; leaves the gradients in S.gW / S.gb.
static isx_status sur_fwd_bwd(isx_ctx* ctx, Sur& S, int64_t n, const float* d_centres, const float* d_halves,
                              const float* d_targets, const float* d_base, int64_t r0, int batch, float* d_loss) {
  hipStream_t s = ctx->stream;
  int wmax = 2;
  for (int l = 0; l <= S.L; ++l) wmax = std::max(wmax, S.w[l]);
  for (int l = 0; l < S.L; ++l) HIPCHK(ensure(ctx->sur_act[l], (size_t)batch * S.w[l] * 4));
  HIPCHK(ensure(ctx->sur_out, (size_t)batch * 8));
  HIPCHK(ensure(ctx->sur_T, (size_t)batch * 8));
  HIPCHK(ensure(ctx->sur_d[0], (size_t)batch * wmax * 4));
  HIPCHK(ensure(ctx->sur_d[1], (size_t)batch * wmax * 4));
  HIPCHK(sur_features(n, r0, batch, d_centres, d_halves, S.size_a, S.size_b, (float*)ctx->sur_act[0].p, d_targets,
                      S.mu_bar, S.scale, d_base, S.s_floor, (float*)ctx->sur_T.p, s));
  for (int l = 0; l < S.L; ++l) {
    float* C = l + 1 < S.L ? (float*)ctx->sur_act[l + 1].p : (float*)ctx->sur_out.p;
    HIPCHK(sur_gemm(batch, S.w[l + 1], S.w[l], (const float*)ctx->sur_act[l].p, S.w[l], false, S.W[l], S.w[l], true, C,
                    S.w[l + 1], S.b[l], l + 1 < S.L, nullptr, 0, s));
  }
  int cur = 0;
  HIPCHK(sur_loss(batch, (const float*)ctx->sur_out.p, (const float*)ctx->sur_T.p, (float*)ctx->sur_d[cur].p, d_loss,
                  s));
  for (int l = S.L - 1; l >= 0; --l) {
    const float* dY = (const float*)ctx->sur_d[cur].p;
    // dW = dY^T H_l,  db = column sums of dY,  dH_l = (dY W_l) . [H_l > 0]
    {
      // (K = batch rows against a few output tiles: split K)
      const size_t we = (size_t)sur_gemm_splits(S.w[l + 1], S.w[l], batch) * S.w[l + 1] * S.w[l];
      HIPCHK(ensure(ctx->sur_work, we * 4));
      HIPCHK(sur_gemm_splitk(S.w[l + 1], S.w[l], batch, dY, S.w[l + 1], true, (const float*)ctx->sur_act[l].p,
                             S.w[l], false, S.gW[l], S.w[l], (float*)ctx->sur_work.p, we, s));
    }
    HIPCHK(sur_colsum(batch, S.w[l + 1], dY, S.gb[l], s));
    if (l > 0) {
      HIPCHK(sur_gemm(batch, S.w[l], S.w[l + 1], dY, S.w[l + 1], false, S.W[l], S.w[l], false,
                      (float*)ctx->sur_d[cur ^ 1].p, S.w[l], nullptr, false, (const float*)ctx->sur_act[l].p, S.w[l],
                      s));
      cur ^= 1;
    }
  }
  return ISX_OK;
}

// Base (f, s) of all n training cells when the surrogate has a base MLP.
static isx_status sur_train_base(isx_ctx* ctx, const Sur& S, int64_t n, const float* d_centres,
                                 const float* d_halves, const float** d_base) {
  *d_base = nullptr;
  if (S.base_mlp < 0) return ISX_OK;
  const Model* base = get_model(ctx, S.base_mlp);
  if (!base) return fail(ctx, ISX_EINVAL, "the surrogate's base MLP was unloaded");
  HIPCHK(ensure(ctx->sur_base, (size_t)n * 8));
  HIPCHK(linearize_cells(ctx, *base, n, d_centres, d_halves, (float*)ctx->sur_base.p, ctx->stream));
  *d_base = (const float*)ctx->sur_base.p;
  return ISX_OK;
}

isx_status isx_surrogate_grad(isx_ctx* ctx, int32_t sur_id, int64_t n, const float* d_centres, const float* d_halves,
                              const float* d_targets, int64_t first_row, int32_t batch, float* const* h_gW,
                              float* const* h_gb, float* h_loss) {
  Sur* Sp = get_sur(ctx, sur_id);
  if (!Sp) return fail(ctx, ISX_EINVAL, "no such surrogate");
  if (n <= 0 || !d_centres || !d_halves || !d_targets || batch < 1 || first_row < 0 || !h_gW || !h_gb)
    return fail(ctx, ISX_EINVAL, "bad arguments");
  (void)hipSetDevice(ctx->device);
  Sur& S = *Sp;
  HIPCHK(ensure(ctx->sp_cnt, sizeof(float) * 2));
  const float* d_base = nullptr;
  isx_status e = sur_train_base(ctx, S, n, d_centres, d_halves, &d_base);
  if (e != ISX_OK) return e;
  e = sur_fwd_bwd(ctx, S, n, d_centres, d_halves, d_targets, d_base, first_row % n, batch, (float*)ctx->sp_cnt.p);
  if (e != ISX_OK) return e;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int l = 0; l < S.L; ++l) {
    HIPCHK(hipMemcpy(h_gW[l], S.gW[l], (size_t)S.w[l] * S.w[l + 1] * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(h_gb[l], S.gb[l], (size_t)S.w[l + 1] * 4, hipMemcpyDeviceToHost));
  }
  if (h_loss) HIPCHK(hipMemcpy(h_loss, ctx->sp_cnt.p, sizeof(float), hipMemcpyDeviceToHost));
  return ISX_OK;
}

isx_status isx_surrogate_train(isx_ctx* ctx, int32_t sur_id, int64_t n, const float* d_centres, const float* d_halves,
                               const float* d_targets, int64_t first_row, int32_t steps, int32_t batch, float lr,
                               float* d_loss) {
  Sur* Sp = get_sur(ctx, sur_id);
  if (!Sp) return fail(ctx, ISX_EINVAL, "no such surrogate");
  Sur& S = *Sp;
  if (n <= 0 || !d_centres || !d_halves || !d_targets || steps < 0 || batch < 1 || first_row < 0 ||
      !(lr > 0.f))
    return fail(ctx, ISX_EINVAL, "bad training arguments");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = ctx->stream;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float* d_base = nullptr;
  {
    isx_status e = sur_train_base(ctx, S, n, d_centres, d_halves, &d_base);
    if (e != ISX_OK) return e;
  }
  for (int st = 0; st < steps; ++st) {
    const int64_t r0 = (first_row + (int64_t)st * batch) % n;
    isx_status e = sur_fwd_bwd(ctx, S, n, d_centres, d_halves, d_targets, d_base, r0, batch,
                               d_loss ? d_loss + st : nullptr);
    if (e != ISX_OK) return e;
    S.t += 1;
    const float c1 = 1.f - std::pow(b1, (float)S.t), c2 = 1.f - std::pow(b2, (float)S.t);
    for (int l = 0; l < S.L; ++l) {
      HIPCHK(sur_adam(S.w[l] * S.w[l + 1], S.W[l], S.gW[l], S.mW[l], S.vW[l], lr, b1, b2, eps, c1, c2, s));
      HIPCHK(sur_adam(S.w[l + 1], S.b[l], S.gb[l], S.mb[l], S.vb[l], lr, b1, b2, eps, c1, c2, s));
    }
  }
  return ISX_OK;
}

isx_status isx_surrogate_predict(isx_ctx* ctx, int32_t sur_id, int64_t n, const float* d_centres,
                                 const float* d_halves, float* d_out) {
  Sur* S = get_sur(ctx, sur_id);
  if (!S) return fail(ctx, ISX_EINVAL, "no such surrogate");
  if (n < 0 || (n > 0 && (!d_centres || !d_halves || !d_out))) return fail(ctx, ISX_EINVAL, "bad arguments");
  if (n == 0) return ISX_OK;
  (void)hipSetDevice(ctx->device);
  return sur_predict_n(ctx, *S, n, d_centres, d_halves, d_out, nullptr);
}

isx_status isx_surrogate_set_base(isx_ctx* ctx, int32_t sur_id, int32_t mlp_id, float s_floor) {
  Sur* S = get_sur(ctx, sur_id);
  if (!S) return fail(ctx, ISX_EINVAL, "no such surrogate");
  if (mlp_id == -1) {
    S->base_mlp = -1;
    return ISX_OK;
  }
  const Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "bad mlp id");
  if (m->act != ISX_RELU) return fail(ctx, ISX_EUNSUPPORTED, "the centre linearisation needs a ReLU net");
  if (!(s_floor > 0.f) || !std::isfinite(s_floor)) return fail(ctx, ISX_EINVAL, "s_floor must be finite and > 0");
  S->base_mlp = mlp_id;
  S->s_floor = s_floor;
  return ISX_OK;
}

isx_status isx_surrogate_attach(isx_ctx* ctx, int32_t mlp_id, int32_t sur_id, int32_t n_levels,
                                const float* h_err_mu, const float* h_err_logsig, const float* h_z,
                                const float* h_z_accept, int32_t accept_leaves) {
  Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "bad mlp id");
  if (sur_id == -1) {
    m->sur_id = -1;
    return ISX_OK;
  }
  if (!get_sur(ctx, sur_id)) return fail(ctx, ISX_EINVAL, "no such surrogate");
  if (n_levels < 1 || n_levels > 16 || !h_err_mu || !h_err_logsig || !h_z || !h_z_accept)
    return fail(ctx, ISX_EINVAL, "bad surrogate band");
  for (int i = 0; i < n_levels; ++i)
    if (!(h_err_mu[i] >= 0.f) || !(h_err_logsig[i] >= 0.f) || !(h_z[i] >= 0.f) || !(h_z_accept[i] >= 0.f) ||
        !std::isfinite(h_err_mu[i]) || !std::isfinite(h_err_logsig[i]) || !std::isfinite(h_z[i]) ||
        !std::isfinite(h_z_accept[i]))
      return fail(ctx, ISX_EINVAL, "bad error scales or bands");
  m->sur_id = sur_id;
  m->sur_levels = n_levels;
  for (int i = 0; i < 16; ++i) {
    m->sur_err_mu[i] = i < n_levels ? h_err_mu[i] : h_err_mu[n_levels - 1];
    m->sur_err_ls[i] = i < n_levels ? h_err_logsig[i] : h_err_logsig[n_levels - 1];
    m->sur_z[i] = i < n_levels ? h_z[i] : h_z[n_levels - 1];
    m->sur_z_acc[i] = i < n_levels ? h_z_accept[i] : h_z_accept[n_levels - 1];
  }
  m->sur_accept_leaves = accept_leaves ? 1 : 0;
  return ISX_OK;
}

isx_status isx_surrogate_partition(isx_ctx* ctx, int32_t mlp_id, int64_t n, const float* d_pred, const float* d_unit,
                                   float k, int32_t level, int32_t leaf, const uint32_t* d_parent_mask,
                                   uint32_t* d_mask, uint32_t* d_fallback) {
  Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "bad mlp id");
  if (m->sur_id < 0) return fail(ctx, ISX_EINVAL, "no surrogate attached to this mlp");
  if (n < 0 || level < 0 || !(k >= 0.f) || !std::isfinite(k) ||
      (n > 0 && (!d_pred || !d_parent_mask || !d_mask || !d_fallback)))
    return fail(ctx, ISX_EINVAL, "bad arguments");
  if (n == 0) return ISX_OK;
  (void)hipSetDevice(ctx->device);
  const int Ls = std::min<int>(level, std::max(0, m->sur_levels - 1));
  HIPCHK(sur_partition(n, d_pred, d_unit, k, iso_list(*m), d_parent_mask, m->sur_err_mu[Ls], m->sur_err_ls[Ls],
                       m->sur_z[Ls], m->sur_z_acc[Ls], leaf ? 1 : 0, m->sur_accept_leaves, d_mask, d_fallback,
                       ctx->stream));
  return ISX_OK;
}


// ------------------------------------------------ surrogate training set and bands
isx_status isx_surrogate_sample_cells(isx_ctx* ctx, int32_t mlp_id, const isx_mesh* visited, int64_t n,
                                      int32_t level_lo, int32_t level_hi, uint64_t seed, float* d_centres,
                                      float* d_halves, int32_t* d_levels) {
  Model* m = get_model(ctx, mlp_id);
  if (!m) return fail(ctx, ISX_EINVAL, "bad mlp id");
  if (n < 0 || level_lo < 0 || level_hi < level_lo || level_hi > 10 ||
      (n > 0 && (!d_centres || !d_halves || !d_levels)))
    return fail(ctx, ISX_EINVAL, "bad arguments");
  if (visited && !visited->kept) return fail(ctx, ISX_EINVAL, "the visited mesh keeps no level cells (ISX_KEEP_LEVELS)");
  if (n == 0) return ISX_OK;
  (void)hipSetDevice(ctx->device);
  std::vector<int64_t> off(1, 0);
  int64_t total = 0;
  if (visited) {
    for (const auto& v : visited->lvl_ids) {
      total += (int64_t)v.size();
      off.push_back(total);
    }
  }
  const int vis_levels = (int)off.size() - 1;
  if (total > 0) {
    HIPCHK(ensure(ctx->sp_vis, (size_t)total * 4));
    HIPCHK(ensure(ctx->sp_vis_off, off.size() * sizeof(int64_t)));
    for (int L = 0; L < vis_levels; ++L)
      HIPCHK(hipMemcpyAsync((uint32_t*)ctx->sp_vis.p + off[L], visited->lvl_ids[L].data(),
                            visited->lvl_ids[L].size() * 4, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->sp_vis_off.p, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                          ctx->stream));
  }
  HIPCHK(launch_sample_cells(n, seed, m->lo, m->hi, level_lo, level_hi, total > 0 ? (const uint32_t*)ctx->sp_vis.p : nullptr,
                             total > 0 ? (const int64_t*)ctx->sp_vis_off.p : nullptr, vis_levels, total, d_centres,
                             d_halves, d_levels, ctx->stream));
  // the host copies of the level ids must outlive the transfers
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ISX_OK;
}

static const float kBandLadder[] = {0.f, 0.5f, 1.f, 1.5f, 2.f, 2.5f, 3.f, 3.5f, 4.f, 5.f, 6.f, 8.f, 12.f};
static constexpr int kLadder = 13;
static constexpr int kPruneFrom = 4;  // prune bands start at 2

isx_status isx_surrogate_calibrate(isx_ctx* ctx, int32_t sur_id, int32_t mlp_id, int64_t n, const float* d_centres,
                                   const float* d_halves, const float* d_targets, const int32_t* d_levels,
                                   int32_t n_levels, float k, float miss_target, float accept_target,
                                   int64_t min_level_kept, int32_t accept_leaves, isx_surrogate_calibration* cal) {
  Sur* Sp = get_sur(ctx, sur_id);
  Model* m = get_model(ctx, mlp_id);
  if (!Sp || !m) return fail(ctx, ISX_EINVAL, "bad surrogate or mlp id");
  if (n <= 0 || !d_centres || !d_halves || !d_targets || !d_levels || !cal || n_levels < 1 || n_levels > 16 ||
      !(k >= 0.f) || !(miss_target >= 0.f) || !(accept_target >= 0.f) || min_level_kept < 0)
    return fail(ctx, ISX_EINVAL, "bad calibration arguments");
  if (m->n_iso < 1) return fail(ctx, ISX_EINVAL, "no iso-values set");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = ctx->stream;
  Sur& S = *Sp;
  const bool based = S.base_mlp >= 0;
  HIPCHK(ensure(ctx->cal_pred, (size_t)n * 8));
  if (based) HIPCHK(ensure(ctx->cal_unit, (size_t)n * 4));
  float* pred = (float*)ctx->cal_pred.p;
  float* unit = based ? (float*)ctx->cal_unit.p : nullptr;
  isx_status st = sur_predict_n(ctx, S, n, d_centres, d_halves, pred, unit);
  if (st != ISX_OK) return st;
  // 1. per-level RMS errors (block partials added in order on the host)
  const int64_t nb = std::min<int64_t>(1024, (n + 255) / 256);
  HIPCHK(ensure(ctx->cal_part, (size_t)nb * n_levels * 3 * sizeof(double)));
  HIPCHK(launch_calib_err(n, pred, d_targets, unit, d_levels, n_levels, (double*)ctx->cal_part.p, nb, s));
  std::vector<double> part((size_t)nb * n_levels * 3);
  HIPCHK(hipMemcpyAsync(part.data(), ctx->cal_part.p, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::memset(cal, 0, sizeof(*cal));
  cal->n_levels = n_levels;
  for (int L = 0; L < n_levels; ++L) {
    double sm = 0.0, sl = 0.0, cnt = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
      const double* q = &part[((size_t)b * n_levels + L) * 3];
      sm += q[0];
      sl += q[1];
      cnt += q[2];
    }
    cal->n_cells[L] = (int64_t)cnt;
    if (cnt < 50.0) {  // too few held-out cells: the previous level's error
      cal->err_mu[L] = L > 0 ? cal->err_mu[L - 1] : S.scale;
      cal->err_logsig[L] = L > 0 ? cal->err_logsig[L - 1] : 1.f;
    } else {
      cal->err_mu[L] = (float)std::sqrt(sm / cnt);
      cal->err_logsig[L] = (float)std::sqrt(sl / cnt);
    }
  }
  // 2. counts per (level, band) of misses and false accepts, and of kept cells
  const size_t ncnt = (size_t)n_levels * kLadder * 2;
  HIPCHK(ensure(ctx->cal_cnt, (ncnt + 16) * sizeof(unsigned long long)));
  HIPCHK(ensure(ctx->cal_vec, 3 * 16 * sizeof(float)));
  float hv[48];
  for (int i = 0; i < 16; ++i) {
    hv[i] = i < n_levels ? cal->err_mu[i] : 0.f;
    hv[16 + i] = i < n_levels ? cal->err_logsig[i] : 0.f;
    hv[32 + i] = i < kLadder ? kBandLadder[i] : 0.f;
  }
  unsigned long long* dcnt = (unsigned long long*)ctx->cal_cnt.p;
  HIPCHK(hipMemcpyAsync(ctx->cal_vec.p, hv, sizeof(hv), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(dcnt, 0, (ncnt + 16) * sizeof(unsigned long long), s));
  const float* dv = (const float*)ctx->cal_vec.p;
  HIPCHK(launch_calib_count(n, pred, d_targets, unit, d_levels, n_levels, k, iso_list(*m), dv, dv + 16, dv + 32,
                            kLadder, dcnt, dcnt + ncnt, s));
  std::vector<unsigned long long> cnt(ncnt + 16);
  HIPCHK(hipMemcpyAsync(cnt.data(), dcnt, cnt.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  auto miss = [&](int L, int zi) { return (double)cnt[((size_t)L * kLadder + zi) * 2 + 0]; };
  auto fals = [&](int L, int zi) { return (double)cnt[((size_t)L * kLadder + zi) * 2 + 1]; };
  double kept_all = 0.0;
  for (int L = 0; L < n_levels; ++L) {
    cal->kept[L] = (int64_t)cnt[ncnt + L];
    kept_all += (double)cal->kept[L];
  }
  const double den = std::max(kept_all, 1.0);
  // 3. the smallest band of the ladder whose rate meets the target, over all
  //    levels, then per level where enough held-out cells are kept
  int zg = kLadder - 1, zag = kLadder - 1;
  for (int zi = kPruneFrom; zi < kLadder; ++zi) {
    double mm = 0.0;
    for (int L = 0; L < n_levels; ++L) mm += miss(L, zi);
    if (mm / den <= miss_target) {
      zg = zi;
      break;
    }
  }
  for (int zi = 0; zi < kLadder; ++zi) {
    double ff = 0.0;
    for (int L = 0; L < n_levels; ++L) ff += fals(L, zi);
    if (ff / den <= accept_target) {
      zag = zi;
      break;
    }
  }
  cal->z_global = kBandLadder[zg];
  cal->z_accept_global = kBandLadder[zag];
  int zl[16], zal[16];
  double hm = 0.0, hf = 0.0;
  for (int L = 0; L < n_levels; ++L) {
    zl[L] = zg;
    zal[L] = zag;
    if (cal->n_cells[L] > 0 && cal->kept[L] >= std::max<int64_t>(min_level_kept, 1)) {
      const double kl = (double)cal->kept[L];
      zl[L] = kLadder - 1;
      for (int zi = kPruneFrom; zi < kLadder; ++zi)
        if (miss(L, zi) / kl <= miss_target) {
          zl[L] = zi;
          break;
        }
      zal[L] = kLadder - 1;
      for (int zi = 0; zi < kLadder; ++zi)
        if (fals(L, zi) / kl <= accept_target) {
          zal[L] = zi;
          break;
        }
    }
    cal->z[L] = kBandLadder[zl[L]];
    cal->z_accept[L] = kBandLadder[zal[L]];
    hm += miss(L, zl[L]);
    hf += fals(L, zal[L]);
  }
  cal->holdout_miss = hm / den;
  cal->holdout_false_accept = hf / den;
  return isx_surrogate_attach(ctx, mlp_id, sur_id, n_levels, cal->err_mu, cal->err_logsig, cal->z, cal->z_accept,
                              accept_leaves);
}

isx_status isx_surrogate_fit(isx_ctx* ctx, int32_t mlp_id, const isx_mesh* visited, const isx_surrogate_fit_params* p,
                             int32_t* sur_id, isx_surrogate_calibration* cal, float* h_loss) {
  Model* m = get_model(ctx, mlp_id);
  if (!m || !p || !sur_id || !cal) return fail(ctx, ISX_EINVAL, "bad arguments");
  if (p->n_pairs < 1 || p->n_holdout < 1 || p->steps < 0 || p->batch < 1 || !(p->lr > 0.f) || p->depth < 0 ||
      p->depth > 10 || p->hidden_width < 1 || p->hidden_width > ISX_MAX_WIDTH || p->hidden_layers < 1 ||
      p->hidden_layers + 1 > ISX_MAX_LINEAR || !(p->scale > 0.f) || !std::isfinite(p->mu_bar))
    return fail(ctx, ISX_EINVAL, "bad surrogate fit parameters");
  (void)hipSetDevice(ctx->device);
  *sur_id = -1;
  const int64_t n = p->n_pairs + p->n_holdout;
  HIPCHK(ensure(ctx->fit_c, (size_t)n * 12));
  HIPCHK(ensure(ctx->fit_h, (size_t)n * 12));
  HIPCHK(ensure(ctx->fit_t, (size_t)n * 8));
  HIPCHK(ensure(ctx->fit_l, (size_t)n * 4));
  float* C = (float*)ctx->fit_c.p;
  float* H = (float*)ctx->fit_h.p;
  float* T = (float*)ctx->fit_t.p;
  int32_t* Lv = (int32_t*)ctx->fit_l.p;
  // 1. cells: visited cells and uniform random cells of levels min(3, D)..D
  isx_status st = isx_surrogate_sample_cells(ctx, mlp_id, visited, n, std::min(3, p->depth), p->depth, p->seed, C, H, Lv);
  if (st != ISX_OK) return st;
  // 2. targets: float32 uncertainty propagation of every cell
  st = run_propagate(ctx, *m, ISX_UP, ISX_FP32, n, C, H, T, nullptr, 0);
  if (st != ISX_OK) return st;
  // 3. network 4 -> hidden^layers -> 2, He-normal weights N(0, 2/fan_in),
  //    biases N(0, (0.1 std)^2), from SplitMix64 streams of the seed
  std::vector<int32_t> widths(p->hidden_layers + 2, p->hidden_width);
  widths.front() = 4;
  widths.back() = 2;
  const int nl = (int)widths.size() - 1;
  std::vector<std::vector<float>> Ws(nl), bs(nl);
  std::vector<const float*> Wp(nl), bp(nl);
  for (int l = 0; l < nl; ++l) {
    const float sd = std::sqrt(2.f / (float)widths[l]);
    Ws[l].resize((size_t)widths[l] * widths[l + 1]);
    bs[l].resize(widths[l + 1]);
    host_normal_fill(p->seed ^ (0xA5A5A5A5ull * (uint64_t)(2 * l + 1)), sd, Ws[l].data(), (int64_t)Ws[l].size());
    host_normal_fill(p->seed ^ (0xA5A5A5A5ull * (uint64_t)(2 * l + 2)), 0.1f * sd, bs[l].data(), (int64_t)bs[l].size());
    Wp[l] = Ws[l].data();
    bp[l] = bs[l].data();
  }
  int32_t sid = -1;
  st = isx_surrogate_load(ctx, nl, widths.data(), Wp.data(), bp.data(), &sid);
  if (st != ISX_OK) return st;
  auto undo = [&](isx_status e) {
    isx_surrogate_free(ctx, sid);
    return e;
  };
  st = isx_surrogate_set_norm(ctx, sid, p->mu_bar, p->scale, 0.25f, 1.f);
  if (st == ISX_OK && p->use_base) st = isx_surrogate_set_base(ctx, sid, mlp_id, 1e-6f * p->scale);
  if (st != ISX_OK) return undo(st);
  // 4. training on the first n_pairs cells
  float* dloss = nullptr;
  if (h_loss && p->steps > 0) {
    HIPCHK(ensure(ctx->fit_loss, (size_t)p->steps * 4));
    dloss = (float*)ctx->fit_loss.p;
  }
  st = isx_surrogate_train(ctx, sid, p->n_pairs, C, H, T, 0, p->steps, p->batch, p->lr, dloss);
  if (st != ISX_OK) return undo(st);
  if (dloss) {
    hipError_t e = hipMemcpyAsync(h_loss, dloss, (size_t)p->steps * 4, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return undo(hip_fail(ctx, e, "surrogate loss copy"));
  }
  // 5. bands calibrated on the held-out cells, then attached to the MLP
  const int64_t o = p->n_pairs;
  st = isx_surrogate_calibrate(ctx, sid, mlp_id, p->n_holdout, C + 3 * o, H + 3 * o, T + 2 * o, Lv + o, p->depth + 1,
                               p->k, p->miss_target, p->accept_target, p->min_level_kept, p->accept_leaves, cal);
  if (st != ISX_OK) return undo(st);
  *sur_id = sid;
  return ISX_OK;
}

}  // extern "C"
