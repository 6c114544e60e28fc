/*
 * isx.h -- C ABI of libisx: hierarchical iso-surface extraction on ReLU
 * coordinate MLPs (implicit neural representations) for AMD MI355X (gfx950).
 *
 * Method: Li & Shen, "Improving Efficiency of Iso-Surface Extraction on
 * Implicit Neural Representations Using Uncertainty Propagation"
 * (arXiv 2402.13861).
 *
 * The library propagates axis-aligned boxes through an MLP with either
 *   - affine arithmetic (range analysis; Sec. III-A/B, Eq. 1-4), giving a hard
 *     bound [x0 - r, x0 + r], or
 *   - uncertainty propagation with probabilistic affine forms (Sec. IV-B/C,
 *     Eq. 6-10, App. D ReLU row), giving a Gaussian N(mu, sigma^2) whose soft
 *     bound is [mu - t sigma, mu + t sigma],
 * classifies cells against iso-values (Alg. 1), searches an octree top-down
 * keeping only active cells (Alg. 1 in 8-way form), evaluates the MLP at the
 * corners of the active leaves and runs marching cubes there (Sec. IV-D).
 *
 * Conventions for every function:
 *   - Returns ISX_OK (0) or a negative isx_status; never throws or aborts.
 *     A human-readable message for the last failure on a context is returned
 *     by isx_last_error().
 *   - "d_" pointers are DEVICE pointers (e.g. torch tensor data_ptr()) owned
 *     by the caller; "h_" pointers are host pointers owned by the caller.
 *     The library never frees caller memory.
 *   - Work is enqueued on the context's HIP stream.  Functions documented as
 *     "asynchronous" return before the GPU work completes; the others
 *     synchronise the stream before returning.
 *   - Float layouts are C-contiguous, float32 unless stated otherwise.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef ISX_H
#define ISX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ISX_OK = 0,
  ISX_EINVAL = -1,       /* bad argument (null pointer, unknown enum, k < 0 ...) */
  ISX_ESHAPE = -2,       /* unsupported or inconsistent layer widths */
  ISX_ENOMEM = -3,       /* device allocation failed */
  ISX_ECAPACITY = -4,    /* a result exceeds a caller-set capacity (never truncated silently) */
  ISX_EHIP = -5,         /* a HIP runtime call or kernel launch failed */
  ISX_ENAN = -6,         /* NaN or Inf in weights, domain or iso-values */
  ISX_EUNSUPPORTED = -7  /* valid request that the library does not implement */
} isx_status;

/* Range analysis by affine arithmetic ("RA-Full", Sec. III), uncertainty
 * propagation with probabilistic affine forms ("UP", Sec. IV-B), or range
 * analysis read off under the uniform assumption ("RA-UA", Sec. IV-A,
 * Eq. 5): the affine form of AA, its symbols taken as independent uniform
 * variables on [-1, 1], gives N(x0, sum_i x_i^2 / 3), whose soft bound is
 * [x0 - t sigma, x0 + t sigma] as for UP.  "RA-Fixed" (the reduced affine form
 * App. A compares against): affine arithmetic that keeps the input symbols
 * and folds every symbol an activation creates into one error magnitude per
 * neuron (a linear layer maps it by |W|); its hard range is
 * [x0 - r, x0 + r].  The affine rule of every activation is that of
 * ISX_AA (Eq. 4). */
typedef enum { ISX_AA = 0, ISX_UP = 1, ISX_RAUA = 2, ISX_RAFIXED = 3 } isx_method;

/* Arithmetic of the propagation and evaluation kernels.
 *   ISX_FP32: float32 everywhere; hidden-layer products on FP32 MFMA.
 *   ISX_BF16: layer products with bfloat16 operands on MFMA, float32
 *             accumulation, statistics and epilogues (centre column float32).
 *   ISX_FP64: float64 everywhere (reference / re-check path). */
typedef enum { ISX_FP32 = 0, ISX_BF16 = 1, ISX_FP64 = 2 } isx_precision;

/* Activation after every hidden linear layer (App. D table rows): ReLU, sine
 * (SIREN nets; any frequency factor omega_0 is folded into the weights), or
 * ELU (x for x > 0, e^x - 1 otherwise). */
typedef enum { ISX_RELU = 0, ISX_SINE = 1, ISX_ELU = 2 } isx_activation;

typedef struct isx_ctx isx_ctx;
typedef struct isx_mesh isx_mesh;

#define ISX_MAX_LINEAR 16 /* maximum number of linear layers */
#define ISX_MAX_WIDTH 1024
#define ISX_MAX_ISO 32    /* iso-values per MLP; cell masks are uint32 */

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  *out receives the
 * context.  Errors: ISX_EINVAL (bad device / out == NULL), ISX_EHIP. */
isx_status isx_create(int device, void* hip_stream, isx_ctx** out);

/* Destroy a context and free all library-owned device memory of it
 * (weights, work buffers).  Meshes must be freed separately. */
isx_status isx_destroy(isx_ctx* ctx);

/* Message of the last failed call on ctx ("" if none); owned by ctx, valid
 * until the next call on ctx.  ctx == NULL gives the last create() error. */
const char* isx_last_error(const isx_ctx* ctx);

/* Load an MLP f: R^3 -> R (Sec. III-B).  n_linear linear layers,
 * widths[0] = 3, widths[n_linear] = 1, 1 <= hidden widths <= ISX_MAX_WIDTH,
 * 2 <= n_linear <= ISX_MAX_LINEAR.  h_W[l] is row-major
 * [widths[l+1]][widths[l]] float32 and h_b[l] is [widths[l+1]], both HOST
 * pointers; a ReLU follows every layer but the last.  Weights are copied to
 * library-owned device memory (float32, float64 and bfloat16 copies, hidden
 * widths zero-padded to a multiple of 32, which leaves every result
 * unchanged), so the caller may free its copy on return.
 * The domain defaults to [-1,1]^3 and the iso-value list to empty.
 * Errors: ISX_EINVAL, ISX_ESHAPE, ISX_ENAN (non-finite weight), ISX_ENOMEM. */
isx_status isx_load_mlp(isx_ctx* ctx, int32_t n_linear, const int32_t* widths,
                        const float* const* h_W, const float* const* h_b, int32_t* mlp_id);

/* Hidden activation of a loaded MLP (default ISX_RELU).  The rules follow
 * the App. D table (UP: Gaussian least-squares lines; AA: the minimax line for
 * ReLU and the convex ELU, a chord with exact error extremes for sine).
 * Sine and ELU nets run in float32, float64 and bfloat16 (the rules
 * themselves in float64 inside the float32 and bfloat16 kernels); the AA
 * rounding margin, isx_linearize and the surrogate's linearisation base need
 * ReLU (ISX_EUNSUPPORTED otherwise).
 * Errors: ISX_EINVAL. */
isx_status isx_set_activation(isx_ctx* ctx, int32_t mlp_id, isx_activation act);

/* Release an MLP's device memory. */
isx_status isx_unload_mlp(isx_ctx* ctx, int32_t mlp_id);

/* Axis-aligned domain [lo, hi] of the octree root (Alg. 1 inputs x_l, x_u).
 * Errors: ISX_EINVAL (hi <= lo on an axis), ISX_ENAN. */
isx_status isx_set_domain(isx_ctx* ctx, int32_t mlp_id, const float h_lo[3], const float h_hi[3]);

/* Iso-values c_j (Alg. 1 input c), 0 <= n_iso <= ISX_MAX_ISO, host array.
 * Bit j of every cell mask refers to h_iso[j].  Errors: ISX_EINVAL, ISX_ENAN. */
isx_status isx_set_isovalues(isx_ctx* ctx, int32_t mlp_id, int32_t n_iso, const float* h_iso);

/* Propagate n_cells boxes through the MLP (the bound computation of Alg. 1, without the
 * test).  d_centres [n][3] and d_halves [n][3] (per-axis half-widths, > 0)
 * are device arrays.  d_out [n][2] receives (centre, spread) as float32:
 * (x0, r) for ISX_AA, whose range is [x0 - r, x0 + r] (Eq. 2),
 * (mu, sigma) for ISX_UP (Eq. 7) and (x0, sigma) for ISX_RAUA (Eq. 5).  With ISX_FP64 the same pair is also
 * written in float64 to d_out64 [n][2] if it is not NULL (it must be NULL
 * for the other precisions).  Asynchronous, except ISX_BF16 with ISX_UP in
 * covariance form with ISX_CANCEL_CHECK on (the default), which synchronises
 * the stream once to count the cells it re-propagates in float64.
 * n_cells == 0 is a no-op.
 * Errors: ISX_EINVAL, ISX_ENOMEM, ISX_EHIP. */
isx_status isx_propagate(isx_ctx* ctx, int32_t mlp_id, isx_method method, isx_precision precision,
                         int64_t n_cells, const float* d_centres, const float* d_halves, float* d_out,
                         double* d_out64);

/* Classify and compact (the pruning test of Alg. 1): cell i keeps iso bit j iff
 * centre - k*spread <= c_j <= centre + k*spread (closed interval) and bit j is
 * set in d_parent_mask[i] (NULL = all bits set); k is the paper's t for UP and
 * must be 1 for the AA hard range.  The indices i of cells with a nonzero
 * mask are written in increasing order to d_active_idx, their masks to
 * d_active_mask, and the count to *d_n_active (device int64).  d_active_idx and
 * d_active_mask must hold n_cells entries.  Asynchronous.
 * Errors: ISX_EINVAL, ISX_EHIP. */
isx_status isx_classify_compact(isx_ctx* ctx, int32_t mlp_id, float k, int64_t n_cells, const float* d_out,
                                const uint32_t* d_parent_mask, uint32_t* d_active_idx,
                                uint32_t* d_active_mask, int64_t* d_n_active);

/* isx_classify_compact_noalloc: isx_classify_compact for callers that cannot
 * allocate device memory -- code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Same arguments, results and
 * asynchrony as isx_classify_compact; it calls no allocating routine.  Its
 * working memory (a uint32 mask per cell and the scan's block partials) is a
 * fixed array of the library, one copy per device, sized for
 * ISX_NOALLOC_MAX_CELLS cells (16 MiB + 16 KiB) and held until the process
 * ends.  n_cells above ISX_NOALLOC_MAX_CELLS fails with ISX_ECAPACITY (split
 * the batch).  Every call on a device uses that device's one array and leaves
 * its contents behind; nothing in it needs to start at zero, but calls that
 * overlap on one device (several streams or host threads) race and must be
 * serialised by the caller.
 * Errors: ISX_EINVAL, ISX_ECAPACITY, ISX_EHIP. */
#define ISX_NOALLOC_MAX_CELLS (1 << 22)
isx_status isx_classify_compact_noalloc(isx_ctx* ctx, int32_t mlp_id, float k, int64_t n_cells,
                                        const float* d_out, const uint32_t* d_parent_mask,
                                        uint32_t* d_active_idx, uint32_t* d_active_mask, int64_t* d_n_active);

/* Plain MLP evaluation f(x) at n points (Sec. III-B; the reconstruction step
 * of Sec. IV-D).  d_points [n][3], d_values [n], float32 device arrays;
 * ISX_FP64 computes in float64 and rounds the result.  Asynchronous. */
isx_status isx_eval_points(isx_ctx* ctx, int32_t mlp_id, isx_precision precision, int64_t n,
                           const float* d_points, float* d_values);

/* Centre linearisation of n cells: the limit of the uncertainty propagation
 * (Sec. IV-C input form, Eq. 6-8) when no ReLU changes sign inside the cell.
 * d_out [n][2] receives (f(c), s) with s = |J(c) diag(h)|_2 / sqrt(3), J the
 * gradient of the MLP at the centre (a ReLU's derivative at 0 taken as 0).
 * d_centres, d_halves [n][3] as in isx_propagate.  float32 (MFMA products),
 * asynchronous; hidden widths up to ISX_MAX_WIDTH.
 * Errors: ISX_EINVAL, ISX_EHIP. */
isx_status isx_linearize(isx_ctx* ctx, int32_t mlp_id, int64_t n, const float* d_centres,
                         const float* d_halves, float* d_out);

/* isx_propagate_segments: isx_propagate for line segments instead of boxes
 * (App. A's ray casting): segment i is {c_i + e v_i : e in [-1, 1]}, d_centres
 * [n][3] its centre and d_halfvec [n][3] its half-vector v_i (float32,
 * device).  It has one input symbol e, with coefficient v (AA, RA-UA,
 * RA-Fixed; range analysis) or v / sqrt 3 (UP: uniform on [-1, 1]).  Methods
 * ISX_AA, ISX_UP, ISX_RAUA, ISX_RAFIXED; precisions ISX_FP32 and ISX_FP64
 * (ISX_BF16 and the AA rounding margin: ISX_EUNSUPPORTED).  Output as
 * isx_propagate.  Asynchronous.  Errors: ISX_EINVAL, ISX_EUNSUPPORTED,
 * ISX_EHIP. */
isx_status isx_propagate_segments(isx_ctx* ctx, int32_t mlp_id, isx_method method, isx_precision precision,
                                  int64_t n, const float* d_centres, const float* d_halfvec, float* d_out,
                                  double* d_out64);

/* Ray casting of the level set f = iso (App. A, following the range-analysis
 * ray caster it compares with).  Ray i starts at t = d_tnear[i] with step
 * step0 and marches along o_i + t d_i (d_origins, d_dirs [n][3], float32;
 * unit directions expected) until t_far = d_tfar[i]: the segment
 * [t, t + de], de = min(step, t_far - t), is bounded by `method` at
 * `precision` (isx_propagate_segments; UP and RA-UA: centre -/+ k spread, AA
 * and RA-Fixed: the hard range).  If the bound excludes iso, t += de and the
 * step doubles (at most step_max), the ray missing once t >= t_far;
 * otherwise the ray hits at t + de / 2 if de <= step_min, else the step
 * becomes de / 2.  Ray state (t, step) is float64; segment centres and
 * half-vectors are formed in float64 and rounded to float32; with ISX_FP64
 * the float64 bounds decide.  d_thit [n] (float32) gets the hit distance or
 * NaN (miss, empty ray, or not finished after max_iter steps), d_iters [n]
 * the steps each ray took; h_stats[2] (host, optional) the segments bounded
 * and the steps taken by the slowest ray.  Synchronises once per step.
 * Errors: ISX_EINVAL, ISX_EUNSUPPORTED (ISX_BF16), ISX_EHIP. */
typedef struct {
  isx_method method;
  isx_precision precision;  /* ISX_FP32 or ISX_FP64 */
  float k;                  /* t of the soft bound (UP, RA-UA) */
  float iso;                /* the level (0 for a signed distance function) */
  float step0, step_min, step_max;
  int32_t max_iter;
} isx_ray_params;
isx_status isx_raycast(isx_ctx* ctx, int32_t mlp_id, const isx_ray_params* params, int64_t n_rays,
                       const float* d_origins, const float* d_dirs, const float* d_tnear, const float* d_tfar,
                       float* d_thit, int32_t* d_iters, int64_t* h_stats);

/* Parameters of a full extraction. */
typedef struct {
  isx_method method;       /* ISX_UP (soft bound) or ISX_AA (hard bound) */
  isx_precision precision; /* arithmetic of propagation and corner evaluation */
  float k;                 /* t of Alg. 1 for UP and RA-UA (ignored for AA, which uses 1) */
  int32_t max_depth;       /* octree depth D: leaves are the (2^D)^3 grid cells, D <= 10 */
  float fp64_band;         /* > 0: cells whose bound endpoint lies within
                              fp64_band of an iso-value are re-propagated in
                              float64 and that result decides (not with ISX_FP64;
                              see also fp64_band_rel) */
  int64_t max_cells;       /* capacity of one level (0 = library default); a
                              level above it fails with ISX_ECAPACITY */
  int64_t chunk_cells;     /* cells propagated per batch (0 = automatic; at most 2^22) */
  int32_t use_surrogate;   /* 1: decide cells with the surrogate attached to
                              the MLP where it is confident (see
                              isx_surrogate_attach), propagate the rest */
  int32_t tree;            /* 0: octree (every level splits a cell into 8 cubes);
                              1: Alg. 1's binary k-d tree, each node split along
                              its widest dimension (ties x, y, z) down to node
                              depth 3 max_depth, so that nodes at half and quarter
                              cells are tested too; needs a cube domain; meshes
                              then record 3 max_depth + 1 levels (node ids: root 0,
                              children 2p and 2p + 1), leaves as octree Morton
                              ids in k-d order; not with use_surrogate */
  float fp64_band_rel;     /* >= 0: widens the re-check band of each cell by this
                              multiple of its own spread (sigma for UP, r for AA):
                              a cell is re-propagated in float64 when a bound
                              endpoint lies within fp64_band + fp64_band_rel *
                              spread of a carried iso-value (the bfloat16 error
                              of the endpoints grows with the spread, so coarse
                              cells need the relative term) */
} isx_params;

/* Full extraction (Alg. 1 followed by corner evaluation and marching cubes)
 * of the MLP's iso-surfaces at all of its iso-values, from the root domain
 * to depth params->max_depth.  *out receives a library-owned mesh.
 * Synchronises the stream.  Errors: ISX_EINVAL, ISX_ECAPACITY, ISX_ENOMEM,
 * ISX_EHIP. */
isx_status isx_extract(isx_ctx* ctx, int32_t mlp_id, const isx_params* params, isx_mesh** out);

/* Dense baseline (the reference point for the range analysis): every cell
 * of the (2^depth)^3 grid is a leaf for every iso-value, so the INR is
 * evaluated at all (2^depth + 1)^3 grid corners (float64 for ISX_FP64, else
 * float32) and marching cubes runs on every (cell, iso) pair (corner
 * evaluation and marching cubes as in isx_extract, Sec. IV-C).  *out
 * receives a library-owned mesh with the same triangle layout as
 * isx_extract's; it records no octree levels, and its times are the leaf
 * list (ms_acp), the corner values (ms_inr) and marching cubes (ms_mc).
 * Synchronises the stream.  Errors: ISX_EINVAL (bad id, precision or depth
 * outside [0, 10], no iso-values), ISX_ECAPACITY (more than 2^28 cells or
 * 2^31 (cell, iso) pairs), ISX_ENOMEM, ISX_EHIP. */
isx_status isx_extract_dense(isx_ctx* ctx, int32_t mlp_id, int32_t depth, isx_precision precision,
                             isx_mesh** out);

/* isx_extract_batch: isx_extract of n INRs (mlp_ids[i], each with its own
 * iso-values and attached surrogate) with the same params; out[i] receives
 * INR i's mesh.  The INRs are dealt to up to ISX_BATCH_WORKERS worker
 * contexts, each with its own stream and scratch and one host thread, so
 * that the level loops of different INRs overlap on the device; each mesh is
 * identical to the one isx_extract returns.  Waits for the caller's stream
 * first; synchronous.  On an error every mesh of the call is freed, out[i]
 * is NULL and isx_last_error names the INR. */
isx_status isx_extract_batch(isx_ctx* ctx, int32_t n, const int32_t* mlp_ids, const isx_params* params,
                             isx_mesh** out);

/* Sizes of a mesh: triangles, active leaves, distinct leaf corners, and the
 * number of octree levels recorded (max_depth + 1). */
isx_status isx_mesh_info(const isx_mesh* mesh, int64_t* n_tris, int64_t* n_leaves, int64_t* n_corners,
                         int32_t* n_levels);

/* Per-level counts: cells examined at that level, cells kept active
 * (mask != 0), cells re-checked in float64, and cells actually propagated
 * (all examined cells unless the surrogate decided some). */
isx_status isx_mesh_level(const isx_mesh* mesh, int32_t level, int64_t* n_cells, int64_t* n_active,
                          int64_t* n_rechecked, int64_t* n_propagated);

/* Cells of a level that the bf16 covariance form flagged for cancellation
 * and propagated again in float64 (ISX_CANCEL_CHECK; 0 for other paths). */
isx_status isx_mesh_level_cancelled(const isx_mesh* mesh, int32_t level, int64_t* n_cancelled);

/* Cells of `level` propagated in float64 by the re-check band (all band
 * cells, or with ISX_RECHECK_CASCADE the inner band's).  ISX_EINVAL on a bad
 * level. */
isx_status isx_mesh_level_rechecked_fp64(const isx_mesh* mesh, int32_t level, int64_t* n_fp64);

/* Phase times in milliseconds measured with HIP events on the context
 * stream: active-cell prediction (all levels), corner evaluation, marching
 * cubes, total. */
isx_status isx_mesh_times(const isx_mesh* mesh, float* ms_acp, float* ms_inr, float* ms_mc, float* ms_total);

/* Copy the triangles to host arrays (each may be NULL to skip it):
 *   h_pos  [n_tris][3][3] float32 vertex positions;
 *   h_keys [n_tris][3]    uint64 vertex keys: (grid-point linear index * 3 +
 *          axis) of the grid edge the vertex lies on, grid of (2^D+1)^3
 *          points, linear index i + (2^D+1) (j + (2^D+1) k);
 *   h_iso  [n_tris]       int32 iso-value index.
 * Triangles are ordered by (active leaf in Morton order, iso index, case
 * table order).  Synchronous. */
isx_status isx_mesh_copy_tris(const isx_mesh* mesh, float* h_pos, uint64_t* h_keys, int32_t* h_iso);

/* Copy the active leaves: Morton ids (x bit lowest, 3*D bits) and iso masks. */
isx_status isx_mesh_copy_leaves(const isx_mesh* mesh, uint32_t* h_ids, uint32_t* h_masks);

/* Copy one level's propagated cells: Morton ids, (centre, spread) and masks
 * after the test.  Only available if the level's data was kept
 * (ISX_KEEP_LEVELS in isx_set_option), else ISX_EUNSUPPORTED. */
isx_status isx_mesh_copy_level(const isx_mesh* mesh, int32_t level, uint32_t* h_ids, float* h_out,
                               uint32_t* h_masks);

isx_status isx_mesh_free(isx_mesh* mesh);

/* ---- Learned surrogate ----------------------------------------------
 * A small ReLU MLP g: (c_x, c_y, c_z, a*log2(cell size)+b) -> standardised
 * ((mu - mu_bar)/S, ln sigma), predicting the propagation's output for a cell
 * at a fraction of its cost.  Trained on the GPU (bf16 MFMA products, float32
 * accumulation and master weights, Adam with beta1 = 0.9, beta2 = 0.999,
 * eps = 1e-8) on (cell, propagated mu/sigma) pairs the caller provides.
 *
 * isx_surrogate_load: n_linear layers, widths[0] = 4, widths[n_linear] = 2,
 *   row-major float32 host weights (copied); Adam state starts at zero.
 * isx_surrogate_get: copy the current weights into host arrays of the same
 *   shapes.
 * isx_surrogate_set_norm: mu_bar, S (> 0) of the targets and a, b of the
 *   size feature.
 * isx_surrogate_set_base: make the two outputs corrections to the centre
 *   linearisation (f, s) of MLP mlp_id (isx_linearize): the network is then
 *   trained on ((mu - f)/s_b, ln(sigma / s_b)) and predicts
 *   mu_hat = f + s_b o_0, sigma_hat = s_b exp(o_1), with s_b = max(s, s_floor)
 *   (s_floor > 0, field units), and the band's err_mu is in units of s_b.
 *   mlp_id = -1 returns to the standardised targets.  The MLP must stay
 *   loaded while the surrogate is used.
 * isx_surrogate_train: `steps` Adam steps on mini-batches of `batch` rows
 *   taken in order from row `first_row` of the n pairs (wrapping around):
 *   d_centres/d_halves [n][3] and d_targets [n][2] = propagated (mu, sigma),
 *   device arrays.  d_loss [steps] (device, may be NULL) receives each step's
 *   loss.  Asynchronous.
 * isx_surrogate_predict: d_out [n][2] = predicted (mu, sigma) in the INR's
 *   units.  Asynchronous.
 * isx_surrogate_attach: use surrogate sur_id in isx_extract of mlp_id (when
 *   params.use_surrogate).  h_err_mu[L], h_err_logsig[L] (L < n_levels) are
 *   the standard deviations of the surrogate's error at octree level L (field
 *   units, or units of s_b with a base; and log-sigma units), h_z[L] and
 *   h_z_accept[L] the level's prune and accept bands in those units (levels
 *   beyond n_levels use the last entry).  A cell at level L is decided
 *   without propagation when for every iso-value c it still carries either
 *     |mu_hat - c| - z err_mu > t sigma_hat exp(+z err_logsig)  (outside), or
 *     |mu_hat - c| + z_accept err_mu < t sigma_hat exp(-z_accept err_logsig)
 *                                                              (inside);
 *   otherwise it is propagated.  A wrongly pruned cell loses surface, a
 *   wrongly accepted one only costs work (its children are classified in
 *   turn; at the leaves it is an extra leaf), so the two bands may differ.  Leaves are always propagated unless
 *   accept_leaves.  sur_id = -1 detaches.
 * Errors: ISX_EINVAL, ISX_ESHAPE, ISX_ENAN, ISX_ENOMEM, ISX_EHIP. */
isx_status isx_surrogate_load(isx_ctx* ctx, int32_t n_linear, const int32_t* widths, const float* const* h_W,
                              const float* const* h_b, int32_t* sur_id);
isx_status isx_surrogate_get(isx_ctx* ctx, int32_t sur_id, float* const* h_W, float* const* h_b);
isx_status isx_surrogate_set_norm(isx_ctx* ctx, int32_t sur_id, float mu_bar, float scale, float size_a,
                                  float size_b);
isx_status isx_surrogate_set_base(isx_ctx* ctx, int32_t sur_id, int32_t mlp_id, float s_floor);
isx_status isx_surrogate_train(isx_ctx* ctx, int32_t sur_id, int64_t n, const float* d_centres,
                               const float* d_halves, const float* d_targets, int64_t first_row, int32_t steps,
                               int32_t batch, float lr, float* d_loss);
/* Gradients of the loss on one mini-batch (rows first_row.. of the n pairs,
 * as in isx_surrogate_train) without updating the weights; copied to host
 * arrays shaped like the weights, and the batch loss to *h_loss (may be
 * NULL).  Synchronous. */
isx_status isx_surrogate_grad(isx_ctx* ctx, int32_t sur_id, int64_t n, const float* d_centres,
                              const float* d_halves, const float* d_targets, int64_t first_row, int32_t batch,
                              float* const* h_gW, float* const* h_gb, float* h_loss);
isx_status isx_surrogate_predict(isx_ctx* ctx, int32_t sur_id, int64_t n, const float* d_centres,
                                 const float* d_halves, float* d_out);
isx_status isx_surrogate_attach(isx_ctx* ctx, int32_t mlp_id, int32_t sur_id, int32_t n_levels,
                                const float* h_err_mu, const float* h_err_logsig, const float* h_z,
                                const float* h_z_accept, int32_t accept_leaves);
isx_status isx_surrogate_free(isx_ctx* ctx, int32_t sur_id);

/* Training set of the surrogate: n cells, each drawn (with probability 1/2
 * when `visited` is given) uniformly from the cells a plain extraction
 * examined -- a mesh made with ISX_KEEP_LEVELS, whose level lists are used --
 * or else as a uniform random cell of a uniform random octree level in
 * [level_lo, level_hi] (<= 10) of the MLP's domain.  Random numbers from
 * SplitMix64 at counters derived from (seed, cell index).  d_centres,
 * d_halves [n][3] float32 and d_levels [n] int32 device arrays receive the
 * boxes and their levels.  Synchronous.  Errors: ISX_EINVAL, ISX_EHIP. */
isx_status isx_surrogate_sample_cells(isx_ctx* ctx, int32_t mlp_id, const isx_mesh* visited, int64_t n,
                                      int32_t level_lo, int32_t level_hi, uint64_t seed, float* d_centres,
                                      float* d_halves, int32_t* d_levels);

/* Calibration of the surrogate's safety bands on held-out cells. */
typedef struct {
  int32_t n_levels;          /* levels 0..n_levels-1 (<= 16) */
  int64_t n_cells[16];       /* held-out cells per level */
  int64_t kept[16];          /* of those, cells the plain soft-bound test keeps for some carried iso-value */
  float err_mu[16];          /* RMS error of mu_hat (field units, or units of s_b with a base); a level with
                                fewer than 50 cells takes the previous level's value (level 0: S, 1) */
  float err_logsig[16];      /* RMS error of ln sigma_hat */
  float z[16], z_accept[16]; /* prune / accept band per level, from the ladder
                                {0, .5, 1, 1.5, 2, 2.5, 3, 3.5, 4, 5, 6, 8, 12} (prune bands >= 2) */
  float z_global, z_accept_global;          /* the bands chosen over all levels together */
  double holdout_miss, holdout_false_accept; /* rates at the chosen per-level bands */
} isx_surrogate_calibration;

/* isx_surrogate_calibrate: predict the n held-out cells (d_centres,
 * d_halves [n][3], propagated d_targets [n][2] = (mu, sigma), octree levels
 * d_levels [n]) with surrogate sur_id, measure its per-level error, and pick
 * bands so that, with t = k and the MLP's iso-values, the prune rule of
 * isx_surrogate_partition drops a kept iso-value of at most miss_target of
 * the kept cells (misses / kept) and the accept rule accepts a rejected
 * iso-value of at most accept_target of them: the smallest ladder value that
 * meets the target over all levels, and per level where at least
 * min_level_kept cells are kept (else the global band).  The surrogate is
 * then attached to mlp_id with those bands (accept_leaves as in
 * isx_surrogate_attach) and *cal receives them.  Error sums are reduced in a
 * fixed order and the rates are integer counts, so the result is
 * deterministic.  Synchronous.  Errors: ISX_EINVAL, ISX_ENOMEM, ISX_EHIP. */
isx_status isx_surrogate_calibrate(isx_ctx* ctx, int32_t sur_id, int32_t mlp_id, int64_t n,
                                   const float* d_centres, const float* d_halves, const float* d_targets,
                                   const int32_t* d_levels, int32_t n_levels, float k, float miss_target,
                                   float accept_target, int64_t min_level_kept, int32_t accept_leaves,
                                   isx_surrogate_calibration* cal);

/* One-call training of a surrogate for MLP mlp_id (the learned part as a
 * whole): n_pairs + n_holdout cells from isx_surrogate_sample_cells (levels
 * min(3, depth)..depth, `visited` optional), their float32 uncertainty
 * propagation as targets, a 4 -> hidden_width^hidden_layers -> 2 network
 * with He-normal weights from the seed, normalisation (mu_bar, scale) and
 * the size feature 0.25 log2(cell size) + 1, optionally corrections to the
 * centre linearisation (use_base, s_floor = 1e-6 scale), `steps` Adam steps
 * of `batch` rows with learning rate lr on the n_pairs cells, and the bands
 * of isx_surrogate_calibrate on the n_holdout cells (attached to mlp_id).
 * *sur_id receives the surrogate, *cal its calibration and h_loss [steps]
 * (host, may be NULL) the training losses.  Synchronous.
 * Errors: ISX_EINVAL, ISX_ESHAPE, ISX_ENOMEM, ISX_EHIP. */
typedef struct {
  int64_t n_pairs, n_holdout;
  int32_t steps, batch;
  float lr;
  uint64_t seed;
  int32_t depth;                       /* octree depth of the extractions it serves */
  int32_t hidden_width, hidden_layers; /* 128, 3 */
  int32_t use_base;
  float mu_bar, scale;                 /* mean and std of the INR output */
  float k;                             /* t of the soft-bound test */
  float miss_target, accept_target;    /* 1e-4, 1e-3 */
  int64_t min_level_kept;              /* 20000 */
  int32_t accept_leaves;
} isx_surrogate_fit_params;
isx_status isx_surrogate_fit(isx_ctx* ctx, int32_t mlp_id, const isx_mesh* visited,
                             const isx_surrogate_fit_params* params, int32_t* sur_id,
                             isx_surrogate_calibration* cal, float* h_loss);

/* isx_surrogate_partition: the band partition isx_extract applies at octree
 * level `level` (bands of that level as attached to mlp_id by
 * isx_surrogate_attach, its iso-values, bound multiplier k = t), on n caller
 * cells.  d_pred [n][2] = (mu_hat, sigma_hat) as from isx_surrogate_predict,
 * d_unit [n] the per-cell unit of err_mu (the base scale s_b for a surrogate
 * with a base; NULL = 1), d_parent_mask [n] the iso bits each cell carries.
 * Per carried iso-value c, with d = |mu_hat - c|: outside if
 * d - z err_mu unit > t sigma_hat exp(z err_logsig), inside if
 * d + z_accept err_mu unit < t sigma_hat exp(-z_accept err_logsig), else
 * unsure.  d_fallback[i] = 1 (propagate; d_mask[i] = 0) if some carried
 * iso-value is unsure or the prediction is not finite, or if leaf != 0, the
 * surrogate may not accept leaves and some bit is inside; otherwise
 * d_fallback[i] = 0 and d_mask[i] = the inside bits (0 = pruned).
 * Float32 arithmetic.  Asynchronous.  Errors: ISX_EINVAL (also when no
 * surrogate is attached), ISX_EHIP. */
isx_status isx_surrogate_partition(isx_ctx* ctx, int32_t mlp_id, int64_t n, const float* d_pred,
                                   const float* d_unit, float k, int32_t level, int32_t leaf,
                                   const uint32_t* d_parent_mask, uint32_t* d_mask, uint32_t* d_fallback);

/* isx_distribution_kl: quality of the predicted output distribution over
 * blocks (Sec. V-E and Eq. 11).  For block b with centre d_centres[b][3] and
 * half-sizes d_halves[b][3] (device, float32), the INR is evaluated (float32)
 * at n_samples Monte Carlo points drawn uniformly in the block: point i,
 * axis a, takes u = (SplitMix64 output number (b n_samples + i) 3 + a of the
 * stream with this seed) >> 40, times 2^-24, and the coordinate
 * c_a + h_a (2u - 1) (float64 product and sum, rounded to float32).  The
 * values' histogram has n_bins equal bins on their [min, max] (bin of v:
 * floor((v - min) / (max - min) n_bins), clamped).  Three Gaussians are
 * scored by the KL divergence of Eq. 11 of the histogram density p from
 * their density q, integrated bin by bin in closed form (ln q is a
 * quadratic): UP's (mu, sigma) and RA-UA's (Eq. 5), both from float64
 * propagation of the block, and the maximum-likelihood Gaussian of the first
 * n_fit samples (the few-sample baseline).  d_out [n_blocks][ISX_DIST_FIELDS]
 * float64, columns in isx_dist_field order; KL is NaN when all samples are
 * equal or a sigma is 0.  d_hist [n_blocks][n_bins] (optional, NULL) gets the
 * counts.  Limits: n_samples in [1, 2^31), n_bins in [1, 8192], n_fit in
 * [1, n_samples].  Asynchronous on the context stream; scratch grows to
 * 16 bytes per sample of up to 2^26 samples at once.  Errors: ISX_EINVAL,
 * ISX_ENOMEM, ISX_EHIP. */
typedef enum {
  ISX_DIST_MC_MEAN = 0, ISX_DIST_MC_STD, ISX_DIST_LO, ISX_DIST_HI, ISX_DIST_UP_MU, ISX_DIST_UP_SIGMA,
  ISX_DIST_RAUA_MU, ISX_DIST_RAUA_SIGMA, ISX_DIST_FIT_MU, ISX_DIST_FIT_SIGMA, ISX_DIST_KL_UP, ISX_DIST_KL_RAUA,
  ISX_DIST_KL_FIT, ISX_DIST_FIELDS
} isx_dist_field;
isx_status isx_distribution_kl(isx_ctx* ctx, int32_t mlp_id, int64_t n_blocks, const float* d_centres,
                               const float* d_halves, int64_t n_samples, int32_t n_bins, int32_t n_fit,
                               uint64_t seed, double* d_out, uint32_t* d_hist);

/* isx_surrogate_save_file: write surrogate sur_id to `path` (binary, little
 * endian): "ISXSUR01", int32 n_linear, int32 widths[n_linear + 1], float32
 * mu_bar, S, a, b, s_floor, int32 has_base, then per layer the row-major
 * float32 W and b.  Synchronous.  ISX_EINVAL on a bad id or an unwritable
 * path.
 * isx_surrogate_load_file: read such a file into a new surrogate (*sur_id);
 * a file written with a base becomes corrections to the linearisation of
 * base_mlp_id (which must then be a loaded MLP; -1 is an error for such a
 * file and is required otherwise).  ISX_EINVAL on a missing or malformed
 * file. */
isx_status isx_surrogate_save_file(isx_ctx* ctx, int32_t sur_id, const char* path);
isx_status isx_surrogate_load_file(isx_ctx* ctx, const char* path, int32_t base_mlp_id, int32_t* sur_id);

/* Copy the library's marching-cubes case table: h_count[256] triangles per
 * case (case bit i set iff corner i < iso-value; corners (0,0,0) (1,0,0)
 * (1,1,0) (0,1,0) (0,0,1) (1,0,1) (1,1,1) (0,1,1)), h_edges[256][15] edge
 * indices, 3 per triangle, -1 padded.  Host only; needs no device. */
isx_status isx_mc_case_table(uint8_t* h_count, int8_t* h_edges);

/* Context options. */
typedef enum {
  ISX_KEEP_LEVELS = 1,     /* value 1: meshes keep every level's cells (for testing) */
  ISX_HIDDEN_KERNEL = 2,   /* 0 = automatic, 1 = force the SIMT kernels, 2 = force MFMA, 3 = MFMA with
                              ISX_FP32 UP products as split bfloat16 MFMAs (as ISX_RECHECK_SPLIT gives the
                              re-check cascade's float32 stage; for measuring that stage directly) */
  ISX_PROFILE = 3,         /* value 1: time every hidden-layer launch with HIP events */
  ISX_SCRATCH_BYTES = 4,   /* bytes of propagation scratch per batch (default 16 GiB) */
  ISX_VERBOSE = 5,         /* value 1: isx_extract prints one line per octree level to stderr */
  ISX_BF16_VARIANT = 6,    /* bf16 hidden-layer tile shape: 0 = default for the width; 1..4 (forced shapes)
                              currently return ISX_EUNSUPPORTED */
  ISX_UP_FORM = 7,         /* bf16 uncertainty propagation: 0 (default) = covariance form (exact
                              alternative to coefficient tracking: C_h = W_h (D C_{h-1} D + diag(gamma^2))
                              W_h^T): on chip, one fused launch per batch, for hidden widths <= 256; with
                              the per-cell N x N matrices in device memory, one launch per layer, for nets
                              whose hidden layers all have width 512 or 1024; else the coefficient form.
                              1 = coefficient form; 2 = the device-memory covariance form for nets whose
                              hidden layers share one width of 256, 512 or 1024 (ISX_EUNSUPPORTED for
                              other nets) */
  ISX_LIN_PRECISION = 8,   /* centre linearisation (isx_linearize and the surrogate's base): 1 (default)
                              = bfloat16 MFMA with every column carried as two bfloat16 parts and three
                              bfloat16 products per layer (f within ~3e-4 of max(|f|, output scale), s
                              within ~2e-3 relative; used when every hidden layer has the same width
                              <= 256, else float32), 0 = float32 MFMA */
  ISX_AA_MARGIN = 9,       /* affine arithmetic: 1 = widen every layer by the rounding margin of its
                              floating-point evaluation (operand rounding 2^-8 for bfloat16 products,
                              accumulation 2^-24 float32 / 2^-53 float64), so that the returned range
                              contains the exact range of the network over the box; 0 (default) = the
                              paper's rule (exact arithmetic assumed) evaluated in floating point */
  ISX_BATCH_WORKERS = 10,  /* isx_extract_batch: worker contexts (streams) that run INRs at once, 1..16
                              (default 4) */
  ISX_CANCEL_CHECK = 11,   /* bf16 uncertainty propagation in covariance form: 1 (default) = a cell with a
                              neuron whose variance sum v = sum_i T_ji W_ji (signed, over bfloat16-rounded
                              covariances) keeps at most 2^-9 of the magnitude a = sum_i |T_ji W_ji| of its
                              terms (Eq. 7 needs the variance; such a sum can lose every digit) while its
                              pre-activation y lies where the rule depends on sigma (ReLU, Eq. 9:
                              |y| < 6 sqrt(max(v, 0) + 2^-7 a); ELU: y below that bound; sine, whose rule
                              depends on v smoothly: (1 + 2|y|) 2^-9 a > 2^-20, the largest shift of the
                              centre that the variance error can cause)
                              is propagated again in float64, and its float64 (mu, sigma) is returned;
                              0 = off */
  ISX_AUTOTUNE = 12,       /* bf16 coefficient-form propagation: 1 = pick the hidden-layer tile shape of
                              each MLP by timing the shapes (1, 3, 4 and the default) on 4096 sample
                              cells at its first such propagation (the shapes give identical results);
                              0 (default) = the default shape for the width, or ISX_BF16_VARIANT;
                              1 currently returns ISX_EUNSUPPORTED (switched off with the forced shapes) */
  ISX_BF16_READOFF = 13,   /* bf16 uncertainty propagation: 0 (default) = the output read-off on bf16 MFMA
                              with hi/lo splits of the row vectors and weights where the widths allow;
                              1 = the float32 MFMA read-off (the same vectors; for comparison) */
  ISX_RECHECK_CASCADE = 14, /* isx_extract with ISX_BF16 and a re-check band: 0 (default) = band cells are
                              propagated again in float64 and that result decides; 1 = they are propagated
                              in float32 first, and only those whose float32 bound endpoint lies within
                              1/8 of the band (fp64_band / 8 + fp64_band_rel / 8 * spread) of a carried
                              iso-value go on to float64; the others keep the float32 decision (float32
                              endpoint errors are far below that eighth: <= 1e-5 of max(|o|, S) in the
                              parity tests); isx_mesh_level_rechecked_fp64 counts the float64 cells */
  ISX_DENSE_FROM_LEVEL = 15, /* isx_extract on the octree: 0 (default) = range analysis down to max_depth
                              (Alg. 1); L in [1, max_depth) = range analysis down to level L only, then
                              every level-max_depth cell below an active level-L cell is a leaf for that
                              cell's iso-values (its corners evaluated and marching cubes run on it, as in
                              isx_extract_dense).  A cost choice beyond the paper: refining a busy level
                              by range analysis can cost more than evaluating its subtrees densely.  The
                              surface contains the one of the full refinement (same computation down to
                              level L, and every leaf the refinement keeps lies below an active level-L
                              cell); the mesh records levels 0..L; isx_extract fails with
                              ISX_ECAPACITY above 2^28 leaves or 2^31 (leaf, iso) pairs, and with
                              ISX_EUNSUPPORTED for the k-d tree */
  ISX_RECHECK_SPLIT = 16    /* with ISX_RECHECK_CASCADE 1: 0 (default) = the float32 stage multiplies on
                              float32 MFMA; 1 = its products are three bfloat16 MFMAs of hi/lo splits of
                              the float32 operands (a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi, float32
                              accumulation; about 3 2^-18 of |a b| per term instead of 2^-24), with the
                              same storage, rule and read-off as the float32 stage; UP only (AA keeps
                              float32 products, which its rounding margin assumes) */
} isx_option;
isx_status isx_set_option(isx_ctx* ctx, isx_option option, int64_t value);

/* Kernel kinds timed by ISX_PROFILE. */
typedef enum {
  ISX_KERNEL_HIDDEN_FP32 = 0,      /* hidden-layer product, FP32 MFMA */
  ISX_KERNEL_HIDDEN_BF16 = 1,      /* hidden-layer product, BF16 MFMA */
  ISX_KERNEL_HIDDEN_SIMT_FP32 = 2, /* hidden-layer product, float32 vector ALUs */
  ISX_KERNEL_HIDDEN_FP64 = 3,      /* hidden-layer product, float64 (re-check band, ISX_FP64) */
  ISX_KERNEL_DENSE = 4,            /* dense forward passes (corner evaluation, linearisation) */
  ISX_KERNEL_OUTPUT = 5,           /* output read-off (spread of the last layer) */
  ISX_KERNEL_HIDDEN_COV_BF16 = 6,  /* every hidden layer of uncertainty propagation in covariance form,
                                      BF16 MFMA (on chip or in device memory; the device-memory form's
                                      launches of one chunk count as one) */
  ISX_KERNEL_LINEARIZE = 7         /* centre linearisation (isx_linearize, the surrogate's base) */
} isx_kernel_kind;

/* Accumulated statistics of one kernel kind since the last reset (ISX_PROFILE
 * on): launches, summed device time in ms (HIP events recorded around each
 * launch on the context stream), algorithmic flops and algorithmic bytes.
 * For the hidden-layer kinds: flops = 2 * n_out * n_in * real columns per
 * cell (the real columns of hidden layer h are the 3 input symbols (+1
 * centre in the float32/float64 layouts) and the true widths of layers
 * 1..h-2); bytes = the coefficient block read plus the block written unless
 * it is the last hidden layer, at the storage precision.  For the covariance
 * kind: flops = for layer 2, 14 n_2 n_1 (T_2 from the rank-3 factor of X_1
 * and the variances) plus 2 n_2^2 n_1 for C_2 = T_2 W_2^T; for each later
 * hidden layer h, 2 n_h n_{h-1}^2 for T = W_h X_{h-1} and 2 n_h^2 n_{h-1} for
 * C_h = T W_h^T (the last hidden layer: 2 n_h n_{h-1} for the diagonal of C_h
 * alone); bytes = the cell's centre and half-sizes
 * read plus the four per-neuron float32 vectors written per hidden layer.
 * Synchronises the
 * stream.  reset != 0 clears the counters of every kind. */
isx_status isx_get_profile(isx_ctx* ctx, int32_t kernel, int64_t* launches, double* ms, double* flops,
                           double* bytes, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* ISX_H */
