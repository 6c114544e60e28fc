// Octree level construction, classification, stream compaction, leaf
// corners and marching cubes (Alg. 1 and Sec. IV-D).
//
// Cells are Morton ids at their level (x bit lowest; 3*level <= 30 bits), so
// the children of an active list in Morton order are again in Morton order
// and the level loop never sorts.  Compaction is stable: a three-phase scan
// (per-block counts, one-block scan of the counts, per-block scatter using
// wavefront ballots), deterministic and free of atomics on values.
#include "isx_internal.h"

#include <algorithm>

namespace isx {

// Every third bit of x starting at bit 0, packed (10 output bits).
__device__ __forceinline__ uint32_t unspread3(uint32_t x) {
  x &= 0x09249249u;
  x = (x ^ (x >> 2)) & 0x030c30c3u;
  x = (x ^ (x >> 4)) & 0x0300f00fu;
  x = (x ^ (x >> 8)) & 0xff0000ffu;
  x = (x ^ (x >> 16)) & 0x000003ffu;
  return x;
}

struct Domain {
  double lo[3];
  double step[3];  // (hi - lo) / 2^(level + 1): half the cell size
};

static Domain make_domain(const Model& m, int level) {
  Domain d;
  for (int a = 0; a < 3; ++a) {
    d.lo[a] = m.lo[a];
    d.step[a] = ((double)m.hi[a] - (double)m.lo[a]) / (double)(1ull << (level + 1));
  }
  return d;
}

// Box of cell (i, j, k) at the level: centre lo + (2i+1) step, half-width step
// (the box of Alg. 1), computed in float64 and rounded once to float32.
__device__ __forceinline__ void cell_box(uint32_t id, const Domain& d, float* c, float* h) {
  const uint32_t ijk[3] = {unspread3(id), unspread3(id >> 1), unspread3(id >> 2)};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    c[a] = (float)(d.lo[a] + (double)(2 * ijk[a] + 1) * d.step[a]);
    h[a] = (float)d.step[a];
  }
}

__global__ void root_kernel(Domain d, uint32_t full, uint32_t* ids, uint32_t* pmask, float* centres,
                            float* halves) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  ids[0] = 0;
  pmask[0] = full;
  cell_box(0, d, centres, halves);
}

__global__ void children_kernel(int64_t n_par, const uint32_t* __restrict__ par_ids,
                                const uint32_t* __restrict__ par_masks, Domain d, uint32_t* __restrict__ ids,
                                uint32_t* __restrict__ pmask, float* __restrict__ centres,
                                float* __restrict__ halves) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 8 * n_par) return;
  const int64_t p = i >> 3;
  const uint32_t id = (par_ids[p] << 3) | (uint32_t)(i & 7);
  ids[i] = id;
  pmask[i] = par_masks[p];
  float c[3], h[3];
  cell_box(id, d, c, h);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    centres[i * 3 + a] = c[a];
    halves[i * 3 + a] = h[a];
  }
}

hipError_t launch_root(const Model& m, uint32_t full_mask, uint32_t* ids, uint32_t* pmask, float* centres,
                       float* halves, hipStream_t s) {
  hipLaunchKernelGGL(root_kernel, dim3(1), dim3(64), 0, s, make_domain(m, 0), full_mask, ids, pmask, centres,
                     halves);
  return hipGetLastError();
}

hipError_t launch_children(const Model& m, int level, int64_t n_par, const uint32_t* par_ids,
                           const uint32_t* par_masks, uint32_t* ids, uint32_t* pmask, float* centres,
                           float* halves, hipStream_t s) {
  if (n_par <= 0) return hipSuccess;
  const int64_t n = 8 * n_par;
  hipLaunchKernelGGL(children_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n_par, par_ids,
                     par_masks, make_domain(m, level), ids, pmask, centres, halves);
  return hipGetLastError();
}

// Every cell of one level as a leaf for every iso-value (the dense
// baseline): ids 0 .. n-1 are the level's Morton codes in order.
__global__ void dense_leaves_kernel(int64_t n, uint32_t full, uint32_t* __restrict__ ids,
                                    uint32_t* __restrict__ masks) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  ids[i] = (uint32_t)i;
  masks[i] = full;
}

hipError_t launch_dense_leaves(int64_t n, uint32_t full, uint32_t* ids, uint32_t* masks, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dense_leaves_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, full, ids, masks);
  return hipGetLastError();
}

__global__ void subtree_leaves_kernel(int64_t n, int shift, const uint32_t* __restrict__ par_ids,
                                      const uint32_t* __restrict__ par_masks, uint32_t* __restrict__ ids,
                                      uint32_t* __restrict__ masks) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p = i >> shift;
  ids[i] = (par_ids[p] << shift) | (uint32_t)(i & (((int64_t)1 << shift) - 1));
  masks[i] = par_masks[p];
}

hipError_t launch_subtree_leaves(int64_t n_par, int levels, const uint32_t* par_ids, const uint32_t* par_masks,
                                 uint32_t* ids, uint32_t* masks, hipStream_t s) {
  const int64_t n = n_par << (3 * levels);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(subtree_leaves_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, 3 * levels,
                     par_ids, par_masks, ids, masks);
  return hipGetLastError();
}

// ------------------------------------------------------------ k-d tree
// Alg. 1's own tree: every node is split in two along its widest dimension,
// ties broken x, then y, then z.  On a cube domain all nodes of a depth have
// the same shape and the split axes cycle x, y, z, so node (depth l, id) --
// children 2 id (lower half) and 2 id + 1 (upper half) -- has, read from the
// top of its l bits, one side bit per split, split s along axis s mod 3.
struct KdDomain {
  double lo[3];
  double ext[3];  // hi - lo
};

__device__ __forceinline__ void kd_box(uint32_t id, int depth, const KdDomain& d, float* c, float* h) {
  uint32_t ijk[3] = {0u, 0u, 0u};
  int cnt[3] = {0, 0, 0};
  for (int s = 0; s < depth; ++s) {
    const int a = s % 3;
    ijk[a] = (ijk[a] << 1) | ((id >> (depth - 1 - s)) & 1u);
    ++cnt[a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double step = d.ext[a] / (double)(2ull << cnt[a]);  // half the node size along a
    c[a] = (float)(d.lo[a] + (double)(2 * ijk[a] + 1) * step);
    h[a] = (float)step;
  }
}

__global__ void children_kd_kernel(int64_t n_par, const uint32_t* __restrict__ par_ids,
                                   const uint32_t* __restrict__ par_masks, int depth, KdDomain d,
                                   uint32_t* __restrict__ ids, uint32_t* __restrict__ pmask,
                                   float* __restrict__ centres, float* __restrict__ halves) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * n_par) return;
  const int64_t p = i >> 1;
  const uint32_t id = (par_ids[p] << 1) | (uint32_t)(i & 1);
  ids[i] = id;
  pmask[i] = par_masks[p];
  float c[3], h[3];
  kd_box(id, depth, d, c, h);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    centres[i * 3 + a] = c[a];
    halves[i * 3 + a] = h[a];
  }
}

static KdDomain make_kd_domain(const Model& m) {
  KdDomain d;
  for (int a = 0; a < 3; ++a) {
    d.lo[a] = m.lo[a];
    d.ext[a] = (double)m.hi[a] - (double)m.lo[a];
  }
  return d;
}

hipError_t launch_children_kd(const Model& m, int depth, int64_t n_par, const uint32_t* par_ids,
                              const uint32_t* par_masks, uint32_t* ids, uint32_t* pmask, float* centres,
                              float* halves, hipStream_t s) {
  if (n_par <= 0) return hipSuccess;
  const int64_t n = 2 * n_par;
  hipLaunchKernelGGL(children_kd_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n_par, par_ids,
                     par_masks, depth, make_kd_domain(m), ids, pmask, centres, halves);
  return hipGetLastError();
}

// k-d node ids of depth 3 D -> octree Morton ids of level D (x bit lowest):
// each triple of k-d bits holds the (x, y, z) sides from the top.
__global__ void kd_to_morton_kernel(int64_t n, int levels, uint32_t* __restrict__ ids) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t v = ids[i];
  uint32_t out = 0;
  for (int q = 0; q < levels; ++q) {
    const uint32_t t = (v >> (3 * q)) & 7u;
    out |= (((t >> 2) & 1u) | (((t >> 1) & 1u) << 1) | ((t & 1u) << 2)) << (3 * q);
  }
  ids[i] = out;
}

hipError_t launch_kd_to_morton(int64_t n, int levels, uint32_t* ids, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(kd_to_morton_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, levels, ids);
  return hipGetLastError();
}

// Soft/hard bound test of Alg. 1 for every iso-value; the interval is
// closed (a bound touching c keeps the cell).
__global__ void classify_kernel(int64_t n, const float* __restrict__ out, float k, IsoList iso,
                                const uint32_t* __restrict__ pmask, uint32_t* __restrict__ mask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float c = out[2 * i], s = out[2 * i + 1];
  // each operation rounded separately (no fused multiply-add), so the test is
  // reproducible as lo = c - (k*s), hi = c + (k*s) in float32
  const float ks = __fmul_rn(k, s);
  const float lo = __fsub_rn(c, ks), hi = __fadd_rn(c, ks);
  uint32_t bits = 0;
  for (int j = 0; j < iso.n; ++j)
    if (lo <= iso.c[j] && iso.c[j] <= hi) bits |= 1u << j;
  mask[i] = bits & (pmask ? pmask[i] : 0xffffffffu);
}

hipError_t launch_classify(int64_t n, const float* out, float k, const IsoList& iso, const uint32_t* pmask,
                           uint32_t* mask, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(classify_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, out, k, iso, pmask,
                     mask);
  return hipGetLastError();
}

// ------------------------------------------------------------------ scans
// Generic exclusive scan of per-element uint32 counts given by a functor,
// in three phases.  SCAN_BLOCK threads, SCAN_ITEMS consecutive elements per
// thread, so a block covers SCAN_TILE consecutive elements.
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* total) {
  // 256 threads = 4 waves of 64
  __shared__ uint64_t wsum[SCAN_BLOCK / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint64_t base = 0, tot = 0;
  for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
    if (w < wave) base += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

template <typename F>
__global__ void scan_reduce_kernel(int64_t n, F f, uint64_t* __restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < n) s += f(base + i);
  uint64_t tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One block: exclusive scan of the block partials in place; total to *d_total.
__global__ void scan_partials_kernel(int64_t nb, uint64_t* __restrict__ partial, int64_t* __restrict__ d_total) {
  uint64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += SCAN_BLOCK) {
    const int64_t i = b0 + threadIdx.x;
    const uint64_t v = i < nb ? partial[i] : 0;
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan(v, &tot);
    if (i < nb) partial[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && d_total) *d_total = (int64_t)carry;
}

// Exclusive offsets per element, out[i] = sum_{j<i} f(j).
template <typename F>
__global__ void scan_apply_kernel(int64_t n, F f, const uint64_t* __restrict__ partial, uint32_t* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = base + i < n ? f(base + i) : 0u;
    s += v[i];
  }
  uint64_t tot;
  uint64_t run = partial[blockIdx.x] + block_exclusive_scan(s, &tot);
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (base + i < n) out[base + i] = (uint32_t)run;
    run += v[i];
  }
}

size_t scan_tmp_bytes(int64_t n) { return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE + 1) * sizeof(uint64_t); }

template <typename F>
static hipError_t exclusive_scan(int64_t n, F f, uint32_t* out, int64_t* d_total, void* tmp, hipStream_t s) {
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  uint64_t* partial = reinterpret_cast<uint64_t*>(tmp);
  if (nb > 0) hipLaunchKernelGGL(scan_reduce_kernel<F>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, n, f, partial);
  hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(SCAN_BLOCK), 0, s, nb, partial, d_total);
  if (nb > 0 && out)
    hipLaunchKernelGGL(scan_apply_kernel<F>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, n, f, partial, out);
  return hipGetLastError();
}

// ------------------------------------------------------------- compaction
struct NonZero {
  const uint32_t* mask;
  __device__ uint32_t operator()(int64_t i) const { return mask[i] != 0u; }
};

// Scatter of the nonzero entries; a block handles SCAN_TILE elements in
// SCAN_ITEMS rounds of 256 consecutive ones, ranks from wavefront ballots.
__global__ void compact_scatter_kernel(int64_t n, const uint32_t* __restrict__ mask, const uint32_t* __restrict__ ids,
                                       const uint64_t* __restrict__ partial, uint32_t* __restrict__ out_idx,
                                       uint32_t* __restrict__ out_mask) {
  __shared__ uint32_t wcnt[SCAN_BLOCK / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t run = partial[blockIdx.x];
  const int64_t tile = (int64_t)blockIdx.x * SCAN_TILE;
  for (int r = 0; r < SCAN_ITEMS; ++r) {
    const int64_t i = tile + (int64_t)r * SCAN_BLOCK + threadIdx.x;
    const uint32_t mk = i < n ? mask[i] : 0u;
    const bool keep = mk != 0u;
    const uint64_t ball = __ballot(keep);
    const uint32_t below = (uint32_t)__popcll(ball & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) wcnt[wave] = (uint32_t)__popcll(ball);
    __syncthreads();
    uint32_t wbase = 0, rtot = 0;
    for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
      if (w < wave) wbase += wcnt[w];
      rtot += wcnt[w];
    }
    if (keep) {
      const uint64_t pos = run + wbase + below;
      out_idx[pos] = ids ? ids[i] : (uint32_t)i;
      if (out_mask) out_mask[pos] = mk;
    }
    run += rtot;
    __syncthreads();
  }
}

size_t compact_tmp_bytes(int64_t n) { return scan_tmp_bytes(n); }

hipError_t launch_compact(int64_t n, const uint32_t* mask, const uint32_t* ids, uint32_t* out_idx,
                          uint32_t* out_mask, int64_t* d_count, void* tmp, hipStream_t s) {
  hipError_t e = exclusive_scan(n, NonZero{mask}, nullptr, d_count, tmp, s);
  if (e != hipSuccess) return e;
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb > 0)
    hipLaunchKernelGGL(compact_scatter_kernel, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, n, mask, ids,
                       reinterpret_cast<const uint64_t*>(tmp), out_idx, out_mask);
  return hipGetLastError();
}

// ---------------------------------------------------------------- corners
__global__ void fill_u32_kernel(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

size_t corner_bitmap_words(int depth) {
  const uint64_t r1 = (1ull << depth) + 1;
  return (size_t)((r1 * r1 * r1 + 31) / 32);
}

__device__ __forceinline__ uint32_t grid_index(uint32_t i, uint32_t j, uint32_t k, uint32_t r1) {
  return i + r1 * (j + r1 * k);
}

// Mark the 8 corners of every active leaf in a bitmap over grid points.
__global__ void corner_mark_kernel(int64_t n, const uint32_t* __restrict__ ids, uint32_t r1,
                                   uint32_t* __restrict__ bitmap) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 8 * n) return;
  const uint32_t id = ids[t >> 3];
  const uint32_t c = (uint32_t)(t & 7);
  const uint32_t g = grid_index(unspread3(id) + (c & 1), unspread3(id >> 1) + ((c >> 1) & 1),
                                unspread3(id >> 2) + ((c >> 2) & 1), r1);
  atomicOr(&bitmap[g >> 5], 1u << (g & 31));
}

hipError_t launch_corner_mark(int depth, int64_t n_leaves, const uint32_t* leaf_ids, uint32_t* bitmap,
                              uint64_t words, hipStream_t s) {
  hipError_t e = launch_fill_u32(bitmap, words, 0u, s);
  if (e != hipSuccess || n_leaves <= 0) return e;
  const int64_t t = 8 * n_leaves;
  hipLaunchKernelGGL(corner_mark_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, n_leaves, leaf_ids,
                     (uint32_t)((1u << depth) + 1), bitmap);
  return hipGetLastError();
}

struct PopWord {
  const uint32_t* w;
  __device__ uint32_t operator()(int64_t i) const { return (uint32_t)__popc(w[i]); }
};

__global__ void corner_list_kernel(uint64_t words, const uint32_t* __restrict__ bitmap,
                                   const uint32_t* __restrict__ word_prefix, uint32_t* __restrict__ corner_g) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= words) return;
  uint32_t w = bitmap[i];
  uint32_t pos = word_prefix[i];
  while (w) {
    const int b = __ffs(w) - 1;
    corner_g[pos++] = (uint32_t)(i * 32 + b);
    w &= w - 1;
  }
}

hipError_t launch_corner_list(int depth, uint64_t words, const uint32_t* bitmap, uint32_t* word_prefix,
                              int64_t* d_count, void* tmp, size_t tmp_bytes, uint32_t* corner_g, hipStream_t s) {
  (void)depth;
  (void)tmp_bytes;
  hipError_t e = exclusive_scan((int64_t)words, PopWord{bitmap}, word_prefix, d_count, tmp, s);
  if (e != hipSuccess) return e;
  if (corner_g)
    hipLaunchKernelGGL(corner_list_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, words, bitmap,
                       word_prefix, corner_g);
  return hipGetLastError();
}

// Grid point coordinates lo + g * (hi - lo) / 2^depth (float64, rounded once).
struct GridGeom {
  double lo[3];
  double cs[3];  // cell size at the leaf level
};

static GridGeom make_grid(const Model& m, int depth) {
  GridGeom g;
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = m.lo[a];
    g.cs[a] = ((double)m.hi[a] - (double)m.lo[a]) / (double)(1ull << depth);
  }
  return g;
}

__global__ void corner_points_kernel(int64_t n, const uint32_t* __restrict__ corner_g, uint32_t r1, GridGeom d,
                                     float* __restrict__ pts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t g = corner_g[i];
  const uint32_t gi[3] = {g % r1, (g / r1) % r1, g / (r1 * r1)};
#pragma unroll
  for (int a = 0; a < 3; ++a) pts[i * 3 + a] = (float)(d.lo[a] + (double)gi[a] * d.cs[a]);
}

hipError_t launch_corner_points(const Model& m, int depth, int64_t n, const uint32_t* corner_g, float* pts,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(corner_points_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, corner_g,
                     (uint32_t)((1u << depth) + 1), make_grid(m, depth), pts);
  return hipGetLastError();
}

// --------------------------------------------------------- marching cubes
__constant__ uint8_t c_tri_count[256];
__constant__ int8_t c_tri_edges[256][15];

hipError_t upload_mc_table() {
  const McTable& t = mc_table();
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_tri_count), t.count, sizeof(t.count));
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_tri_edges), t.edges, sizeof(t.edges));
}

// Each edge's (lower, upper) corners and axis.
__constant__ uint8_t c_edge_lo[12] = {0, 1, 3, 0, 4, 5, 7, 4, 0, 1, 2, 3};
__constant__ uint8_t c_edge_hi[12] = {1, 2, 2, 3, 5, 6, 6, 7, 4, 5, 6, 7};
__constant__ uint8_t c_edge_axis[12] = {0, 1, 0, 1, 0, 1, 0, 1, 2, 2, 2, 2};

struct LeafCtx {
  const uint32_t* ids;
  const uint32_t* masks;
  const uint32_t* bitmap;
  const uint32_t* prefix;
  const float* vals;
  uint32_t r1;
  int n_iso;
  IsoList iso;
};

__device__ __forceinline__ float corner_value(const LeafCtx& L, uint32_t g) {
  const uint32_t w = L.bitmap[g >> 5];
  const uint32_t below = w & ((1u << (g & 31)) - 1u);
  return L.vals[L.prefix[g >> 5] + __popc(below)];
}

// Corner c of a cell in marching-cubes order: (0,0,0) (1,0,0) (1,1,0)
// (0,1,0) (0,0,1) (1,0,1) (1,1,1) (0,1,1).
__constant__ uint8_t c_corner_dx[8] = {0, 1, 1, 0, 0, 1, 1, 0};
__constant__ uint8_t c_corner_dy[8] = {0, 0, 1, 1, 0, 0, 1, 1};
__constant__ uint8_t c_corner_dz[8] = {0, 0, 0, 0, 1, 1, 1, 1};

__device__ __forceinline__ void leaf_corners(const LeafCtx& L, uint32_t id, uint32_t g[8], float v[8]) {
  const uint32_t i = unspread3(id), j = unspread3(id >> 1), k = unspread3(id >> 2);
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    g[c] = grid_index(i + c_corner_dx[c], j + c_corner_dy[c], k + c_corner_dz[c], L.r1);
    v[c] = corner_value(L, g[c]);
  }
}

__device__ __forceinline__ uint32_t mc_case(const float v[8], float c) {
  uint32_t k = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) k |= (v[i] < c ? 1u : 0u) << i;
  return k;
}

struct TriCount {
  LeafCtx L;
  __device__ uint32_t operator()(int64_t p) const {
    const int64_t leaf = p / L.n_iso;
    const int j = (int)(p - leaf * L.n_iso);
    if (!((L.masks[leaf] >> j) & 1u)) return 0u;
    uint32_t g[8];
    float v[8];
    leaf_corners(L, L.ids[leaf], g, v);
    return c_tri_count[mc_case(v, L.iso.c[j])];
  }
};

static LeafCtx make_leaf_ctx(const Model& m, int depth, const uint32_t* ids, const uint32_t* masks,
                             const uint32_t* bitmap, const uint32_t* prefix, const float* vals) {
  LeafCtx L;
  L.ids = ids;
  L.masks = masks;
  L.bitmap = bitmap;
  L.prefix = prefix;
  L.vals = vals;
  L.r1 = (1u << depth) + 1;
  L.n_iso = m.n_iso;
  L.iso.n = m.n_iso;
  for (int j = 0; j < ISX_MAX_ISO; ++j) L.iso.c[j] = j < m.n_iso ? m.iso[j] : 0.f;
  return L;
}

hipError_t launch_mc_count(const Model& m, int depth, int64_t n_leaves, const uint32_t* leaf_ids,
                           const uint32_t* leaf_masks, const uint32_t* bitmap, const uint32_t* word_prefix,
                           const float* corner_vals, uint32_t* tri_offsets, int64_t* d_total, void* tmp,
                           size_t tmp_bytes, hipStream_t s) {
  (void)tmp_bytes;
  TriCount f{make_leaf_ctx(m, depth, leaf_ids, leaf_masks, bitmap, word_prefix, corner_vals)};
  return exclusive_scan(n_leaves * m.n_iso, f, tri_offsets, d_total, tmp, s);
}

// Emit the triangles of one (leaf, iso) pair: vertices interpolated along
// the grid edge from its lower to its upper corner, keyed by the edge.
__global__ void mc_emit_kernel(int64_t n_pairs, LeafCtx L, GridGeom geo, const uint32_t* __restrict__ offsets,
                               float* __restrict__ tri_pos, uint64_t* __restrict__ tri_keys,
                               int32_t* __restrict__ tri_iso) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const int64_t leaf = p / L.n_iso;
  const int j = (int)(p - leaf * L.n_iso);
  if (!((L.masks[leaf] >> j) & 1u)) return;
  uint32_t g[8];
  float v[8];
  leaf_corners(L, L.ids[leaf], g, v);
  const float c = L.iso.c[j];
  const uint32_t cs = mc_case(v, c);
  const int nt = c_tri_count[cs];
  const uint32_t base = offsets[p];
  for (int t = 0; t < nt; ++t) {
    const uint64_t o = (uint64_t)base + t;
    tri_iso[o] = j;
    for (int q = 0; q < 3; ++q) {
      const int e = c_tri_edges[cs][3 * t + q];
      const int a = c_edge_lo[e], b = c_edge_hi[e], ax = c_edge_axis[e];
      const float frac = (c - v[a]) / (v[b] - v[a]);
      const uint32_t ga = g[a];
      const uint32_t gi[3] = {ga % L.r1, (ga / L.r1) % L.r1, ga / (L.r1 * L.r1)};
      for (int d = 0; d < 3; ++d) {
        double x = geo.lo[d] + (double)gi[d] * geo.cs[d];
        if (d == ax) x += (double)frac * geo.cs[d];
        tri_pos[o * 9 + q * 3 + d] = (float)x;
      }
      tri_keys[o * 3 + q] = (uint64_t)ga * 3u + (uint64_t)ax;
    }
  }
}

hipError_t launch_mc_emit(const Model& m, int depth, int64_t n_leaves, const uint32_t* leaf_ids,
                          const uint32_t* leaf_masks, const uint32_t* bitmap, const uint32_t* word_prefix,
                          const float* corner_vals, const uint32_t* tri_offsets, float* tri_pos,
                          uint64_t* tri_keys, int32_t* tri_iso, hipStream_t s) {
  const int64_t n = n_leaves * m.n_iso;
  if (n <= 0) return hipSuccess;
  LeafCtx L = make_leaf_ctx(m, depth, leaf_ids, leaf_masks, bitmap, word_prefix, corner_vals);
  hipLaunchKernelGGL(mc_emit_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, L, make_grid(m, depth),
                     tri_offsets, tri_pos, tri_keys, tri_iso);
  return hipGetLastError();
}

}  // namespace isx

namespace isx {

// ------------------------------------------------------ float64 re-check
// Cells whose float32/bfloat16 bound endpoint lies within `band` of an
// iso-value they still carry are re-propagated in float64, and the float64
// bound decides their mask.
__global__ void band_flags_kernel(int64_t n, const float* __restrict__ out, float k, IsoList iso,
                                  const uint32_t* __restrict__ pmask, float band, float band_rel,
                                  uint32_t* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float c = out[2 * i], s = out[2 * i + 1];
  const float ks = __fmul_rn(k, s);
  const float lo = __fsub_rn(c, ks), hi = __fadd_rn(c, ks);
  const uint32_t pm = pmask ? pmask[i] : 0xffffffffu;
  const float bw = band + band_rel * s;  // this cell's band
  uint32_t f = 0;
  for (int j = 0; j < iso.n; ++j) {
    if (!((pm >> j) & 1u)) continue;
    const float d = fminf(fabsf(lo - iso.c[j]), fabsf(hi - iso.c[j]));
    if (!(d > bw)) f = 1;  // also catches NaN
  }
  flags[i] = f;
}

hipError_t launch_band_flags(int64_t n, const float* out, float k, const IsoList& iso, const uint32_t* pmask,
                             float band, float band_rel, uint32_t* flags, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(band_flags_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, out, k, iso, pmask,
                     band, band_rel, flags);
  return hipGetLastError();
}

__global__ void gather_boxes_kernel(int64_t n, const uint32_t* __restrict__ idx, const float* __restrict__ centres,
                                    const float* __restrict__ halves, float* __restrict__ c_out,
                                    float* __restrict__ h_out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t i = idx[t];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    c_out[t * 3 + a] = centres[i * 3 + a];
    h_out[t * 3 + a] = halves[i * 3 + a];
  }
}

hipError_t launch_gather_boxes(int64_t n, const uint32_t* idx, const float* centres, const float* halves,
                               float* c_out, float* h_out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_boxes_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, idx, centres,
                     halves, c_out, h_out);
  return hipGetLastError();
}

__global__ void recheck_apply_kernel(int64_t n, const uint32_t* __restrict__ idx, const double* __restrict__ out64,
                                     double k, IsoList iso, const uint32_t* __restrict__ pmask, float* __restrict__ out,
                                     uint32_t* __restrict__ mask) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t i = idx[t];
  const double c = out64[2 * t], s = out64[2 * t + 1];
  const double lo = c - k * s, hi = c + k * s;
  uint32_t bits = 0;
  for (int j = 0; j < iso.n; ++j) {
    const double cj = (double)iso.c[j];
    if (lo <= cj && cj <= hi) bits |= 1u << j;
  }
  mask[i] = bits & (pmask ? pmask[i] : 0xffffffffu);
  out[2 * i] = (float)c;
  out[2 * i + 1] = (float)s;
}

// float32 (centre, spread) pairs widened to float64
__global__ void widen_pairs_kernel(int64_t n, const float* __restrict__ src, double* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  dst[2 * t] = (double)src[2 * t];
  dst[2 * t + 1] = (double)src[2 * t + 1];
}

hipError_t launch_widen_pairs(int64_t n, const float* src, double* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(widen_pairs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, src, dst);
  return hipGetLastError();
}

// dst[idx[t]] = src[t] for float64 pairs
__global__ void scatter_pairs_kernel(int64_t n, const uint32_t* __restrict__ idx, const double* __restrict__ src,
                                     double* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t i = idx[t];
  dst[2 * i] = src[2 * t];
  dst[2 * i + 1] = src[2 * t + 1];
}

hipError_t launch_scatter_pairs(int64_t n, const uint32_t* idx, const double* src, double* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_pairs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, idx, src, dst);
  return hipGetLastError();
}

hipError_t launch_recheck_apply(int64_t n, const uint32_t* idx, const double* out64, double k, const IsoList& iso,
                                const uint32_t* pmask, float* out, uint32_t* mask, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(recheck_apply_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, idx, out64, k, iso,
                     pmask, out, mask);
  return hipGetLastError();
}

}  // namespace isx
