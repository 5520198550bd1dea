// Internal definitions shared by the gfx950 kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "seele.h"

namespace seele {

constexpr int kMaxViewsPre = 8;       // views handled by one preprocess launch
constexpr int kMaxSegs = 16;          // active segments per preprocess call
constexpr int kMaxViewsBin = 256;     // views per bin_sort call (kernel-argument table)
constexpr int kMaxViewsRaster = 64;   // views per raster launch (kernel-argument table)

constexpr int kSortBlock = 256;       // threads per sort/scan block (4 waves)
constexpr int kSortItems = 16;        // items per thread
constexpr int kSortTile = kSortBlock * kSortItems;


struct CamK {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float C[3];  // camera centre -R^T t (computed on the host in double)
  int W, H, gridW, gridH;
};

struct PreArgs {
  int64_t n;
  int sh_degree;
  int n_views;        // views in this launch (<= kMaxViewsPre)
  int64_t view0;      // index of this launch's first view
  int tile;
  int extent;
  float alpha_min, lowpass, z_near;
  int n_segs;
  int64_t seg_begin[kMaxSegs];
  int64_t seg_end[kMaxSegs];
  CamK cam[kMaxViewsPre];
};

// Super-tiles: square blocks of kSuperTile x kSuperTile tiles (row-major per
// view, numbered after the previous views' super-tiles).  A super-tile list
// entry key is the record's tile rectangle clipped to the super-tile (local
// inclusive x0, x1, y0, y1 of 2 bits each) above the global super-tile id.
constexpr int kSuperTile = 4;
constexpr int kClipShift = 24;
constexpr uint32_t kStMask = (1u << kClipShift) - 1u;

// 16-bit coverage mask of an entry over its super-tile's tiles (bit 4 iy + ix).
__device__ __forceinline__ uint32_t clip_mask(uint32_t clip) {
  const uint32_t xm = ((2u << ((clip >> 2) & 3u)) - 1u) & ~((1u << (clip & 3u)) - 1u);
  const uint32_t y0 = (clip >> 4) & 3u, y1 = (clip >> 6) & 3u;
  const uint32_t rows = ((2u << (4u * y1 + 3u)) - 1u) & ~((1u << (4u * y0)) - 1u);
  return (xm * 0x1111u) & rows;
}

struct BinView {
  int32_t tile_base;  // first global tile of the view
  int32_t st_base;    // first global super-tile of the view
  uint16_t grid_w, grid_h;
};

struct BinViews {
  int n_views;
  int64_t n;     // Gaussians per view
  int64_t n_st;  // super-tiles over all views
  BinView v[kMaxViewsBin];
};

struct RasterView {
  int32_t tile_begin;  // first tile of this view, relative to the launch
  int32_t st_base;     // global id of the view's first super-tile
  int32_t W, H, grid_w;
  int64_t pix_base;    // first pixel of this view in final_T / n_contrib
};

struct RasterViews {
  int n_views;
  int32_t tile_base;   // global id of the launch's first tile
  RasterView v[kMaxViewsRaster];
};

struct RasterParams {
  float alpha_min, alpha_max, T_min;
  float log2_inv_alpha_min;  // log2(1 / alpha_min), for the culling bound
  float bg0, bg1, bg2;
  int group_w, group_h;
};

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Inclusive prefix sum across the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (l >= d) x += y;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Block-wide exclusive scan for blockDim.x == kSortBlock; returns the
// exclusive prefix of `x` and the block total in `total`.  `smem` holds at
// least kSortBlock/64 + 1 elements.  Contains barriers: call uniformly.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T x, T* smem, T& total) {
  constexpr int kWaves = kSortBlock / 64;
  const int w = threadIdx.x >> 6;
  const T inc = wave_inclusive_scan(x);
  if (lane_id() == 63) smem[w] = inc;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const T s = smem[i];
    if (i < w) base += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return base + inc - x;
}

// -------------------------------------------------------------- blending math
// The rasterizers evaluate q = d^T A d (A = conic, d = pixel centre - mean) as
// a sum of squares through the Cholesky factor of A scaled by sqrt(k),
// k = log2(e)/2:
//   A k = L L^T,  L = [[l11, 0], [l21, l22]],
//   k q = (l11 dx + l21 dy)^2 + (l22 dy)^2,   exp(-q/2) = exp2(-k q).
// Unlike the expanded quadratic, the sum of squares does not cancel for
// elongated footprints and needs no clamp at zero.  Preprocessing computes the
// factor once per record, in double precision, from the float32 conic, and
// stores it in the record.
struct Chol {
  float l11, l21, l22;
};

__device__ __forceinline__ Chol conic_factor(float a, float b, float c) {
  const double k = 0.72134752044448170;  // log2(e)/2
  const double ad = a > 0.0f ? (double)a : 0.0;
  const double det = (double)a * (double)c - (double)b * (double)b;  // exact products
  Chol f;
  if (ad > 0.0) {
    const double sa = sqrt(ad);
    f.l11 = (float)(sqrt(k) * sa);
    f.l21 = (float)(sqrt(k) * (double)b / sa);
    f.l22 = (float)sqrt(k * fmax(det / ad, 0.0));
  } else {
    f.l11 = 0.0f;
    f.l21 = 0.0f;
    f.l22 = (float)sqrt(k * fmax((double)c, 0.0));
  }
  return f;
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// The exponent of the unclamped alpha in base 2 with the opacity folded in:
// o exp2(-(u^2 + w^2)) = exp2(-qo) with qo = u^2 + w^2 - log2(o), u and w the
// two linear forms of the pixel offset (d = pixel - mean) through the
// Cholesky factor.  The forward, its leader tests and the backward all use
// this one expression, so they agree on every alpha bit.
__device__ __forceinline__ float splat_qo(float px, float py, float mx, float my, float l11,
                                          float l21, float l22, float log2o, float& dx,
                                          float& dy) {
  dx = px - mx;
  dy = py - my;
  const float u = __builtin_fmaf(l21, dy, l11 * dx);
  const float w = l22 * dy;
  return __builtin_fmaf(u, u, __builtin_fmaf(w, w, -log2o));
}

// alpha = min(alpha_max, raw) for raw = o * exp2(p) >= 0 and alpha_max > 0,
// as one median-of-three (which needs no NaN canonicalisation of alpha_max).
__device__ __forceinline__ float clamp_alpha(float raw, float alpha_max) {
  return __builtin_amdgcn_fmed3f(raw, 0.0f, alpha_max);
}

// Wave-level culling mask of one record for one tile whose top-left pixel is
// (x0, y0).  Bit q (q = 2*row + column of the 8x8 block that wave q owns) is
// cleared only if alpha < alpha_min at every pixel centre of block q as the
// blending loops compute it in float32 (splat_qo, fast_exp2, clamp_alpha).
// Over a block's centres the two linear forms u = l11 dx + l21 dy and
// w = l22 dy range over intervals (l11, l22 > 0); the squared distances of
// those intervals from zero add up to a lower bound of k q.  alpha >=
// alpha_min needs k q <= log2(o / alpha_min), so a block is cleared when the
// bound exceeds that by a margin covering the float32 rounding of the loop's
// evaluation and of the bound itself (relative to the squared magnitude S^2
// of the terms, taken over the whole tile), plus 1e-3 for the logarithms and
// exp2.  A NaN or infinite input makes the margin NaN or infinite and leaves
// every bit set.  log2o = log2(o) as the loops use it; log2_inv_amin =
// log2(1 / alpha_min).
template <int TS>
__device__ __forceinline__ uint32_t quad_mask(float mx, float my, float l11, float l21, float l22,
                                              float log2o, float log2_inv_amin, int x0, int y0) {
  constexpr int NB = TS / 8;  // 8x8 blocks per tile row
  const float X0 = ((float)x0 + 0.5f) - mx, Y0 = ((float)y0 + 0.5f) - my;
  const float ax = __builtin_fabsf(X0) + (float)(TS - 1);
  const float ay = __builtin_fabsf(Y0) + (float)(TS - 1);
  const float S = l11 * ax + __builtin_fabsf(l21) * ay, Wm = l22 * ay;
  const float thr = ((log2o + log2_inv_amin) + 1e-3f) + 4e-6f * (S * S + Wm * Wm);
  const float ux = l11 * X0, ux7 = ux + 7.0f * l11, step = 8.0f * l11;
  uint32_t m = 0;
#pragma unroll
  for (int by = 0; by < NB; ++by) {
    const float ylo = Y0 + (float)(8 * by), yhi = ylo + 7.0f;
    const float a = l21 * ylo, b = l21 * yhi;
    const float lo = ux + __builtin_fminf(a, b), hi = ux7 + __builtin_fmaxf(a, b);
    const float dw = l22 * __builtin_fmaxf(__builtin_fmaxf(ylo, -yhi), 0.0f);
    const float w2 = dw * dw;
#pragma unroll
    for (int bx = 0; bx < NB; ++bx) {
      const float ulo = bx ? lo + step : lo, uhi = bx ? hi + step : hi;
      const float du = __builtin_fmaxf(__builtin_fmaxf(ulo, -uhi), 0.0f);
      if (!(__builtin_fmaf(du, du, w2) > thr)) m |= 1u << (by * NB + bx);
    }
  }
  return m;
}

// Binning input staged by preprocessing (in the bin-sort workspace): per span
// (view v, preprocess workgroup b; span = v * n_blocks + b, 256 records) the
// visible records' depth keys and ids compacted to the span's start, the
// span's count, and every record's packed tile rectangle.
struct BinStage {
  uint32_t* keys;
  uint32_t* ids;
  uint32_t* prect;  // packed tile rectangle per slot (pack_rect8), beside the ids
  uint64_t* span_count;
  uint2* rid;
  int64_t n_blocks;  // ceil(n / 256)
};

// A non-empty tile rectangle [x0, x1) x [y0, y1) inside a grid of at most
// 256 x 256 tiles in 32 bits: x0, x1 - 1, y0, y1 - 1, one byte each (rect_x /
// rect_y hold x0 | x1 << 16 and y0 | y1 << 16).  Outside such grids the
// value is not used.
__host__ __device__ inline uint32_t pack_rect8(uint32_t rect_x, uint32_t rect_y) {
  return (rect_x & 0xffu) | (((rect_x >> 16) - 1u) & 0xffu) << 8 | (rect_y & 0xffu) << 16 |
         (((rect_y >> 16) - 1u) & 0xffu) << 24;
}

// ------------------------------------------------------------- host launchers
hipError_t launch_preprocess(const PreArgs& a, const seele_gaussians& g, seele_splat* splats,
                             int32_t* n_tiles, hipStream_t stream,
                             const BinStage* stage = nullptr);

struct BinSortPlan {
  int64_t n_records;      // n_views * n
  int64_t capacity;       // pair capacity
  int64_t n_tiles_total;
  int64_t max_st;         // bound on super-tiles (n_tiles_total)
  int64_t max_seg;        // bound on write segments
  // workspace carve-up (byte offsets)
  size_t off_hdr, off_partial, off_partial2, off_dkeys0, off_dkeys1, off_dvals0, off_dvals1;
  size_t off_skeys0, off_skeys1, off_svals0, off_svals1, off_rx, off_ry, off_rid, off_span;
  size_t off_prect0, off_prect1;  // packed rectangles riding along the depth sort
  size_t off_hist, off_digits, off_st_range, off_st_seg, off_seg_st, off_seg_cnt;
  size_t off_tile_cnt, off_tile_start, total;
};
BinSortPlan plan_bin_sort(int64_t n_records, int64_t capacity, int64_t n_tiles_total);
// Per-tile lists (sorted_ids, tile_ranges), or (super) the super-tile lists:
// entry keys and ids (sorted_ids) in list order and super-tile ranges
// (tile_ranges then holds n_st pairs).  staged: the visible records come from
// the stage that preprocessing wrote into ws (bin_stage_of), not from
// splats / n_tiles.
hipError_t launch_bin_sort(const BinSortPlan& p, const BinViews& views, const seele_splat* splats,
                           const int32_t* n_tiles, void* ws, uint32_t* sorted_ids,
                           int32_t* tile_ranges, int64_t* num_pairs, hipStream_t stream,
                           bool super = false, uint32_t* entry_keys = nullptr,
                           bool staged = false);
// Where preprocessing stages the binning input inside a bin-sort workspace.
BinStage bin_stage_of(const BinSortPlan& p, void* ws, int64_t n);

bool raster_batch_supported(int tile, int batch);

// Offline contribution pass: per-pixel top-k (k <= 32) marks and sums.
hipError_t launch_contrib_topk(int tile, const RasterViews& views, int n_tiles_launch,
                               const RasterParams& rp, const seele_splat* splats,
                               const uint32_t* sorted_ids, const int32_t* tile_ranges, int k_top,
                               uint8_t* mark, float* contrib_sum, hipStream_t stream);

// Forward over super-tile lists (one LDS batch of two entries per thread).
hipError_t launch_raster_fwd_super(int tile, int mode, const RasterViews& views,
                                   int n_tiles_launch, const RasterParams& rp,
                                   const seele_splat* splats, const uint32_t* entry_keys,
                                   const uint32_t* entry_ids, const int32_t* st_ranges,
                                   float* image, float* final_T, int32_t* n_contrib,
                                   unsigned long long* counters, int32_t* last_entry,
                                   hipStream_t stream);

hipError_t launch_raster_fwd(int tile, int mode, int batch, const RasterViews& views,
                             int n_tiles_launch, const RasterParams& rp,
                             const seele_splat* splats, const uint32_t* sorted_ids,
                             const int32_t* tile_ranges, float* image, float* final_T,
                             int32_t* n_contrib, unsigned long long* counters,
                             hipStream_t stream);

hipError_t launch_raster_fwd_queue(int tile, int mode, int batch, const RasterViews& views,
                                   int n_tiles_launch, const RasterParams& rp,
                                   const seele_splat* splats, const uint32_t* sorted_ids,
                                   const int32_t* tile_ranges, float* image, float* final_T,
                                   int32_t* n_contrib, uint32_t* counter, const uint32_t* order,
                                   int n_workgroups, hipStream_t stream);

hipError_t launch_tile_order_keys(const int32_t* tile_ranges, int32_t tile_base, uint32_t n,
                                  uint32_t* keys, uint32_t* vals, uint32_t* counter,
                                  hipStream_t stream);
hipError_t launch_zero_counter(uint32_t* counter, hipStream_t stream);

size_t radix_sort_workspace_size(int64_t n);
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, int64_t n, int bits, void* ws,
                            hipStream_t stream);

hipError_t launch_preprocess_bwd(const PreArgs& a, const seele_gaussians& g,
                                 const int32_t* n_tiles, const float* grad2d,
                                 const seele_gaussian_grads& out, bool accumulate,
                                 hipStream_t stream);

hipError_t launch_raster_bwd_quad(int mode, const RasterViews& views, int n_st_launch,
                                  const RasterParams& rp, const seele_splat* splats,
                                  const uint32_t* entry_ids, const uint32_t* entry_keys,
                                  const int32_t* st_ranges, const float* final_T,
                                  const int32_t* last_entry, const float* dL_dimage, float* grad2d,
                                  hipStream_t stream);
hipError_t launch_raster_bwd(int tile, int mode, const RasterViews& views, int n_tiles_launch,
                             const RasterParams& rp, const seele_splat* splats,
                             const uint32_t* sorted_ids, const int32_t* tile_ranges,
                             const float* final_T, const int32_t* n_contrib,
                             const float* dL_dimage, float* grad2d, hipStream_t stream);

}  // namespace seele
