// extern "C" entry points of libseele: argument validation on the host, then
// kernel launches on the caller's stream.  Nothing here allocates device
// memory or synchronises.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <algorithm>
#include <array>
#include <string>
#include <vector>

#include "finetune_internal.h"
#include "layout_internal.h"
#include "seele_internal.h"

using namespace seele;

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int32_t hip_fail(hipError_t e, const char* where) {
  return fail(SEELE_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

bool is_finite(float v) { return std::isfinite(v); }

int32_t check_camera(const seele_camera& c, int v, int tile) {
  for (int k = 0; k < 9; ++k)
    if (!is_finite(c.R[k])) return fail(SEELE_ERR_INVALID_ARG, "camera %d: non-finite R", v);
  for (int k = 0; k < 3; ++k)
    if (!is_finite(c.t[k])) return fail(SEELE_ERR_INVALID_ARG, "camera %d: non-finite t", v);
  if (!is_finite(c.fx) || !is_finite(c.fy) || !is_finite(c.cx) || !is_finite(c.cy) || c.fx <= 0 ||
      c.fy <= 0)
    return fail(SEELE_ERR_INVALID_ARG, "camera %d: bad intrinsics", v);
  if (c.width < 1 || c.height < 1)
    return fail(SEELE_ERR_INVALID_ARG, "camera %d: image size %dx%d", v, c.width, c.height);
  const int64_t gw = (c.width + tile - 1) / tile, gh = (c.height + tile - 1) / tile;
  if (gw > 65535 || gh > 65535)
    return fail(SEELE_ERR_UNSUPPORTED, "camera %d: more than 65535 tiles along an axis", v);
  return SEELE_OK;
}

int32_t check_cams(const seele_camera* cams, int32_t n_views, int tile, int max_views) {
  if (!cams) return fail(SEELE_ERR_INVALID_ARG, "cams is null");
  if (n_views < 1) return fail(SEELE_ERR_INVALID_ARG, "n_views must be >= 1 (got %d)", n_views);
  if (n_views > max_views)
    return fail(SEELE_ERR_UNSUPPORTED, "n_views %d exceeds %d", n_views, max_views);
  if (tile != 8 && tile != 16) return fail(SEELE_ERR_INVALID_ARG, "tile must be 8 or 16");
  for (int v = 0; v < n_views; ++v) {
    const int32_t s = check_camera(cams[v], v, tile);
    if (s != SEELE_OK) return s;
  }
  return SEELE_OK;
}

int64_t super_tiles_of(const seele_camera& c, int tile) {
  const int64_t gw = (c.width + tile - 1) / tile, gh = (c.height + tile - 1) / tile;
  return ((gw + kSuperTile - 1) / kSuperTile) * ((gh + kSuperTile - 1) / kSuperTile);
}

int64_t tiles_of(const seele_camera& c, int tile) {
  return (int64_t)((c.width + tile - 1) / tile) * ((c.height + tile - 1) / tile);
}

CamK to_camk(const seele_camera& c, int tile) {
  CamK k{};
  for (int i = 0; i < 9; ++i) k.R[i] = c.R[i];
  for (int i = 0; i < 3; ++i) k.t[i] = c.t[i];
  k.fx = c.fx;
  k.fy = c.fy;
  k.cx = c.cx;
  k.cy = c.cy;
  // camera centre C = -R^T t, in double
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int j = 0; j < 3; ++j) s -= (double)c.R[j * 3 + i] * (double)c.t[j];
    k.C[i] = (float)s;
  }
  k.W = c.width;
  k.H = c.height;
  k.gridW = (c.width + tile - 1) / tile;
  k.gridH = (c.height + tile - 1) / tile;
  return k;
}

int32_t check_gaussians(const seele_gaussians* g) {
  if (!g) return fail(SEELE_ERR_INVALID_ARG, "gaussians is null");
  if (g->n < 0 || g->n >= ((int64_t)1 << 31))
    return fail(SEELE_ERR_INVALID_ARG, "n = %lld out of range", (long long)g->n);
  if (g->sh_degree < 0 || g->sh_degree > 3)
    return fail(SEELE_ERR_INVALID_ARG, "sh_degree %d not in 0..3", g->sh_degree);
  if (g->n > 0) {
    const void* p[5] = {g->means, g->log_scales, g->quats, g->opacity_logits, g->sh};
    const char* nm[5] = {"means", "log_scales", "quats", "opacity_logits", "sh"};
    for (int k = 0; k < 5; ++k) {
      if (!p[k]) return fail(SEELE_ERR_INVALID_ARG, "%s is null", nm[k]);
      if (!aligned(p[k], 4)) return fail(SEELE_ERR_INVALID_ARG, "%s is misaligned", nm[k]);
    }
  }
  return SEELE_OK;
}

int32_t check_preprocess_opts(const seele_preprocess_opts* o, int64_t n) {
  if (!o) return fail(SEELE_ERR_INVALID_ARG, "opts is null");
  if (o->tile != 8 && o->tile != 16) return fail(SEELE_ERR_INVALID_ARG, "tile must be 8 or 16");
  if (o->extent != SEELE_EXTENT_3SIGMA && o->extent != SEELE_EXTENT_OPACITY)
    return fail(SEELE_ERR_INVALID_ARG, "unknown extent mode %d", o->extent);
  if (!(o->alpha_min > 0.0f && o->alpha_min < 1.0f))
    return fail(SEELE_ERR_INVALID_ARG, "alpha_min must be in (0, 1)");
  if (!(o->lowpass >= 0.0f) || !is_finite(o->lowpass))
    return fail(SEELE_ERR_INVALID_ARG, "lowpass must be finite and >= 0");
  if (!(o->z_near > 0.0f) || !is_finite(o->z_near))
    return fail(SEELE_ERR_INVALID_ARG, "z_near must be finite and > 0");
  if (o->n_segs < 0 || o->n_segs > kMaxSegs)
    return fail(SEELE_ERR_UNSUPPORTED, "n_segs %d not in 0..%d", o->n_segs, kMaxSegs);
  if (o->n_segs > 0 && (!o->seg_begin || !o->seg_count))
    return fail(SEELE_ERR_INVALID_ARG, "segment arrays are null");
  for (int s = 0; s < o->n_segs; ++s) {
    const int64_t b = o->seg_begin[s], c = o->seg_count[s];
    if (b < 0 || c < 0 || b > n || c > n - b)
      return fail(SEELE_ERR_INVALID_ARG, "segment %d [%lld, +%lld) outside [0, %lld)", s,
                  (long long)b, (long long)c, (long long)n);
  }
  return SEELE_OK;
}

int32_t check_raster_opts(const seele_raster_opts* o) {
  if (!o) return fail(SEELE_ERR_INVALID_ARG, "raster opts is null");
  if (o->tile != 8 && o->tile != 16) return fail(SEELE_ERR_INVALID_ARG, "tile must be 8 or 16");
  if (o->mode != SEELE_RASTER_PLAIN && o->mode != SEELE_RASTER_CONTRIB)
    return fail(SEELE_ERR_INVALID_ARG, "unknown raster mode %d", o->mode);
  if (o->mode == SEELE_RASTER_CONTRIB) {
    auto ok = [](int g) { return g == 1 || g == 2 || g == 4; };
    if (!ok(o->group_w) || !ok(o->group_h) || o->group_w * o->group_h > 16)
      return fail(SEELE_ERR_INVALID_ARG, "group %dx%d unsupported (each of 1, 2, 4; area <= 16)",
                  o->group_w, o->group_h);
  }
  if (!(o->alpha_min > 0.0f && o->alpha_min < 1.0f))
    return fail(SEELE_ERR_INVALID_ARG, "alpha_min must be in (0, 1)");
  if (!(o->alpha_max > o->alpha_min && o->alpha_max < 1.0f))
    return fail(SEELE_ERR_INVALID_ARG, "alpha_max must be in (alpha_min, 1)");
  if (!(o->T_min > 0.0f && o->T_min < 1.0f))
    return fail(SEELE_ERR_INVALID_ARG, "T_min must be in (0, 1)");
  for (int c = 0; c < 3; ++c)
    if (!is_finite(o->bg[c])) return fail(SEELE_ERR_INVALID_ARG, "non-finite background");
  if (o->lds_batch != 0 && !raster_batch_supported(o->tile, o->lds_batch))
    return fail(SEELE_ERR_INVALID_ARG, "lds_batch %d unsupported for tile %d", o->lds_batch,
                o->tile);
  return SEELE_OK;
}

int batch_of(const seele_raster_opts* o) {
  return o->lds_batch != 0 ? o->lds_batch : o->tile * o->tile;
}

PreArgs make_pre_args(const seele_gaussians* g, const seele_preprocess_opts* opts) {
  PreArgs a{};
  a.n = g->n;
  a.sh_degree = g->sh_degree;
  a.tile = opts->tile;
  a.extent = opts->extent;
  a.alpha_min = opts->alpha_min;
  a.lowpass = opts->lowpass;
  a.z_near = opts->z_near;
  a.n_segs = opts->n_segs;
  for (int k = 0; k < opts->n_segs; ++k) {
    a.seg_begin[k] = opts->seg_begin[k];
    a.seg_end[k] = opts->seg_begin[k] + opts->seg_count[k];
  }
  return a;
}

RasterParams make_raster_params(const seele_raster_opts* opts) {
  RasterParams rp{};
  rp.alpha_min = opts->alpha_min;
  rp.log2_inv_alpha_min = (float)std::log2(1.0 / (double)opts->alpha_min);
  rp.alpha_max = opts->alpha_max;
  rp.T_min = opts->T_min;
  rp.bg0 = opts->bg[0];
  rp.bg1 = opts->bg[1];
  rp.bg2 = opts->bg[2];
  rp.group_w = opts->mode == SEELE_RASTER_CONTRIB ? opts->group_w : 1;
  rp.group_h = opts->mode == SEELE_RASTER_CONTRIB ? opts->group_h : 1;
  return rp;
}

// Views [v0, v0 + nv) as one raster launch; tile_base / pix_base are the
// global tile and pixel offsets of view v0.
RasterViews make_raster_views(const seele_camera* cams, int v0, int nv, int tile,
                              int64_t tile_base, int64_t pix_base, int64_t& n_tiles_out,
                              int64_t& n_pix_out) {
  RasterViews rv{};
  rv.n_views = nv;
  rv.tile_base = (int32_t)tile_base;
  int64_t st = 0;
  for (int k = 0; k < v0; ++k) st += super_tiles_of(cams[k], tile);
  int64_t t = 0, px = 0;
  for (int k = 0; k < nv; ++k) {
    const seele_camera& c = cams[v0 + k];
    rv.v[k].tile_begin = (int32_t)t;
    rv.v[k].st_base = (int32_t)st;
    st += super_tiles_of(c, tile);
    rv.v[k].W = c.width;
    rv.v[k].H = c.height;
    rv.v[k].grid_w = (c.width + tile - 1) / tile;
    rv.v[k].pix_base = pix_base + px;
    t += tiles_of(c, tile);
    px += (int64_t)c.width * c.height;
  }
  n_tiles_out = t;
  n_pix_out = px;
  return rv;
}

// Per Gaussian i, over the n_views records v*n + i of one cluster's views:
// shared |= any top-k mark; the summed contribution replaces best_sum (and
// the cluster best_cluster) if strictly larger, so ties keep the earlier
// cluster.
__global__ void k_hp_accumulate(const uint8_t* __restrict__ mark, const float* __restrict__ sums,
                                int32_t n_views, int64_t n, int32_t cluster,
                                uint8_t* __restrict__ shared, float* __restrict__ best_sum,
                                int32_t* __restrict__ best_cluster) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint8_t any = 0;
  float s = 0.0f;
  for (int v = 0; v < n_views; ++v) {
    any |= mark[(int64_t)v * n + i];
    s += sums[(int64_t)v * n + i];
  }
  if (any) shared[i] = 1;
  if (s > best_sum[i]) {
    best_sum[i] = s;
    best_cluster[i] = cluster;
  }
}

// dst[c] = src[perm[c]] for every attribute (SoA: component-major arrays).
__global__ void k_gather_gaussians(seele_gaussians src, const int64_t* __restrict__ perm,
                                   int64_t n_out, seele_gaussian_grads dst, int n_sh) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_out) return;
  const int64_t i = perm[c];
  const int64_t ns = src.n, nd = n_out;
  for (int k = 0; k < 3; ++k) {
    dst.means[k * nd + c] = src.means[k * ns + i];
    dst.log_scales[k * nd + c] = src.log_scales[k * ns + i];
  }
  for (int k = 0; k < 4; ++k) dst.quats[k * nd + c] = src.quats[k * ns + i];
  dst.opacity_logits[c] = src.opacity_logits[i];
  for (int k = 0; k < n_sh; ++k) dst.sh[k * nd + c] = src.sh[k * ns + i];
}

// Zeroes p[0, n) (p 4-byte aligned): the body with 16-byte stores over a
// bounded grid, the up to three floats before the first 16-byte boundary
// and after the last one singly.
__global__ __launch_bounds__(256) void k_zero_f32(float* p, int64_t n) {
  const int64_t lead = (int64_t)((16u - ((uint32_t)(uintptr_t)p & 15u)) & 15u) / 4;
  const int64_t head = lead < n ? lead : n;
  const int64_t nq = (n - head) / 4;
  const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float4* q = reinterpret_cast<float4*>(p + head);
  for (int64_t i = tid; i < nq; i += (int64_t)gridDim.x * 256) q[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (tid < head) p[tid] = 0.0f;
  const int64_t t0 = head + 4 * nq;
  if (tid < n - t0) p[t0 + tid] = 0.0f;
}

}  // namespace

extern "C" {

const char* seele_last_error(void) { return g_err.c_str(); }

const char* seele_status_string(int32_t s) {
  switch (s) {
    case SEELE_OK: return "SEELE_OK";
    case SEELE_ERR_INVALID_ARG: return "SEELE_ERR_INVALID_ARG";
    case SEELE_ERR_UNSUPPORTED: return "SEELE_ERR_UNSUPPORTED";
    case SEELE_ERR_CAPACITY: return "SEELE_ERR_CAPACITY";
    case SEELE_ERR_HIP: return "SEELE_ERR_HIP";
    default: return "SEELE_ERR_UNKNOWN";
  }
}

int32_t seele_abi_version(void) { return 102; }

int64_t seele_total_tiles(const seele_camera* cams, int32_t n_views, int32_t tile) {
  if (!cams || n_views < 1 || (tile != 8 && tile != 16)) return -1;
  int64_t t = 0;
  for (int v = 0; v < n_views; ++v) {
    if (cams[v].width < 1 || cams[v].height < 1) return -1;
    t += tiles_of(cams[v], tile);
  }
  return t;
}

}  // extern "C"

namespace {

int32_t preprocess_impl(const seele_gaussians* g, const seele_camera* cams, int32_t n_views,
                        const seele_preprocess_opts* opts, seele_splat* splats, int32_t* n_tiles,
                        void* stream, const BinStage* stage) {
  int32_t s = check_gaussians(g);
  if (s != SEELE_OK) return s;
  if ((s = check_preprocess_opts(opts, g->n)) != SEELE_OK) return s;
  if ((s = check_cams(cams, n_views, opts->tile, 1 << 20)) != SEELE_OK) return s;
  if ((int64_t)n_views * g->n >= ((int64_t)1 << 32))
    return fail(SEELE_ERR_UNSUPPORTED, "n_views * n must be < 2^32");
  if (g->n > 0) {
    if (!splats || !aligned(splats, 16))
      return fail(SEELE_ERR_INVALID_ARG, "splats must be non-null and 16-byte aligned");
    if (!n_tiles || !aligned(n_tiles, 4))
      return fail(SEELE_ERR_INVALID_ARG, "n_tiles must be non-null and 4-byte aligned");
  }
  if (g->n == 0) return SEELE_OK;
  PreArgs a = make_pre_args(g, opts);
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int v0 = 0; v0 < n_views; v0 += kMaxViewsPre) {
    const int nv = std::min(kMaxViewsPre, n_views - v0);
    a.n_views = nv;
    a.view0 = v0;
    for (int k = 0; k < nv; ++k) a.cam[k] = to_camk(cams[v0 + k], opts->tile);
    const hipError_t e = launch_preprocess(a, *g, splats, n_tiles, st, stage);
    if (e != hipSuccess) return hip_fail(e, "preprocess launch");
  }
  return SEELE_OK;
}

}  // namespace

extern "C" {

int32_t seele_preprocess(const seele_gaussians* g, const seele_camera* cams, int32_t n_views,
                         const seele_preprocess_opts* opts, seele_splat* splats,
                         int32_t* n_tiles, void* stream) {
  return preprocess_impl(g, cams, n_views, opts, splats, n_tiles, stream, nullptr);
}

int32_t seele_preprocess_staged(const seele_gaussians* g, const seele_camera* cams,
                                int32_t n_views, const seele_preprocess_opts* opts,
                                seele_splat* splats, int32_t* n_tiles, void* workspace,
                                size_t workspace_bytes, int64_t capacity, void* stream) {
  if (!g || !opts) return fail(SEELE_ERR_INVALID_ARG, "null gaussians or options");
  int32_t s = check_cams(cams, n_views, opts->tile, kMaxViewsBin);
  if (s != SEELE_OK) return s;
  if (capacity < 0 || capacity >= ((int64_t)1 << 31))
    return fail(SEELE_ERR_INVALID_ARG, "capacity must be in [0, 2^31)");
  const int64_t R = (int64_t)n_views * g->n;
  if (R >= ((int64_t)1 << 32)) return fail(SEELE_ERR_UNSUPPORTED, "n_views * n must be < 2^32");
  const BinSortPlan plan = plan_bin_sort(R, capacity, seele_total_tiles(cams, n_views, opts->tile));
  if (!workspace || !aligned(workspace, 256))
    return fail(SEELE_ERR_INVALID_ARG, "workspace null or not 256-byte aligned");
  if (workspace_bytes < plan.total)
    return fail(SEELE_ERR_CAPACITY, "workspace %zu bytes < required %zu", workspace_bytes,
                plan.total);
  const BinStage bs = bin_stage_of(plan, workspace, g->n);
  return preprocess_impl(g, cams, n_views, opts, splats, n_tiles, stream, &bs);
}

size_t seele_bin_sort_workspace_size(int64_t n_records, int64_t capacity, int64_t n_tiles_total) {
  if (n_records < 0 || capacity < 0 || n_tiles_total < 0) return 0;
  return plan_bin_sort(n_records, capacity, n_tiles_total).total;
}

}  // extern "C"

namespace {

// Shared by both list forms: per-tile lists into (sorted_ids, ranges), or
// (super) super-tile lists into (entry_keys, sorted_ids, ranges).
int32_t bin_sort_impl(bool super, bool staged, const seele_splat* splats, const int32_t* n_tiles,
                      int64_t n,
                      const seele_camera* cams, int32_t n_views, int32_t tile, void* workspace,
                      size_t workspace_bytes, uint32_t* entry_keys, uint32_t* sorted_ids,
                      int64_t capacity, int32_t* ranges, int64_t* num_pairs, void* stream) {
  int32_t* tile_ranges = ranges;
  int32_t s = check_cams(cams, n_views, tile, kMaxViewsBin);
  if (s != SEELE_OK) return s;
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(SEELE_ERR_INVALID_ARG, "n out of range");
  const int64_t R = (int64_t)n_views * n;
  if (R >= ((int64_t)1 << 32)) return fail(SEELE_ERR_UNSUPPORTED, "n_views * n must be < 2^32");
  if (capacity < 0 || capacity >= ((int64_t)1 << 31))
    return fail(SEELE_ERR_INVALID_ARG, "capacity must be in [0, 2^31)");
  const int64_t TT = seele_total_tiles(cams, n_views, tile);
  if (TT >= ((int64_t)1 << 31)) return fail(SEELE_ERR_UNSUPPORTED, "too many tiles");
  if (R > 0 && !staged && (!splats || !aligned(splats, 16) || !n_tiles || !aligned(n_tiles, 4)))
    return fail(SEELE_ERR_INVALID_ARG, "splats/n_tiles null or misaligned");
  if (capacity > 0 && (!sorted_ids || !aligned(sorted_ids, 4)))
    return fail(SEELE_ERR_INVALID_ARG, "sorted_ids null or misaligned");
  if (super && capacity > 0 && (!entry_keys || !aligned(entry_keys, 4)))
    return fail(SEELE_ERR_INVALID_ARG, "entry_keys null or misaligned");
  if (!tile_ranges || !aligned(tile_ranges, 4))
    return fail(SEELE_ERR_INVALID_ARG, "tile_ranges null or misaligned");
  if (!num_pairs || !aligned(num_pairs, 8))
    return fail(SEELE_ERR_INVALID_ARG, "num_pairs null or misaligned");
  const BinSortPlan plan = plan_bin_sort(R, capacity, TT);
  if (!workspace || !aligned(workspace, 256))
    return fail(SEELE_ERR_INVALID_ARG, "workspace null or not 256-byte aligned");
  if (workspace_bytes < plan.total)
    return fail(SEELE_ERR_CAPACITY, "workspace %zu bytes < required %zu", workspace_bytes,
                plan.total);
  BinViews bv{};
  bv.n_views = n_views;
  bv.n = n;
  int64_t base = 0, st_base = 0;
  for (int v = 0; v < n_views; ++v) {
    const int gw = (cams[v].width + tile - 1) / tile, gh = (cams[v].height + tile - 1) / tile;
    bv.v[v].tile_base = (int32_t)base;
    bv.v[v].st_base = (int32_t)st_base;
    bv.v[v].grid_w = (uint16_t)gw;
    bv.v[v].grid_h = (uint16_t)gh;
    base += tiles_of(cams[v], tile);
    st_base += (int64_t)((gw + kSuperTile - 1) / kSuperTile) * ((gh + kSuperTile - 1) / kSuperTile);
  }
  if (st_base > ((int64_t)1 << 24))
    return fail(SEELE_ERR_UNSUPPORTED, "more than 2^24 super-tiles (%lld)", (long long)st_base);
  bv.n_st = st_base;
  const hipError_t e =
      launch_bin_sort(plan, bv, splats, n_tiles, workspace, sorted_ids, tile_ranges, num_pairs,
                      static_cast<hipStream_t>(stream), super, entry_keys, staged);
  if (e != hipSuccess) return hip_fail(e, "bin_sort launch");
  return SEELE_OK;
}

}  // namespace

extern "C" {

int32_t seele_bin_sort(const seele_splat* splats, const int32_t* n_tiles, int64_t n,
                       const seele_camera* cams, int32_t n_views, int32_t tile,
                       void* workspace, size_t workspace_bytes, uint32_t* sorted_ids,
                       int64_t capacity, int32_t* tile_ranges, int64_t* num_pairs,
                       void* stream) {
  return bin_sort_impl(false, false, splats, n_tiles, n, cams, n_views, tile, workspace,
                       workspace_bytes, nullptr, sorted_ids, capacity, tile_ranges, num_pairs,
                       stream);
}

int64_t seele_total_super_tiles(const seele_camera* cams, int32_t n_views, int32_t tile) {
  if (seele_total_tiles(cams, n_views, tile) < 0) return -1;
  int64_t t = 0;
  for (int v = 0; v < n_views; ++v) t += super_tiles_of(cams[v], tile);
  return t;
}

int32_t seele_bin_sort_super(const seele_splat* splats, const int32_t* n_tiles, int64_t n,
                             const seele_camera* cams, int32_t n_views, int32_t tile,
                             void* workspace, size_t workspace_bytes, uint32_t* entry_keys,
                             uint32_t* entry_ids, int64_t capacity, int32_t* st_ranges,
                             int64_t* num_pairs, void* stream) {
  return bin_sort_impl(true, false, splats, n_tiles, n, cams, n_views, tile, workspace,
                       workspace_bytes, entry_keys, entry_ids, capacity, st_ranges, num_pairs,
                       stream);
}

int32_t seele_bin_sort_ex(int32_t flags, const seele_splat* splats, const int32_t* n_tiles,
                          int64_t n, const seele_camera* cams, int32_t n_views, int32_t tile,
                          void* workspace, size_t workspace_bytes, uint32_t* entry_keys,
                          uint32_t* ids, int64_t capacity, int32_t* ranges, int64_t* num_pairs,
                          void* stream) {
  if (flags & ~(SEELE_BIN_SUPER | SEELE_BIN_STAGED))
    return fail(SEELE_ERR_INVALID_ARG, "unknown bin_sort flags 0x%x", (unsigned)flags);
  const bool super = (flags & SEELE_BIN_SUPER) != 0;
  return bin_sort_impl(super, (flags & SEELE_BIN_STAGED) != 0, splats, n_tiles, n, cams, n_views,
                       tile, workspace, workspace_bytes, super ? entry_keys : nullptr, ids,
                       capacity, ranges, num_pairs, stream);
}

}  // extern "C"

namespace {

// Workspace of seele_bin_sort_noalloc: one copy per GPU, in the code object's
// zero-initialised device data.  In host code `scratch` is only a stand-in
// symbol; its device address comes from hipGetSymbolAddress, per device.
__device__ __align__(256) unsigned char scratch[SEELE_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, looked up once per
// device with that device current.
int32_t scratch_for_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(SEELE_ERR_UNSUPPORTED, "device %d beyond the %d the scratch table holds", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(SEELE_ERR_HIP, "hipGetSymbolAddress(scratch) gave a null address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SEELE_OK;
}

}  // namespace

extern "C" {

int32_t seele_bin_sort_noalloc(int32_t flags, const seele_splat* splats, const int32_t* n_tiles,
                               int64_t n, const seele_camera* cams, int32_t n_views, int32_t tile,
                               uint32_t* entry_keys, uint32_t* ids, int64_t capacity,
                               int32_t* ranges, int64_t* num_pairs, void* stream) {
  if (flags & ~SEELE_BIN_SUPER)
    return fail(SEELE_ERR_INVALID_ARG, "bin_sort_noalloc flags must be 0 or SEELE_BIN_SUPER");
  // size check before the device is touched, so an oversized call fails the
  // same way on any host
  const int32_t s = check_cams(cams, n_views, tile, kMaxViewsBin);
  if (s != SEELE_OK) return s;
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(SEELE_ERR_INVALID_ARG, "n out of range");
  if (capacity < 0 || capacity >= ((int64_t)1 << 31))
    return fail(SEELE_ERR_INVALID_ARG, "capacity must be in [0, 2^31)");
  const size_t need =
      plan_bin_sort((int64_t)n_views * n, capacity, seele_total_tiles(cams, n_views, tile)).total;
  if (need > SEELE_NOALLOC_SCRATCH_BYTES)
    return fail(SEELE_ERR_CAPACITY,
                "bin_sort_noalloc needs %zu workspace bytes, more than the %zu of its scratch "
                "array; use seele_bin_sort_ex with a caller workspace",
                need, (size_t)SEELE_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  const int32_t sc = scratch_for_current_device(&ws);
  if (sc != SEELE_OK) return sc;
  const bool super = (flags & SEELE_BIN_SUPER) != 0;
  return bin_sort_impl(super, false, splats, n_tiles, n, cams, n_views, tile, ws,
                       SEELE_NOALLOC_SCRATCH_BYTES, super ? entry_keys : nullptr, ids, capacity,
                       ranges, num_pairs, stream);
}

}  // extern "C"

namespace {

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// super: (sorted_ids, tile_ranges) are super-tile lists (entry ids,
// super-tile ranges) with their entry keys.
int32_t rasterize(const seele_splat* splats, const uint32_t* sorted_ids,
                  const int32_t* tile_ranges, const seele_camera* cams, int32_t n_views,
                  const seele_raster_opts* opts, float* image, float* final_T,
                  int32_t* n_contrib, uint64_t* counters, void* stream, bool super = false,
                  const uint32_t* entry_keys = nullptr, int32_t* last_entry = nullptr) {
  int32_t s = check_raster_opts(opts);
  if (s != SEELE_OK) return s;
  if ((s = check_cams(cams, n_views, opts->tile, 1 << 20)) != SEELE_OK) return s;
  const int64_t TT = seele_total_tiles(cams, n_views, opts->tile);
  if (TT >= ((int64_t)1 << 31)) return fail(SEELE_ERR_UNSUPPORTED, "too many tiles");
  if (super) {
    if (batch_of(opts) != opts->tile * opts->tile)
      return fail(SEELE_ERR_UNSUPPORTED, "super-tile lists take the default LDS batch only");
    if (seele_total_super_tiles(cams, n_views, opts->tile) > ((int64_t)1 << 24))
      return fail(SEELE_ERR_UNSUPPORTED, "more than 2^24 super-tiles");
    if (entry_keys && !aligned(entry_keys, 4))
      return fail(SEELE_ERR_INVALID_ARG, "entry_keys misaligned");
    if (last_entry && !aligned(last_entry, 4))
      return fail(SEELE_ERR_INVALID_ARG, "last_entry misaligned");
  }
  if (!tile_ranges || !aligned(tile_ranges, 4))
    return fail(SEELE_ERR_INVALID_ARG, "tile_ranges null or misaligned");
  if (!image || !aligned(image, 4) || !final_T || !aligned(final_T, 4) || !n_contrib ||
      !aligned(n_contrib, 4))
    return fail(SEELE_ERR_INVALID_ARG, "output buffers null or misaligned");
  if ((splats && !aligned(splats, 16)) || (sorted_ids && !aligned(sorted_ids, 4)))
    return fail(SEELE_ERR_INVALID_ARG, "splats/sorted_ids misaligned");
  const RasterParams rp = make_raster_params(opts);
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(counters);
  if (cnt) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, cnt, 6);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "counter reset");
  }
  int64_t tile_base = 0, pix_base = 0;
  for (int v0 = 0; v0 < n_views; v0 += kMaxViewsRaster) {
    const int nv = std::min(kMaxViewsRaster, n_views - v0);
    int64_t t = 0, npx = 0;
    const RasterViews rv = make_raster_views(cams, v0, nv, opts->tile, tile_base, pix_base, t, npx);
    pix_base += npx;
    const hipError_t e =
        super ? launch_raster_fwd_super(opts->tile, opts->mode, rv, (int)t, rp, splats,
                                        entry_keys, sorted_ids, tile_ranges, image, final_T,
                                        n_contrib, cnt, last_entry, st)
              : launch_raster_fwd(opts->tile, opts->mode, batch_of(opts), rv, (int)t, rp, splats,
                                  sorted_ids, tile_ranges, image, final_T, n_contrib, cnt, st);
    if (e != hipSuccess) return hip_fail(e, "raster launch");
    tile_base += t;
  }
  return SEELE_OK;
}

}  // namespace

extern "C" {

int32_t seele_rasterize_fwd(const seele_splat* splats, const uint32_t* sorted_ids,
                            const int32_t* tile_ranges, const seele_camera* cams,
                            int32_t n_views, const seele_raster_opts* opts, float* image,
                            float* final_T, int32_t* n_contrib, void* stream) {
  return rasterize(splats, sorted_ids, tile_ranges, cams, n_views, opts, image, final_T,
                   n_contrib, nullptr, stream);
}

int32_t seele_contrib_topk(const seele_splat* splats, const uint32_t* sorted_ids,
                           const int32_t* tile_ranges, const seele_camera* cams, int32_t n_views,
                           int64_t n, const seele_raster_opts* opts, int32_t k,
                           uint8_t* topk_mark, float* contrib_sum, void* stream) {
  int32_t s = check_raster_opts(opts);
  if (s != SEELE_OK) return s;
  if (opts->mode != SEELE_RASTER_PLAIN)
    return fail(SEELE_ERR_UNSUPPORTED, "the contribution pass blends in the plain form");
  if (k < 1 || k > 32) return fail(SEELE_ERR_INVALID_ARG, "k must be in [1, 32]");
  if ((s = check_cams(cams, n_views, opts->tile, 1 << 20)) != SEELE_OK) return s;
  if (n < 0 || (int64_t)n_views * n >= ((int64_t)1 << 32))
    return fail(SEELE_ERR_INVALID_ARG, "n out of range");
  const int64_t TT = seele_total_tiles(cams, n_views, opts->tile);
  if (TT >= ((int64_t)1 << 31)) return fail(SEELE_ERR_UNSUPPORTED, "too many tiles");
  if (!tile_ranges || !aligned(tile_ranges, 4))
    return fail(SEELE_ERR_INVALID_ARG, "tile_ranges null or misaligned");
  if (n > 0 && (!topk_mark || !contrib_sum || !aligned(contrib_sum, 4)))
    return fail(SEELE_ERR_INVALID_ARG, "topk_mark / contrib_sum null or misaligned");
  if ((splats && !aligned(splats, 16)) || (sorted_ids && !aligned(sorted_ids, 4)))
    return fail(SEELE_ERR_INVALID_ARG, "splats/sorted_ids misaligned");
  const RasterParams rp = make_raster_params(opts);
  hipStream_t st = static_cast<hipStream_t>(stream);
  int64_t tile_base = 0, pix_base = 0;
  for (int v0 = 0; v0 < n_views; v0 += kMaxViewsRaster) {
    const int nv = std::min(kMaxViewsRaster, n_views - v0);
    int64_t t = 0, npx = 0;
    const RasterViews rv = make_raster_views(cams, v0, nv, opts->tile, tile_base, pix_base, t, npx);
    pix_base += npx;
    const hipError_t e = launch_contrib_topk(opts->tile, rv, (int)t, rp, splats, sorted_ids,
                                             tile_ranges, k, topk_mark, contrib_sum, st);
    if (e != hipSuccess) return hip_fail(e, "contribution pass launch");
    tile_base += t;
  }
  return SEELE_OK;
}

int32_t seele_rasterize_fwd_super(const seele_splat* splats, const uint32_t* entry_keys,
                                  const uint32_t* entry_ids, const int32_t* st_ranges,
                                  const seele_camera* cams, int32_t n_views,
                                  const seele_raster_opts* opts, float* image, float* final_T,
                                  int32_t* n_contrib, int32_t* last_entry, uint64_t* counters,
                                  void* stream) {
  return rasterize(splats, entry_ids, st_ranges, cams, n_views, opts, image, final_T, n_contrib,
                   counters, stream, true, entry_keys, last_entry);
}

size_t seele_raster_queue_workspace_size(int64_t n_tiles_total) {
  if (n_tiles_total < 0) return 0;
  const int64_t n = std::max<int64_t>(n_tiles_total, 1);
  return 256 + 2 * ((4 * (size_t)n + 255) & ~(size_t)255) + radix_sort_workspace_size(n);
}

int32_t seele_rasterize_fwd_queue(const seele_splat* splats, const uint32_t* sorted_ids,
                                  const int32_t* tile_ranges, const seele_camera* cams,
                                  int32_t n_views, const seele_raster_opts* opts, int32_t order,
                                  void* workspace, size_t workspace_bytes, float* image,
                                  float* final_T, int32_t* n_contrib, void* stream) {
  int32_t s = check_raster_opts(opts);
  if (s != SEELE_OK) return s;
  if ((s = check_cams(cams, n_views, opts->tile, 1 << 20)) != SEELE_OK) return s;
  if (order != SEELE_QUEUE_LIST && order != SEELE_QUEUE_HEAVIEST_FIRST)
    return fail(SEELE_ERR_INVALID_ARG, "unknown queue order %d", order);
  const int64_t TT = seele_total_tiles(cams, n_views, opts->tile);
  if (TT >= ((int64_t)1 << 31)) return fail(SEELE_ERR_UNSUPPORTED, "too many tiles");
  if (!tile_ranges || !aligned(tile_ranges, 4))
    return fail(SEELE_ERR_INVALID_ARG, "tile_ranges null or misaligned");
  if (!image || !aligned(image, 4) || !final_T || !aligned(final_T, 4) || !n_contrib ||
      !aligned(n_contrib, 4))
    return fail(SEELE_ERR_INVALID_ARG, "output buffers null or misaligned");
  if ((splats && !aligned(splats, 16)) || (sorted_ids && !aligned(sorted_ids, 4)))
    return fail(SEELE_ERR_INVALID_ARG, "splats/sorted_ids misaligned");
  if (!workspace || !aligned(workspace, 256))
    return fail(SEELE_ERR_INVALID_ARG, "workspace null or not 256-byte aligned");
  // the largest chunk of views decides the workspace
  int64_t max_chunk = 0;
  for (int v0 = 0; v0 < n_views; v0 += kMaxViewsRaster) {
    const int64_t t = seele_total_tiles(cams + v0, std::min(kMaxViewsRaster, n_views - v0),
                                        opts->tile);
    max_chunk = std::max(max_chunk, t);
  }
  const size_t need = seele_raster_queue_workspace_size(max_chunk);
  if (workspace_bytes < need)
    return fail(SEELE_ERR_CAPACITY, "workspace %zu bytes < required %zu", workspace_bytes, need);
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      return fail(SEELE_ERR_HIP, "cannot query the compute-unit count");
    cus = n;
  }
  const int workgroups = cus * (opts->tile == 16 ? 8 : 32);
  char* base = static_cast<char*>(workspace);
  uint32_t* counter = reinterpret_cast<uint32_t*>(base);
  const size_t tb = (4 * (size_t)std::max<int64_t>(max_chunk, 1) + 255) & ~(size_t)255;
  uint32_t* keys = reinterpret_cast<uint32_t*>(base + 256);
  uint32_t* vals = reinterpret_cast<uint32_t*>(base + 256 + tb);
  void* sort_ws = base + 256 + 2 * tb;
  const RasterParams rp = make_raster_params(opts);
  hipStream_t st = static_cast<hipStream_t>(stream);
  int64_t tile_base = 0, pix_base = 0;
  for (int v0 = 0; v0 < n_views; v0 += kMaxViewsRaster) {
    const int nv = std::min(kMaxViewsRaster, n_views - v0);
    int64_t t = 0, npx = 0;
    const RasterViews rv = make_raster_views(cams, v0, nv, opts->tile, tile_base, pix_base, t, npx);
    hipError_t e;
    const uint32_t* ord = nullptr;
    if (order == SEELE_QUEUE_HEAVIEST_FIRST) {
      e = launch_tile_order_keys(tile_ranges, (int32_t)tile_base, (uint32_t)t, keys, vals, counter,
                                 st);
      if (e == hipSuccess) e = radix_sort_pairs(keys, vals, t, 32, sort_ws, st);
      ord = vals;
    } else {
      e = launch_zero_counter(counter, st);
    }
    if (e == hipSuccess)
      e = launch_raster_fwd_queue(opts->tile, opts->mode, batch_of(opts), rv, (int)t, rp, splats,
                                  sorted_ids, tile_ranges, image, final_T, n_contrib, counter, ord,
                                  workgroups, st);
    if (e != hipSuccess) return hip_fail(e, "queued raster launch");
    tile_base += t;
    pix_base += npx;
  }
  return SEELE_OK;
}

int32_t seele_rasterize_fwd_counted(const seele_splat* splats, const uint32_t* sorted_ids,
                                    const int32_t* tile_ranges, const seele_camera* cams,
                                    int32_t n_views, const seele_raster_opts* opts, float* image,
                                    float* final_T, int32_t* n_contrib, uint64_t* counters,
                                    void* stream) {
  if (!counters || !aligned(counters, 8))
    return fail(SEELE_ERR_INVALID_ARG, "counters null or misaligned");
  return rasterize(splats, sorted_ids, tile_ranges, cams, n_views, opts, image, final_T,
                   n_contrib, counters, stream);
}

}  // extern "C"

namespace {

// Shared by both list forms: per-tile lists (sorted_ids, tile_ranges) or
// (super) super-tile lists (entry ids, entry keys, super-tile ranges).
int32_t rasterize_bwd_impl(bool super, const seele_gaussians* g, const seele_camera* cams,
                           int32_t n_views, const seele_preprocess_opts* popts,
                           const seele_raster_opts* ropts, const seele_splat* splats,
                           const int32_t* n_tiles, const uint32_t* ids, const uint32_t* entry_keys,
                           const int32_t* ranges, const float* final_T, const int32_t* n_contrib,
                           const float* dL_dimage, float* grad2d,
                           const seele_gaussian_grads* grads, void* stream) {
  // super: n_contrib holds the last-entry indices of seele_rasterize_fwd_super
  int32_t s = check_gaussians(g);
  if (s != SEELE_OK) return s;
  if ((s = check_preprocess_opts(popts, g->n)) != SEELE_OK) return s;
  if ((s = check_raster_opts(ropts)) != SEELE_OK) return s;
  if (popts->tile != ropts->tile)
    return fail(SEELE_ERR_INVALID_ARG, "preprocess and raster tile sizes differ");
  if (super && ropts->tile != 16)
    return fail(SEELE_ERR_UNSUPPORTED, "the super-tile backward takes 16x16 tiles");
  if ((s = check_cams(cams, n_views, ropts->tile, 1 << 20)) != SEELE_OK) return s;
  const int64_t R = (int64_t)n_views * g->n;
  if (R >= ((int64_t)1 << 32)) return fail(SEELE_ERR_UNSUPPORTED, "n_views * n must be < 2^32");
  const int64_t TT = seele_total_tiles(cams, n_views, ropts->tile);
  if (TT >= ((int64_t)1 << 31)) return fail(SEELE_ERR_UNSUPPORTED, "too many tiles");
  if (!grads) return fail(SEELE_ERR_INVALID_ARG, "grads is null");
  if (!ranges || !aligned(ranges, 4) || !final_T || !aligned(final_T, 4) ||
      !n_contrib || !aligned(n_contrib, 4) || !dL_dimage || !aligned(dL_dimage, 4))
    return fail(SEELE_ERR_INVALID_ARG, "ranges/final_T/n_contrib/dL_dimage null or misaligned");
  if (super && (!entry_keys || !aligned(entry_keys, 4) || !ids || !aligned(ids, 4)))
    return fail(SEELE_ERR_INVALID_ARG, "entry_keys/entry_ids null or misaligned");
  if (R > 0) {
    if (!splats || !aligned(splats, 16) || !n_tiles || !aligned(n_tiles, 4) || !grad2d ||
        !aligned(grad2d, 4))
      return fail(SEELE_ERR_INVALID_ARG, "splats/n_tiles/grad2d null or misaligned");
    const void* p[5] = {grads->means, grads->log_scales, grads->quats, grads->opacity_logits,
                        grads->sh};
    for (int k = 0; k < 5; ++k)
      if (!p[k] || !aligned(p[k], 4))
        return fail(SEELE_ERR_INVALID_ARG, "gradient output %d null or misaligned", k);
  }
  if (g->n == 0) return SEELE_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // 1. per-record 2D gradients, accumulated by the blend backward
  const int64_t n2 = R * 9;
  hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)std::min<int64_t>((n2 / 4 + 255) / 256 + 1, 4096)),
                     dim3(256), 0, st, grad2d, n2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "grad2d reset");
  const RasterParams rp = make_raster_params(ropts);
  int64_t tile_base = 0, pix_base = 0;
  for (int v0 = 0; v0 < n_views; v0 += kMaxViewsRaster) {
    const int nv = std::min(kMaxViewsRaster, n_views - v0);
    int64_t t = 0, npx = 0;
    const RasterViews rv = make_raster_views(cams, v0, nv, ropts->tile, tile_base, pix_base, t, npx);
    if (super) {
      int64_t nst = 0;
      for (int k = 0; k < nv; ++k) nst += super_tiles_of(cams[v0 + k], ropts->tile);
      e = launch_raster_bwd_quad(ropts->mode, rv, (int)nst, rp, splats, ids, entry_keys, ranges,
                                 final_T, n_contrib /* last_entry */, dL_dimage, grad2d, st);
    } else {
      e = launch_raster_bwd(ropts->tile, ropts->mode, rv, (int)t, rp, splats, ids, ranges,
                            final_T, n_contrib, dL_dimage, grad2d, st);
    }
    if (e != hipSuccess) return hip_fail(e, "raster backward launch");
    tile_base += t;
    pix_base += npx;
  }
  // 2. chain to the raw parameters, views summed
  PreArgs a = make_pre_args(g, popts);
  for (int v0 = 0; v0 < n_views; v0 += kMaxViewsPre) {
    const int nv = std::min(kMaxViewsPre, n_views - v0);
    a.n_views = nv;
    a.view0 = v0;
    for (int k = 0; k < nv; ++k) a.cam[k] = to_camk(cams[v0 + k], popts->tile);
    e = launch_preprocess_bwd(a, *g, n_tiles, grad2d, *grads, v0 > 0, st);
    if (e != hipSuccess) return hip_fail(e, "preprocess backward launch");
  }
  return SEELE_OK;
}

}  // namespace

extern "C" {

int32_t seele_rasterize_bwd(const seele_gaussians* g, const seele_camera* cams, int32_t n_views,
                            const seele_preprocess_opts* popts, const seele_raster_opts* ropts,
                            const seele_splat* splats, const int32_t* n_tiles,
                            const uint32_t* sorted_ids, const int32_t* tile_ranges,
                            const float* final_T, const int32_t* n_contrib,
                            const float* dL_dimage, float* grad2d,
                            const seele_gaussian_grads* grads, void* stream) {
  return rasterize_bwd_impl(false, g, cams, n_views, popts, ropts, splats, n_tiles, sorted_ids,
                            nullptr, tile_ranges, final_T, n_contrib, dL_dimage, grad2d, grads,
                            stream);
}

int32_t seele_rasterize_bwd_super(const seele_gaussians* g, const seele_camera* cams,
                                  int32_t n_views, const seele_preprocess_opts* popts,
                                  const seele_raster_opts* ropts, const seele_splat* splats,
                                  const int32_t* n_tiles, const uint32_t* entry_keys,
                                  const uint32_t* entry_ids, const int32_t* st_ranges,
                                  const float* final_T, const int32_t* last_entry,
                                  const float* dL_dimage, float* grad2d,
                                  const seele_gaussian_grads* grads, void* stream) {
  return rasterize_bwd_impl(true, g, cams, n_views, popts, ropts, splats, n_tiles, entry_ids,
                            entry_keys, st_ranges, final_T, last_entry, dL_dimage, grad2d, grads,
                            stream);
}

}  // extern "C"

namespace {

// Pose feature of Sec. 3.3 "Offline Clustering": the camera centre divided
// by pos_scale, then beta times the viewing direction (camera +z in world
// coordinates).
void pose_feature(const seele_camera* cam, float pos_scale, float beta, double* f) {
  for (int i = 0; i < 3; ++i) {
    double c = 0.0;
    for (int j = 0; j < 3; ++j) c -= (double)cam->R[j * 3 + i] * (double)cam->t[j];
    f[i] = c / (double)pos_scale;
    f[3 + i] = (double)beta * (double)cam->R[6 + i];
  }
}

double dist2_6(const double* a, const double* b) {
  double s = 0.0;
  for (int i = 0; i < 6; ++i) s += (a[i] - b[i]) * (a[i] - b[i]);
  return s;
}

}  // namespace

extern "C" {

float seele_hp_pos_scale(const seele_camera* cams, int32_t n_cams) {
  if (!cams || n_cams < 1) {
    fail(SEELE_ERR_INVALID_ARG, "need at least one camera");
    return -1.0f;
  }
  double best = 0.0;
  for (int p = 0; p < n_cams; ++p) {
    double f[6];
    pose_feature(&cams[p], 1.0f, 0.0f, f);
    const double r = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!std::isfinite(r)) {
      fail(SEELE_ERR_INVALID_ARG, "non-finite camera centre");
      return -1.0f;
    }
    best = std::max(best, r);
  }
  return (float)best;
}

int32_t seele_hp_kmeans(const seele_camera* cams, int32_t n_cams, float pos_scale, float beta,
                        int32_t K, int32_t iters, float* centroids, int32_t* labels) {
  if (!cams || !centroids || !labels) return fail(SEELE_ERR_INVALID_ARG, "null argument");
  if (n_cams < 1 || K < 1 || K > n_cams || iters < 0)
    return fail(SEELE_ERR_INVALID_ARG, "need 1 <= K <= n_cams and iters >= 0");
  if (!is_finite(pos_scale) || !is_finite(beta))
    return fail(SEELE_ERR_INVALID_ARG, "bad pos_scale/beta");
  if (pos_scale <= 0.0f) {
    pos_scale = seele_hp_pos_scale(cams, n_cams);
    if (!(pos_scale > 0.0f))
      return fail(SEELE_ERR_INVALID_ARG, "every sampled camera centre is at the origin");
  }
  std::vector<double> f((size_t)n_cams * 6), c((size_t)K * 6), dmin((size_t)n_cams);
  for (int p = 0; p < n_cams; ++p) pose_feature(&cams[p], pos_scale, beta, &f[(size_t)p * 6]);
  // farthest-point seeding: pose 0, then each time the pose farthest from
  // every chosen centroid (the lowest index on ties)
  for (int i = 0; i < 6; ++i) c[i] = f[i];
  for (int p = 0; p < n_cams; ++p) dmin[p] = dist2_6(&f[(size_t)p * 6], &c[0]);
  for (int k = 1; k < K; ++k) {
    int far = 0;
    for (int p = 1; p < n_cams; ++p)
      if (dmin[p] > dmin[far]) far = p;
    for (int i = 0; i < 6; ++i) c[(size_t)k * 6 + i] = f[(size_t)far * 6 + i];
    for (int p = 0; p < n_cams; ++p)
      dmin[p] = std::min(dmin[p], dist2_6(&f[(size_t)p * 6], &c[(size_t)k * 6]));
  }
  // Lloyd: nearest centroid (lowest index on ties), then member means; an
  // empty cluster keeps its centroid; stops when no label changes
  std::vector<int> lab((size_t)n_cams, -1);
  for (int it = 0; it <= iters; ++it) {
    bool changed = false;
    for (int p = 0; p < n_cams; ++p) {
      int best = 0;
      double bd = dist2_6(&f[(size_t)p * 6], &c[0]);
      for (int k = 1; k < K; ++k) {
        const double d = dist2_6(&f[(size_t)p * 6], &c[(size_t)k * 6]);
        if (d < bd) {
          bd = d;
          best = k;
        }
      }
      changed |= lab[p] != best;
      lab[p] = best;
    }
    if (!changed || it == iters) break;
    std::vector<double> sum((size_t)K * 6, 0.0);
    std::vector<int> cnt((size_t)K, 0);
    for (int p = 0; p < n_cams; ++p) {
      ++cnt[lab[p]];
      for (int i = 0; i < 6; ++i) sum[(size_t)lab[p] * 6 + i] += f[(size_t)p * 6 + i];
    }
    for (int k = 0; k < K; ++k)
      if (cnt[k] > 0)
        for (int i = 0; i < 6; ++i) c[(size_t)k * 6 + i] = sum[(size_t)k * 6 + i] / cnt[k];
  }
  for (int k = 0; k < K * 6; ++k) centroids[k] = (float)c[k];
  for (int p = 0; p < n_cams; ++p) labels[p] = lab[p];
  return SEELE_OK;
}

int32_t seele_hp_accumulate(const uint8_t* topk_mark, const float* contrib_sum, int32_t n_views,
                            int64_t n, int32_t cluster, uint8_t* shared, float* best_sum,
                            int32_t* best_cluster, void* stream) {
  if (n_views < 1 || n < 0 || cluster < 0)
    return fail(SEELE_ERR_INVALID_ARG, "need n_views >= 1, n >= 0, cluster >= 0");
  if (n == 0) return SEELE_OK;
  if (!topk_mark || !contrib_sum || !shared || !best_sum || !best_cluster ||
      !aligned(contrib_sum, 4) || !aligned(best_sum, 4) || !aligned(best_cluster, 4))
    return fail(SEELE_ERR_INVALID_ARG, "null or misaligned argument");
  hipLaunchKernelGGL(k_hp_accumulate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), topk_mark, contrib_sum, n_views, n, cluster,
                     shared, best_sum, best_cluster);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SEELE_OK : hip_fail(e, "hp accumulate launch");
}

int32_t seele_gather_gaussians(const seele_gaussians* src, const int64_t* perm, int64_t n_out,
                               const seele_gaussian_grads* dst, void* stream) {
  int32_t s = check_gaussians(src);
  if (s != SEELE_OK) return s;
  if (n_out < 0 || n_out >= ((int64_t)1 << 31) || !dst)
    return fail(SEELE_ERR_INVALID_ARG, "bad n_out or null dst");
  if (n_out == 0) return SEELE_OK;
  if (src->n == 0) return fail(SEELE_ERR_INVALID_ARG, "gather from an empty set");
  if (!perm || !aligned(perm, 8)) return fail(SEELE_ERR_INVALID_ARG, "perm null or misaligned");
  const void* p[5] = {dst->means, dst->log_scales, dst->quats, dst->opacity_logits, dst->sh};
  for (int k = 0; k < 5; ++k)
    if (!p[k] || !aligned(p[k], 4)) return fail(SEELE_ERR_INVALID_ARG, "dst array null/misaligned");
  const int n_sh = 3 * (src->sh_degree + 1) * (src->sh_degree + 1);
  hipLaunchKernelGGL(k_gather_gaussians, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), *src, perm, n_out, *dst, n_sh);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SEELE_OK : hip_fail(e, "gather launch");
}

int32_t seele_hp_partition(const uint8_t* shared, const float* best_sum,
                           const int32_t* best_cluster, int64_t n, int32_t K, int64_t* perm,
                           int64_t* layout_begin, int64_t* layout_count) {
  if (n < 0 || K < 1) return fail(SEELE_ERR_INVALID_ARG, "need n >= 0 and K >= 1");
  if (n > 0 && (!shared || !best_sum || !best_cluster || !perm))
    return fail(SEELE_ERR_INVALID_ARG, "null argument");
  if (!layout_begin || !layout_count) return fail(SEELE_ERR_INVALID_ARG, "null layout");
  // segment of each Gaussian: 0 shared, 1 + c exclusive to cluster c, K + 1 discarded
  auto seg_of = [&](int64_t i) -> int64_t {
    if (shared[i]) return 0;
    const int32_t c = best_cluster[i];
    if (best_sum[i] > 0.0f && c >= 0 && c < K) return 1 + c;
    return (int64_t)K + 1;
  };
  std::vector<int64_t> cnt((size_t)K + 2, 0);
  for (int64_t i = 0; i < n; ++i) ++cnt[(size_t)seg_of(i)];
  std::vector<int64_t> next((size_t)K + 2, 0);
  for (int s = 1; s < K + 2; ++s) next[(size_t)s] = next[(size_t)s - 1] + cnt[(size_t)s - 1];
  for (int s = 0; s < K + 1; ++s) {
    layout_begin[s] = next[(size_t)s];
    layout_count[s] = cnt[(size_t)s];
  }
  for (int64_t i = 0; i < n; ++i) perm[next[(size_t)seg_of(i)]++] = i;
  return SEELE_OK;
}

int32_t seele_hp_select(const float* centroids, int32_t K, const seele_camera* cam,
                        float pos_scale, float beta, int32_t M, int32_t* clusters) {
  if (!centroids || !cam || !clusters) return fail(SEELE_ERR_INVALID_ARG, "null argument");
  if (K < 1 || M < 0 || M > K - 1) return fail(SEELE_ERR_INVALID_ARG, "need K >= 1, 0 <= M < K");
  if (!(pos_scale > 0.0f) || !is_finite(pos_scale) || !is_finite(beta))
    return fail(SEELE_ERR_INVALID_ARG, "bad pos_scale/beta");
  double f[6];
  pose_feature(cam, pos_scale, beta, f);
  auto dist2 = [&](int k, const double* p) {
    double s = 0.0;
    for (int i = 0; i < 6; ++i) {
      const double d = (double)centroids[k * 6 + i] - p[i];
      s += d * d;
    }
    return s;
  };
  int best = 0;
  double bd = dist2(0, f);
  for (int k = 1; k < K; ++k) {
    const double d = dist2(k, f);
    if (d < bd) {
      bd = d;
      best = k;
    }
  }
  clusters[0] = best;
  double c[6];
  for (int i = 0; i < 6; ++i) c[i] = centroids[best * 6 + i];
  // M nearest other centroids to the chosen one; selection keeps ties in index order
  for (int m = 0; m < M; ++m) {
    int pick = -1;
    double pd = 0.0;
    for (int k = 0; k < K; ++k) {
      bool used = false;
      for (int q = 0; q <= m; ++q) used |= clusters[q] == k;
      if (used) continue;
      const double d = dist2(k, c);
      if (pick < 0 || d < pd) {
        pick = k;
        pd = d;
      }
    }
    clusters[1 + m] = pick;
  }
  return SEELE_OK;
}

int32_t seele_hp_segments(const int64_t* layout_begin, const int64_t* layout_count, int32_t K,
                          const int32_t* clusters, int32_t n_sel, int64_t* out_begin,
                          int64_t* out_count, int32_t* n_out) {
  if (!layout_begin || !layout_count || !out_begin || !out_count || !n_out ||
      (n_sel > 0 && !clusters))
    return fail(SEELE_ERR_INVALID_ARG, "null argument");
  if (K < 0 || n_sel < 0) return fail(SEELE_ERR_INVALID_ARG, "negative K or n_sel");
  int cnt = 0;
  auto add = [&](int64_t b, int64_t c) {
    if (c <= 0) return;
    for (int i = 0; i < cnt; ++i)
      if (out_begin[i] == b) return;  // a cluster chosen twice
    out_begin[cnt] = b;
    out_count[cnt] = c;
    ++cnt;
  };
  add(layout_begin[0], layout_count[0]);
  for (int s = 0; s < n_sel; ++s) {
    const int c = clusters[s];
    if (c < 0 || c >= K) return fail(SEELE_ERR_INVALID_ARG, "cluster %d not in 0..%d", c, K - 1);
    add(layout_begin[1 + c], layout_count[1 + c]);
  }
  // insertion sort by begin
  for (int i = 1; i < cnt; ++i)
    for (int j = i; j > 0 && out_begin[j] < out_begin[j - 1]; --j) {
      std::swap(out_begin[j], out_begin[j - 1]);
      std::swap(out_count[j], out_count[j - 1]);
    }
  *n_out = cnt;
  return SEELE_OK;
}

}  // extern "C"

// ---- scene prefetching (Sec. 3.3 "Scene Prefetching")

namespace {

using M3 = std::array<double, 9>;  // row-major

M3 mat_of(const float* r) {
  M3 m;
  for (int k = 0; k < 9; ++k) m[k] = (double)r[k];
  return m;
}

M3 mul(const M3& a, const M3& b) {
  M3 c{};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) c[i * 3 + j] += a[i * 3 + k] * b[k * 3 + j];
  return c;
}

M3 transpose(const M3& a) {
  M3 t;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) t[i * 3 + j] = a[j * 3 + i];
  return t;
}

// Rotation vector (axis times angle) of a rotation matrix.
void rot_log(const M3& r, double* w) {
  const double v[3] = {r[7] - r[5], r[2] - r[6], r[3] - r[1]};  // 2 sin(theta) axis
  const double c = std::min(1.0, std::max(-1.0, 0.5 * (r[0] + r[4] + r[8] - 1.0)));
  const double th = std::acos(c);
  if (th < 1e-6) {  // theta / (2 sin theta) -> 1/2
    for (int i = 0; i < 3; ++i) w[i] = 0.5 * v[i];
    return;
  }
  if (th < 3.14159) {
    const double f = th / (2.0 * std::sin(th));
    for (int i = 0; i < 3; ++i) w[i] = f * v[i];
    return;
  }
  // near pi: the axis from the symmetric part (R + I) / 2 = a a^T (+ O(pi - theta))
  int k = 0;
  for (int i = 1; i < 3; ++i)
    if (r[i * 4] > r[k * 4]) k = i;
  double a[3];
  const double akk = std::sqrt(std::max(0.0, 0.5 * (r[k * 4] + 1.0)));
  for (int i = 0; i < 3; ++i)
    a[i] = i == k ? akk : 0.25 * (r[i * 3 + k] + r[k * 3 + i]) / akk;
  const double nrm = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  const double sg = (a[0] * v[0] + a[1] * v[1] + a[2] * v[2]) < 0.0 ? -1.0 : 1.0;
  for (int i = 0; i < 3; ++i) w[i] = sg * th * a[i] / nrm;
}

// Rotation matrix of a rotation vector (Rodrigues' formula).
M3 rot_exp(const double* w) {
  const double th = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  M3 r{1, 0, 0, 0, 1, 0, 0, 0, 1};
  if (th == 0.0) return r;
  const double x = w[0] / th, y = w[1] / th, z = w[2] / th;
  const M3 k{0, -z, y, z, 0, -x, -y, x, 0};
  const M3 k2 = mul(k, k);
  const double s = std::sin(th), c1 = 1.0 - std::cos(th);
  for (int i = 0; i < 9; ++i) r[i] += s * k[i] + c1 * k2[i];
  return r;
}

}  // namespace

extern "C" {

int32_t seele_pose_extrapolate(const seele_camera* prev, const seele_camera* cur, float s,
                               seele_camera* out) {
  if (!prev || !cur || !out) return fail(SEELE_ERR_INVALID_ARG, "null argument");
  if (!is_finite(s)) return fail(SEELE_ERR_INVALID_ARG, "non-finite step");
  int32_t st = check_camera(*prev, 0, 16);
  if (st == SEELE_OK) st = check_camera(*cur, 1, 16);
  if (st != SEELE_OK) return st;
  const M3 rp = mat_of(prev->R), rc = mat_of(cur->R);
  double cp[3], cc[3], co[3];
  for (int i = 0; i < 3; ++i) {
    cp[i] = cc[i] = 0.0;
    for (int j = 0; j < 3; ++j) {
      cp[i] -= rp[j * 3 + i] * (double)prev->t[j];
      cc[i] -= rc[j * 3 + i] * (double)cur->t[j];
    }
    co[i] = cc[i] + (double)s * (cc[i] - cp[i]);
  }
  double w[3];
  rot_log(mul(rc, transpose(rp)), w);
  for (int i = 0; i < 3; ++i) w[i] *= (double)s;
  const M3 ro = mul(rot_exp(w), rc);
  seele_camera o = *cur;
  for (int k = 0; k < 9; ++k) o.R[k] = (float)ro[k];
  for (int i = 0; i < 3; ++i) {
    double t = 0.0;
    for (int j = 0; j < 3; ++j) t -= ro[i * 3 + j] * co[j];
    o.t[i] = (float)t;
  }
  *out = o;
  return SEELE_OK;
}

int32_t seele_resident_plan(int32_t* slot_cluster, int64_t* slot_stamp, int32_t n_slots,
                            const int64_t* cluster_count, int32_t K, int64_t slot_cap,
                            const int32_t* need, int32_t n_need, const int32_t* want,
                            int32_t n_want, int64_t frame, int32_t* load_cluster,
                            int32_t* load_slot, int32_t* n_loads, int32_t* n_demand) {
  if (!slot_cluster || !slot_stamp || !cluster_count || !load_cluster || !load_slot || !n_loads ||
      !n_demand || (n_need > 0 && !need) || (n_want > 0 && !want))
    return fail(SEELE_ERR_INVALID_ARG, "null argument");
  if (n_slots < 1 || K < 1 || slot_cap < 0 || n_need < 0 || n_want < 0)
    return fail(SEELE_ERR_INVALID_ARG, "need n_slots >= 1, K >= 1, sizes >= 0");
  std::vector<int> slot_of((size_t)K, -1);
  for (int s = 0; s < n_slots; ++s) {
    const int c = slot_cluster[s];
    if (c < -1 || c >= K) return fail(SEELE_ERR_INVALID_ARG, "slot %d holds cluster %d", s, c);
    if (c >= 0) {
      if (slot_of[c] >= 0) return fail(SEELE_ERR_INVALID_ARG, "cluster %d in two slots", c);
      slot_of[c] = s;
    }
  }
  auto check_c = [&](int c) -> int32_t {
    if (c < 0 || c >= K) return fail(SEELE_ERR_INVALID_ARG, "cluster %d not in 0..%d", c, K - 1);
    if (cluster_count[c] > slot_cap)
      return fail(SEELE_ERR_CAPACITY, "cluster %d (%lld Gaussians) exceeds the slot size %lld", c,
                  (long long)cluster_count[c], (long long)slot_cap);
    return SEELE_OK;
  };
  std::vector<char> needed((size_t)K, 0), wanted((size_t)K, 0), held((size_t)n_slots, 0);
  int distinct = 0;
  for (int i = 0; i < n_need; ++i) {
    const int32_t st = check_c(need[i]);
    if (st != SEELE_OK) return st;
    distinct += !needed[need[i]];
    needed[need[i]] = 1;
  }
  if (distinct > n_slots)
    return fail(SEELE_ERR_CAPACITY, "%d clusters needed at once, %d slots", distinct, n_slots);
  for (int i = 0; i < n_want; ++i) {
    const int32_t st = check_c(want[i]);
    if (st != SEELE_OK) return st;
    wanted[want[i]] = 1;
  }
  int nl = 0;
  // a slot for cluster c: the lowest empty slot, else the least recently
  // stamped slot that is not held (lowest index on ties), preferring slots
  // whose cluster is not wanted; for a predicted load only unwanted, older
  // slots qualify
  auto pick = [&](bool demand) -> int {
    for (int s = 0; s < n_slots; ++s)
      if (slot_cluster[s] < 0) return s;
    int best = -1;
    for (int s = 0; s < n_slots; ++s) {
      if (held[s]) continue;
      const bool w = wanted[slot_cluster[s]] != 0;
      if (!demand && (w || slot_stamp[s] >= frame)) continue;
      if (best < 0) {
        best = s;
        continue;
      }
      const bool wb = wanted[slot_cluster[best]] != 0;
      if (w != wb ? !w : slot_stamp[s] < slot_stamp[best]) best = s;
    }
    return best;
  };
  auto load = [&](int c, int s) {
    if (slot_cluster[s] >= 0) slot_of[slot_cluster[s]] = -1;
    slot_cluster[s] = c;
    slot_of[c] = s;
    slot_stamp[s] = frame;
    held[s] = 1;
    load_cluster[nl] = c;
    load_slot[nl] = s;
    ++nl;
  };
  for (int i = 0; i < n_need; ++i) {  // resident needed clusters are held
    const int s = slot_of[need[i]];
    if (s >= 0) {
      held[s] = 1;
      slot_stamp[s] = frame;
    }
  }
  for (int i = 0; i < n_need; ++i) {  // demand loads
    const int c = need[i];
    if (slot_of[c] >= 0) continue;
    load(c, pick(true));  // a slot exists: distinct needs <= n_slots
  }
  *n_demand = nl;
  for (int i = 0; i < n_want; ++i) {  // predicted loads
    const int c = want[i];
    if (slot_of[c] >= 0) {
      held[slot_of[c]] = 1;
      continue;
    }
    const int s = pick(false);
    if (s < 0) break;
    load(c, s);
  }
  *n_loads = nl;
  return SEELE_OK;
}

int32_t seele_load_segments(const float* host_src, int64_t src_stride, float* dev_pool,
                            int64_t dst_stride, int32_t rows, const int64_t* src_begin,
                            const int64_t* dst_begin, const int64_t* count, int32_t n_loads,
                            void* stream) {
  if (n_loads < 0 || rows < 0 || src_stride < 0 || dst_stride < 0)
    return fail(SEELE_ERR_INVALID_ARG, "negative size");
  if (n_loads == 0 || rows == 0) return SEELE_OK;
  if (!host_src || !dev_pool || !src_begin || !dst_begin || !count)
    return fail(SEELE_ERR_INVALID_ARG, "null argument");
  for (int j = 0; j < n_loads; ++j)
    if (count[j] < 0 || src_begin[j] < 0 || dst_begin[j] < 0 ||
        src_begin[j] + count[j] > src_stride || dst_begin[j] + count[j] > dst_stride)
      return fail(SEELE_ERR_INVALID_ARG, "load %d out of bounds", j);
  for (int j = 0; j < n_loads; ++j) {
    if (count[j] == 0) continue;
    const hipError_t e = hipMemcpy2DAsync(
        dev_pool + dst_begin[j], (size_t)dst_stride * sizeof(float), host_src + src_begin[j],
        (size_t)src_stride * sizeof(float), (size_t)count[j] * sizeof(float), (size_t)rows,
        hipMemcpyHostToDevice, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "segment copy");
  }
  return SEELE_OK;
}

}  // extern "C"

// ---- fine-tuning (Sec. 3.5)

namespace {

struct LossPlan {
  int64_t elems = 0, blocks = 0;
  size_t bytes = 0;
};

LossPlan loss_plan(const seele_camera* cams, int32_t n_views) {
  LossPlan p;
  for (int v = 0; v < n_views; ++v) {
    p.elems += 3 * (int64_t)cams[v].width * cams[v].height;
    p.blocks += loss_blocks(cams[v].width, cams[v].height);
  }
  // 3 maps of all elements + 2 floats per block (each chunk of views reuses it)
  p.bytes = (size_t)(3 * p.elems + 2 * p.blocks) * sizeof(float) + 256;
  return p;
}

}  // namespace

extern "C" {

size_t seele_photometric_loss_workspace_size(const seele_camera* cams, int32_t n_views) {
  if (!cams || n_views < 1) return 0;
  return loss_plan(cams, n_views).bytes;
}

int32_t seele_photometric_loss(const float* image, const float* target, const seele_camera* cams,
                               int32_t n_views, float lambda, void* workspace,
                               size_t workspace_bytes, float* loss, float* dL_dimage,
                               void* stream) {
  if (!cams || n_views < 1) return fail(SEELE_ERR_INVALID_ARG, "need cameras, n_views >= 1");
  for (int v = 0; v < n_views; ++v) {
    const int32_t st = check_camera(cams[v], v, 16);
    if (st != SEELE_OK) return st;
  }
  if (!(lambda >= 0.0f && lambda <= 1.0f)) return fail(SEELE_ERR_INVALID_ARG, "lambda not in [0, 1]");
  if (!image || !target || !loss || !dL_dimage || !aligned(image, 4) || !aligned(target, 4) ||
      !aligned(loss, 4) || !aligned(dL_dimage, 4))
    return fail(SEELE_ERR_INVALID_ARG, "null or misaligned array");
  const LossPlan plan = loss_plan(cams, n_views);
  if (!workspace || !aligned(workspace, 256) || workspace_bytes < plan.bytes)
    return fail(SEELE_ERR_CAPACITY, "workspace needs %zu bytes", plan.bytes);
  if (plan.blocks >= ((int64_t)1 << 31)) return fail(SEELE_ERR_UNSUPPORTED, "images too large");
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* maps = static_cast<float*>(workspace);
  int64_t e0 = 0;
  for (int v0 = 0; v0 < n_views; v0 += kMaxViewsLoss) {
    const int nv = std::min(kMaxViewsLoss, n_views - v0);
    LossViews lv{};
    lv.n_views = nv;
    int64_t e = 0, b = 0;
    for (int k = 0; k < nv; ++k) {
      const seele_camera& c = cams[v0 + k];
      lv.elem_off[k] = e;
      lv.blk_off[k] = (int32_t)b;
      lv.w[k] = c.width;
      lv.h[k] = c.height;
      e += 3 * (int64_t)c.width * c.height;
      b += loss_blocks(c.width, c.height);
    }
    lv.elem_off[nv] = e;
    lv.blk_off[nv] = (int32_t)b;
    float* blk = maps + 3 * e;
    const hipError_t err = launch_photometric_loss(
        lv, (int)b, image + e0, target + e0, lambda, 1.0f / (float)n_views, maps, e, blk,
        loss + v0, dL_dimage + e0, s);
    if (err != hipSuccess) return hip_fail(err, "photometric loss launch");
    e0 += e;
  }
  return SEELE_OK;
}

int32_t seele_adam_step(const seele_gaussian_grads* params, const seele_gaussian_grads* grads,
                        const seele_gaussian_grads* m, const seele_gaussian_grads* v, int64_t n,
                        int32_t sh_degree, const seele_adam_opts* opts, int64_t step,
                        void* stream) {
  if (!params || !grads || !m || !v || !opts) return fail(SEELE_ERR_INVALID_ARG, "null argument");
  if (n < 0 || sh_degree < 0 || sh_degree > 3 || step < 1)
    return fail(SEELE_ERR_INVALID_ARG, "need n >= 0, 0 <= sh_degree <= 3, step >= 1");
  const float lrs[6] = {opts->lr_means, opts->lr_log_scales, opts->lr_quats,
                        opts->lr_opacity, opts->lr_sh_dc, opts->lr_sh_rest};
  for (float x : lrs)
    if (!(x >= 0.0f) || !is_finite(x)) return fail(SEELE_ERR_INVALID_ARG, "bad learning rate");
  if (!(opts->beta1 >= 0.0f && opts->beta1 < 1.0f) || !(opts->beta2 >= 0.0f && opts->beta2 < 1.0f) ||
      !(opts->eps > 0.0f))
    return fail(SEELE_ERR_INVALID_ARG, "bad beta1/beta2/eps");
  if (n == 0) return SEELE_OK;
  const int n_sh = 3 * (sh_degree + 1) * (sh_degree + 1);
  const int64_t len[6] = {3 * n, 3 * n, 4 * n, n, 3 * n, (int64_t)(n_sh - 3) * n};
  const seele_gaussian_grads* t[4] = {params, grads, m, v};
  float* ptr[4][6];
  for (int k = 0; k < 4; ++k) {
    const seele_gaussian_grads& a = *t[k];
    float* base[6] = {a.means, a.log_scales, a.quats, a.opacity_logits, a.sh,
                      a.sh ? a.sh + 3 * n : nullptr};
    for (int s = 0; s < 6; ++s) {
      if (len[s] > 0 && (!base[s] || !aligned(base[s], 4)))
        return fail(SEELE_ERR_INVALID_ARG, "null or misaligned attribute array");
      ptr[k][s] = base[s];
    }
  }
  const hipError_t e = launch_adam(ptr[0], ptr[1], ptr[2], ptr[3], len, lrs, opts->beta1,
                                   opts->beta2, opts->eps, step, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SEELE_OK : hip_fail(e, "adam launch");
}

}  // extern "C"

// ---- FLIP view-consistency term (Sec. 3.5)

namespace {

constexpr double kPi = 3.14159265358979323846;

struct FlipHost {
  FlipFilt f;
  FlipConst k;
};

void flip_lab(const double* m, const double* white, const double* lin, double* lab) {
  double n[3];
  for (int i = 0; i < 3; ++i)
    n[i] = (m[i * 3] * lin[0] + m[i * 3 + 1] * lin[1] + m[i * 3 + 2] * lin[2]) / white[i];
  const double d = 6.0 / 29.0;
  double f[3];
  for (int i = 0; i < 3; ++i) f[i] = n[i] > d * d * d ? std::cbrt(n[i]) : n[i] / (3 * d * d) + 4.0 / 29.0;
  lab[0] = 116 * f[1] - 16;
  lab[1] = 0.01 * lab[0] * 500 * (f[0] - f[1]);  // Hunt-adjusted
  lab[2] = 0.01 * lab[0] * 200 * (f[1] - f[2]);
}

int32_t flip_setup(float ppd, FlipHost& h) {
  if (!(ppd > 0.0f) || !is_finite(ppd)) return fail(SEELE_ERR_INVALID_ARG, "bad pixels per degree");
  const double P = ppd;
  const double bA = 0.0047, bRG = 0.0053, a1 = 34.1, b1 = 0.04, a2 = 13.5, b2 = 0.025;
  const int rc = (int)std::ceil(3.0 * std::sqrt(0.04 / (2 * kPi * kPi)) * P);
  const double sd = 0.5 * 0.082 * P;
  const int rf = (int)std::ceil(3.0 * sd);
  if (rc > kMaxFlipRadius || rf > kMaxFlipRadius)
    return fail(SEELE_ERR_UNSUPPORTED, "pixels per degree above %d-pixel filter radii",
                kMaxFlipRadius);
  FlipFilt& f = h.f;
  f = FlipFilt{};
  f.rc = rc;
  f.rf = rf;
  auto gauss = [&](double b, int t) { return std::exp(-kPi * kPi * (t / P) * (t / P) / b); };
  double sA = 0, sRG = 0, s1 = 0, s2 = 0;
  for (int t = -rc; t <= rc; ++t) {
    sA += gauss(bA, t);
    sRG += gauss(bRG, t);
    s1 += gauss(b1, t);
    s2 += gauss(b2, t);
  }
  const double w1 = a1 * std::sqrt(kPi / b1), w2 = a2 * std::sqrt(kPi / b2);
  const double S = w1 * s1 * s1 + w2 * s2 * s2;
  f.c1 = (float)(w1 / S);
  f.c2 = (float)(w2 / S);
  for (int t = -rc; t <= rc; ++t) {
    f.gA[t + rc] = (float)(gauss(bA, t) / sA);
    f.gRG[t + rc] = (float)(gauss(bRG, t) / sRG);
    f.u1[t + rc] = (float)gauss(b1, t);
    f.u2[t + rc] = (float)gauss(b2, t);
  }
  double G = 0, ep = 0, en = 0, pp = 0, pn = 0;
  for (int t = -rf; t <= rf; ++t) {
    const double g = std::exp(-(double)t * t / (2 * sd * sd));
    const double e = -t * g, q = ((double)t * t / (sd * sd) - 1) * g;
    G += g;
    if (e > 0) ep += e; else en -= e;
    if (q > 0) pp += q; else pn -= q;
  }
  for (int t = -rf; t <= rf; ++t) {
    const double g = std::exp(-(double)t * t / (2 * sd * sd));
    const double e = -t * g, q = ((double)t * t / (sd * sd) - 1) * g;
    f.gn[t + rf] = (float)(g / G);
    f.fe[t + rf] = (float)(e > 0 ? e / ep : e / en);
    f.fp[t + rf] = (float)(q > 0 ? q / pp : q / pn);
  }
  // colour constants: linear sRGB -> XYZ (D65) and its inverse
  const double m[9] = {10135552.0 / 24577794, 8788810.0 / 24577794, 4435075.0 / 24577794,
                       2613072.0 / 12288897,  8788810.0 / 12288897, 887015.0 / 12288897,
                       1425312.0 / 73733382,  8788810.0 / 73733382, 70074185.0 / 73733382};
  const double det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                     m[2] * (m[3] * m[7] - m[4] * m[6]);
  const double mi[9] = {(m[4] * m[8] - m[5] * m[7]) / det, (m[2] * m[7] - m[1] * m[8]) / det,
                        (m[1] * m[5] - m[2] * m[4]) / det, (m[5] * m[6] - m[3] * m[8]) / det,
                        (m[0] * m[8] - m[2] * m[6]) / det, (m[2] * m[3] - m[0] * m[5]) / det,
                        (m[3] * m[7] - m[4] * m[6]) / det, (m[1] * m[6] - m[0] * m[7]) / det,
                        (m[0] * m[4] - m[1] * m[3]) / det};
  double white[3];
  for (int i = 0; i < 3; ++i) white[i] = m[i * 3] + m[i * 3 + 1] + m[i * 3 + 2];
  FlipConst& k = h.k;
  for (int i = 0; i < 3; ++i) {
    k.white[i] = (float)white[i];
    k.inv_white[i] = (float)(1.0 / white[i]);
    for (int j = 0; j < 3; ++j) {
      k.m[i][j] = (float)m[i * 3 + j];
      k.mi[i][j] = (float)mi[i * 3 + j];
    }
  }
  k.qc = 0.7f;
  k.qf = 0.5f;
  k.pc = 0.4f;
  k.pt = 0.95f;
  k.eps = 1e-15f;
  const double green[3] = {0, 1, 0}, blue[3] = {0, 0, 1};
  double lg[3], lb[3];
  flip_lab(m, white, green, lg);
  flip_lab(m, white, blue, lb);
  const double hy = std::fabs(lg[0] - lb[0]) +
                    std::sqrt(std::max((lg[1] - lb[1]) * (lg[1] - lb[1]) +
                                       (lg[2] - lb[2]) * (lg[2] - lb[2]), 1e-15));
  k.cmax = (float)std::pow(hy, 0.7);
  k.lo_slope = (float)(0.95 / (0.4 * (double)k.cmax));
  k.hi_slope = (float)((1.0 - 0.95) / ((double)k.cmax - 0.4 * (double)k.cmax));
  return SEELE_OK;
}

struct FlipPlan {
  int64_t pix = 0, blocks = 0;
  size_t bytes = 0;
};

FlipPlan flip_plan(const seele_camera* cams, int32_t n_views) {
  FlipPlan p;
  for (int v = 0; v < n_views; ++v) {
    p.pix += (int64_t)cams[v].width * cams[v].height;
    p.blocks += std::max(flip_blocks(cams[v].width, cams[v].height),
                         flip_tile_blocks(cams[v].width, cams[v].height));
  }
  // 27 maps for the untiled path (7 for the tiled one) + a float per block
  p.bytes = (size_t)(27 * p.pix + p.blocks) * sizeof(float) + 256;
  return p;
}

}  // namespace

extern "C" {

size_t seele_flip_loss_workspace_size(const seele_camera* cams, int32_t n_views) {
  if (!cams || n_views < 1) return 0;
  return flip_plan(cams, n_views).bytes;
}

int32_t seele_flip_loss(const float* image, const float* reference, const seele_camera* cams,
                        int32_t n_views, float ppd, float scale, int32_t accumulate,
                        void* workspace, size_t workspace_bytes, float* flip, float* dL_dimage,
                        void* stream) {
  if (!cams || n_views < 1) return fail(SEELE_ERR_INVALID_ARG, "need cameras, n_views >= 1");
  for (int v = 0; v < n_views; ++v) {
    const int32_t st = check_camera(cams[v], v, 16);
    if (st != SEELE_OK) return st;
  }
  if (!is_finite(scale)) return fail(SEELE_ERR_INVALID_ARG, "non-finite scale");
  if (!image || !reference || !flip || !dL_dimage || !aligned(image, 4) ||
      !aligned(reference, 4) || !aligned(flip, 4) || !aligned(dL_dimage, 4))
    return fail(SEELE_ERR_INVALID_ARG, "null or misaligned array");
  FlipHost h;
  int32_t st = flip_setup(ppd, h);
  if (st != SEELE_OK) return st;
  const FlipPlan plan = flip_plan(cams, n_views);
  if (!workspace || !aligned(workspace, 256) || workspace_bytes < plan.bytes)
    return fail(SEELE_ERR_CAPACITY, "workspace needs %zu bytes", plan.bytes);
  if (plan.blocks >= ((int64_t)1 << 31)) return fail(SEELE_ERR_UNSUPPORTED, "images too large");
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* maps = static_cast<float*>(workspace);
  // LDS-tiled kernels when both filter radii fit their halo
  const bool tiled = std::max(h.f.rc, h.f.rf) <= flip_tile_halo();
  int64_t p0 = 0;
  for (int v0 = 0; v0 < n_views; v0 += kMaxViewsFlip) {
    const int nv = std::min(kMaxViewsFlip, n_views - v0);
    FlipViews fv{};
    fv.n_views = nv;
    int64_t P = 0, b = 0;
    for (int k = 0; k < nv; ++k) {
      const seele_camera& c = cams[v0 + k];
      fv.pix_off[k] = P;
      fv.blk_off[k] = (int32_t)b;
      fv.w[k] = c.width;
      fv.h[k] = c.height;
      P += (int64_t)c.width * c.height;
      b += tiled ? flip_tile_blocks(c.width, c.height) : flip_blocks(c.width, c.height);
    }
    fv.pix_off[nv] = P;
    fv.blk_off[nv] = (int32_t)b;
    const hipError_t e =
        tiled ? launch_flip_tiled(fv, (int)b, h.f, h.k, image + 3 * p0, reference + 3 * p0,
                                  maps, P, maps + 27 * P, scale / (float)n_views,
                                  accumulate != 0, flip + v0, dL_dimage + 3 * p0, s)
              : launch_flip(fv, (int)b, h.f, h.k, image + 3 * p0, reference + 3 * p0, maps, P,
                            maps + 27 * P, scale / (float)n_views, accumulate != 0, flip + v0,
                            dL_dimage + 3 * p0, s);
    if (e != hipSuccess) return hip_fail(e, "flip launch");
    p0 += P;
  }
  return SEELE_OK;
}

}  // extern "C"

// ---- scene storage order

extern "C" {

size_t seele_spatial_order_workspace_size(int64_t n) {
  return n < 0 ? 0 : spatial_order_workspace_size(n);
}

int32_t seele_spatial_order(const seele_gaussians* g, void* workspace, size_t workspace_bytes,
                            int64_t* perm, void* stream) {
  const int32_t st = check_gaussians(g);
  if (st != SEELE_OK) return st;
  if (g->n >= ((int64_t)1 << 32)) return fail(SEELE_ERR_UNSUPPORTED, "more than 2^32 Gaussians");
  if (g->n == 0) return SEELE_OK;
  if (!perm || !aligned(perm, 8)) return fail(SEELE_ERR_INVALID_ARG, "perm null or misaligned");
  const size_t need = spatial_order_workspace_size(g->n);
  if (!workspace || !aligned(workspace, 256) || workspace_bytes < need)
    return fail(SEELE_ERR_CAPACITY, "workspace needs %zu bytes", need);
  const hipError_t e = launch_spatial_order(g->means, g->n, workspace, perm,
                                            static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SEELE_OK : hip_fail(e, "spatial order launch");
}

}  // extern "C"
