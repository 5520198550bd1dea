// Front-to-back blending on gfx950: plain (Sec. 3.1, Eqs. 1-2) and
// contribution-aware (Sec. 3.4, Algorithm 1).
//
// One workgroup per (view, tile), one lane per pixel.  Each wave owns an 8x8
// pixel block laid out as pixel groups (2x2 by default): lanes
// [k*g, (k+1)*g) hold group k with its leader (top-left pixel) first.  The
// tile's depth-ordered list is staged through LDS in batches of one record
// per thread; there the conic is replaced by the Cholesky factor of
// (log2(e)/2) * conic, so that exp(-q/2) = exp2(-(u^2 + w^2)) with two linear
// forms u, w of the pixel offset.
//
// Plain form: every live lane evaluates every Gaussian of the batch.
// Contribution-aware form: the leader tests are packed -- lane l tests group
// (l mod G) against Gaussian (l div G), so one wave instruction stream tests
// 64/G Gaussians against all G group leaders (4 Gaussians for 2x2 groups).
// The ballot of those tests is wave-uniform: a Gaussian no leader accepts is
// skipped by the whole wave without any per-pixel work (the divergence-free
// skip of Sec. 3.4 "GPU Parallelism"); otherwise only lanes of accepting
// groups evaluate and blend it.  Leaders keep testing after they stop.
//
// Early exit: a wave leaves a batch when all its lanes are done; the block
// stops loading batches when all its pixels are done.
#include "seele_internal.h"

namespace seele {

namespace {

struct LdsBatch {
  float4 a;  // mean_x, mean_y, l11, l21  (Cholesky factor of k * conic)
  float4 b;  // l22, opacity, r, g
};

__device__ __forceinline__ float alpha_at(float px, float py, const float4& a, const float4& b,
                                          float alpha_max) {
  float dx, dy;
  const float p = splat_power(px, py, a.x, a.y, a.z, a.w, b.x, dx, dy);
  return __builtin_fminf(alpha_max, b.y * fast_exp2(p));
}

// COUNT instantiations also accumulate the method's work counters:
// [0] alpha evaluations by pixels that have not stopped (contribution-aware:
// only in groups whose leader accepted), [1] blends, [2] leader tests of
// groups holding a live pixel, [3] of those, acceptances.
template <int TS, int MODE, bool COUNT>
__global__ __launch_bounds__(TS* TS) void k_raster_fwd(RasterViews views, RasterParams rp,
                                                       const seele_splat* __restrict__ splats,
                                                       const uint32_t* __restrict__ ids,
                                                       const int32_t* __restrict__ ranges,
                                                       float* __restrict__ image,
                                                       float* __restrict__ final_T,
                                                       int32_t* __restrict__ n_contrib,
                                                       unsigned long long* __restrict__ counters) {
  constexpr int NT = TS * TS;
  __shared__ LdsBatch s_ab[NT];
  __shared__ float s_blue[NT];
  __shared__ unsigned long long s_cnt[4];
  uint32_t c_eval = 0, c_blend = 0, c_ltest = 0, c_lpass = 0;
  if (COUNT) {
    if (threadIdx.x < 4) s_cnt[threadIdx.x] = 0;
  }

  const int gt = blockIdx.x;
  int v = 0;
  for (int k = 1; k < views.n_views; ++k)
    if (views.v[k].tile_begin <= gt) v = k;
  const RasterView rv = views.v[v];
  const int lt = gt - rv.tile_begin;
  const int tile_x = lt % rv.grid_w, tile_y = lt / rv.grid_w;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wx = (TS == 16) ? (wave & 1) * 8 : 0;
  const int wy = (TS == 16) ? (wave >> 1) * 8 : 0;
  const int gw = MODE ? rp.group_w : 1, gh = MODE ? rp.group_h : 1;
  const int gsz = gw * gh, G = 64 / gsz, gpr = 8 / gw;
  const int grp = lane / gsz, r = lane % gsz;
  const int x = tile_x * TS + wx + (grp % gpr) * gw + r % gw;
  const int y = tile_y * TS + wy + (grp / gpr) * gh + r / gw;
  const bool inside = x < rv.W && y < rv.H;
  const float fx = (float)x + 0.5f, fy = (float)y + 0.5f;
  // leader this lane tests in the packed contribution-aware test
  const int tg = lane % G, sub = lane / G;
  const float lfx = (float)(tile_x * TS + wx + (tg % gpr) * gw) + 0.5f;
  const float lfy = (float)(tile_y * TS + wy + (tg / gpr) * gh) + 0.5f;
  const uint64_t gmask = G >= 64 ? ~0ull : ((1ull << G) - 1ull);

  const int64_t ri = 2 * ((int64_t)views.tile_base + gt);
  const int start = ranges[ri], n = ranges[ri + 1] - start;
  const float amin = rp.alpha_min, amax = rp.alpha_max, tmin = rp.T_min;

  float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
  int last = 0;
  bool done = !inside;

  for (int base = 0; base < n; base += NT) {
    if (__syncthreads_count(done) == NT) break;
    const int j = base + tid;
    if (j < n) {
      const float4* src = reinterpret_cast<const float4*>(splats + ids[start + j]);
      const float4 A = src[0], Bv = src[1];
      const float blue = src[2].x;
      const Chol L = conic_factor(A.z, A.w, Bv.x);
      s_ab[tid].a = make_float4(A.x, A.y, L.l11, L.l21);
      s_ab[tid].b = make_float4(L.l22, Bv.y, Bv.z, Bv.w);
      s_blue[tid] = blue;
    }
    __syncthreads();
    const int cnt = min(NT, n - base);
    if (MODE == 0) {
      for (int k = 0; k < cnt; ++k) {
        if (__ballot(!done) == 0) break;
        if (!done) {
          if (COUNT) ++c_eval;
          const float4 a = s_ab[k].a, b = s_ab[k].b;
          const float alpha = alpha_at(fx, fy, a, b, amax);
          if (alpha >= amin) {
            const float Tn = T * (1.0f - alpha);
            if (Tn < tmin) {
              done = true;
            } else {
              const float wgt = alpha * T;
              c0 = __builtin_fmaf(wgt, b.z, c0);
              c1 = __builtin_fmaf(wgt, b.w, c1);
              c2 = __builtin_fmaf(wgt, s_blue[k], c2);
              T = Tn;
              last = base + k + 1;
              if (COUNT) ++c_blend;
            }
          }
        }
      }
    } else {
      const int per = 64 / G;
      for (int k0 = 0; k0 < cnt; k0 += per) {
        if (__ballot(!done) == 0) break;
        const int kk = k0 + sub;
        bool pass = false;
        if (kk < cnt) pass = alpha_at(lfx, lfy, s_ab[kk].a, s_ab[kk].b, amax) >= amin;
        const uint64_t bal = __ballot(pass);
        for (int s = 0; s < per; ++s) {
          const uint64_t gm = (bal >> (s * G)) & gmask;
          if (COUNT && k0 + s < cnt) {
            const uint64_t live = __ballot(!done);  // all lanes take part in the ballot
            uint64_t glive = 0;
            const uint64_t gl = gsz >= 64 ? ~0ull : ((1ull << gsz) - 1ull);
            for (int q = 0; q < G; ++q)
              if ((live >> (q * gsz)) & gl) glive |= 1ull << q;
            if (lane == 0) {
              c_ltest += (uint32_t)__popcll(glive);
              c_lpass += (uint32_t)__popcll(glive & gm);
            }
          }
          if (gm == 0) continue;  // no leader of this wave accepts it: wave-uniform skip
          if (!done && ((gm >> grp) & 1ull)) {
            const int k = k0 + s;
            if (COUNT) ++c_eval;
            const float4 a = s_ab[k].a, b = s_ab[k].b;
            const float alpha = alpha_at(fx, fy, a, b, amax);
            if (alpha >= amin) {
              const float Tn = T * (1.0f - alpha);
              if (Tn < tmin) {
                done = true;
              } else {
                const float wgt = alpha * T;
                c0 = __builtin_fmaf(wgt, b.z, c0);
                c1 = __builtin_fmaf(wgt, b.w, c1);
                c2 = __builtin_fmaf(wgt, s_blue[k], c2);
                T = Tn;
                last = base + k + 1;
                if (COUNT) ++c_blend;
              }
            }
          }
        }
      }
    }
    __syncthreads();
  }

  if (COUNT) {
    __syncthreads();
    atomicAdd(&s_cnt[0], (unsigned long long)c_eval);
    atomicAdd(&s_cnt[1], (unsigned long long)c_blend);
    atomicAdd(&s_cnt[2], (unsigned long long)c_ltest);
    atomicAdd(&s_cnt[3], (unsigned long long)c_lpass);
    __syncthreads();
    if (threadIdx.x < 4) atomicAdd(&counters[threadIdx.x], s_cnt[threadIdx.x]);
  }

  if (inside) {
    const int64_t hw = (int64_t)rv.W * rv.H;
    const int64_t pix = (int64_t)y * rv.W + x;
    float* img = image + 3 * rv.pix_base;
    img[pix] = c0 + T * rp.bg0;
    img[hw + pix] = c1 + T * rp.bg1;
    img[2 * hw + pix] = c2 + T * rp.bg2;
    final_T[rv.pix_base + pix] = T;
    n_contrib[rv.pix_base + pix] = last;
  }
}

template <int TS, bool COUNT>
void launch_ts(int mode, dim3 grid, const RasterViews& views, const RasterParams& rp,
               const seele_splat* splats, const uint32_t* ids, const int32_t* ranges, float* image,
               float* final_T, int32_t* n_contrib, unsigned long long* counters,
               hipStream_t stream) {
  if (mode == SEELE_RASTER_CONTRIB)
    hipLaunchKernelGGL((k_raster_fwd<TS, 1, COUNT>), grid, dim3(TS * TS), 0, stream, views, rp,
                       splats, ids, ranges, image, final_T, n_contrib, counters);
  else
    hipLaunchKernelGGL((k_raster_fwd<TS, 0, COUNT>), grid, dim3(TS * TS), 0, stream, views, rp,
                       splats, ids, ranges, image, final_T, n_contrib, counters);
}

}  // namespace

hipError_t launch_raster_fwd(int tile, int mode, const RasterViews& views, int n_tiles_launch,
                             const RasterParams& rp, const seele_splat* splats,
                             const uint32_t* sorted_ids, const int32_t* tile_ranges, float* image,
                             float* final_T, int32_t* n_contrib, unsigned long long* counters,
                             hipStream_t stream) {
  if (n_tiles_launch <= 0) return hipSuccess;
  const dim3 grid(n_tiles_launch);
  if (tile == 16) {
    if (counters)
      launch_ts<16, true>(mode, grid, views, rp, splats, sorted_ids, tile_ranges, image, final_T,
                          n_contrib, counters, stream);
    else
      launch_ts<16, false>(mode, grid, views, rp, splats, sorted_ids, tile_ranges, image, final_T,
                           n_contrib, counters, stream);
  } else {
    if (counters)
      launch_ts<8, true>(mode, grid, views, rp, splats, sorted_ids, tile_ranges, image, final_T,
                         n_contrib, counters, stream);
    else
      launch_ts<8, false>(mode, grid, views, rp, splats, sorted_ids, tile_ranges, image, final_T,
                          n_contrib, counters, stream);
  }
  return hipGetLastError();
}

}  // namespace seele
