// Backward of front-to-back blending on gfx950 (fine-tuning, Sec. 3.5), for
// the plain (Eqs. 1-2) and contribution-aware (Algorithm 1) forms.
//
// No per-pixel lists are stored by the forward pass: each pixel walks its
// tile list backwards from its last blended position (n_contrib) with the
// final transmittance T, recomputing alpha with the forward's own device
// function, so every skip / leader / blend decision is reproduced exactly.
// For a blended entry j with colour c_j and the colour S accumulated behind
// it (background included):
//   T_j = T / (1 - alpha_j)                     (transmittance before j)
//   dL/dalpha_j = T_j (g . c_j) - (g . S) / (1 - alpha_j)
//   dL/dc_j = T_j alpha_j g
// and through alpha = o exp(-q/2), q = d^T A d (zero where the alpha clamp
// was active).  Only the scalar g . S is carried (S itself is never needed).
// Per-record terms are reduced across the wave (DPP), summed over the
// block's waves in LDS, turned into the record's 9 gradient slots and added
// to HBM with one set of float atomics per tile.
//
// As in the forward kernels, each wave visits only the records whose culling
// bit for its 8x8 block is set (quad_mask), and only those below the largest
// n_contrib of its pixels: a skipped record is blended by none of its pixels
// and so has no gradient from them.
#include "seele_internal.h"

namespace seele {

namespace {

struct LdsBwd {
  float4 a;  // mean_x, mean_y, l11, l21
  float4 b;  // l22, log2(opacity), r, g
  float4 c;  // blue, conic a, conic b, conic c
  float inv_o, pad0, pad1, pad2;  // 1 / opacity
};

// Sum of x over the 64 lanes of a wave, returned to every lane: inclusive
// row sums by DPP row shifts (1, 2, 4, 8 within each 16-lane row), then the
// row totals carried across rows by the row broadcasts of lanes 15 and 31,
// so lane 63 holds the total.  Masked or out-of-row source lanes add 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_shifted(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf,
                                                    false));
}

__device__ __forceinline__ float wave_total(float x) {
  x += dpp_shifted<0x111, 0xf>(x);  // row_shr:1
  x += dpp_shifted<0x112, 0xf>(x);  // row_shr:2
  x += dpp_shifted<0x114, 0xf>(x);  // row_shr:4
  x += dpp_shifted<0x118, 0xf>(x);  // row_shr:8
  x += dpp_shifted<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_shifted<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Add the wave sums of nine per-lane values to acc[0..8] (LDS).  Eight of
// them are reduced transposed: a 32-lane swap pairs v0/v1, v2/v3, ... so that
// one register holds half-sums of one value in lanes 0-31 and of the other
// in lanes 32-63; a 16-lane swap then leaves each 16-lane row of a register
// with quarter-sums of a single value; row shifts finish each row, and the
// last lane of each row adds its value's total.  The ninth takes the plain
// DPP reduction.
__device__ __forceinline__ float row_total(float x) {
  x += dpp_shifted<0x111, 0xf>(x);  // row_shr:1
  x += dpp_shifted<0x112, 0xf>(x);  // row_shr:2
  x += dpp_shifted<0x114, 0xf>(x);  // row_shr:4
  x += dpp_shifted<0x118, 0xf>(x);  // row_shr:8
  return x;                         // lane 15 of each row: the row's sum
}

__device__ __forceinline__ float pair_half(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float pair_quarter(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ void wave_accumulate9(const float (&v)[9], float* acc, int lane) {
  // rows of t0: v0, v2, v1, v3; rows of t1: v4, v6, v5, v7
  const float t0 = row_total(pair_quarter(pair_half(v[0], v[1]), pair_half(v[2], v[3])));
  const float t1 = row_total(pair_quarter(pair_half(v[4], v[5]), pair_half(v[6], v[7])));
  const float t8 = wave_total(v[8]);
  if ((lane & 15) == 15) {
    const int row = lane >> 4;
    const int idx = ((row & 1) << 1) | (row >> 1);
    atomicAdd(acc + idx, t0);
    atomicAdd(acc + 4 + idx, t1);
    if (lane == 63) atomicAdd(acc + 8, t8);
  }
}

// One record of the reverse walk for one pixel (pixel_terms): recompute
// alpha, undo the blend (T and GS = g . S, the loss gradient dotted with the
// colour S accumulated behind the record, background included) if the
// forward blended it, and give the record's per-pixel terms v; blend_grad
// adds them, reduced over the wave, to the record's LDS accumulator `acc` (9
// floats, shared by the block's waves and turned into gradients once per
// batch).  With d = pixel - mean, A = conic and
// p = alpha dL/dalpha below the alpha clamp:
//   dL/do    = p / o
//   dL/dA    = -p d d^T / 2   (off-diagonal: -p dx dy for the b of q)
//   dL/dmean = p A d
// so the accumulated terms are p, p dx, p dy, p dx^2, p dx dy, p dy^2 and
// the colour terms T_j alpha g; the record's constants (A, 1/o) multiply the
// sums once per batch.
template <int MODE>
__device__ __forceinline__ bool pixel_terms(const LdsBwd& e, bool need, float fx, float fy,
                                            int leader_lane, float amin, float amax, float g0,
                                            float g1, float g2, float& T, float& GS,
                                            float (&v)[9]) {
  const float4 a = e.a, b = e.b;  // b.y = log2(opacity), as the forward stages it
  float dx, dy;
  const float qo = splat_qo(fx, fy, a.x, a.y, a.z, a.w, b.x, b.y, dx, dy);
  const float raw = fast_exp2(-qo);
  const float alpha = clamp_alpha(raw, amax);
  bool blended = need && alpha >= amin;
  if (MODE) {
    // the leader's alpha is the leader lane's own alpha (same function, same pixel)
    const float lead = __shfl(alpha, leader_lane, 64);
    blended = blended && lead >= amin;
  }
  // branch-free: every lane computes the step, the selects keep only the
  // blended lanes' effects (1 - alpha >= 1 - alpha_max > 0 everywhere)
  const float cb = e.c.x;
  const float om = 1.0f - alpha;
  const float rom = __builtin_amdgcn_rcpf(om);
  const float Tj = T * rom;
  const float ta = Tj * alpha;
  // fused multiply-adds from here on: the gradient chain needs no
  // bit-identity with the forward (only alpha and the decisions do)
  const float gc = __builtin_fmaf(g2, cb, __builtin_fmaf(g1, b.w, g0 * b.z));  // g . c
  // dL/dalpha = T_j (g . c) - (g . S) / (1 - alpha)
  const float dal = __builtin_fmaf(Tj, gc, -(rom * GS));
  GS = blended ? __builtin_fmaf(ta, gc, GS) : GS;
  T = blended ? Tj : T;
  const float wc = blended ? ta : 0.0f;
  const float gr = wc * g0, gg = wc * g1, gbl = wc * g2;
  // p = alpha dL/dalpha where the clamp is inactive (d alpha / d o = alpha / o)
  const float tp = (blended && raw <= amax) ? alpha * dal : 0.0f;
  const float tx = tp * dx, ty = tp * dy;
  v[0] = tx;
  v[1] = ty;
  v[2] = tx * dx;
  v[3] = tx * dy;
  v[4] = ty * dy;
  v[5] = tp;
  v[6] = gr;
  v[7] = gg;
  v[8] = gbl;
  return blended;
}

template <int MODE>
__device__ __forceinline__ void blend_grad(const LdsBwd& e, bool need, float fx, float fy,
                                           int leader_lane, int lane, float amin, float amax,
                                           float g0, float g1, float g2, float& T, float& GS,
                                           float* acc) {
  float v[9];
  const bool blended =
      pixel_terms<MODE>(e, need, fx, fy, leader_lane, amin, amax, g0, g1, g2, T, GS, v);
  if (__ballot(blended) != 0) wave_accumulate9(v, acc, lane);
}

// Gradient slots of a record (mean x, mean y, conic a, b, c, opacity, r, g,
// b) from its accumulated terms {sum p dx, sum p dy, sum p dx^2,
// sum p dx dy, sum p dy^2, sum p, colour x3}.
__device__ __forceinline__ void record_grads(const LdsBwd& e, const float* t, float* out) {
  const float ca = e.c.y, cbb = e.c.z, cc = e.c.w;
  out[0] = __builtin_fmaf(ca, t[0], cbb * t[1]);
  out[1] = __builtin_fmaf(cbb, t[0], cc * t[1]);
  out[2] = -0.5f * t[2];
  out[3] = -t[3];
  out[4] = -0.5f * t[4];
  out[5] = t[5] * e.inv_o;
  out[6] = t[6];
  out[7] = t[7];
  out[8] = t[8];
}

// Gradient slot k of record_grads alone.
__device__ __forceinline__ float record_grad(const LdsBwd& e, const float* t, int k) {
  if (k < 2) {
    const float ca = e.c.y, cbb = e.c.z, cc = e.c.w;
    return k == 0 ? __builtin_fmaf(ca, t[0], cbb * t[1]) : __builtin_fmaf(cbb, t[0], cc * t[1]);
  }
  const float sc = k == 5 ? e.inv_o : (k == 2 || k == 4) ? -0.5f : k == 3 ? -1.0f : 1.0f;
  return sc * t[k];
}

template <int TS, int MODE>
__global__ __launch_bounds__(TS* TS) void k_raster_bwd(RasterViews views, RasterParams rp,
                                                       const seele_splat* __restrict__ splats,
                                                       const uint32_t* __restrict__ ids,
                                                       const int32_t* __restrict__ ranges,
                                                       const float* __restrict__ final_T,
                                                       const int32_t* __restrict__ n_contrib,
                                                       const float* __restrict__ dL_dimage,
                                                       float* __restrict__ grad2d) {
  constexpr int NT = TS * TS;
  // records staged per batch: half the block for 16 x 16 tiles keeps the LDS
  // at 13 KB, so the VGPR budget (9 waves per SIMD), not the LDS, bounds the
  // occupancy
  constexpr int NBATCH = NT > 64 ? NT / 2 : NT;
  __shared__ LdsBwd s_e[NBATCH];
  __shared__ uint32_t s_id[NBATCH];
  __shared__ uint8_t s_qm[NBATCH];
  __shared__ float s_g[NBATCH][9];  // per staged record: the block's 2D gradient sum
  __shared__ int s_max;

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
  const int gsz = gw * gh, gpr = 8 / gw;
  const int grp = lane / gsz, r = lane % gsz;
  const int leader_lane = lane - r;
  const int x = tile_x * TS + wx + (grp % gpr) * gw + r % gw;
  const int y = tile_y * TS + wy + (grp / gpr) * gh + r / gw;
  const bool inside = x < rv.W && y < rv.H;
  const float fx = (float)x + 0.5f, fy = (float)y + 0.5f;

  const int64_t ri = 2 * ((int64_t)views.tile_base + gt);
  const int start = ranges[ri];
  const float amin = rp.alpha_min, l2ia = rp.log2_inv_alpha_min, amax = rp.alpha_max;

  float T = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
  int last = 0;
  if (inside) {
    const int64_t hw = (int64_t)rv.W * rv.H;
    const int64_t pix = (int64_t)y * rv.W + x;
    T = final_T[rv.pix_base + pix];
    last = n_contrib[rv.pix_base + pix];
    const float* g = dL_dimage + 3 * rv.pix_base;
    g0 = g[pix];
    g1 = g[hw + pix];
    g2 = g[2 * hw + pix];
  }
  // g . S with S = T bg, the colour behind the last blended record
  float GS = T * __builtin_fmaf(g2, rp.bg2, __builtin_fmaf(g1, rp.bg1, g0 * rp.bg0));

  if (tid == 0) s_max = 0;
  __syncthreads();
  atomicMax(&s_max, last);
  __syncthreads();
  const int jmax = s_max;
  int wave_last = last;
  for (int o = 32; o > 0; o >>= 1) wave_last = max(wave_last, __shfl_xor(wave_last, o, 64));

  for (int hi = jmax; hi > 0; hi -= NBATCH) {
    const int lo = hi > NBATCH ? hi - NBATCH : 0;
    if (tid < hi - lo) {
      const uint32_t id = ids[start + lo + tid];
      const float4* src = reinterpret_cast<const float4*>(splats + id);
      const float4 A = src[0], Bv = src[1];
      const float l2o = __log2f(Bv.y);
      s_e[tid].a = A;
      s_e[tid].b = make_float4(Bv.x, l2o, Bv.z, Bv.w);
      s_e[tid].c = src[2];  // blue, conic a, b, c
      s_e[tid].inv_o = __builtin_amdgcn_rcpf(Bv.y);
      s_id[tid] = id;
      s_qm[tid] = (uint8_t)quad_mask<TS>(A.x, A.y, A.z, A.w, Bv.x, l2o, l2ia, tile_x * TS,
                                         tile_y * TS);
#pragma unroll
      for (int q = 0; q < 9; ++q) s_g[tid][q] = 0.0f;
    }
    __syncthreads();
    // this wave's records of the batch, highest position first, 64 at a time;
    // the ballot is walked in scalar registers (readfirstlane keeps it there)
    const int nb = min(hi, wave_last) - lo;
    for (int c = (nb - 1) & ~63; c >= 0; c -= 64) {
      const int jj = c + lane;
      const uint64_t bal = __ballot(jj < nb && ((s_qm[jj] >> wave) & 1u));
      const uint32_t blo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)bal);
      const uint32_t bhi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(bal >> 32));
      uint64_t bits = ((uint64_t)bhi << 32) | (uint64_t)blo;
      while (bits != 0) {
        const int top = 63 - __builtin_clzll(bits);
        bits &= ~(1ull << top);
        const int k = c + top;
        blend_grad<MODE>(s_e[k], lo + k < last, fx, fy, leader_lane, lane, amin, amax, g0, g1,
                         g2, T, GS, s_g[k]);
      }
    }
    __syncthreads();
    // one set of global atomics per record and tile
    if (tid < hi - lo) {
      float* dst = grad2d + (int64_t)s_id[tid] * 9;
      float gq[9];
      record_grads(s_e[tid], s_g[tid], gq);
#pragma unroll
      for (int q = 0; q < 9; ++q)
        if (gq[q] != 0.0f) atomicAdd(dst + q, gq[q]);
    }
  }
}

// ---- the same backward over super-tile lists, one workgroup per quadrant
//
// A workgroup takes a 2 x 2-tile quadrant of a super-tile and walks the
// super-tile's depth-ordered entry list backwards, keeping the entries whose
// clipped rectangle covers a tile of the quadrant.  The forward over the same
// lists recorded, per pixel, the list index of the last entry it blended
// (last_entry, 1-based), so a pixel's records are the entries covering its
// tile up to that index: no positions in the per-tile lists are needed, and
// the walk starts at the quadrant's largest index.  Every pixel step is
// pixel_terms', so the gradients equal the per-tile kernel's up to the order
// of the float sums; but every record is flushed to HBM once per quadrant
// instead of once per tile of it.
//
// Two pixels per lane: 8 waves, wave w on the 16 x 8 half w % 2 of quadrant
// tile w / 2, a lane on the same pixel of the half's two 8 x 8 blocks (left
// and right).  A visit runs the pixel step twice and reduces the nine values
// once for 128 pixels; a wave visits a record when either block's bit is set
// (a block whose bit is clear cannot blend it: the cull bound is
// conservative, so its pixels blend nothing).  Measured per 8 x 720p call
// (plain): one pixel per lane in 16 waves 3.01 ms, two in 8 waves 2.78, four
// in 4 waves (a wave per tile, 88 VGPRs) 3.29.
constexpr int kQuadPx = 2;                     // pixels per lane (2: 16 x 8 per wave, 4: 16 x 16)
constexpr int kQuadThreads = 1024 / kQuadPx;
constexpr int kQuadBatch = 256;  // entries scanned per batch (threads 0..255)

// (x0, x1, y0, y1) of an entry's clip cover local tile (lx, ly)?
__device__ __forceinline__ bool clip_covers(uint32_t key, int lx, int ly) {
  const uint32_t c = key >> kClipShift;
  const int x0 = (int)(c & 3u), x1 = (int)((c >> 2) & 3u);
  const int y0 = (int)((c >> 4) & 3u), y1 = (int)((c >> 6) & 3u);
  return x0 <= lx && lx <= x1 && y0 <= ly && ly <= y1;
}

template <int MODE>
__global__ __launch_bounds__(kQuadThreads) __attribute__((amdgpu_waves_per_eu(6)))
void k_raster_bwd_quad(
    RasterViews views, RasterParams rp, const seele_splat* __restrict__ splats,
    const uint32_t* __restrict__ entry_ids, const uint32_t* __restrict__ entry_keys,
    const int32_t* __restrict__ st_ranges, const float* __restrict__ final_T,
    const int32_t* __restrict__ last_entry, const float* __restrict__ dL_dimage,
    float* __restrict__ grad2d) {
  constexpr int NB = kQuadBatch;
  constexpr int SW = NB / 64;  // staging waves
  __shared__ LdsBwd s_e[NB];
  __shared__ uint32_t s_id[NB];
  __shared__ uint32_t s_qm[NB];   // 4 block bits per quadrant tile (bit 4 t + block)
  __shared__ int32_t s_ent[NB];   // list index of the staged entry
  __shared__ float s_g[NB][9];
  __shared__ int s_L[4];          // per quadrant tile: largest last_entry of its pixels
  __shared__ uint32_t s_cnt[SW];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t s = (int64_t)views.v[0].st_base + (blockIdx.x >> 2);
  int v = 0;
  for (int k = 1; k < views.n_views; ++k)
    if (views.v[k].st_base <= s) v = k;
  const RasterView rv = views.v[v];
  const int sgw = (rv.grid_w + kSuperTile - 1) / kSuperTile;
  const int ls = (int)(s - rv.st_base);
  const int sy = ls / sgw, sx = ls - sy * sgw;
  constexpr int PX = kQuadPx;
  const int q = blockIdx.x & 3;
  const int tq = PX == 2 ? wave >> 1 : wave, half = PX == 2 ? wave & 1 : 0;
  const int lxq0 = 2 * (q & 1), lyq0 = 2 * (q >> 1);
  const int lx = lxq0 + (tq & 1), ly = lyq0 + (tq >> 1);
  const int tile_x = sx * kSuperTile + lx, tile_y = sy * kSuperTile + ly;
  const int grid_h = (rv.H + 15) / 16;
  const bool tile_ok = tile_x < rv.grid_w && tile_y < grid_h;
  const int gw = MODE ? rp.group_w : 1, gh = MODE ? rp.group_h : 1;
  const int gsz = gw * gh, gpr = 8 / gw;
  const int grp = lane / gsz, r = lane % gsz;
  const int leader_lane = lane - r;
  const int x0 = tile_x * 16 + (grp % gpr) * gw + r % gw;  // left block; right: + 8
  const int y0 = tile_y * 16 + half * 8 + (grp / gpr) * gh + r / gw;  // top; bottom: + 8
  const int start = st_ranges[2 * s];
  const float amin = rp.alpha_min, l2ia = rp.log2_inv_alpha_min, amax = rp.alpha_max;

  float fx[PX], fy[PX], T[PX], GS[PX], g0[PX], g1[PX], g2[PX];
  int last[PX];  // 1 + list index of the pixel's last blended entry (0: none)
#pragma unroll
  for (int p = 0; p < PX; ++p) {
    const int x = x0 + 8 * (p & 1), y = y0 + 8 * (p >> 1);
    fx[p] = (float)x + 0.5f;
    fy[p] = (float)y + 0.5f;
    T[p] = 1.0f;
    g0[p] = g1[p] = g2[p] = 0.0f;
    last[p] = 0;
    if (tile_ok && x < rv.W && y < rv.H) {
      const int64_t hw = (int64_t)rv.W * rv.H;
      const int64_t pix = (int64_t)y * rv.W + x;
      T[p] = final_T[rv.pix_base + pix];
      last[p] = last_entry[rv.pix_base + pix];
      const float* g = dL_dimage + 3 * rv.pix_base;
      g0[p] = g[pix];
      g1[p] = g[hw + pix];
      g2[p] = g[2 * hw + pix];
    }
    GS[p] = T[p] * __builtin_fmaf(g2[p], rp.bg2, __builtin_fmaf(g1[p], rp.bg1, g0[p] * rp.bg0));
  }
  if (tid < 4) s_L[tid] = 0;
  int wave_last = last[0];
#pragma unroll
  for (int p = 1; p < PX; ++p) wave_last = max(wave_last, last[p]);
  for (int o = 32; o > 0; o >>= 1) wave_last = max(wave_last, __shfl_xor(wave_last, o, 64));
  __syncthreads();
  if (lane == 0 && wave_last > 0) atomicMax(&s_L[tq], wave_last);
  __syncthreads();
  int L[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) L[t] = s_L[t];
  const int top = max(max(L[0], L[1]), max(L[2], L[3])) - 1;

  // this wave's block bits
  const uint32_t bits2 = (PX == 2 ? 3u : 15u) << (4 * tq + 2 * half);
  uint32_t nkey = 0, nid = 0;
  if (wave < SW && top - tid >= 0) {
    nkey = entry_keys[start + top - tid];
    nid = entry_ids[start + top - tid];
  }
  for (int hi = top; hi >= 0; hi -= NB) {
    const int e = hi - tid;
    const uint32_t key = nkey, id = nid;
    uint32_t cb = 0;  // quadrant tiles this entry covers and that need it
    uint32_t slot = 0;
    if (wave < SW) {  // uniform per wave
      if (e - NB >= 0) {
        nkey = entry_keys[start + e - NB];
        nid = entry_ids[start + e - NB];
      }
      if (e >= 0) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (e < L[t] && clip_covers(key, lxq0 + (t & 1), lyq0 + (t >> 1))) cb |= 1u << t;
      }
      const uint64_t nb = __ballot(cb != 0u);
      if (lane == 0) s_cnt[wave] = (uint32_t)__popcll(nb);
      slot = __builtin_amdgcn_mbcnt_hi((uint32_t)(nb >> 32),
                                       __builtin_amdgcn_mbcnt_lo((uint32_t)nb, 0u));
    }
    __syncthreads();
    uint32_t nslots = 0;
#pragma unroll
    for (int k = 0; k < SW; ++k) {
      const uint32_t c = s_cnt[k];
      if (k < wave) slot += c;
      nslots += c;
    }
    if (cb != 0u) {
      const float4* src = reinterpret_cast<const float4*>(splats + id);
      const float4 A = src[0], Bv = src[1];
      const float l2o = __log2f(Bv.y);
      s_e[slot].a = A;
      s_e[slot].b = make_float4(Bv.x, l2o, Bv.z, Bv.w);
      s_e[slot].c = src[2];
      s_e[slot].inv_o = __builtin_amdgcn_rcpf(Bv.y);
      s_id[slot] = id;
      s_ent[slot] = e;
      uint32_t qm = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if ((cb >> t) & 1u) {
          const int tx = sx * kSuperTile + lxq0 + (t & 1), ty = sy * kSuperTile + lyq0 + (t >> 1);
          qm |= quad_mask<16>(A.x, A.y, A.z, A.w, Bv.x, l2o, l2ia, tx * 16, ty * 16) << (4 * t);
        }
      }
      s_qm[slot] = qm;
#pragma unroll
      for (int k = 0; k < 9; ++k) s_g[slot][k] = 0.0f;
    }
    __syncthreads();
    for (int c0 = 0; c0 < (int)nslots; c0 += 64) {
      const int k0 = c0 + lane;
      const bool vis = k0 < (int)nslots && (s_qm[k0] & bits2) != 0u && s_ent[k0] < wave_last;
      const uint64_t bal = __ballot(vis);
      const uint32_t blo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)bal);
      const uint32_t bhi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(bal >> 32));
      uint64_t bits = ((uint64_t)bhi << 32) | (uint64_t)blo;
      while (bits != 0) {
        const int b0 = __builtin_ctzll(bits);
        bits &= bits - 1;
        const int k = c0 + b0;
        const int ent = s_ent[k];
        float vs[9], vp[9];
        bool any = pixel_terms<MODE>(s_e[k], ent < last[0], fx[0], fy[0], leader_lane, amin,
                                     amax, g0[0], g1[0], g2[0], T[0], GS[0], vs);
#pragma unroll
        for (int p = 1; p < PX; ++p) {
          any |= pixel_terms<MODE>(s_e[k], ent < last[p], fx[p], fy[p], leader_lane, amin, amax,
                                   g0[p], g1[p], g2[p], T[p], GS[p], vp);
#pragma unroll
          for (int j = 0; j < 9; ++j) vs[j] += vp[j];
        }
        if (__ballot(any) != 0) wave_accumulate9(vs, s_g[k], lane);
      }
    }
    __syncthreads();
    for (int i = tid; i < 9 * (int)nslots; i += kQuadThreads) {
      const int sl = i / 9, k = i - 9 * sl;
      const float gk = record_grad(s_e[sl], s_g[sl], k);
      if (gk != 0.0f) atomicAdd(grad2d + (int64_t)s_id[sl] * 9 + k, gk);
    }
  }
}

}  // namespace

hipError_t launch_raster_bwd(int tile, int mode, const RasterViews& views, int n_tiles_launch,
                             const RasterParams& rp, const seele_splat* splats,
                             const uint32_t* sorted_ids, const int32_t* tile_ranges,
                             const float* final_T, const int32_t* n_contrib,
                             const float* dL_dimage, float* grad2d, hipStream_t stream) {
  if (n_tiles_launch <= 0) return hipSuccess;
  const dim3 grid(n_tiles_launch);
  if (tile == 16) {
    if (mode == SEELE_RASTER_CONTRIB)
      hipLaunchKernelGGL((k_raster_bwd<16, 1>), grid, dim3(256), 0, stream, views, rp, splats,
                         sorted_ids, tile_ranges, final_T, n_contrib, dL_dimage, grad2d);
    else
      hipLaunchKernelGGL((k_raster_bwd<16, 0>), grid, dim3(256), 0, stream, views, rp, splats,
                         sorted_ids, tile_ranges, final_T, n_contrib, dL_dimage, grad2d);
  } else {
    if (mode == SEELE_RASTER_CONTRIB)
      hipLaunchKernelGGL((k_raster_bwd<8, 1>), grid, dim3(64), 0, stream, views, rp, splats,
                         sorted_ids, tile_ranges, final_T, n_contrib, dL_dimage, grad2d);
    else
      hipLaunchKernelGGL((k_raster_bwd<8, 0>), grid, dim3(64), 0, stream, views, rp, splats,
                         sorted_ids, tile_ranges, final_T, n_contrib, dL_dimage, grad2d);
  }
  return hipGetLastError();
}

hipError_t launch_raster_bwd_quad(int mode, const RasterViews& views, int n_st_launch,
                                  const RasterParams& rp, const seele_splat* splats,
                                  const uint32_t* entry_ids, const uint32_t* entry_keys,
                                  const int32_t* st_ranges, const float* final_T,
                                  const int32_t* last_entry, const float* dL_dimage, float* grad2d,
                                  hipStream_t stream) {
  if (n_st_launch <= 0) return hipSuccess;
  const dim3 grid((unsigned)(4 * n_st_launch));
  if (mode == SEELE_RASTER_CONTRIB)
    hipLaunchKernelGGL(k_raster_bwd_quad<1>, grid, dim3(kQuadThreads), 0, stream, views, rp,
                       splats, entry_ids, entry_keys, st_ranges, final_T, last_entry, dL_dimage,
                       grad2d);
  else
    hipLaunchKernelGGL(k_raster_bwd_quad<0>, grid, dim3(kQuadThreads), 0, stream, views, rp,
                       splats, entry_ids, entry_keys, st_ranges, final_T, last_entry, dL_dimage,
                       grad2d);
  return hipGetLastError();
}

}  // namespace seele
