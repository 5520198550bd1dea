// Front-to-back blending on gfx950: plain (Sec. 3.1, Eqs. 1-2) and
// contribution-aware (Sec. 3.4, Algorithm 1).
//
// One workgroup per (view, tile), one lane per pixel.  Each wave owns an 8x8
// pixel block laid out as pixel groups (2x2 by default): lanes
// [k*g, (k+1)*g) hold group k with its leader (top-left pixel) first.  The
// tile's depth-ordered list is staged through LDS in batches of one record
// per thread; each record carries the Cholesky factor of (log2(e)/2) * conic,
// so that exp(-q/2) = exp2(-(u^2 + w^2)) with two linear forms u, w of the
// pixel offset.
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
// Wave-level culling: when a batch is staged, each record also gets a bit per
// 8x8 wave block that its alpha >= alpha_min region can reach (a conservative
// bound, see quad_mask).  A wave then visits only the records whose bit it
// holds, walking the ballot of those bits with scalar bit scans.  A record a
// wave skips has alpha < alpha_min at every pixel of its block, so no pixel
// (and no group leader) of that block blends it or passes its test: results
// are identical to visiting every record.  The instrumented (COUNT) kernels
// visit every record, as the method states, to count its work.
//
// Early exit: a wave leaves a batch when all its lanes are done; the block
// stops loading batches when all its pixels are done.
#include "seele_internal.h"

namespace seele {

namespace {

struct LdsRec {
  float4 a;  // mean_x, mean_y, l11, l21  (Cholesky factor of k * conic)
  float4 b;  // l22, log2(opacity), r, g
  float blue;
  int entry;  // super-tile lists: the record's index in the list
  float pad1, pad2;
};

__device__ __forceinline__ float alpha_at(float px, float py, const float4& a, const float4& b,
                                          float alpha_max) {
  float dx, dy;
  const float qo = splat_qo(px, py, a.x, a.y, a.z, a.w, b.x, b.y, dx, dy);
  return clamp_alpha(fast_exp2(-qo), alpha_max);
}

// One front-to-back step of Eqs. 1-2 for one pixel, with the alpha skip, the
// clamp and the termination rule.  The blend weight is w = T alpha and the
// next transmittance T - w (= T (1 - alpha)).  A pixel's state is (T,
// colour, last); a pixel that has stopped carries -T (T >= T_min > 0 while it
// runs): its T - w stays negative, so every later step leaves it unchanged
// without a separate flag.  True if blended.
__device__ __forceinline__ bool blend_step(float fx, float fy, const float4& a, const float4& b,
                                           float blue, int pos, float amin, float amax,
                                           float tmin, float& T, float& c0, float& c1, float& c2,
                                           int& last, float* w_out = nullptr) {
  const float alpha = alpha_at(fx, fy, a, b, amax);
  const bool pass = alpha >= amin;
  const float wgt = T * alpha;
  const float Tn = T - wgt;
  const bool keep = Tn >= tmin;
  const bool take = pass && keep;
  if (w_out) *w_out = take ? wgt : 0.0f;  // the blend weight T alpha (0 if not blended)
  if (take) {
    c0 = __builtin_fmaf(wgt, b.z, c0);
    c1 = __builtin_fmaf(wgt, b.w, c1);
    c2 = __builtin_fmaf(wgt, blue, c2);
    last = pos;
  }
  const float Tk = keep ? Tn : -__builtin_fabsf(T);
  T = pass ? Tk : T;
  return take;
}

// The same step without branches (selects only), for the production loops:
// a step that does not blend adds 0 * colour (colours are finite and >= 0,
// the sums start at +0), so it writes the same bits as blend_step.  acc =
// false (a group whose leader did not accept the Gaussian) leaves the pixel
// unchanged, as if blend_step were not called.
__device__ __forceinline__ void blend_select(float fx, float fy, const float4& a, const float4& b,
                                             float blue, int pos, float amin, float amax,
                                             float tmin, float& T, float& c0, float& c1,
                                             float& c2, int& last, bool acc = true) {
  const float alpha = alpha_at(fx, fy, a, b, amax);
  const bool pass = acc && alpha >= amin;
  const float w = T * alpha;
  const float Tn = T - w;
  const bool keep = Tn >= tmin;
  const bool take = pass && keep;
  const float wgt = take ? w : 0.0f;
  c0 = __builtin_fmaf(wgt, b.z, c0);
  c1 = __builtin_fmaf(wgt, b.w, c1);
  c2 = __builtin_fmaf(wgt, blue, c2);
  last = take ? pos : last;
  const float Tk = keep ? Tn : -__builtin_fabsf(T);
  T = pass ? Tk : T;
}

// COUNT instantiations also accumulate the method's work counters:
// [0] alpha evaluations by pixels that have not stopped (contribution-aware:
// only in groups whose leader accepted), [1] blends, [2] leader tests of
// groups holding a live pixel, [3] of those, acceptances; and the work left
// to the culled kernels: [4] evaluations of [0] on records whose block bit is
// set, [5] (wave, record) visits with the bit set while the wave has a live
// pixel.
// The tile list is consumed in LDS batches of BATCH records (<= TS*TS: threads
// tid < BATCH stage one record each); BATCH trades barrier and early-exit
// granularity against LDS latency and is chosen by the autotuner.
//
// SUPER: the tile reads its super-tile's depth-ordered entry list instead of
// a list of its own (ids = entry record ids, ekeys = entry keys, ranges =
// super-tile ranges).  Each staging thread takes two entries per batch; the
// entries whose clipped rectangle covers the tile are compacted, in list
// order, into the batch (so a batch holds up to 2 * BATCH records), and the
// running count of covered entries gives each record's position in the
// tile's own list.  Everything after staging is shared, so the outputs are
// bit-identical to the per-tile lists'.  With last_entry, each pixel also
// gets 1 + the super-list index of its last blended entry: the staged
// records carry their list index, and once per batch a pixel whose last
// blend fell in the batch reads it from its record's slot.
template <int TS, int MODE, bool COUNT, int BATCH, bool SUPER = false>
__device__ __forceinline__ void raster_tile(const int gt, const RasterViews& views,
                                            const RasterParams& rp,
                                            const seele_splat* __restrict__ splats,
                                            const uint32_t* __restrict__ ids,
                                            const uint32_t* __restrict__ ekeys,
                                            const int32_t* __restrict__ ranges,
                                            float* __restrict__ image,
                                            float* __restrict__ final_T,
                                            int32_t* __restrict__ n_contrib,
                                            unsigned long long* __restrict__ counters,
                                            int32_t* __restrict__ last_entry = nullptr) {
  constexpr int NT = TS * TS;
  constexpr int NW = NT / 64;
  static_assert((BATCH <= NT && BATCH % 64 == 0) || BATCH == NT, "batch depth");
  constexpr int CAP = SUPER ? 2 * BATCH : BATCH;  // records per LDS batch
  constexpr int E = CAP;                          // list entries per batch
  constexpr int SW = BATCH / 64;                  // staging waves
  __shared__ LdsRec s_rec[CAP];
  __shared__ uint8_t s_qm[CAP];
  // s_need[c][w]: bit i set if record 64 c + i of the batch can reach wave
  // w's block (the ballots of the s_qm bits, taken once at staging)
  __shared__ uint64_t s_need[CAP / 64][NW];
  __shared__ uint32_t s_dead[NW];
  __shared__ uint8_t s_list[NW][64];
  __shared__ uint32_t s_wc[2][SW];
  __shared__ unsigned long long s_cnt[6];
  uint32_t c_eval = 0, c_blend = 0, c_ltest = 0, c_lpass = 0, c_need = 0, c_visit = 0;
  if (COUNT) {
    if (threadIdx.x < 6) s_cnt[threadIdx.x] = 0;
  }

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

  int start, n;
  // SUPER: an entry covers this tile iff its clip's x nibble (x0 | x1 << 2)
  // has x0 <= lx <= x1 and its y nibble likewise; mx / my hold, per nibble
  // value, whether it does (one bit each).
  uint32_t mx = 0, my = 0;
  if (SUPER) {
    const int sgw = (rv.grid_w + kSuperTile - 1) / kSuperTile;
    const int64_t s = (int64_t)rv.st_base + (tile_y / kSuperTile) * sgw + tile_x / kSuperTile;
    start = ranges[2 * s];
    n = ranges[2 * s + 1] - start;
    const int lx = tile_x % kSuperTile, ly = tile_y % kSuperTile;
#pragma unroll
    for (int v0 = 0; v0 < 16; ++v0) {
      const int lo = v0 & 3, hi = v0 >> 2;
      if (lo <= lx && lx <= hi) mx |= 1u << v0;
      if (lo <= ly && ly <= hi) my |= 1u << v0;
    }
  } else {
    const int64_t ri = 2 * ((int64_t)views.tile_base + gt);
    start = ranges[ri];
    n = ranges[ri + 1] - start;
  }
  const float amin = rp.alpha_min, l2ia = rp.log2_inv_alpha_min;
  const float amax = rp.alpha_max, tmin = rp.T_min;

  // pixels outside the image start stopped
  float T = inside ? 1.0f : -1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
  int last = 0;
  int last_e = 0;  // SUPER with last_entry: 1 + list index of the last blend
  const bool want_e = SUPER && last_entry != nullptr;  // uniform

  // Staging loads are software-pipelined: while a batch is blended, each
  // staging thread already has the next batch's record and the id of the
  // batch after in flight.  Once three quarters of the tile's pixels have
  // stopped, the tile is likely to end within the batch, so the look-ahead
  // stops (ahead = false) and a batch that is still needed loads its records
  // when it starts (pid then holds the current batch's id).
  const bool stager = tid < BATCH;
  bool ahead = true;  // uniform over the block
  float4 pa = make_float4(0.0f, 0.0f, 0.0f, 0.0f), pb = pa;
  float pblue = 0.0f;
  uint32_t pid = 0;
  // SUPER state of the thread's two entries r = 0, 1 (entries base + r*BATCH
  // + tid): covered flag and record of the batch to stage; key and id of the
  // next batch (of the current one while ahead is false).
  bool cv0 = false, cv1 = false;
  float4 qa1 = pa, qb1 = pa;
  float ql1 = 0.0f;
  uint32_t nk0 = 0, nk1 = 0, ni1 = 0;
  int run = 0;  // SUPER: covered entries before the batch (block-uniform)
  auto covers = [&](uint32_t key) {
    return ((mx >> ((key >> kClipShift) & 15u)) & (my >> (key >> (kClipShift + 4))) & 1u) != 0u;
  };
  auto load_rec = [&](uint32_t id, float4& a, float4& b, float& bl) {
    const float4* src = reinterpret_cast<const float4*>(splats + id);
    a = src[0];
    b = src[1];
    bl = src[2].x;
  };
  // staged form of a record's second quarter: opacity as log2(o)
  auto staged_b = [](const float4& b) { return make_float4(b.x, __log2f(b.y), b.z, b.w); };
  // SUPER: make (cv, q) the batch of entries j0, j0 + BATCH from (nk, ni),
  // then load the keys and ids of the batch after into (nk, ni)
  auto super_step = [&](int j0) {
    const int j1 = j0 + BATCH;
    cv0 = j0 < n && covers(nk0);
    cv1 = j1 < n && covers(nk1);
    if (cv0) load_rec(pid, pa, pb, pblue);
    if (cv1) load_rec(ni1, qa1, qb1, ql1);
    if (j0 + E < n) {
      nk0 = ekeys[start + j0 + E];
      pid = ids[start + j0 + E];
    }
    if (j1 + E < n) {
      nk1 = ekeys[start + j1 + E];
      ni1 = ids[start + j1 + E];
    }
  };
  if (SUPER) {
    if (stager && tid < n) {
      nk0 = ekeys[start + tid];
      pid = ids[start + tid];
    }
    if (stager && BATCH + tid < n) {
      nk1 = ekeys[start + BATCH + tid];
      ni1 = ids[start + BATCH + tid];
    }
    if (stager) super_step(tid);
  } else {
    if (stager && tid < n) load_rec(ids[start + tid], pa, pb, pblue);
    if (stager && BATCH + tid < n) pid = ids[start + BATCH + tid];
  }

  for (int base = 0; base < n; base += E) {
    // pixels stopped so far: per-wave ballot counts through LDS
    {
      const uint64_t dead = __ballot(T < 0.0f);
      if (lane == 0) s_dead[wave] = (uint32_t)__popcll(dead);
    }
    __syncthreads();
    int stopped = 0;
#pragma unroll
    for (int w2 = 0; w2 < NW; ++w2) stopped += (int)s_dead[w2];
    if (stopped == NT) break;
    const int j = base + tid;
    int cnt;
    if (SUPER) {
      if (!ahead && stager) super_step(j);
      const uint64_t b0 = __ballot(cv0), b1 = __ballot(cv1);
      if (stager && lane == 0) {
        s_wc[0][wave] = (uint32_t)__popcll(b0);
        s_wc[1][wave] = (uint32_t)__popcll(b1);
      }
      __syncthreads();
      uint32_t off0 = 0, off1 = 0, tot0 = 0, tot1 = 0;
#pragma unroll
      for (int w2 = 0; w2 < SW; ++w2) {
        const uint32_t c0w = s_wc[0][w2], c1w = s_wc[1][w2];
        if (w2 < wave) {
          off0 += c0w;
          off1 += c1w;
        }
        tot0 += c0w;
        tot1 += c1w;
      }
      cnt = (int)(tot0 + tot1);
      const uint32_t r0 = __builtin_amdgcn_mbcnt_hi((uint32_t)(b0 >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)b0, 0u));
      const uint32_t r1 = __builtin_amdgcn_mbcnt_hi((uint32_t)(b1 >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)b1, 0u));
      if (cv0) {
        const uint32_t sl = off0 + r0;
        s_rec[sl].a = pa;
        s_rec[sl].b = staged_b(pb);
        s_rec[sl].blue = pblue;
        if (want_e) s_rec[sl].entry = j;
      }
      if (cv1) {
        const uint32_t sl = tot0 + off1 + r1;
        s_rec[sl].a = qa1;
        s_rec[sl].b = staged_b(qb1);
        s_rec[sl].blue = ql1;
        if (want_e) s_rec[sl].entry = j + BATCH;
      }
      __syncthreads();
      // culling masks over the compacted records, one per thread, so that
      // every lane of a wave has a record to bound
      for (int k0 = 0; k0 < cnt; k0 += NT) {
        const int k = k0 + tid;
        uint32_t qm = 0;
        if (k < cnt) {
          const float4 a = s_rec[k].a;
          const float4 b = s_rec[k].b;
          qm = quad_mask<TS>(a.x, a.y, a.z, a.w, b.x, b.y, l2ia, tile_x * TS, tile_y * TS);
          s_qm[k] = (uint8_t)qm;
        }
        if (k0 + 64 * wave < cnt) {  // uniform per wave
#pragma unroll
          for (int q = 0; q < NW; ++q) {
            const uint64_t bq = __ballot((qm >> q) & 1u);
            if (lane == 0) s_need[(k0 >> 6) + wave][q] = bq;
          }
        }
      }
      __syncthreads();
      ahead = 4 * stopped < 3 * NT;
      if (ahead && stager) super_step(j + E);
    } else {
      if (!ahead) {
        if (stager && j < n) {
          const float4* src = reinterpret_cast<const float4*>(splats + pid);
          pa = src[0];
          pb = src[1];
          pblue = src[2].x;
        }
        if (stager && j + BATCH < n) pid = ids[start + j + BATCH];
      }
      uint32_t qm = 0;
      if (stager && j < n) {
        const float4 sb = staged_b(pb);
        s_rec[tid].a = pa;
        s_rec[tid].b = sb;
        s_rec[tid].blue = pblue;
        qm = quad_mask<TS>(pa.x, pa.y, pa.z, pa.w, sb.x, sb.y, l2ia, tile_x * TS, tile_y * TS);
        s_qm[tid] = (uint8_t)qm;
      }
      if (stager) {  // uniform per wave (BATCH is a multiple of 64)
#pragma unroll
        for (int q = 0; q < NW; ++q) {
          const uint64_t bq = __ballot((qm >> q) & 1u);
          if (lane == 0) s_need[wave][q] = bq;
        }
      }
      __syncthreads();
      ahead = 4 * stopped < 3 * NT;
      if (ahead && stager && j + BATCH < n) {
        const float4* src = reinterpret_cast<const float4*>(splats + pid);
        pa = src[0];
        pb = src[1];
        pblue = src[2].x;
        if (j + 2 * BATCH < n) pid = ids[start + j + 2 * BATCH];
      }
      cnt = min(BATCH, n - base);
    }
    const int lbase = SUPER ? run : base;  // list position of the batch's first record
    if (COUNT && MODE == 0) {
      for (int k = 0; k < cnt; ++k) {
        if (__ballot(T >= 0.0f) == 0) break;
        const bool bit = (s_qm[k] >> wave) & 1u;
        if (bit && lane == 0) ++c_visit;
        if (T >= 0.0f) {
          ++c_eval;
          if (bit) ++c_need;
          if (blend_step(fx, fy, s_rec[k].a, s_rec[k].b, s_rec[k].blue, lbase + k + 1, amin,
                         amax, tmin, T, c0, c1, c2, last))
            ++c_blend;
        }
      }
    } else if (COUNT) {
      const int per = 64 / G;
      const uint64_t gl = gsz >= 64 ? ~0ull : ((1ull << gsz) - 1ull);
      for (int k0 = 0; k0 < cnt; k0 += per) {
        if (__ballot(T >= 0.0f) == 0) break;
        const int kk = k0 + sub;
        bool pass = false;
        if (kk < cnt) pass = alpha_at(lfx, lfy, s_rec[kk].a, s_rec[kk].b, amax) >= amin;
        const uint64_t bal = __ballot(pass);
        for (int s = 0; s < per && k0 + s < cnt; ++s) {
          const uint64_t gm = (bal >> (s * G)) & gmask;
          const uint64_t live = __ballot(T >= 0.0f);  // all lanes take part in the ballot
          uint64_t glive = 0;
          for (int q = 0; q < G; ++q)
            if ((live >> (q * gsz)) & gl) glive |= 1ull << q;
          if (lane == 0) {
            c_ltest += (uint32_t)__popcll(glive);
            c_lpass += (uint32_t)__popcll(glive & gm);
            if (live != 0 && ((s_qm[k0 + s] >> wave) & 1u)) ++c_visit;
          }
          if (gm == 0) continue;
          if (T >= 0.0f && ((gm >> grp) & 1ull)) {
            const int k = k0 + s;
            ++c_eval;
            ++c_need;
            if (blend_step(fx, fy, s_rec[k].a, s_rec[k].b, s_rec[k].blue, lbase + k + 1, amin,
                           amax, tmin, T, c0, c1, c2, last))
              ++c_blend;
          }
        }
      }
    } else {
      for (int c = 0; c < cnt; c += 64) {
        if (__ballot(T >= 0.0f) == 0) break;
        const uint64_t nb = s_need[c >> 6][wave];
        // (readfirstlane returns int: widen through uint32_t, not by sign)
        const uint32_t nlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)nb);
        const uint32_t nhi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(nb >> 32));
        uint64_t bits = ((uint64_t)nhi << 32) | (uint64_t)nlo;
        if (bits == 0) continue;
        const bool need = (bits >> lane) & 1ull;
        if (MODE == 0) {
          // Walk the wave-uniform ballot in depth order with scalar
          // find-first-set, two records at a time: the next record's LDS
          // reads are in flight while the current one is blended.  (When the
          // ballot runs out, the record read ahead is a repeat of the last
          // one and is not blended.)
          int ka = c + __builtin_ctzll(bits);
          bits &= bits - 1;
          float4 aa = s_rec[ka].a, ab = s_rec[ka].b;
          float abl = s_rec[ka].blue;
          for (;;) {
            const int kb = bits ? c + __builtin_ctzll(bits) : ka;
            const float4 ba = s_rec[kb].a, bb = s_rec[kb].b;
            const float bbl = s_rec[kb].blue;
            blend_select(fx, fy, aa, ab, abl, lbase + ka + 1, amin, amax, tmin, T, c0, c1, c2, last);
            if (bits == 0) break;
            bits &= bits - 1;
            ka = bits ? c + __builtin_ctzll(bits) : kb;
            aa = s_rec[ka].a;
            ab = s_rec[ka].b;
            abl = s_rec[ka].blue;
            blend_select(fx, fy, ba, bb, bbl, lbase + kb + 1, amin, amax, tmin, T, c0, c1, c2, last);
            if (bits == 0) break;
            bits &= bits - 1;
          }
        } else {
          // compact this wave's records of the chunk, then run the packed
          // leader test on per = 64/G of them at a time
          const int nsel = __popcll(bits);
          const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bits >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)bits, 0u));
          if (need) s_list[wave][rank] = (uint8_t)lane;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const int per = 64 / G;
          for (int i = 0; i < nsel; i += per) {
            const int li = i + sub;
            const int kk = li < nsel ? c + (int)s_list[wave][li] : 0;
            const bool pass =
                li < nsel && alpha_at(lfx, lfy, s_rec[kk].a, s_rec[kk].b, amax) >= amin;
            const uint64_t bal = __ballot(pass);
            const int ns = min(per, nsel - i);
            for (int s = 0; s < ns; ++s) {
              const uint64_t gm = (bal >> (s * G)) & gmask;
              if (gm == 0) continue;  // no leader of this wave accepts it: wave-uniform skip
              const int k = __builtin_amdgcn_readlane(kk, s * G);
              blend_select(fx, fy, s_rec[k].a, s_rec[k].b, s_rec[k].blue, lbase + k + 1, amin,
                           amax, tmin, T, c0, c1, c2, last, ((gm >> grp) & 1ull) != 0);
            }
            if (__ballot(T >= 0.0f) == 0) break;
          }
          __builtin_amdgcn_wave_barrier();  // list reads finish before the next chunk's writes
        }
      }
    }
    if (SUPER) {
      // the batch's records are still staged (the next batch writes them
      // after the barrier below)
      if (want_e && last > run) last_e = s_rec[last - run - 1].entry + 1;
      run += cnt;
    }
    __syncthreads();
  }

  if (COUNT) {
    __syncthreads();
    atomicAdd(&s_cnt[0], (unsigned long long)c_eval);
    atomicAdd(&s_cnt[1], (unsigned long long)c_blend);
    atomicAdd(&s_cnt[2], (unsigned long long)c_ltest);
    atomicAdd(&s_cnt[3], (unsigned long long)c_lpass);
    atomicAdd(&s_cnt[4], (unsigned long long)c_need);
    atomicAdd(&s_cnt[5], (unsigned long long)c_visit);
    __syncthreads();
    if (threadIdx.x < 6) atomicAdd(&counters[threadIdx.x], s_cnt[threadIdx.x]);
  }

  if (inside) {
    const float Tf = __builtin_fabsf(T);
    const int64_t hw = (int64_t)rv.W * rv.H;
    const int64_t pix = (int64_t)y * rv.W + x;
    float* img = image + 3 * rv.pix_base;
    img[pix] = c0 + Tf * rp.bg0;
    img[hw + pix] = c1 + Tf * rp.bg1;
    img[2 * hw + pix] = c2 + Tf * rp.bg2;
    final_T[rv.pix_base + pix] = Tf;
    n_contrib[rv.pix_base + pix] = last;
    if (want_e) last_entry[rv.pix_base + pix] = last_e;
  }
}

template <int TS, int MODE, bool COUNT, int BATCH>
__global__ __launch_bounds__(TS* TS) void k_raster_fwd(RasterViews views, RasterParams rp,
                                                       const seele_splat* __restrict__ splats,
                                                       const uint32_t* __restrict__ ids,
                                                       const int32_t* __restrict__ ranges,
                                                       float* __restrict__ image,
                                                       float* __restrict__ final_T,
                                                       int32_t* __restrict__ n_contrib,
                                                       unsigned long long* __restrict__ counters) {
  raster_tile<TS, MODE, COUNT, BATCH>(blockIdx.x, views, rp, splats, ids, nullptr, ranges, image,
                                      final_T, n_contrib, counters);
}

// One workgroup per (view, tile) reading the tile's super-tile list.
template <int TS, int MODE, bool COUNT, int BATCH>
__global__ __launch_bounds__(TS* TS) void k_raster_fwd_super(
    RasterViews views, RasterParams rp, const seele_splat* __restrict__ splats,
    const uint32_t* __restrict__ entry_ids, const uint32_t* __restrict__ entry_keys,
    const int32_t* __restrict__ st_ranges, float* __restrict__ image, float* __restrict__ final_T,
    int32_t* __restrict__ n_contrib, unsigned long long* __restrict__ counters,
    int32_t* __restrict__ last_entry) {
  raster_tile<TS, MODE, COUNT, BATCH, true>(blockIdx.x, views, rp, splats, entry_ids, entry_keys,
                                            st_ranges, image, final_T, n_contrib, counters,
                                            last_entry);
}

// Persistent form for batches of views: a fixed grid of workgroups pulls
// (view, tile) items from a device counter until the queue is empty, in list
// order or in the order given by `order` (heaviest tile lists first, so the
// longest items start early and the tail stays short).  Every workgroup exits
// once the counter passes the item count.
template <int TS, int MODE, int BATCH>
__global__ __launch_bounds__(TS* TS) void k_raster_fwd_queue(
    RasterViews views, RasterParams rp, const seele_splat* __restrict__ splats,
    const uint32_t* __restrict__ ids, const int32_t* __restrict__ ranges,
    float* __restrict__ image, float* __restrict__ final_T, int32_t* __restrict__ n_contrib,
    uint32_t* __restrict__ counter, const uint32_t* __restrict__ order, uint32_t n_items) {
  __shared__ uint32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t item = s_item;
    __syncthreads();
    if (item >= n_items) break;
    const int t = (int)(order ? order[item] : item);
    raster_tile<TS, MODE, false, BATCH>(t, views, rp, splats, ids, nullptr, ranges, image,
                                        final_T, n_contrib, nullptr);
  }
}

// Offline contribution pass (Sec. 3.3 "Offline Clustering"): the plain blend
// of every pixel, exactly as the forward computes it (blend_step), keeping
// the pixel's K largest contributions T alpha with their record ids in
// registers; a larger contribution wins, equal ones go to the lower record
// id.  At the end every pixel marks its top records; every blend also adds
// its T alpha to the record's sum (one atomic per record and wave, after a
// wave reduction).  One workgroup per (view, tile), one lane per pixel, the
// tile list staged through LDS one record per thread.
template <int TS, int K>
__global__ __launch_bounds__(TS* TS) void k_contrib_topk(RasterViews views, RasterParams rp,
                                                         const seele_splat* __restrict__ splats,
                                                         const uint32_t* __restrict__ ids,
                                                         const int32_t* __restrict__ ranges,
                                                         int k_top, uint8_t* __restrict__ mark,
                                                         float* __restrict__ contrib_sum) {
  constexpr int NT = TS * TS;
  __shared__ LdsRec s_rec[NT];
  __shared__ uint32_t s_id[NT];
  const int gt = blockIdx.x;
  int v = 0;
  for (int q = 1; q < views.n_views; ++q)
    if (views.v[q].tile_begin <= gt) v = q;
  const RasterView rv = views.v[v];
  const int lt = gt - rv.tile_begin;
  const int tile_x = lt % rv.grid_w, tile_y = lt / rv.grid_w;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wx = (TS == 16) ? (wave & 1) * 8 : 0, wy = (TS == 16) ? (wave >> 1) * 8 : 0;
  const int x = tile_x * TS + wx + (lane & 7), y = tile_y * TS + wy + (lane >> 3);
  const bool inside = x < rv.W && y < rv.H;
  const float fx = (float)x + 0.5f, fy = (float)y + 0.5f;
  const int64_t ri = 2 * ((int64_t)views.tile_base + gt);
  const int start = ranges[ri], n = ranges[ri + 1] - start;
  const float amin = rp.alpha_min, amax = rp.alpha_max, tmin = rp.T_min;

  float T = inside ? 1.0f : -1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
  int last = 0;
  float tw[K];
  uint32_t tr[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    tw[j] = -1.0f;  // empty slot: below every contribution
    tr[j] = 0xffffffffu;
  }
  for (int base = 0; base < n; base += NT) {
    if (__syncthreads_count(T < 0.0f) == NT) break;
    if (tid < n - base) {
      const uint32_t id = ids[start + base + tid];
      const float4* src = reinterpret_cast<const float4*>(splats + id);
      const float4 b = src[1];
      s_rec[tid].a = src[0];
      s_rec[tid].b = make_float4(b.x, __log2f(b.y), b.z, b.w);
      s_rec[tid].blue = src[2].x;
      s_id[tid] = id;
    }
    __syncthreads();
    const int cnt = min(NT, n - base);
    for (int q = 0; q < cnt; ++q) {
      if (__ballot(T >= 0.0f) == 0) break;
      float w;
      const bool took = blend_step(fx, fy, s_rec[q].a, s_rec[q].b, s_rec[q].blue, base + q + 1,
                                   amin, amax, tmin, T, c0, c1, c2, last, &w);
      const uint32_t rid = s_id[q];
      if (took) {
        // replace the worst kept entry (smallest weight, then largest id) if w beats it
        int wj = 0;
#pragma unroll
        for (int j = 1; j < K; ++j) {
          const bool worse = tw[j] < tw[wj] || (tw[j] == tw[wj] && tr[j] > tr[wj]);
          wj = (j < k_top && worse) ? j : wj;
        }
        float ww = 0.0f;
        uint32_t wr = 0u;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          ww = j == wj ? tw[j] : ww;
          wr = j == wj ? tr[j] : wr;
        }
        if (w > ww || (w == ww && rid < wr)) {
#pragma unroll
          for (int j = 0; j < K; ++j) {
            tw[j] = j == wj ? w : tw[j];
            tr[j] = j == wj ? rid : tr[j];
          }
        }
      }
      const float ws = wave_sum(w);
      if (lane == 0 && ws != 0.0f) atomicAdd(contrib_sum + rid, ws);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (j < k_top && tr[j] != 0xffffffffu) mark[tr[j]] = 1;
}

// Sort keys for heaviest-first scheduling: ~(list length) so an ascending
// stable sort puts long lists first (ties in tile order).
__global__ void k_tile_len_keys(const int32_t* __restrict__ ranges, int32_t tile_base,
                                uint32_t n, uint32_t* __restrict__ keys,
                                uint32_t* __restrict__ vals, uint32_t* __restrict__ counter) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *counter = 0u;
  if (i >= n) return;
  const int64_t r = 2 * ((int64_t)tile_base + i);
  keys[i] = ~(uint32_t)(ranges[r + 1] - ranges[r]);
  vals[i] = i;
}

__global__ void k_zero_counter(uint32_t* counter) {
  if (threadIdx.x == 0) *counter = 0u;
}

template <int TS, int BATCH>
void launch_fwd(int mode, bool count, dim3 grid, const RasterViews& views, const RasterParams& rp,
                const seele_splat* splats, const uint32_t* ids, const int32_t* ranges,
                float* image, float* final_T, int32_t* n_contrib, unsigned long long* counters,
                hipStream_t stream) {
  const dim3 block(TS * TS);
  if (mode == SEELE_RASTER_CONTRIB) {
    if (count)
      hipLaunchKernelGGL((k_raster_fwd<TS, 1, true, BATCH>), grid, block, 0, stream, views, rp,
                         splats, ids, ranges, image, final_T, n_contrib, counters);
    else
      hipLaunchKernelGGL((k_raster_fwd<TS, 1, false, BATCH>), grid, block, 0, stream, views, rp,
                         splats, ids, ranges, image, final_T, n_contrib, counters);
  } else {
    if (count)
      hipLaunchKernelGGL((k_raster_fwd<TS, 0, true, BATCH>), grid, block, 0, stream, views, rp,
                         splats, ids, ranges, image, final_T, n_contrib, counters);
    else
      hipLaunchKernelGGL((k_raster_fwd<TS, 0, false, BATCH>), grid, block, 0, stream, views, rp,
                         splats, ids, ranges, image, final_T, n_contrib, counters);
  }
}

template <int TS, int BATCH>
void launch_queue(int mode, dim3 grid, const RasterViews& views, const RasterParams& rp,
                  const seele_splat* splats, const uint32_t* ids, const int32_t* ranges,
                  float* image, float* final_T, int32_t* n_contrib, uint32_t* counter,
                  const uint32_t* order, uint32_t n_items, hipStream_t stream) {
  const dim3 block(TS * TS);
  if (mode == SEELE_RASTER_CONTRIB)
    hipLaunchKernelGGL((k_raster_fwd_queue<TS, 1, BATCH>), grid, block, 0, stream, views, rp,
                       splats, ids, ranges, image, final_T, n_contrib, counter, order, n_items);
  else
    hipLaunchKernelGGL((k_raster_fwd_queue<TS, 0, BATCH>), grid, block, 0, stream, views, rp,
                       splats, ids, ranges, image, final_T, n_contrib, counter, order, n_items);
}

template <int TS>
void launch_super(int mode, bool count, dim3 grid, const RasterViews& views,
                  const RasterParams& rp, const seele_splat* splats, const uint32_t* entry_keys,
                  const uint32_t* entry_ids, const int32_t* st_ranges, float* image,
                  float* final_T, int32_t* n_contrib, unsigned long long* counters,
                  int32_t* last_entry, hipStream_t stream) {
  constexpr int BT = TS * TS;
  const dim3 block(BT);
#define SEELE_SUPER(M, C)                                                                       \
  hipLaunchKernelGGL((k_raster_fwd_super<TS, M, C, BT>), grid, block, 0, stream, views, rp,     \
                     splats, entry_ids, entry_keys, st_ranges, image, final_T, n_contrib,       \
                     counters, last_entry)
  if (mode == SEELE_RASTER_CONTRIB) {
    if (count) SEELE_SUPER(1, true);
    else SEELE_SUPER(1, false);
  } else {
    if (count) SEELE_SUPER(0, true);
    else SEELE_SUPER(0, false);
  }
#undef SEELE_SUPER
}

}  // namespace

hipError_t launch_raster_fwd_super(int tile, int mode, const RasterViews& views,
                                   int n_tiles_launch, const RasterParams& rp,
                                   const seele_splat* splats, const uint32_t* entry_keys,
                                   const uint32_t* entry_ids, const int32_t* st_ranges,
                                   float* image, float* final_T, int32_t* n_contrib,
                                   unsigned long long* counters, int32_t* last_entry,
                                   hipStream_t stream) {
  if (n_tiles_launch <= 0) return hipSuccess;
  const dim3 grid(n_tiles_launch);
  if (tile == 16)
    launch_super<16>(mode, counters != nullptr, grid, views, rp, splats, entry_keys, entry_ids,
                     st_ranges, image, final_T, n_contrib, counters, last_entry, stream);
  else
    launch_super<8>(mode, counters != nullptr, grid, views, rp, splats, entry_keys, entry_ids,
                    st_ranges, image, final_T, n_contrib, counters, last_entry, stream);
  return hipGetLastError();
}

hipError_t launch_contrib_topk(int tile, const RasterViews& views, int n_tiles_launch,
                               const RasterParams& rp, const seele_splat* splats,
                               const uint32_t* sorted_ids, const int32_t* tile_ranges, int k_top,
                               uint8_t* mark, float* contrib_sum, hipStream_t stream) {
  if (n_tiles_launch <= 0) return hipSuccess;
  const dim3 grid(n_tiles_launch);
  if (tile == 16)
    hipLaunchKernelGGL((k_contrib_topk<16, 32>), grid, dim3(256), 0, stream, views, rp, splats,
                       sorted_ids, tile_ranges, k_top, mark, contrib_sum);
  else
    hipLaunchKernelGGL((k_contrib_topk<8, 32>), grid, dim3(64), 0, stream, views, rp, splats,
                       sorted_ids, tile_ranges, k_top, mark, contrib_sum);
  return hipGetLastError();
}

// Batch depths offered per tile size (the default is one record per thread).
bool raster_batch_supported(int tile, int batch) {
  if (tile == 16) return batch == 64 || batch == 128 || batch == 256;
  return batch == 64;
}

hipError_t launch_raster_fwd(int tile, int mode, int batch, const RasterViews& views,
                             int n_tiles_launch, const RasterParams& rp,
                             const seele_splat* splats, const uint32_t* sorted_ids,
                             const int32_t* tile_ranges, float* image, float* final_T,
                             int32_t* n_contrib, unsigned long long* counters,
                             hipStream_t stream) {
  if (n_tiles_launch <= 0) return hipSuccess;
  const dim3 grid(n_tiles_launch);
  const bool cnt = counters != nullptr;
  if (tile == 16) {
    if (batch == 64)
      launch_fwd<16, 64>(mode, cnt, grid, views, rp, splats, sorted_ids, tile_ranges, image,
                         final_T, n_contrib, counters, stream);
    else if (batch == 128)
      launch_fwd<16, 128>(mode, cnt, grid, views, rp, splats, sorted_ids, tile_ranges, image,
                          final_T, n_contrib, counters, stream);
    else
      launch_fwd<16, 256>(mode, cnt, grid, views, rp, splats, sorted_ids, tile_ranges, image,
                          final_T, n_contrib, counters, stream);
  } else {
    launch_fwd<8, 64>(mode, cnt, grid, views, rp, splats, sorted_ids, tile_ranges, image,
                      final_T, n_contrib, counters, stream);
  }
  return hipGetLastError();
}

hipError_t launch_raster_fwd_queue(int tile, int mode, int batch, const RasterViews& views,
                                   int n_tiles_launch, const RasterParams& rp,
                                   const seele_splat* splats, const uint32_t* sorted_ids,
                                   const int32_t* tile_ranges, float* image, float* final_T,
                                   int32_t* n_contrib, uint32_t* counter, const uint32_t* order,
                                   int n_workgroups, hipStream_t stream) {
  if (n_tiles_launch <= 0) return hipSuccess;
  const dim3 grid(std::min(n_workgroups, n_tiles_launch));
  const uint32_t items = (uint32_t)n_tiles_launch;
  if (tile == 16) {
    if (batch == 64)
      launch_queue<16, 64>(mode, grid, views, rp, splats, sorted_ids, tile_ranges, image, final_T,
                           n_contrib, counter, order, items, stream);
    else if (batch == 128)
      launch_queue<16, 128>(mode, grid, views, rp, splats, sorted_ids, tile_ranges, image,
                            final_T, n_contrib, counter, order, items, stream);
    else
      launch_queue<16, 256>(mode, grid, views, rp, splats, sorted_ids, tile_ranges, image,
                            final_T, n_contrib, counter, order, items, stream);
  } else {
    launch_queue<8, 64>(mode, grid, views, rp, splats, sorted_ids, tile_ranges, image, final_T,
                        n_contrib, counter, order, items, stream);
  }
  return hipGetLastError();
}

hipError_t launch_tile_order_keys(const int32_t* tile_ranges, int32_t tile_base, uint32_t n,
                                  uint32_t* keys, uint32_t* vals, uint32_t* counter,
                                  hipStream_t stream) {
  if (n == 0) {
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, stream, counter);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_tile_len_keys, dim3((n + 255) / 256), dim3(256), 0, stream, tile_ranges,
                     tile_base, n, keys, vals, counter);
  return hipGetLastError();
}

hipError_t launch_zero_counter(uint32_t* counter, hipStream_t stream) {
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, stream, counter);
  return hipGetLastError();
}

}  // namespace seele
