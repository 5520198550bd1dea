// Tile binning and per-tile depth order on gfx950 (Sec. 3.1 "Preprocessing"
// finds Gaussian-tile intersections, "Sorting" orders each tile's Gaussians
// from the closest to the furthest).
//
// The required order is lexicographic in (global tile, float32 depth bits,
// record id).  It is built without sorting one key per Gaussian-tile pair:
//  1. The visible records are sorted by depth alone (4 stable 8-bit LSD
//     passes over N_vis records, input in id order so ties stay in id order).
//  2. Super-tiles of 4 x 4 tiles: every depth-ordered record emits one entry
//     per super-tile its tile rectangle touches, carrying the rectangle
//     clipped to that super-tile (2 bits per edge) above the super-tile id.
//     The entries (several times fewer than pairs) are stably sorted by
//     super-tile id, so each super-tile's list is in depth order.
//  3. Each super-tile list is cut into segments of kSegLen entries.  Per
//     segment and tile, the entries covering the tile are counted; a prefix
//     over the super-tile's segments and one scan over all tiles give the
//     tile ranges.  A last pass writes every record id straight to its slot:
//     inside a wave the rank among entries covering a tile is a ballot count.
// Every step is stable, so the result is exactly the lexicographic order.
//
// Every count (visible records, pairs, entries, segments) stays on the
// device: grids are sized for the maximum and loop over the live work, so the
// whole stage can be captured in a graph and never synchronises with the
// host.
#include "seele_internal.h"

namespace seele {

namespace {

constexpr int B = kSortBlock;
constexpr int ITEMS = kSortItems;
constexpr int TILE = kSortTile;
constexpr int WAVES = B / 64;
constexpr int ST = kSuperTile;
constexpr int ST2 = ST * ST;
constexpr int kSegLen = 1024;      // super-tile list entries per write segment
constexpr int kClipShift = 24;     // entry key = clipped rectangle << 24 | super-tile
constexpr uint32_t kStMask = (1u << kClipShift) - 1u;
constexpr int kMaxGrid = 2048;     // workgroups of the loops over device-side counts

struct Hdr {
  uint32_t n_vis;      // visible records
  uint32_t n_pairs;    // pairs: P if P <= capacity, else 0
  uint64_t p_total;    // pairs the frame needs
  uint32_t n_ent;      // super-tile entries (0 when the frame overflows)
  uint32_t n_seg;      // write segments
};

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_zero_hdr(Hdr* h) {
  if (threadIdx.x == 0) {
    h->n_vis = 0;
    h->n_pairs = 0;
    h->p_total = 0;
    h->n_ent = 0;
    h->n_seg = 0;
  }
}

// Tile rectangle [x0, x1) x [y0, y1) of a record, clipped to its view's grid
// (preprocessing already keeps it inside; the clip guards the indexing).
struct Rect {
  uint32_t x0, x1, y0, y1;
};

__device__ __forceinline__ Rect rect_of(const seele_splat& s, const BinView& bv) {
  Rect r;
  r.x1 = min(s.rect_x >> 16, (uint32_t)bv.grid_w);
  r.y1 = min(s.rect_y >> 16, (uint32_t)bv.grid_h);
  r.x0 = min(s.rect_x & 0xffffu, r.x1);
  r.y0 = min(s.rect_y & 0xffffu, r.y1);
  return r;
}

__device__ __forceinline__ uint32_t st_count(const Rect& r) {
  if (r.x1 <= r.x0 || r.y1 <= r.y0) return 0u;
  return ((r.x1 - 1) / ST - r.x0 / ST + 1) * ((r.y1 - 1) / ST - r.y0 / ST + 1);
}

// Where super-tile s lies: its view's global tile of the super-tile's top-left
// tile, the view's grid width and how many of its 4 x 4 tiles are inside.
struct StLoc {
  int32_t tile0;
  int grid_w, nx, ny;
};

__device__ __forceinline__ StLoc st_locate(const BinViews& views, uint32_t s) {
  int lo = 0, hi = views.n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((uint32_t)views.v[mid].st_base <= s) lo = mid;
    else hi = mid - 1;
  }
  const BinView bv = views.v[lo];
  const int sgw = (bv.grid_w + ST - 1) / ST;
  const int ls = (int)(s - (uint32_t)bv.st_base);
  const int sy = ls / sgw, sx = ls - sy * sgw;
  StLoc L;
  L.grid_w = bv.grid_w;
  L.tile0 = bv.tile_base + sy * ST * bv.grid_w + sx * ST;
  L.nx = min(ST, bv.grid_w - sx * ST);
  L.ny = min(ST, bv.grid_h - sy * ST);
  return L;
}

// Does an entry with clipped rectangle `clip` cover tile t (t = 4 iy + ix)
// of its super-tile?
__device__ __forceinline__ bool clip_covers(uint32_t clip, int t) {
  const uint32_t ix = (uint32_t)(t & 3), iy = (uint32_t)(t >> 2);
  return ix >= (clip & 3u) && ix <= ((clip >> 2) & 3u) && iy >= ((clip >> 4) & 3u) &&
         iy <= ((clip >> 6) & 3u);
}

// ---- visible-record compaction: count per block, scan, then write (depth, id)
__global__ __launch_bounds__(B) void k_vis_count(const int32_t* __restrict__ n_tiles, int64_t n,
                                                  uint64_t* __restrict__ partial) {
  const int64_t begin = (int64_t)blockIdx.x * TILE;
  uint32_t c = 0;
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int64_t idx = begin + it * B + threadIdx.x;
    if (idx < n && n_tiles[idx] > 0) ++c;
  }
  __shared__ uint32_t s[WAVES];
  c = wave_sum(c);
  if (lane_id() == 0) s[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < WAVES; ++w) t += s[w];
    partial[blockIdx.x] = t;
  }
}

// Exclusive scan of nb partial sums in place by one block; the total goes to
// mode 0: hdr->n_vis.  1: hdr->p_total, *num_pairs and hdr->n_pairs (zero
// when the total exceeds capacity).  2: hdr->n_ent (zero when the pairs
// exceed capacity).  3: hdr->n_seg.  4: nowhere.
__global__ __launch_bounds__(B) void k_scan_partials(uint64_t* __restrict__ partial, int64_t nb,
                                                      Hdr* __restrict__ hdr, int mode,
                                                      int64_t capacity,
                                                      int64_t* __restrict__ num_pairs) {
  __shared__ uint64_t s[WAVES + 1];
  uint64_t carry = 0;
  for (int64_t base = 0; base < nb; base += B) {
    const int64_t idx = base + threadIdx.x;
    const uint64_t x = idx < nb ? partial[idx] : 0;
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan<uint64_t>(x, s, tot);
    if (idx < nb) partial[idx] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    if (mode == 0) {
      hdr->n_vis = (uint32_t)carry;
    } else if (mode == 1) {
      hdr->p_total = carry;
      *num_pairs = (int64_t)carry;
      hdr->n_pairs = carry <= (uint64_t)capacity ? (uint32_t)carry : 0u;
    } else if (mode == 2) {
      hdr->n_ent = hdr->p_total <= (uint64_t)capacity ? (uint32_t)carry : 0u;
    } else if (mode == 3) {
      hdr->n_seg = (uint32_t)carry;
    }
  }
}

__global__ __launch_bounds__(B) void k_vis_compact(const int32_t* __restrict__ n_tiles, int64_t n,
                                                    const seele_splat* __restrict__ splats,
                                                    const uint64_t* __restrict__ partial,
                                                    uint32_t* __restrict__ keys,
                                                    uint32_t* __restrict__ vals) {
  __shared__ uint32_t s[WAVES + 1];
  const int64_t begin = (int64_t)blockIdx.x * TILE;
  uint32_t carry = (uint32_t)partial[blockIdx.x];
#pragma unroll 1
  for (int it = 0; it < ITEMS; ++it) {
    const int64_t idx = begin + it * B + threadIdx.x;
    const uint32_t f = (idx < n && n_tiles[idx] > 0) ? 1u : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t>(f, s, tot);
    if (f) {
      const uint32_t pos = carry + ex;
      keys[pos] = __float_as_uint(splats[idx].depth);
      vals[pos] = (uint32_t)idx;
    }
    carry += tot;
  }
}

// ---- stable LSD radix sort of (u32 key, u32 value) with a device-side count
//
// A radix block owns BLK = 256 * IT consecutive items.  Items either come
// from arrays (LOAD) or are generated on the fly as the super-tile entries
// [b*BLK, (b+1)*BLK) of the depth-ordered records (GEN: the entry emission
// fused into the first pass, so the entries are never written unsorted).
// A fixed grid loops over the live blocks.  hist layout: [digit][block] with
// row stride `stride`.

constexpr int kGenIT = 8;                 // GEN blocks hold 2048 entries
constexpr int kGenBlk = B * kGenIT;
// GEN window arrays (W <= BLK + 1 records each): first entry, id, global
// super-tile of the top-left covered super-tile, covered super-tile columns |
// super-tile grid width << 16, tile rectangle x0 | x1 << 16 and y0 | y1 << 16,
// and the block position -> window record map.
enum { kWinOff, kWinId, kWinT0, kWinWg, kWinRx, kWinRy, kWinRec, kWinArrays };

struct GenSrc {
  const uint32_t* ids;          // depth-ordered visible records
  const seele_splat* splats;
  const uint32_t* goff;         // first entry of each depth-ordered record
  const uint32_t* block_first;  // record holding the first entry of each GEN block
  const Hdr* hdr;
};

// Block-wide inclusive max-scan of IT consecutive values per thread (in place).
template <int IT>
__device__ __forceinline__ void block_inclusive_max(uint32_t* s_rec, uint32_t* s_tmp) {
  const int tid = threadIdx.x, w = tid >> 6, l = lane_id();
  uint32_t v[IT];
  uint32_t m = 0;
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    v[i] = s_rec[tid * IT + i];
    m = v[i] > m ? v[i] : m;
    v[i] = m;
  }
  // inclusive max over lanes, then over waves
  uint32_t x = m;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (l >= d) x = y > x ? y : x;
  }
  if (l == 63) s_tmp[w] = x;
  __syncthreads();
  uint32_t prev = __shfl_up(x, 1, 64);
  if (l == 0) prev = 0;
  for (int i = 0; i < w; ++i) prev = s_tmp[i] > prev ? s_tmp[i] : prev;
#pragma unroll
  for (int i = 0; i < IT; ++i) s_rec[tid * IT + i] = v[i] > prev ? v[i] : prev;
  __syncthreads();
}

// Exact k / w for 1 <= w < 2^16: a float reciprocal estimate is within one of
// the quotient for k < 2^22 and is corrected once; larger k divide exactly.
__device__ __forceinline__ uint32_t div_small(uint32_t k, uint32_t w) {
  if (k < (1u << 22)) {
    uint32_t q = (uint32_t)((float)k * __builtin_amdgcn_rcpf((float)w));
    const int32_t r = (int32_t)(k - q * w);
    if (r < 0) --q;
    else if (r >= (int32_t)w) ++q;
    return q;
  }
  return k / w;
}

// Stage the records covering entries [S, S + BLK) in the LDS window and map
// every position of the block to its record: each record marks the block
// position of its first entry and an inclusive max-scan spreads the marks
// over the record's entries.
template <int IT>
__device__ __forceinline__ void gen_window(const GenSrc& g, const BinViews& views, uint32_t blk,
                                           uint32_t nblk, uint32_t* s_win, uint32_t* s_tmp) {
  constexpr int BLK = B * IT;
  constexpr int L = BLK + 1;
  uint32_t* s_rec = s_win + kWinRec * L;
  const uint32_t nv = g.hdr->n_vis;
  const uint32_t S = blk * (uint32_t)BLK;
  const uint32_t g_lo = g.block_first[blk];
  const uint32_t g_hi = blk + 1 < nblk ? g.block_first[blk + 1] : nv - 1;
  // records without entries (only from malformed rectangles) could widen the
  // window past its LDS arrays; the cap keeps every access inside
  const int W = min((int)(g_hi - g_lo + 1), L);
  const uint32_t n = (uint32_t)views.n;
  for (int j = threadIdx.x; j < BLK; j += B) s_rec[j] = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < W; j += B) {
    const uint32_t id = g.ids[g_lo + j];
    const uint32_t o = g.goff[g_lo + j];
    const BinView bv = views.v[id / n];
    const Rect r = rect_of(g.splats[id], bv);
    const uint32_t sgw = ((uint32_t)bv.grid_w + ST - 1) / ST;
    const uint32_t sx0 = r.x0 / ST, sy0 = r.y0 / ST;
    const uint32_t sw = r.x1 > r.x0 ? (r.x1 - 1) / ST - sx0 + 1 : 1u;
    s_win[kWinOff * L + j] = o;
    s_win[kWinId * L + j] = id;
    s_win[kWinT0 * L + j] = (uint32_t)bv.st_base + sy0 * sgw + sx0;
    s_win[kWinWg * L + j] = sw | (sgw << 16);
    s_win[kWinRx * L + j] = r.x0 | (r.x1 << 16);
    s_win[kWinRy * L + j] = r.y0 | (r.y1 << 16);
    // records without entries own no position (their offset is the next one's)
    if (j > 0 && st_count(r) > 0 && o - S < (uint32_t)BLK) s_rec[o - S] = (uint32_t)j;
  }
  __syncthreads();
  block_inclusive_max<IT>(s_rec, s_tmp);
}

// Entry at block position p (global position q).
template <int IT>
__device__ __forceinline__ void gen_entry(uint32_t q, uint32_t p, const uint32_t* s_win,
                                          uint32_t& key, uint32_t& val) {
  constexpr int L = B * IT + 1;
  const uint32_t j = s_win[kWinRec * L + p];
  const uint32_t k = q - s_win[kWinOff * L + j];
  const uint32_t wg = s_win[kWinWg * L + j];
  const uint32_t sw = wg & 0xffffu;
  const uint32_t dy = div_small(k, sw);
  const uint32_t dx = k - dy * sw;
  const uint32_t rx = s_win[kWinRx * L + j], ry = s_win[kWinRy * L + j];
  const uint32_t x0 = rx & 0xffffu, x1 = rx >> 16, y0 = ry & 0xffffu, y1 = ry >> 16;
  const uint32_t ox = (x0 / ST + dx) * ST, oy = (y0 / ST + dy) * ST;
  const uint32_t cx0 = max(x0, ox) - ox, cx1 = min(x1, ox + ST) - 1u - ox;
  const uint32_t cy0 = max(y0, oy) - oy, cy1 = min(y1, oy + ST) - 1u - oy;
  const uint32_t clip = cx0 | (cx1 << 2) | (cy0 << 4) | (cy1 << 6);
  key = (clip << kClipShift) | (s_win[kWinT0 * L + j] + dy * (wg >> 16) + dx);
  val = s_win[kWinId * L + j];
}

template <int IT>
constexpr int gen_lds_words() {
  return kWinArrays * (B * IT + 1);
}

template <int IT, bool GEN>
__global__ __launch_bounds__(B) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ d_count,
                                                   GenSrc gs, BinViews views, int shift,
                                                   int bits, uint32_t* __restrict__ hist,
                                                   int stride) {
  constexpr int BLK = B * IT;
  constexpr int kWin = GEN ? gen_lds_words<IT>() : 1;
  __shared__ uint32_t h[WAVES][256];
  __shared__ uint32_t s_win[kWin];
  __shared__ uint32_t s_tmp[WAVES + 1];
  const int radix = 1 << bits;
  const int w = threadIdx.x >> 6;
  const uint32_t count = *d_count;
  const uint32_t nbl = (uint32_t)(((uint64_t)count + BLK - 1) / BLK);
  const uint32_t mask = (uint32_t)radix - 1u;
  for (uint32_t vb = blockIdx.x; vb < nbl; vb += gridDim.x) {
    for (int d = threadIdx.x; d < WAVES * 256; d += B) (&h[0][0])[d] = 0;
    if (GEN) gen_window<IT>(gs, views, vb, nbl, s_win, s_tmp);
    __syncthreads();
    const int64_t begin = (int64_t)vb * BLK;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const uint32_t p = it * B + threadIdx.x;
      const int64_t idx = begin + p;
      if (idx < count) {
        uint32_t k, v;
        if (GEN)
          gen_entry<IT>((uint32_t)idx, p, s_win, k, v);
        else
          k = keys[idx];
        atomicAdd(&h[w][(k >> shift) & mask], 1u);
      }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < radix; d += B) {
      uint32_t t = 0;
#pragma unroll
      for (int ww = 0; ww < WAVES; ++ww) t += h[ww][d];
      hist[(int64_t)d * stride + vb] = t;
    }
    __syncthreads();
  }
}

// One block per digit: exclusive scan of that digit's per-block counts over
// the live blocks, in place (16 consecutive entries per thread); the digit
// total goes to digit_total[d].
__global__ __launch_bounds__(B) void k_radix_rowscan(uint32_t* __restrict__ hist, int stride,
                                                      const uint32_t* __restrict__ d_count,
                                                      int blk, uint32_t* __restrict__ digit_total) {
  constexpr int R = 16;
  __shared__ uint32_t s[WAVES + 1];
  const int nblocks = (int)(((uint64_t)*d_count + blk - 1) / blk);
  uint32_t* row = hist + (int64_t)blockIdx.x * stride;
  uint32_t carry = 0;
  for (int base = 0; base < nblocks; base += B * R) {
    const int i0 = base + threadIdx.x * R;
    uint32_t v[R];
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v[r] = i0 + r < nblocks ? row[i0 + r] : 0u;
      sum += v[r];
    }
    uint32_t tot;
    uint32_t run = carry + block_exclusive_scan<uint32_t>(sum, s, tot);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (i0 + r < nblocks) row[i0 + r] = run;
      run += v[r];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) digit_total[blockIdx.x] = carry;
}

// Stable scatter.  Wave w owns the contiguous quarter w of the block,
// processed 64 items at a time in index order.  Within a 64-item step a
// lane's rank among equal digits comes from ballots over the digit bits;
// per-wave running counts in LDS order the steps; per-digit wave offsets
// order the waves.  Items are first placed in LDS in block-sorted order and
// then written out digit run by digit run, so consecutive lanes store to
// consecutive addresses.  Input order is preserved among equal digits.
template <int IT, bool GEN>
__global__ __launch_bounds__(B) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, const uint32_t* __restrict__ d_count,
    GenSrc gs, BinViews views, int shift, int bits, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ digit_total, int stride) {
  constexpr int BLK = B * IT;
  constexpr int kWords = GEN ? gen_lds_words<IT>() : 2 * BLK;
  __shared__ uint32_t s_mem[kWords];  // GEN window, then the staged (key, value) pairs
  __shared__ uint32_t s_dig[256];     // global start of each digit
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_loc[256];
  __shared__ uint32_t s_w[WAVES][256];
  __shared__ uint32_t s_tmp[WAVES + 1];
  const uint32_t count = *d_count;
  const uint32_t nbl = (uint32_t)(((uint64_t)count + BLK - 1) / BLK);
  if (blockIdx.x >= nbl) return;  // uniform per block
  const int radix = 1 << bits;
  const uint32_t mask = (uint32_t)radix - 1u;
  const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
  {
    const uint32_t t = tid < radix ? digit_total[tid] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t>(t, s_tmp, tot);
    if (tid < radix) s_dig[tid] = ex;
  }
  const uint64_t lt = lanemask_lt();
  for (uint32_t vb = blockIdx.x; vb < nbl; vb += gridDim.x) {
    const int64_t begin = (int64_t)vb * BLK;
    if (tid < radix) s_base[tid] = s_dig[tid] + hist[(int64_t)tid * stride + vb];
    for (int d = tid; d < WAVES * 256; d += B) (&s_w[0][0])[d] = 0;
    if (GEN) gen_window<IT>(gs, views, vb, nbl, s_mem, s_tmp);
    __syncthreads();

    uint32_t k[IT], v[IT], rank[IT];
    const int64_t wbase = begin + (int64_t)w * 64 * IT;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int64_t idx = wbase + it * 64 + lane;
      k[it] = 0u;
      v[it] = 0u;
      if (idx < count) {
        if (GEN)
          gen_entry<IT>((uint32_t)idx, (uint32_t)(idx - begin), s_mem, k[it], v[it]);
        else {
          k[it] = kin[idx];
          v[it] = vin[idx];
        }
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int64_t idx = wbase + it * 64 + lane;
      const bool valid = idx < count;
      const uint32_t d = (k[it] >> shift) & mask;
      uint64_t peers = __ballot(valid);
      for (int b = 0; b < bits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        peers &= bit ? bb : ~bb;
      }
      const uint32_t below = (uint32_t)__popcll(peers & lt);
      const uint32_t before = s_w[w][d];
      rank[it] = before + below;
      if (valid && below == 0) s_w[w][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();  // s_w complete; the GEN window is no longer read
    // per digit: wave offsets, block total, block-local digit start
    uint32_t dtot = 0;
    if (tid < radix) {
#pragma unroll
      for (int ww = 0; ww < WAVES; ++ww) {
        const uint32_t c = s_w[ww][tid];
        s_w[ww][tid] = dtot;
        dtot += c;
      }
    }
    {
      uint32_t tot;
      const uint32_t ex = block_exclusive_scan<uint32_t>(tid < radix ? dtot : 0u, s_tmp, tot);
      if (tid < radix) s_loc[tid] = ex;
    }
    __syncthreads();
    uint32_t* s_k = s_mem;
    uint32_t* s_v = s_mem + BLK;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int64_t idx = wbase + it * 64 + lane;
      if (idx < count) {
        const uint32_t d = (k[it] >> shift) & mask;
        const uint32_t lp = s_loc[d] + s_w[w][d] + rank[it];
        s_k[lp] = k[it];
        s_v[lp] = v[it];
      }
    }
    __syncthreads();
    const uint32_t n_here = (uint32_t)min<int64_t>(BLK, (int64_t)count - begin);
    for (uint32_t j = tid; j < n_here; j += B) {
      const uint32_t kk = s_k[j];
      const uint32_t d = (kk >> shift) & mask;
      const uint32_t pos = s_base[d] + (j - s_loc[d]);
      kout[pos] = kk;
      vout[pos] = s_v[j];
    }
    __syncthreads();  // LDS is reused by the next block
  }
}

// ---- super-tile entries of the depth-ordered records
// Per record: pairs (tiles of its rectangle) and entries (super-tiles it
// touches); block sums of both.
__global__ __launch_bounds__(B) void k_pair_count(const uint32_t* __restrict__ ids,
                                                   const seele_splat* __restrict__ splats,
                                                   BinViews views, const Hdr* __restrict__ hdr,
                                                   uint32_t* __restrict__ ecount,
                                                   uint64_t* __restrict__ partial,
                                                   uint64_t* __restrict__ partial2) {
  const uint32_t nv = hdr->n_vis;
  const int64_t begin = (int64_t)blockIdx.x * TILE;
  uint64_t c = 0, q = 0;
  const uint32_t n = (uint32_t)views.n;
  if (begin < nv) {
#pragma unroll 4
    for (int it = 0; it < ITEMS; ++it) {
      const int64_t i = begin + it * B + threadIdx.x;
      if (i < nv) {
        const uint32_t id = ids[i];
        const Rect r = rect_of(splats[id], views.v[id / n]);
        const uint32_t m = st_count(r);
        if (m > 0) c += (uint64_t)(r.x1 - r.x0) * (r.y1 - r.y0);
        ecount[i] = m;
        q += m;
      }
    }
  }
  __shared__ uint64_t s[2][WAVES];
  c = wave_sum(c);
  q = wave_sum(q);
  if (lane_id() == 0) {
    s[0][threadIdx.x >> 6] = c;
    s[1][threadIdx.x >> 6] = q;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0, u = 0;
    for (int w = 0; w < WAVES; ++w) {
      t += s[0][w];
      u += s[1][w];
    }
    partial[blockIdx.x] = t;
    partial2[blockIdx.x] = u;
  }
}

// Per-record entry offsets in depth order (exclusive scan of entry counts),
// and for every GEN block of kGenBlk entries the record holding its first
// entry.  Skipped when the frame overflows the pair capacity.
__global__ __launch_bounds__(B) void k_entry_offsets(const uint32_t* __restrict__ ecount,
                                                      const Hdr* __restrict__ hdr,
                                                      const uint64_t* __restrict__ partial,
                                                      int64_t capacity,
                                                      uint32_t* __restrict__ goff,
                                                      uint32_t* __restrict__ block_first) {
  __shared__ uint64_t s[WAVES + 1];
  const uint32_t nv = hdr->n_vis;
  const int64_t begin = (int64_t)blockIdx.x * TILE;
  if (begin >= nv || hdr->p_total > (uint64_t)capacity) return;  // uniform per block
  uint64_t carry = partial[blockIdx.x];
#pragma unroll 1
  for (int it = 0; it < ITEMS; ++it) {
    const int64_t i = begin + it * B + threadIdx.x;
    const uint32_t c = i < nv ? ecount[i] : 0u;
    uint64_t tot;
    const uint64_t off = carry + block_exclusive_scan<uint64_t>((uint64_t)c, s, tot);
    carry += tot;
    if (i < nv) {
      goff[i] = (uint32_t)off;
      // GEN blocks whose first entry belongs to this record
      for (uint64_t b = (off + kGenBlk - 1) / kGenBlk; b * kGenBlk < off + c; ++b)
        block_first[b] = (uint32_t)i;
    }
  }
}

// Super-tile list ranges [a, b) from the sorted entry keys.
__global__ void k_st_ranges(const uint32_t* __restrict__ keys, const Hdr* __restrict__ hdr,
                            int32_t* __restrict__ st_range) {
  const int64_t cnt = hdr->n_ent;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t s = keys[i] & kStMask;
    if (i == 0 || (keys[i - 1] & kStMask) != s) st_range[2 * (int64_t)s] = (int32_t)i;
    if (i == cnt - 1 || (keys[i + 1] & kStMask) != s)
      st_range[2 * (int64_t)s + 1] = (int32_t)(i + 1);
  }
}

__device__ __forceinline__ uint32_t n_segments(const int32_t* st_range, int64_t s) {
  const int32_t len = st_range[2 * s + 1] - st_range[2 * s];
  return (uint32_t)((len + kSegLen - 1) / kSegLen);
}

// Segments per super-tile: block sums, then (after the scan) each
// super-tile's first segment and the segment -> super-tile table.
__global__ __launch_bounds__(B) void k_seg_count(const int32_t* __restrict__ st_range,
                                                  int64_t n_st, uint64_t* __restrict__ partial) {
  const int64_t begin = (int64_t)blockIdx.x * TILE;
  uint32_t c = 0;
#pragma unroll 4
  for (int it = 0; it < ITEMS; ++it) {
    const int64_t s = begin + it * B + threadIdx.x;
    if (s < n_st) c += n_segments(st_range, s);
  }
  __shared__ uint32_t sm[WAVES];
  c = wave_sum(c);
  if (lane_id() == 0) sm[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < WAVES; ++w) t += sm[w];
    partial[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(B) void k_seg_emit(const int32_t* __restrict__ st_range,
                                                 int64_t n_st, const uint64_t* __restrict__ partial,
                                                 uint32_t* __restrict__ st_seg,
                                                 uint32_t* __restrict__ seg_st) {
  __shared__ uint32_t sm[WAVES + 1];
  const int64_t begin = (int64_t)blockIdx.x * TILE;
  uint32_t carry = (uint32_t)partial[blockIdx.x];
#pragma unroll 1
  for (int it = 0; it < ITEMS; ++it) {
    const int64_t s = begin + it * B + threadIdx.x;
    const uint32_t c = s < n_st ? n_segments(st_range, s) : 0u;
    uint32_t tot;
    const uint32_t first = carry + block_exclusive_scan<uint32_t>(c, sm, tot);
    carry += tot;
    if (s < n_st) {
      st_seg[s] = first;
      for (uint32_t k = 0; k < c; ++k) seg_st[first + k] = (uint32_t)s;
    }
  }
}

// Entries [a, e) of segment `seg` and its super-tile.
struct Seg {
  uint32_t st;
  int32_t a, e;
};

__device__ __forceinline__ Seg segment(uint32_t seg, const uint32_t* seg_st,
                                       const uint32_t* st_seg, const int32_t* st_range) {
  Seg g;
  g.st = seg_st[seg];
  const int32_t lo = st_range[2 * (int64_t)g.st], hi = st_range[2 * (int64_t)g.st + 1];
  g.a = lo + (int32_t)(seg - st_seg[g.st]) * kSegLen;
  g.e = min(hi, g.a + kSegLen);
  return g;
}

// Per segment and tile of its super-tile: entries covering the tile.
__global__ __launch_bounds__(B) void k_seg_tile_count(const Hdr* __restrict__ hdr,
                                                       const uint32_t* __restrict__ seg_st,
                                                       const uint32_t* __restrict__ st_seg,
                                                       const int32_t* __restrict__ st_range,
                                                       const uint32_t* __restrict__ ekeys,
                                                       uint32_t* __restrict__ seg_cnt) {
  __shared__ uint32_t s_c[WAVES][ST2];
  const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
  const uint32_t nseg = hdr->n_seg;
  for (uint32_t seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
    const Seg g = segment(seg, seg_st, st_seg, st_range);
    uint32_t c[ST2];
#pragma unroll
    for (int t = 0; t < ST2; ++t) c[t] = 0;
    for (int32_t base = g.a + w * 64; base < g.e; base += B) {
      const int32_t i = base + lane;
      const bool valid = i < g.e;
      const uint32_t clip = valid ? ekeys[i] >> kClipShift : 0u;
#pragma unroll
      for (int t = 0; t < ST2; ++t) c[t] += (uint32_t)__popcll(__ballot(valid && clip_covers(clip, t)));
    }
    if (lane < ST2) {
      uint32_t x = 0;
#pragma unroll
      for (int t = 0; t < ST2; ++t)
        if (t == lane) x = c[t];
      s_c[w][lane] = x;
    }
    __syncthreads();
    if (tid < ST2) {
      uint32_t t = 0;
#pragma unroll
      for (int ww = 0; ww < WAVES; ++ww) t += s_c[ww][tid];
      seg_cnt[(int64_t)seg * ST2 + tid] = t;
    }
    __syncthreads();
  }
}

// One thread per (super-tile, tile): exclusive prefix of the tile's counts
// over the super-tile's segments (in place) and the tile's total pair count.
__global__ void k_st_tile_prefix(const int32_t* __restrict__ st_range,
                                 const uint32_t* __restrict__ st_seg, int64_t n_st,
                                 BinViews views, uint32_t* __restrict__ seg_cnt,
                                 uint32_t* __restrict__ tile_cnt) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_st * ST2) return;
  const int64_t s = g / ST2;
  const int t = (int)(g % ST2);
  const uint32_t ns = n_segments(st_range, s);
  const uint32_t first = st_seg[s];
  uint32_t run = 0;
  for (uint32_t k = 0; k < ns; ++k) {
    uint32_t* p = seg_cnt + (int64_t)(first + k) * ST2 + t;
    const uint32_t c = *p;
    *p = run;
    run += c;
  }
  const StLoc L = st_locate(views, (uint32_t)s);
  const int ix = t & 3, iy = t >> 2;
  if (ix < L.nx && iy < L.ny) tile_cnt[L.tile0 + iy * L.grid_w + ix] = run;
}

__global__ __launch_bounds__(B) void k_tile_partials(const uint32_t* __restrict__ tile_cnt,
                                                      int64_t n, uint64_t* __restrict__ partial) {
  const int64_t begin = (int64_t)blockIdx.x * TILE;
  uint64_t c = 0;
#pragma unroll 4
  for (int it = 0; it < ITEMS; ++it) {
    const int64_t t = begin + it * B + threadIdx.x;
    if (t < n) c += tile_cnt[t];
  }
  __shared__ uint64_t sm[WAVES];
  c = wave_sum(c);
  if (lane_id() == 0) sm[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < WAVES; ++w) t += sm[w];
    partial[blockIdx.x] = t;
  }
}

// Tile starts and ranges: [start, start + count) for a non-empty tile,
// (0, 0) for an empty one or when the frame overflows the pair capacity.
__global__ __launch_bounds__(B) void k_tile_ranges(const uint32_t* __restrict__ tile_cnt,
                                                    int64_t n, const uint64_t* __restrict__ partial,
                                                    const Hdr* __restrict__ hdr,
                                                    uint32_t* __restrict__ tile_start,
                                                    int32_t* __restrict__ ranges) {
  __shared__ uint64_t sm[WAVES + 1];
  const int64_t begin = (int64_t)blockIdx.x * TILE;
  const bool fits = hdr->n_pairs > 0;
  uint64_t carry = partial[blockIdx.x];
#pragma unroll 1
  for (int it = 0; it < ITEMS; ++it) {
    const int64_t t = begin + it * B + threadIdx.x;
    const uint32_t c = t < n ? tile_cnt[t] : 0u;
    uint64_t tot;
    const uint64_t start = carry + block_exclusive_scan<uint64_t>((uint64_t)c, sm, tot);
    carry += tot;
    if (t < n) {
      tile_start[t] = (uint32_t)start;
      const bool any = fits && c > 0;
      ranges[2 * t] = any ? (int32_t)start : 0;
      ranges[2 * t + 1] = any ? (int32_t)(start + c) : 0;
    }
  }
}

// Write every record id of a segment to its slots: for each tile of the
// super-tile, the segment's base slot, plus the entries covering the tile in
// earlier 256-entry steps, earlier waves of this step, and (ballot count)
// lower lanes of this wave.
__global__ __launch_bounds__(B) void k_seg_write(const Hdr* __restrict__ hdr,
                                                  const uint32_t* __restrict__ seg_st,
                                                  const uint32_t* __restrict__ st_seg,
                                                  const int32_t* __restrict__ st_range,
                                                  const uint32_t* __restrict__ ekeys,
                                                  const uint32_t* __restrict__ evals,
                                                  const uint32_t* __restrict__ seg_cnt,
                                                  const uint32_t* __restrict__ tile_start,
                                                  BinViews views, uint32_t* __restrict__ out) {
  __shared__ uint32_t s_run[ST2];
  __shared__ uint32_t s_c[WAVES][ST2];
  const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
  const uint64_t lt = lanemask_lt();
  const uint32_t nseg = hdr->n_seg;
  for (uint32_t seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
    const Seg g = segment(seg, seg_st, st_seg, st_range);
    if (tid < ST2) {
      const StLoc L = st_locate(views, g.st);
      const int ix = tid & 3, iy = tid >> 2;
      s_run[tid] = (ix < L.nx && iy < L.ny)
                       ? tile_start[L.tile0 + iy * L.grid_w + ix] + seg_cnt[(int64_t)seg * ST2 + tid]
                       : 0u;
    }
    for (int32_t base = g.a; base < g.e; base += B) {
      const int32_t i = base + tid;
      const bool valid = i < g.e;
      const uint32_t clip = valid ? ekeys[i] >> kClipShift : 0u;
      const uint32_t id = valid ? evals[i] : 0u;
      uint64_t bal[ST2];
#pragma unroll
      for (int t = 0; t < ST2; ++t) bal[t] = __ballot(valid && clip_covers(clip, t));
      if (lane < ST2) {
        uint32_t x = 0;
#pragma unroll
        for (int t = 0; t < ST2; ++t)
          if (t == lane) x = (uint32_t)__popcll(bal[t]);
        s_c[w][lane] = x;
      }
      __syncthreads();
      if (tid < ST2) {
        uint32_t o = s_run[tid];
#pragma unroll
        for (int ww = 0; ww < WAVES; ++ww) {
          const uint32_t c = s_c[ww][tid];
          s_c[ww][tid] = o;
          o += c;
        }
        s_run[tid] = o;
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < ST2; ++t)
        if ((bal[t] >> lane) & 1ull) out[s_c[w][t] + (uint32_t)__popcll(bal[t] & lt)] = id;
      __syncthreads();
    }
  }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t nblocks_for(int64_t n) { return (n + TILE - 1) / TILE; }

int grid_for(int64_t nb) { return (int)std::max<int64_t>(1, std::min<int64_t>(nb, kMaxGrid)); }

// One radix pass over a device-side count of at most max_count items.
template <int IT, bool GEN>
hipError_t radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                      const uint32_t* d_count, int64_t max_count, const GenSrc& gs,
                      const BinViews& views, int shift, int bits, uint32_t* hist,
                      uint32_t* digits, hipStream_t stream) {
  constexpr int BLK = B * IT;
  const int64_t nb = (max_count + BLK - 1) / BLK;
  if (nb == 0) return hipSuccess;
  const int stride = (int)nb;
  const dim3 grid(grid_for(nb));
  hipLaunchKernelGGL((k_radix_hist<IT, GEN>), grid, dim3(B), 0, stream, kin, d_count, gs, views,
                     shift, bits, hist, stride);
  hipLaunchKernelGGL(k_radix_rowscan, dim3(1 << bits), dim3(B), 0, stream, hist, stride, d_count,
                     BLK, digits);
  hipLaunchKernelGGL((k_radix_scatter<IT, GEN>), grid, dim3(B), 0, stream, kin, vin, kout, vout,
                     d_count, gs, views, shift, bits, hist, digits, stride);
  return hipGetLastError();
}

__global__ void k_set_count(uint32_t* d_count, uint32_t n) {
  if (threadIdx.x == 0) *d_count = n;
}

int64_t max_segments(int64_t capacity, int64_t max_st) {
  return (capacity + kSegLen - 1) / kSegLen + max_st;
}

}  // namespace

size_t radix_sort_workspace_size(int64_t n) {
  const int64_t nb = std::max<int64_t>(nblocks_for(n), 1);
  return align_up(256) + 4 * align_up(4 * (size_t)std::max<int64_t>(n, 1)) +
         align_up(4 * 256 * (size_t)nb) + align_up(4 * 256);
}

// Stable LSD sort of (key, value) pairs by the low `bits` key bits (8-bit
// passes); the result is left in (keys, vals).  ws holds the count, the
// ping-pong buffers and the digit histograms.
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, int64_t n, int bits, void* ws,
                            hipStream_t stream) {
  if (n <= 1) return hipSuccess;
  char* b = static_cast<char*>(ws);
  uint32_t* d_count = reinterpret_cast<uint32_t*>(b);
  size_t off = align_up(256);
  uint32_t* k1 = reinterpret_cast<uint32_t*>(b + off);
  off += align_up(4 * (size_t)n);
  uint32_t* v1 = reinterpret_cast<uint32_t*>(b + off);
  off += align_up(4 * (size_t)n);
  off += 2 * align_up(4 * (size_t)n);  // reserved
  uint32_t* hist = reinterpret_cast<uint32_t*>(b + off);
  off += align_up(4 * 256 * (size_t)std::max<int64_t>(nblocks_for(n), 1));
  uint32_t* digits = reinterpret_cast<uint32_t*>(b + off);
  hipLaunchKernelGGL(k_set_count, dim3(1), dim3(64), 0, stream, d_count, (uint32_t)n);
  uint32_t* k[2] = {keys, k1};
  uint32_t* v[2] = {vals, v1};
  const int passes = (bits + 7) / 8;
  BinViews none{};
  for (int pass = 0; pass < passes; ++pass) {
    const int src = pass & 1, dst = src ^ 1;
    const int pb = std::min(8, bits - 8 * pass);
    const hipError_t e = radix_pass<ITEMS, false>(k[src], v[src], k[dst], v[dst], d_count, n,
                                                  GenSrc{}, none, 8 * pass, pb, hist, digits,
                                                  stream);
    if (e != hipSuccess) return e;
  }
  if (passes % 2 == 1) {
    hipError_t e = hipMemcpyAsync(keys, k1, 4 * (size_t)n, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(vals, v1, 4 * (size_t)n, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

BinSortPlan plan_bin_sort(int64_t n_records, int64_t capacity, int64_t n_tiles_total) {
  BinSortPlan p{};
  p.n_records = n_records;
  p.capacity = capacity;
  p.n_tiles_total = n_tiles_total;
  p.max_st = std::max<int64_t>(n_tiles_total, 1);
  p.max_seg = max_segments(capacity, p.max_st);
  const int64_t nb_rec = std::max<int64_t>(nblocks_for(n_records), 1);
  const int64_t nb_hist = std::max<int64_t>(
      {nb_rec, (capacity + kGenBlk - 1) / kGenBlk, nblocks_for(capacity), 1});
  const int64_t nb_part =
      std::max<int64_t>({nb_rec, nblocks_for(p.max_st), nblocks_for(n_tiles_total), 1});
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  p.off_hdr = take(sizeof(Hdr));
  p.off_partial = take(8 * (size_t)nb_part);
  p.off_partial2 = take(8 * (size_t)nb_rec);
  p.off_dkeys0 = take(4 * (size_t)n_records);
  p.off_dkeys1 = take(4 * (size_t)n_records);
  p.off_dvals0 = take(4 * (size_t)n_records);
  p.off_dvals1 = take(4 * (size_t)n_records);
  p.off_skeys0 = take(4 * (size_t)capacity);
  p.off_skeys1 = take(4 * (size_t)capacity);
  p.off_svals0 = take(4 * (size_t)capacity);
  p.off_svals1 = 0;  // the second value buffer is the caller's sorted_ids
  p.off_mcount = take(4 * (size_t)n_records);
  p.off_goff = take(4 * (size_t)n_records);
  p.off_bfirst = take(4 * (size_t)(capacity / kGenBlk + 2));
  p.off_hist = take(4 * 256 * (size_t)nb_hist);
  p.off_digits = take(4 * 256);
  p.off_st_range = take(8 * (size_t)p.max_st);
  p.off_st_seg = take(4 * (size_t)p.max_st);
  p.off_seg_st = take(4 * (size_t)p.max_seg);
  p.off_seg_cnt = take(4 * ST2 * (size_t)p.max_seg);
  p.off_tile_cnt = take(4 * (size_t)std::max<int64_t>(n_tiles_total, 1));
  p.off_tile_start = take(4 * (size_t)std::max<int64_t>(n_tiles_total, 1));
  p.total = off;
  return p;
}

hipError_t launch_bin_sort(const BinSortPlan& p, const BinViews& views, const seele_splat* splats,
                           const int32_t* n_tiles, void* ws, uint32_t* sorted_ids,
                           int32_t* tile_ranges, int64_t* num_pairs, hipStream_t stream) {
  char* base = static_cast<char*>(ws);
  auto at = [&](size_t o) { return reinterpret_cast<uint32_t*>(base + o); };
  Hdr* hdr = reinterpret_cast<Hdr*>(base + p.off_hdr);
  uint64_t* partial = reinterpret_cast<uint64_t*>(base + p.off_partial);
  uint64_t* partial2 = reinterpret_cast<uint64_t*>(base + p.off_partial2);
  uint32_t* dk[2] = {at(p.off_dkeys0), at(p.off_dkeys1)};
  uint32_t* dv[2] = {at(p.off_dvals0), at(p.off_dvals1)};
  uint32_t* sk[2] = {at(p.off_skeys0), at(p.off_skeys1)};
  uint32_t* ecount = at(p.off_mcount);
  uint32_t* goff = at(p.off_goff);
  uint32_t* bfirst = at(p.off_bfirst);
  uint32_t* hist = at(p.off_hist);
  uint32_t* digits = at(p.off_digits);
  int32_t* st_range = reinterpret_cast<int32_t*>(base + p.off_st_range);
  uint32_t* st_seg = at(p.off_st_seg);
  uint32_t* seg_st = at(p.off_seg_st);
  uint32_t* seg_cnt = at(p.off_seg_cnt);
  uint32_t* tile_cnt = at(p.off_tile_cnt);
  uint32_t* tile_start = at(p.off_tile_start);
  const uint32_t* d_nvis = &hdr->n_vis;
  const uint32_t* d_nent = &hdr->n_ent;
  const int64_t n_st = views.n_st;
  const int64_t TT = p.n_tiles_total;
  hipError_t e;

  hipLaunchKernelGGL(k_zero_hdr, dim3(1), dim3(64), 0, stream, hdr);
  if (n_st > 0)
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((2 * n_st + 255) / 256)), dim3(256), 0, stream,
                       st_range, 2 * n_st, 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t R = p.n_records;
  const int nbR = (int)nblocks_for(R);
  if (nbR > 0) {
    // 1. visible records (n_tiles > 0) in id order with their depth keys
    hipLaunchKernelGGL(k_vis_count, dim3(nbR), dim3(B), 0, stream, n_tiles, R, partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(B), 0, stream, partial, (int64_t)nbR, hdr, 0,
                       p.capacity, num_pairs);
    hipLaunchKernelGGL(k_vis_compact, dim3(nbR), dim3(B), 0, stream, n_tiles, R, splats, partial,
                       dk[0], dv[0]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    //    stable sort by float32 depth bits (4 x 8-bit passes, ends in buffer 0)
    for (int pass = 0; pass < 4; ++pass) {
      const int src = pass & 1, dst = src ^ 1;
      e = radix_pass<ITEMS, false>(dk[src], dv[src], dk[dst], dv[dst], d_nvis, R, GenSrc{}, views,
                                   8 * pass, 8, hist, digits, stream);
      if (e != hipSuccess) return e;
    }
    // 2. pair and entry totals (pairs -> num_pairs), entry offsets
    hipLaunchKernelGGL(k_pair_count, dim3(nbR), dim3(B), 0, stream, dv[0], splats, views, hdr,
                       ecount, partial, partial2);
  }
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(B), 0, stream, partial, (int64_t)nbR, hdr, 1,
                     p.capacity, num_pairs);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(B), 0, stream, partial2, (int64_t)nbR, hdr, 2,
                     p.capacity, num_pairs);
  if (nbR > 0)
    hipLaunchKernelGGL(k_entry_offsets, dim3(nbR), dim3(B), 0, stream, ecount, hdr, partial2,
                       p.capacity, goff, bfirst);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  //    entries sorted by super-tile id (balanced digit widths <= 8); the first
  //    pass generates them; the value buffers alternate between svals0 and
  //    sorted_ids so that the last pass ends in svals0
  int st_bits = 0;
  while (st_bits < 24 && ((int64_t)1 << st_bits) < n_st) ++st_bits;
  const int passes = std::max(1, (st_bits + 7) / 8);
  const int per = (st_bits + passes - 1) / passes;
  uint32_t* sv_final = at(p.off_svals0);
  uint32_t* sv[2] = {(passes % 2 == 1) ? sv_final : sorted_ids,
                     (passes % 2 == 1) ? sorted_ids : sv_final};
  int shift = std::min(per, st_bits);
  {
    const GenSrc gs{dv[0], splats, goff, bfirst, hdr};
    e = radix_pass<kGenIT, true>(nullptr, nullptr, sk[0], sv[0], d_nent, p.capacity, gs, views, 0,
                                 shift, hist, digits, stream);
    if (e != hipSuccess) return e;
  }
  int cur = 0;
  for (int pass = 1; pass < passes; ++pass) {
    const int bits = std::min(per, st_bits - shift);
    e = radix_pass<ITEMS, false>(sk[cur], sv[cur], sk[cur ^ 1], sv[cur ^ 1], d_nent, p.capacity,
                                 GenSrc{}, views, shift, bits, hist, digits, stream);
    if (e != hipSuccess) return e;
    cur ^= 1;
    shift += bits;
  }
  const uint32_t* ekeys = sk[cur];
  const uint32_t* evals = sv[cur];
  // 3. super-tile ranges, segments, per-tile counts, tile ranges, write
  if (p.capacity > 0)
    hipLaunchKernelGGL(k_st_ranges, dim3(grid_for((p.capacity + 255) / 256)), dim3(256), 0,
                       stream, ekeys, hdr, st_range);
  const int nbS = (int)nblocks_for(n_st);
  if (nbS > 0) {
    hipLaunchKernelGGL(k_seg_count, dim3(nbS), dim3(B), 0, stream, st_range, n_st, partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(B), 0, stream, partial, (int64_t)nbS, hdr, 3,
                       p.capacity, num_pairs);
    hipLaunchKernelGGL(k_seg_emit, dim3(nbS), dim3(B), 0, stream, st_range, n_st, partial, st_seg,
                       seg_st);
  }
  const int seg_grid = grid_for(p.max_seg);
  hipLaunchKernelGGL(k_seg_tile_count, dim3(seg_grid), dim3(B), 0, stream, hdr, seg_st, st_seg,
                     st_range, ekeys, seg_cnt);
  if (n_st > 0)
    hipLaunchKernelGGL(k_st_tile_prefix, dim3((unsigned)((n_st * ST2 + 255) / 256)), dim3(256), 0,
                       stream, st_range, st_seg, n_st, views, seg_cnt, tile_cnt);
  const int nbT = (int)nblocks_for(TT);
  if (nbT > 0) {
    hipLaunchKernelGGL(k_tile_partials, dim3(nbT), dim3(B), 0, stream, tile_cnt, TT, partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(B), 0, stream, partial, (int64_t)nbT, hdr, 4,
                       p.capacity, num_pairs);
    hipLaunchKernelGGL(k_tile_ranges, dim3(nbT), dim3(B), 0, stream, tile_cnt, TT, partial, hdr,
                       tile_start, tile_ranges);
  }
  hipLaunchKernelGGL(k_seg_write, dim3(seg_grid), dim3(B), 0, stream, hdr, seg_st, st_seg,
                     st_range, ekeys, evals, seg_cnt, tile_start, views, sorted_ids);
  return hipGetLastError();
}

}  // namespace seele
