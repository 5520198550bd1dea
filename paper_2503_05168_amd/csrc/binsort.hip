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
//  3. Each super-tile list is cut into segments of kSegLen entries, each
//     segment into four wave quarters.  Per quarter and tile, the entries
//     covering the tile are counted; a prefix over the super-tile's quarters
//     and one scan over all tiles give the tile ranges.  A last pass writes
//     every record id straight to its slot: inside a wave the rank among
//     entries covering a tile is a ballot count.
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
constexpr int kMaxGrid = 2048;     // workgroups of the loops over device-side counts

struct Hdr {
  uint32_t n_vis;      // visible records
  uint32_t n_pairs;    // pairs: P if P <= capacity, else 0
  uint64_t p_total;    // pairs the frame needs
  uint32_t n_ent;      // super-tile entries (0 when the frame overflows)
  uint32_t n_seg;      // write segments
  uint64_t e_total;    // entries the frame needs (counted with atomics)
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
    h->e_total = 0;
  }
}

// Tile rectangle [x0, x1) x [y0, y1) of a record, clipped to its view's grid
// (preprocessing already keeps it inside; the clip guards the indexing).
struct Rect {
  uint32_t x0, x1, y0, y1;
};

// Tile rectangle from a record's packed rect_x / rect_y, clipped to its view.
__device__ __forceinline__ Rect rect_of(uint32_t rect_x, uint32_t rect_y, const BinView& bv) {
  Rect r;
  r.x1 = min(rect_x >> 16, (uint32_t)bv.grid_w);
  r.y1 = min(rect_y >> 16, (uint32_t)bv.grid_h);
  r.x0 = min(rect_x & 0xffffu, r.x1);
  r.y0 = min(rect_y & 0xffffu, r.y1);
  return r;
}

// View of record id = view * n + i: id / n < n_views <= 256, so a float
// reciprocal estimate is off by at most one and one correction makes it exact.
__device__ __forceinline__ uint32_t view_of(uint32_t id, const BinViews& views) {
  if (views.n_views == 1) return 0u;
  const uint64_t n = (uint64_t)views.n;
  uint32_t q = (uint32_t)((float)id * __builtin_amdgcn_rcpf((float)n));
  if ((uint64_t)q * n > id) --q;
  else if ((uint64_t)(q + 1) * n <= id) ++q;
  return q;
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

// ---- visible-record compaction.  Wave w of block b owns records
// [b*kSpanBlock + w*kWaveSpan, +kWaveSpan): per-wave counts, one scan, then each
// wave writes its (depth, id) pairs independently (ballot ranks).
// Radix passes of the binning: 512 threads x 8 items (4096 per block); 8
// waves per block shorten each block's serial chain (the passes are bound by
// latency, one round of blocks; measured on a 1080p frame of 3M Gaussians,
// bin/sort: 256 x 8 0.284 ms, 512 x 4 0.272, 512 x 8 0.269, 512 x 12 0.275,
// 512 x 16 0.297, 768 x 8 0.293, 1024 x 4 0.282)
constexpr int kRadixIT = 8;
constexpr int kRadixThreads = 512;
constexpr int kWaveSpan = 256;                    // records per wave (4 steps of 64)
constexpr int kSpanBlock = WAVES * kWaveSpan;      // records per workgroup

__global__ __launch_bounds__(B) void k_vis_count(const int32_t* __restrict__ n_tiles, int64_t n,
                                                  uint64_t* __restrict__ partial) {
  const int w = threadIdx.x >> 6, lane = lane_id();
  const int64_t begin = (int64_t)blockIdx.x * kSpanBlock + w * kWaveSpan;
  uint32_t c = 0;
#pragma unroll
  for (int it = 0; it < kWaveSpan / 64; ++it) {
    const int64_t idx = begin + it * 64 + lane;
    if (idx < n && n_tiles[idx] > 0) ++c;
  }
  c = wave_sum(c);
  if (lane == 0) partial[(int64_t)blockIdx.x * WAVES + w] = c;
}

// Exclusive scan of nb partial sums in place by one block; the total goes to
// mode 0: hdr->n_vis.  1: hdr->p_total, *num_pairs and hdr->n_pairs (zero
// when the total exceeds capacity).  2: hdr->n_ent (zero when the pairs
// exceed capacity).  3: hdr->n_seg.  4: nowhere.
constexpr int kScanThreads = 1024;

// Chunks of 12288 partials (one chunk for a 1080p frame's 3M records) go
// through LDS: coalesced loads, then each thread scans 12 consecutive values,
// then coalesced stores.  In place; returns the total (to every thread).
__device__ uint64_t scan_in_place(uint64_t* __restrict__ partial, int64_t nb) {
  constexpr int R = 12;
  constexpr int CH = kScanThreads * R;
  constexpr int NW = kScanThreads / 64;
  __shared__ uint64_t s_v[CH];
  __shared__ uint64_t s_w[NW];
  const int tid = threadIdx.x, w = tid >> 6;
  uint64_t carry = 0;
  for (int64_t base = 0; base < nb; base += CH) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = base + r * kScanThreads + tid;
      s_v[r * kScanThreads + tid] = i < nb ? partial[i] : 0;
    }
    __syncthreads();
    uint64_t v[R];
    uint64_t sum = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v[r] = s_v[tid * R + r];
      sum += v[r];
    }
    const uint64_t inc = wave_inclusive_scan(sum);
    if (lane_id() == 63) s_w[w] = inc;
    __syncthreads();
    uint64_t wbase = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const uint64_t x = s_w[i];
      if (i < w) wbase += x;
      tot += x;
    }
    uint64_t run = carry + wbase + inc - sum;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      s_v[tid * R + r] = run;
      run += v[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = base + r * kScanThreads + tid;
      if (i < nb) partial[i] = s_v[r * kScanThreads + tid];
    }
    carry += tot;
    __syncthreads();
  }
  return carry;
}

// One workgroup.  mode 1 with partial2 also scans the entry partials after
// the pair partials (mode 2's result), in the same launch.
// With super_lists the entries, not the pairs, must fit the capacity, and
// num_pairs[1] receives the entry count.
__global__ __launch_bounds__(kScanThreads) void k_scan_partials(uint64_t* __restrict__ partial,
                                                                 int64_t nb, Hdr* __restrict__ hdr,
                                                                 int mode, int64_t capacity,
                                                                 int64_t* __restrict__ num_pairs,
                                                                 uint64_t* __restrict__ partial2 =
                                                                     nullptr,
                                                                 int super_lists = 0) {
  const uint64_t carry = scan_in_place(partial, nb);
  uint64_t carry2 = 0;
  if (partial2) carry2 = scan_in_place(partial2, nb);
  if (threadIdx.x == 0) {
    if (mode == 0) {
      hdr->n_vis = (uint32_t)carry;
    } else if (mode == 1) {
      hdr->p_total = carry;
      hdr->e_total = carry2;
      num_pairs[0] = (int64_t)carry;
      if (super_lists) num_pairs[1] = (int64_t)carry2;
      hdr->n_pairs = carry <= (uint64_t)capacity ? (uint32_t)carry : 0u;
      const bool fits = (super_lists ? carry2 : carry) <= (uint64_t)capacity;
      if (partial2) hdr->n_ent = fits ? (uint32_t)carry2 : 0u;
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
                                                    uint32_t* __restrict__ vals,
                                                    uint2* __restrict__ rid,
                                                    uint32_t* __restrict__ prect) {
  const int w = threadIdx.x >> 6, lane = lane_id();
  const int64_t begin = (int64_t)blockIdx.x * kSpanBlock + w * kWaveSpan;
  if (begin >= n) return;  // per wave; no barriers below
  uint32_t carry = (uint32_t)partial[(int64_t)blockIdx.x * WAVES + w];
  const uint64_t lt = lanemask_lt();
#pragma unroll 4
  for (int it = 0; it < kWaveSpan / 64; ++it) {
    const int64_t idx = begin + it * 64 + lane;
    const bool in = idx < n;
    const bool f = in && n_tiles[idx] > 0;
    const uint64_t bal = __ballot(f);
    uint2 rr = make_uint2(0u, 0u);
    if (f) {
      // depth, rect_x, rect_y: the record's fourth 16-byte quarter
      const float4 q = reinterpret_cast<const float4*>(splats + idx)[3];
      const uint32_t pos = carry + (uint32_t)__popcll(bal & lt);
      keys[pos] = __float_as_uint(q.x);
      vals[pos] = (uint32_t)idx;
      rr = make_uint2(__float_as_uint(q.y), __float_as_uint(q.z));
      prect[pos] = pack_rect8(rr.x, rr.y);
    }
    if (in) rid[idx] = rr;
    carry += (uint32_t)__popcll(bal);
  }
}

// ---- stable LSD radix sort of (u32 key, u32 value) with a device-side count
//
// A radix block of NT threads owns BLK = NT * IT consecutive items; a fixed
// grid loops over the live blocks.  hist layout: [digit][block] with row
// stride `stride`.

// Input items: either [0, *d_count) or (staged, d_count null) the stage
// slots [0, nslots) of which slot j is live when j % 256 < span_cnt[j / 256];
// the staged pass also clears the header's totals for the later kernels.
__device__ __forceinline__ bool radix_item_live(int64_t idx, uint32_t count,
                                                const uint64_t* __restrict__ span_cnt) {
  if (idx >= count) return false;
  return !span_cnt || (uint64_t)(idx & 255) < span_cnt[idx >> 8];
}

// Exclusive scan over the NT threads of a block; returns the prefix and the
// total in `total` (smem: NT / 64 + 1 elements).  Contains barriers.
template <int NT, typename T>
__device__ __forceinline__ T block_scan_nt(T x, T* smem, T& total) {
  constexpr int NW = NT / 64;
  const int w = threadIdx.x >> 6;
  const T inc = wave_inclusive_scan(x);
  if (lane_id() == 63) smem[w] = inc;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const T v = smem[q];
    if (q < w) base += v;
    tot += v;
  }
  __syncthreads();
  total = tot;
  return base + inc - x;
}

template <int IT, int NT>
__global__ __launch_bounds__(NT) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ d_count, int shift,
                                                   int bits, uint32_t* __restrict__ hist,
                                                   int stride,
                                                   const uint64_t* __restrict__ span_cnt = nullptr,
                                                   uint32_t nslots = 0, Hdr* hdr = nullptr) {
  constexpr int BLK = NT * IT;
  constexpr int NW = NT / 64;
  __shared__ uint32_t h[NW][256];
  const int radix = 1 << bits;
  const int w = threadIdx.x >> 6;
  const uint32_t count = d_count ? *d_count : nslots;
  const uint32_t nbl = (uint32_t)(((uint64_t)count + BLK - 1) / BLK);
  const uint32_t mask = (uint32_t)radix - 1u;
  if (hdr && blockIdx.x == 0 && threadIdx.x == 0) {
    hdr->n_pairs = 0;
    hdr->p_total = 0;
    hdr->n_ent = 0;
    hdr->n_seg = 0;
    hdr->e_total = 0;
  }
  for (uint32_t vb = blockIdx.x; vb < nbl; vb += gridDim.x) {
    for (int d = threadIdx.x; d < NW * 256; d += NT) (&h[0][0])[d] = 0;
    __syncthreads();
    const int64_t begin = (int64_t)vb * BLK;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int64_t idx = begin + it * NT + threadIdx.x;
      if (radix_item_live(idx, count, span_cnt))
        atomicAdd(&h[w][(keys[idx] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < radix; d += NT) {
      uint32_t t = 0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) t += h[ww][d];
      hist[(int64_t)d * stride + vb] = t;
    }
    __syncthreads();
  }
}

// One block per digit: exclusive scan of that digit's per-block counts over
// the live blocks, in place (16 consecutive entries per thread); the digit
// total goes to digit_total[d].
// (d_count null: the count is nslots.)
__global__ __launch_bounds__(B) void k_radix_rowscan(uint32_t* __restrict__ hist, int stride,
                                                      const uint32_t* __restrict__ d_count,
                                                      int blk, uint32_t* __restrict__ digit_total,
                                                      uint32_t nslots = 0) {
  constexpr int R = 16;
  __shared__ uint32_t s[WAVES + 1];
  const int nblocks = (int)(((uint64_t)(d_count ? *d_count : nslots) + blk - 1) / blk);
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
// PAY: a second 32-bit value (pin -> pout) moves with each item.
template <int IT, int NT, bool PAY>
__global__ __launch_bounds__(NT) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, const uint32_t* __restrict__ d_count,
    int shift, int bits, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ digit_total, int stride,
    const uint64_t* __restrict__ span_cnt, uint32_t nslots, Hdr* hdr,
    const uint32_t* __restrict__ pin, uint32_t* __restrict__ pout) {
  constexpr int BLK = NT * IT;
  constexpr int NW = NT / 64;
  __shared__ uint32_t s_k[BLK];
  __shared__ uint32_t s_v[BLK];
  __shared__ uint32_t s_p[PAY ? BLK : 1];
  __shared__ uint32_t s_dig[256];     // global start of each digit
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_loc[256];
  __shared__ uint32_t s_w[NW][256];
  __shared__ uint32_t s_tmp[NW + 1];
  const uint32_t count = d_count ? *d_count : nslots;
  const uint32_t nbl = (uint32_t)(((uint64_t)count + BLK - 1) / BLK);
  if (blockIdx.x >= nbl) return;  // uniform per block
  const int radix = 1 << bits;
  const uint32_t mask = (uint32_t)radix - 1u;
  const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
  {
    const uint32_t t = tid < radix ? digit_total[tid] : 0u;
    uint32_t tot;
    const uint32_t ex = block_scan_nt<NT, uint32_t>(t, s_tmp, tot);
    if (tid < radix) s_dig[tid] = ex;
    // a staged pass learns the number of live items here
    if (hdr && blockIdx.x == 0 && tid == 0) hdr->n_vis = tot;
  }
  const uint64_t lt = lanemask_lt();
  for (uint32_t vb = blockIdx.x; vb < nbl; vb += gridDim.x) {
    const int64_t begin = (int64_t)vb * BLK;
    if (tid < radix) s_base[tid] = s_dig[tid] + hist[(int64_t)tid * stride + vb];
    for (int d = tid; d < NW * 256; d += NT) (&s_w[0][0])[d] = 0;
    __syncthreads();

    uint32_t k[IT], v[IT], pl[IT], rank[IT];
    const int64_t wbase = begin + (int64_t)w * 64 * IT;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int64_t idx = wbase + it * 64 + lane;
      const bool live = radix_item_live(idx, count, span_cnt);
      k[it] = live ? kin[idx] : 0u;
      v[it] = live ? vin[idx] : 0u;
      pl[it] = (PAY && live) ? pin[idx] : 0u;
      rank[it] = live ? 0u : 0xffffffffu;  // marks a dead slot until ranked
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const bool valid = rank[it] == 0u;
      const uint32_t d = (k[it] >> shift) & mask;
      uint64_t peers = __ballot(valid);
      for (int b = 0; b < bits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        peers &= bit ? bb : ~bb;
      }
      const uint32_t below = (uint32_t)__popcll(peers & lt);
      const uint32_t before = s_w[w][d];
      rank[it] = valid ? before + below : 0xffffffffu;
      if (valid && below == 0) s_w[w][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();  // s_w complete
    // per digit: wave offsets, block total, block-local digit start
    uint32_t dtot = 0, n_here = 0;
    if (tid < radix) {
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) {
        const uint32_t c = s_w[ww][tid];
        s_w[ww][tid] = dtot;
        dtot += c;
      }
    }
    {
      uint32_t tot;
      const uint32_t ex = block_scan_nt<NT, uint32_t>(tid < radix ? dtot : 0u, s_tmp, tot);
      if (tid < radix) s_loc[tid] = ex;
      n_here = tot;  // live items of the block
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      if (rank[it] != 0xffffffffu) {
        const uint32_t d = (k[it] >> shift) & mask;
        const uint32_t lp = s_loc[d] + s_w[w][d] + rank[it];
        s_k[lp] = k[it];
        s_v[lp] = v[it];
        if (PAY) s_p[lp] = pl[it];
      }
    }
    __syncthreads();
    for (uint32_t j = tid; j < n_here; j += NT) {
      const uint32_t kk = s_k[j];
      const uint32_t d = (kk >> shift) & mask;
      const uint32_t pos = s_base[d] + (j - s_loc[d]);
      kout[pos] = kk;
      vout[pos] = s_v[j];
      if (PAY) pout[pos] = s_p[j];
    }
    __syncthreads();  // LDS is reused by the next block
  }
}

// ---- super-tile entries of the depth-ordered records
// Per record: its clipped rectangle (kept for the emission), pairs (tiles of
// the rectangle) and entries (super-tiles it touches); per-wave sums of both
// over the same wave spans as the compaction.
__global__ __launch_bounds__(B) void k_pair_count(const uint32_t* __restrict__ ids,
                                                   const uint2* __restrict__ rid,
                                                   BinViews views, const Hdr* __restrict__ hdr,
                                                   uint32_t* __restrict__ rx_s,
                                                   uint32_t* __restrict__ ry_s,
                                                   uint64_t* __restrict__ partial,
                                                   uint64_t* __restrict__ partial2) {
  const int w = threadIdx.x >> 6, lane = lane_id();
  const uint32_t nv = hdr->n_vis;
  const int64_t begin = (int64_t)blockIdx.x * kSpanBlock + w * kWaveSpan;
  uint64_t c = 0, q = 0;
  if (begin < nv) {
#pragma unroll 4
    for (int it = 0; it < kWaveSpan / 64; ++it) {
      const int64_t i = begin + it * 64 + lane;
      if (i < nv) {
        const uint32_t id = ids[i];
        const uint2 rr = rid[id];
        const Rect r = rect_of(rr.x, rr.y, views.v[view_of(id, views)]);
        const uint32_t m = st_count(r);
        if (m > 0) c += (uint64_t)(r.x1 - r.x0) * (r.y1 - r.y0);
        rx_s[i] = r.x0 | (r.x1 << 16);
        ry_s[i] = r.y0 | (r.y1 << 16);
        q += m;
      }
    }
  }
  c = wave_sum(c);
  q = wave_sum(q);
  if (lane == 0) {
    partial[(int64_t)blockIdx.x * WAVES + w] = c;
    partial2[(int64_t)blockIdx.x * WAVES + w] = q;
  }
}

// Entry k (row-major over the covered super-tiles) of a record with tile
// rectangle r: key = clipped rectangle << 24 | global super-tile.  For
// k < 2^22 a float quotient estimate is within one of k / sw and is corrected
// once; larger k divide exactly.
__device__ __forceinline__ uint32_t entry_key(const Rect& r, uint32_t k, uint32_t sw, uint32_t sgw,
                                              uint32_t st_base) {
  uint32_t dy;
  if (k < (1u << 22)) {
    dy = (uint32_t)((float)k * __builtin_amdgcn_rcpf((float)sw));
    const int32_t rem = (int32_t)(k - dy * sw);
    if (rem < 0) --dy;
    else if (rem >= (int32_t)sw) ++dy;
  } else {
    dy = k / sw;
  }
  const uint32_t dx = k - dy * sw;
  const uint32_t sx = r.x0 / ST + dx, sy = r.y0 / ST + dy;
  const uint32_t ox = sx * ST, oy = sy * ST;
  const uint32_t clip = (max(r.x0, ox) - ox) | (min(r.x1, ox + ST) - 1u - ox) << 2 |
                        (max(r.y0, oy) - oy) << 4 | (min(r.y1, oy + ST) - 1u - oy) << 6;
  return (clip << kClipShift) | (st_base + sy * sgw + sx);
}

// Order a wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Emit the entries of every depth-ordered record at its offset (exclusive
// scan of entry counts), value = record id.  Each wave handles 64 records at
// a time; their entries form one contiguous output range.  When that range
// fits the wave's LDS map (kStage entries), the map gives each position of
// the range its owning lane, and the wave then writes the range in order, 64
// consecutive entries per store (each lane computing the entry it writes from
// its owner's rectangle).  Otherwise a record with few entries is emitted by
// its own lane and a larger one by the whole wave.  Skipped when the frame
// overflows the pair capacity.
constexpr uint32_t kStage = 1024;
constexpr uint32_t kLaneEntries = 8;

__global__ __launch_bounds__(B) void k_entry_emit(const uint32_t* __restrict__ ids,
                                                   const uint32_t* __restrict__ rx_s,
                                                   const uint32_t* __restrict__ ry_s,
                                                   BinViews views, const Hdr* __restrict__ hdr,
                                                   const uint64_t* __restrict__ partial,
                                                   int64_t capacity, uint32_t* __restrict__ ekeys,
                                                   uint32_t* __restrict__ evals) {
  __shared__ uint8_t s_own[WAVES][kStage];
  const int w = threadIdx.x >> 6, lane = lane_id();
  const uint32_t nv = hdr->n_vis;
  const int64_t begin = (int64_t)blockIdx.x * kSpanBlock + w * kWaveSpan;
  if (begin >= nv || hdr->n_ent == 0) return;  // overflow (or nothing to emit); per wave
  uint64_t carry = partial[(int64_t)blockIdx.x * WAVES + w];
#pragma unroll 1
  for (int it = 0; it < kWaveSpan / 64; ++it) {
    const int64_t i = begin + it * 64 + lane;
    Rect r{0u, 0u, 0u, 0u};
    uint32_t id = 0;
    if (i < nv) {
      id = ids[i];
      const uint32_t rx = rx_s[i], ry = ry_s[i];
      r.x0 = rx & 0xffffu;
      r.x1 = rx >> 16;
      r.y0 = ry & 0xffffu;
      r.y1 = ry >> 16;
    }
    const uint32_t m = st_count(r);
    const uint32_t inc = wave_inclusive_scan(m);
    const uint32_t rel = inc - m;
    const uint64_t base = carry;
    const uint64_t off = base + rel;
    const uint32_t total = __builtin_amdgcn_readlane(inc, 63);
    carry += total;
    uint32_t sgw = 0, stb = 0, sw = 1;
    if (m > 0) {
      const BinView bv = views.v[view_of(id, views)];
      sgw = ((uint32_t)bv.grid_w + ST - 1) / ST;
      stb = (uint32_t)bv.st_base;
      sw = (r.x1 - 1) / ST - r.x0 / ST + 1;
    }
    if (total <= kStage) {
      // owner map: every record with entries marks its first slot with its
      // lane, a prefix max spreads the marks (lane l scans the chunk
      // [l*C, (l+1)*C) after a max-scan of the chunk maxima); then ordered
      // coalesced stores
      for (uint32_t j = lane; j < total; j += 64) s_own[w][j] = 0;
      wave_lds_sync();
      if (m > 0) s_own[w][rel] = (uint8_t)lane;
      wave_lds_sync();
      {
        const uint32_t C = (total + 63) / 64;
        const uint32_t c0 = (uint32_t)lane * C;
        uint32_t run = 0;
        for (uint32_t c = 0; c < C; ++c)
          if (c0 + c < total) run = max(run, (uint32_t)s_own[w][c0 + c]);
        uint32_t inc_max = run;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const uint32_t y = __shfl_up(inc_max, d, 64);
          if (lane >= d) inc_max = max(inc_max, y);
        }
        uint32_t cur = __shfl_up(inc_max, 1, 64);
        if (lane == 0) cur = 0;
        wave_lds_sync();
        for (uint32_t c = 0; c < C; ++c)
          if (c0 + c < total) {
            cur = max(cur, (uint32_t)s_own[w][c0 + c]);
            s_own[w][c0 + c] = (uint8_t)cur;
          }
      }
      wave_lds_sync();
      const uint32_t rxp = r.x0 | (r.x1 << 16), ryp = r.y0 | (r.y1 << 16);
      const uint32_t swg = sw | (sgw << 16);
      for (uint32_t j0 = 0; j0 < total; j0 += 64) {
        const uint32_t j = j0 + (uint32_t)lane;
        const int o = j < total ? (int)s_own[w][j] : 0;
        const uint32_t ro = __shfl(rel, o, 64);
        const uint32_t rxo = __shfl(rxp, o, 64), ryo = __shfl(ryp, o, 64);
        const uint32_t swgo = __shfl(swg, o, 64), stbo = __shfl(stb, o, 64);
        const uint32_t ido = __shfl(id, o, 64);
        if (j < total) {
          const Rect ro_r{rxo & 0xffffu, rxo >> 16, ryo & 0xffffu, ryo >> 16};
          ekeys[base + j] = entry_key(ro_r, j - ro, swgo & 0xffffu, swgo >> 16, stbo);
          evals[base + j] = ido;
        }
      }
      wave_lds_sync();  // map reads finish before the next group's writes
      continue;
    }
    if (m > 0 && m <= kLaneEntries) {
      // row-major walk of the covered super-tiles (no division)
      uint64_t o = off;
      for (uint32_t sy = r.y0 / ST; sy <= (r.y1 - 1) / ST; ++sy) {
        const uint32_t oy = sy * ST;
        const uint32_t cy = (max(r.y0, oy) - oy) << 4 | (min(r.y1, oy + ST) - 1u - oy) << 6;
        for (uint32_t sx = r.x0 / ST; sx <= (r.x1 - 1) / ST; ++sx, ++o) {
          const uint32_t ox = sx * ST;
          const uint32_t clip = cy | (max(r.x0, ox) - ox) | (min(r.x1, ox + ST) - 1u - ox) << 2;
          ekeys[o] = (clip << kClipShift) | (stb + sy * sgw + sx);
          evals[o] = id;
        }
      }
    }
    uint64_t big = __ballot(m > kLaneEntries);
    while (big != 0) {
      const int src = __builtin_ctzll(big);
      big &= big - 1;
      Rect rb;
      rb.x0 = __builtin_amdgcn_readlane(r.x0, src);
      rb.x1 = __builtin_amdgcn_readlane(r.x1, src);
      rb.y0 = __builtin_amdgcn_readlane(r.y0, src);
      rb.y1 = __builtin_amdgcn_readlane(r.y1, src);
      const uint32_t mb = __builtin_amdgcn_readlane(m, src);
      const uint32_t swb = __builtin_amdgcn_readlane(sw, src);
      const uint32_t sgwb = __builtin_amdgcn_readlane(sgw, src);
      const uint32_t stbb = __builtin_amdgcn_readlane(stb, src);
      const uint32_t idb = __builtin_amdgcn_readlane(id, src);
      const uint32_t olo = __builtin_amdgcn_readlane((uint32_t)off, src);
      const uint32_t ohi = __builtin_amdgcn_readlane((uint32_t)(off >> 32), src);
      const uint64_t ob = ((uint64_t)ohi << 32) | olo;
      for (uint32_t k = lane; k < mb; k += 64) {
        ekeys[ob + k] = entry_key(rb, k, swb, sgwb, stbb);
        evals[ob + k] = idb;
      }
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

// ---- one-pass super-tile bucketing (frames with at most kEmitMaxSt
// super-tiles over all views)
//
// The depth-ordered records are cut into blocks of EW waves x kEmitWaveRecs
// records.  k_st_count counts each block's entries per super-tile
// (hist[s][block]) and the frame's pair and entry totals; a row scan over the
// blocks of every super-tile and a scan of the super-tile totals give each
// (super-tile, block) its first slot; k_st_emit then writes every entry
// straight to its slot.  Inside a block, per-wave counts order the waves;
// inside a wave the entries are walked in (record, row-major super-tile)
// order, 64 at a time, and an entry's rank among the step's entries of the
// same super-tile comes from ballots over the super-tile bits.  A record has
// at most one entry per super-tile, so entries of one super-tile keep the
// records' depth order: the lists equal those of the stable radix sort by
// super-tile id.  Each wave takes 64 records (one step) and issues all their
// loads first; many waves per block keep the per-block count table small
// while the chip stays full.  A wave's time grows with its records' entries,
// and the nearest records have hundreds each: short waves keep the slowest
// ones short (measured on a 1080p frame of 3M Gaussians: 256, 128 and 64
// records per wave, bin/sort 0.319, 0.296 and 0.285 ms).
// (Measured: with up to 2048 super-tiles -- eight 720p views -- the one pass
// was slower than the radix passes it replaces, so larger frames take those.)
constexpr int kEmitMaxSt = 512;
constexpr int kEmitWaveRecs = 64;                   // records per wave
constexpr int kEmitSteps = kEmitWaveRecs / 64;
constexpr int kEmitWaves = 16;                      // waves per block
constexpr int kEmitBlock = kEmitWaves * kEmitWaveRecs;  // records per block

// k / d for k < 2^22 (float quotient estimate, corrected once).
__device__ __forceinline__ uint32_t div_small(uint32_t k, uint32_t d) {
  uint32_t q = (uint32_t)((float)k * __builtin_amdgcn_rcpf((float)d));
  const int32_t rem = (int32_t)(k - q * d);
  if (rem < 0) --q;
  else if (rem >= (int32_t)d) ++q;
  return q;
}

// One depth-ordered record: its clipped rectangle, entry count, entry-row
// width, its view's super-tile grid width and first super-tile.
struct EmitRec {
  Rect r;
  uint32_t m, sw, sgw, stb, id;
};

__device__ __forceinline__ EmitRec emit_rec(uint32_t id, uint32_t rx, uint32_t ry,
                                            const BinViews& views) {
  EmitRec e;
  e.id = id;
  e.r = Rect{rx & 0xffffu, rx >> 16, ry & 0xffffu, ry >> 16};
  e.m = st_count(e.r);
  e.sw = 1;
  e.sgw = 0;
  e.stb = 0;
  if (e.m > 0) {
    const BinView bv = views.v[view_of(id, views)];
    e.sgw = ((uint32_t)bv.grid_w + ST - 1) / ST;
    e.stb = (uint32_t)bv.st_base;
    e.sw = (e.r.x1 - 1) / ST - e.r.x0 / ST + 1;
  }
  return e;
}

// The rx / ry words (x0 | x1 << 16, y0 | y1 << 16) of a pack_rect8 value.
__device__ __forceinline__ void unpack_rect8(uint32_t p, uint32_t& rx, uint32_t& ry) {
  rx = (p & 0xffu) | (((p >> 8) & 0xffu) + 1u) << 16;
  ry = ((p >> 16) & 0xffu) | ((p >> 24) + 1u) << 16;
}

__device__ __forceinline__ EmitRec no_rec() {
  EmitRec e{};
  e.sw = 1;
  return e;
}

// Add every record's entries to the LDS counts h[super-tile]: rectangles of
// at most kLaneEntries super-tiles by their own lane, larger ones by the
// whole wave.  Call with the whole wave.
__device__ __forceinline__ void count_entries(const EmitRec& e, uint32_t* h, int lane) {
  if (e.m > 0 && e.m <= kLaneEntries) {
    for (uint32_t sy = e.r.y0 / ST; sy <= (e.r.y1 - 1) / ST; ++sy)
      for (uint32_t sx = e.r.x0 / ST; sx <= (e.r.x1 - 1) / ST; ++sx)
        atomicAdd(&h[e.stb + sy * e.sgw + sx], 1u);
  }
  uint64_t big = __ballot(e.m > kLaneEntries);
  while (big != 0) {
    const int src = __builtin_ctzll(big);
    big &= big - 1;
    const uint32_t mb = __builtin_amdgcn_readlane(e.m, src);
    const uint32_t swb = __builtin_amdgcn_readlane(e.sw, src);
    const uint32_t sgwb = __builtin_amdgcn_readlane(e.sgw, src);
    const uint32_t s0 = __builtin_amdgcn_readlane(
        e.stb + (e.r.y0 / ST) * e.sgw + e.r.x0 / ST, src);
    for (uint32_t k = lane; k < mb; k += 64) {
      const uint32_t dy = div_small(k, swb);
      atomicAdd(&h[s0 + dy * sgwb + (k - dy * swb)], 1u);
    }
  }
}

// Exclusive scan over the NTH threads of a block (NTH / 64 waves); returns
// the prefix and the total in `total`.  Contains barriers.
template <int NTH, typename T>
__device__ __forceinline__ T block_scan_n(T x, T* smem, T& total) {
  constexpr int NW = NTH / 64;
  const int w = threadIdx.x >> 6;
  const T inc = wave_inclusive_scan(x);
  if (lane_id() == 63) smem[w] = inc;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const T s = smem[i];
    if (i < w) base += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return base + inc - x;
}

// Pairs of block b go to ppart[b] (no atomics: same-address device atomics
// from every wave serialise across the chip).  PACKED: the rectangles come
// in depth order with the ids (prect, carried by the depth sort) instead of
// from the id-indexed rid, and rx_s / ry_s are not written.
template <int NST, int EW, bool PACKED>
__global__ __launch_bounds__(EW * 64) void k_st_count(const uint32_t* __restrict__ ids,
                                                       const uint2* __restrict__ rid,
                                                       const uint32_t* __restrict__ prect,
                                                       BinViews views, const Hdr* __restrict__ hdr,
                                                       uint32_t* __restrict__ rx_s,
                                                       uint32_t* __restrict__ ry_s,
                                                       uint32_t* __restrict__ hist, int stride,
                                                       uint64_t* __restrict__ ppart) {
  constexpr int NTH = EW * 64;
  constexpr int EBLK = EW * kEmitWaveRecs;
  __shared__ uint32_t s_h[NST];
  __shared__ uint64_t s_p[EW];
  const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
  const int n_st = (int)views.n_st;
  const uint32_t nv = hdr->n_vis;
  const uint32_t nbl = (nv + EBLK - 1) / EBLK;
  for (uint32_t vb = blockIdx.x; vb < nbl; vb += gridDim.x) {
    for (int t = tid; t < n_st; t += NTH) s_h[t] = 0u;
    // every load of the thread's records first: ids, then their rectangles
    uint32_t id[kEmitSteps];
    uint2 rr[kEmitSteps];
#pragma unroll
    for (int it = 0; it < kEmitSteps; ++it) {
      const int64_t i = (int64_t)vb * EBLK + it * NTH + tid;
      id[it] = i < nv ? ids[i] : 0u;
      if (PACKED) {
        uint32_t rx = 0, ry = 0;
        if (i < nv) unpack_rect8(prect[i], rx, ry);
        rr[it] = make_uint2(rx, ry);
      }
    }
    if (!PACKED) {
#pragma unroll
      for (int it = 0; it < kEmitSteps; ++it) {
        const int64_t i = (int64_t)vb * EBLK + it * NTH + tid;
        rr[it] = i < nv ? rid[id[it]] : make_uint2(0u, 0u);
      }
    }
    __syncthreads();  // s_h cleared
    uint64_t c = 0;  // pairs of this thread's records
#pragma unroll
    for (int it = 0; it < kEmitSteps; ++it) {
      const int64_t i = (int64_t)vb * EBLK + it * NTH + tid;
      EmitRec e = no_rec();
      if (i < nv) {
        const Rect r = rect_of(rr[it].x, rr[it].y, views.v[view_of(id[it], views)]);
        const uint32_t rx = r.x0 | (r.x1 << 16), ry = r.y0 | (r.y1 << 16);
        if (!PACKED) {
          rx_s[i] = rx;
          ry_s[i] = ry;
        }
        e = emit_rec(id[it], rx, ry, views);
        if (e.m > 0) c += (uint64_t)(r.x1 - r.x0) * (r.y1 - r.y0);
      }
      count_entries(e, s_h, lane);
    }
    const uint64_t cw = wave_sum(c);
    if (lane == 0) s_p[w] = cw;
    __syncthreads();
    for (int t = tid; t < n_st; t += NTH) hist[(int64_t)t * stride + vb] = s_h[t];
    if (tid == 0) {
      uint64_t tot = 0;
#pragma unroll
      for (int k = 0; k < EW; ++k) tot += s_p[k];
      ppart[vb] = tot;
    }
    __syncthreads();
  }
}

// Owner map of positions [0, W) of a wave's entry window: every position
// takes the largest lane that marked a position at or before it (lane l
// scans the chunk [l*C, (l+1)*C) after a max-scan of the chunk maxima).
__device__ __forceinline__ void owner_fill(uint8_t* own, uint32_t W, int lane) {
  const uint32_t C = (W + 63) / 64;
  const uint32_t c0 = (uint32_t)lane * C;
  uint32_t run = 0;
  for (uint32_t c = 0; c < C; ++c)
    if (c0 + c < W) run = max(run, (uint32_t)own[c0 + c]);
  uint32_t inc_max = run;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc_max, d, 64);
    if (lane >= d) inc_max = max(inc_max, y);
  }
  uint32_t cur = __shfl_up(inc_max, 1, 64);
  if (lane == 0) cur = 0;
  wave_lds_sync();
  for (uint32_t c = 0; c < C; ++c)
    if (c0 + c < W) {
      cur = max(cur, (uint32_t)own[c0 + c]);
      own[c0 + c] = (uint8_t)cur;
    }
}

// NST: LDS capacity in super-tiles (>= n_st; NBITS = log2 NST bits rank the
// super-tile ids); EW waves per block.  Block 0
// also writes every super-tile range ([0, 0) when empty or when the frame
// overflows the capacity), the counts and the header totals; on overflow no
// entry is written.
template <int NST, int EW, bool PACKED, int NBITS = (NST <= 512 ? 9 : 11)>
__global__ __launch_bounds__(EW * 64) void k_st_emit(const uint32_t* __restrict__ ids,
                                                      const uint32_t* __restrict__ rx_s,
                                                      const uint32_t* __restrict__ ry_s,
                                                      const uint32_t* __restrict__ prect,
                                                      BinViews views, Hdr* __restrict__ hdr,
                                                      const uint32_t* __restrict__ hist,
                                                      int stride,
                                                      const uint32_t* __restrict__ st_total,
                                                      int64_t capacity,
                                                      uint32_t* __restrict__ ekeys,
                                                      uint32_t* __restrict__ evals,
                                                      int32_t* __restrict__ st_range,
                                                      int64_t* __restrict__ num_pairs,
                                                      int super_lists,
                                                      const uint64_t* __restrict__ ppart) {
  constexpr int NTH = EW * 64;
  constexpr int EBLK = EW * kEmitWaveRecs;
  constexpr int PT = (NST + NTH - 1) / NTH;  // super-tiles per thread in the scans
  __shared__ uint32_t s_base[NST];
  __shared__ uint32_t s_w[EW][NST];
  __shared__ uint8_t s_own[EW][kStage];
  __shared__ uint64_t s_tmp[EW + 1];
  const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
  const int n_st = (int)views.n_st;
  const uint32_t nv = hdr->n_vis;
  const uint32_t nbl = (nv + EBLK - 1) / EBLK;
  // the frame's entries (sum of the super-tile totals) and pairs (sum of the
  // per-block partials), and the first slot of every super-tile (exclusive
  // scan of the totals)
  uint64_t tv[PT], start[PT], sum = 0, psum = 0;
#pragma unroll
  for (int r = 0; r < PT; ++r) {
    const int st = tid * PT + r;
    tv[r] = st < n_st ? st_total[st] : 0u;
    sum += tv[r];
  }
  for (uint32_t b = tid; b < nbl; b += NTH) psum += ppart[b];
  uint64_t E, P;
  uint64_t run = block_scan_n<NTH, uint64_t>(sum, s_tmp, E);
  block_scan_n<NTH, uint64_t>(psum, s_tmp, P);
  // the stored lists must fit: entries for super-tile lists, pairs otherwise
  const bool fits = (super_lists ? E : P) <= (uint64_t)capacity;
#pragma unroll
  for (int r = 0; r < PT; ++r) {
    start[r] = run;
    run += tv[r];
  }
  if (blockIdx.x == 0) {
#pragma unroll
    for (int r = 0; r < PT; ++r) {
      const int st = tid * PT + r;
      if (st < n_st) {
        const bool ok = fits && tv[r] > 0;
        st_range[2 * (int64_t)st] = ok ? (int32_t)start[r] : 0;
        st_range[2 * (int64_t)st + 1] = ok ? (int32_t)(start[r] + tv[r]) : 0;
      }
    }
    if (tid == 0) {
      num_pairs[0] = (int64_t)P;
      if (super_lists) num_pairs[1] = (int64_t)E;
      hdr->n_pairs = P <= (uint64_t)capacity ? (uint32_t)P : 0u;
      hdr->n_ent = fits ? (uint32_t)E : 0u;
    }
  }
  if (!fits) return;  // uniform over the grid
  const uint64_t lt = lanemask_lt();
  uint32_t* next = s_w[w];
  uint8_t* own = s_own[w];
  for (uint32_t vb = blockIdx.x; vb < nbl; vb += gridDim.x) {
    const int64_t wbeg = (int64_t)vb * EBLK + w * kEmitWaveRecs;
    // this wave's records (all loads first)
    uint32_t rid_[kEmitSteps], rx[kEmitSteps], ry[kEmitSteps];
#pragma unroll
    for (int st = 0; st < kEmitSteps; ++st) {
      const int64_t i = wbeg + st * 64 + lane;
      const bool in = i < nv;
      rid_[st] = in ? ids[i] : 0u;
      if (PACKED) {
        rx[st] = 0u;
        ry[st] = 0u;
        if (in) unpack_rect8(prect[i], rx[st], ry[st]);
      } else {
        rx[st] = in ? rx_s[i] : 0u;
        ry[st] = in ? ry_s[i] : 0u;
      }
    }
#pragma unroll
    for (int r = 0; r < PT; ++r) {
      const int st = tid * PT + r;
      if (st < n_st) s_base[st] = (uint32_t)start[r] + hist[(int64_t)st * stride + vb];
    }
    for (int t = tid; t < EW * NST; t += NTH) (&s_w[0][0])[t] = 0u;
    __syncthreads();
    // this wave's entries per super-tile (rx = ry = 0: no entries)
#pragma unroll
    for (int st = 0; st < kEmitSteps; ++st)
      count_entries(emit_rec(rid_[st], rx[st], ry[st], views), next, lane);
    __syncthreads();
    // wave w's first slot per super-tile
    for (int st = tid; st < n_st; st += NTH) {
      uint32_t b = s_base[st];
#pragma unroll
      for (int ww = 0; ww < EW; ++ww) {
        const uint32_t c = s_w[ww][st];
        s_w[ww][st] = b;
        b += c;
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int step = 0; step < kEmitSteps; ++step) {
      if (wbeg + step * 64 >= (int64_t)nv) break;  // wave-uniform
      const EmitRec e = emit_rec(rid_[step], rx[step], ry[step], views);
      const uint32_t inc = wave_inclusive_scan(e.m);
      const uint32_t rel = inc - e.m;
      const uint32_t T = __builtin_amdgcn_readlane(inc, 63);
      const uint32_t rxp = e.r.x0 | (e.r.x1 << 16), ryp = e.r.y0 | (e.r.y1 << 16);
      const uint32_t swg = e.sw | (e.sgw << 16);
      for (uint32_t a = 0; a < T; a += kStage) {
        const uint32_t W = min(kStage, T - a);
        for (uint32_t j = lane; j < W; j += 64) own[j] = 0;
        wave_lds_sync();
        if (e.m > 0 && rel < a + W && rel + e.m > a) own[max(rel, a) - a] = (uint8_t)lane;
        wave_lds_sync();
        owner_fill(own, W, lane);
        wave_lds_sync();
        for (uint32_t j0 = 0; j0 < W; j0 += 64) {
          const uint32_t j = j0 + (uint32_t)lane;
          const bool valid = j < W;
          const int o = valid ? (int)own[j] : 0;
          const int o0 = __builtin_amdgcn_readfirstlane(o);
          if (__ballot(valid && o != o0) == 0) {
            // every entry of the chunk belongs to one record: distinct
            // super-tiles, so each lane's rank is 0 and its count 1
            const uint32_t ro = __builtin_amdgcn_readlane(rel, o0);
            const uint32_t rxo = __builtin_amdgcn_readlane(rxp, o0);
            const uint32_t ryo = __builtin_amdgcn_readlane(ryp, o0);
            const uint32_t swgo = __builtin_amdgcn_readlane(swg, o0);
            const uint32_t stbo = __builtin_amdgcn_readlane(e.stb, o0);
            const uint32_t ido = __builtin_amdgcn_readlane(e.id, o0);
            if (valid) {
              const Rect ro_r{rxo & 0xffffu, rxo >> 16, ryo & 0xffffu, ryo >> 16};
              const uint32_t key = entry_key(ro_r, a + j - ro, swgo & 0xffffu, swgo >> 16, stbo);
              const uint32_t st = key & kStMask;
              const uint32_t pos = next[st];
              next[st] = pos + 1u;
              ekeys[pos] = key;
              evals[pos] = ido;
            }
            continue;
          }
          const uint32_t ro = __shfl(rel, o, 64);
          const uint32_t rxo = __shfl(rxp, o, 64), ryo = __shfl(ryp, o, 64);
          const uint32_t swgo = __shfl(swg, o, 64), stbo = __shfl(e.stb, o, 64);
          const uint32_t ido = __shfl(e.id, o, 64);
          uint32_t key = 0, st = 0;
          if (valid) {
            const Rect ro_r{rxo & 0xffffu, rxo >> 16, ryo & 0xffffu, ryo >> 16};
            key = entry_key(ro_r, a + j - ro, swgo & 0xffffu, swgo >> 16, stbo);
            st = key & kStMask;
          }
          // lanes whose super-tile equals this lane's: the AND over the
          // super-tile bits of (ballot of the bit, inverted where this
          // lane's bit is 0)
          uint64_t peers = __ballot(valid);
#pragma unroll
          for (int b = 0; b < NBITS; ++b) {
            const uint64_t bb = __ballot((st >> b) & 1u);
            const uint64_t flip = ((st >> b) & 1u) ? 0ull : ~0ull;
            peers &= bb ^ flip;
          }
          const uint32_t below = (uint32_t)__popcll(peers & lt);
          const uint32_t before = next[st];
          if (valid && below == 0) next[st] = before + (uint32_t)__popcll(peers);
          if (valid) {
            ekeys[before + below] = key;
            evals[before + below] = ido;
          }
        }
        wave_lds_sync();  // map reads finish before the next window's writes
      }
    }
    __syncthreads();  // s_base and s_w are rewritten for the next block
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
                                                 uint4* __restrict__ seg_meta) {
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
      const int32_t lo = st_range[2 * s], hi = st_range[2 * s + 1];
      for (uint32_t k = 0; k < c; ++k) {
        const int32_t a = lo + (int32_t)k * kSegLen;
        seg_meta[first + k] =
            make_uint4((uint32_t)s, (uint32_t)a, (uint32_t)min(hi, a + kSegLen), 0u);
      }
    }
  }
}

// Entries [a, e) of quarter w of a segment, and its super-tile, from the
// segment's record {super-tile, begin, end}.
struct Quarter {
  uint32_t st;
  int32_t a, e;
};

__device__ __forceinline__ Quarter quarter(const uint4& m, int w) {
  Quarter g;
  g.st = m.x;
  const int32_t a = (int32_t)m.y + w * (kSegLen / WAVES);
  g.a = min((int32_t)m.z, a);
  g.e = min((int32_t)m.z, a + kSegLen / WAVES);
  return g;
}

// Per wave quarter of a segment and tile of its super-tile: entries covering
// the tile.  seg_cnt layout: [segment][wave quarter][tile].
__global__ __launch_bounds__(B) void k_seg_tile_count(const Hdr* __restrict__ hdr,
                                                       const uint4* __restrict__ seg_meta,
                                                       const uint32_t* __restrict__ ekeys,
                                                       uint32_t* __restrict__ seg_cnt) {
  const int w = threadIdx.x >> 6, lane = lane_id();
  const uint32_t nseg = hdr->n_seg;
  for (uint32_t seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
    const Quarter g = quarter(seg_meta[seg], w);
    uint32_t mine = 0;  // lane t < 16: count of tile t
    for (int32_t base = g.a; base < g.e; base += 64) {
      const int32_t i = base + lane;
      const bool valid = i < g.e;
      const uint32_t cov = valid ? clip_mask(ekeys[i] >> kClipShift) : 0u;
#pragma unroll
      for (int t = 0; t < ST2; ++t) {
        const uint32_t c = (uint32_t)__popcll(__ballot((cov >> t) & 1u));
        if (lane == t) mine += c;
      }
    }
    if (lane < ST2) seg_cnt[((int64_t)seg * WAVES + w) * ST2 + lane] = mine;
  }
}

// One thread per (super-tile, tile): exclusive prefix of the tile's counts
// over the super-tile's wave quarters in order (in place) and the tile's
// total pair count.
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
  // Quarter counts of four segments at a time are loaded before any is
  // rewritten, so sixteen loads are in flight.
  constexpr int KS = 4, Q = KS * WAVES;
  uint32_t run = 0;
  uint32_t* p = seg_cnt + (int64_t)first * WAVES * ST2 + t;
  uint32_t k = 0;
  for (; k + KS <= ns; k += KS, p += Q * ST2) {
    uint32_t c[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) c[j] = p[j * ST2];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      p[j * ST2] = run;
      run += c[j];
    }
  }
  for (; k < ns; ++k, p += WAVES * ST2) {
    uint32_t c[WAVES];
#pragma unroll
    for (int j = 0; j < WAVES; ++j) c[j] = p[j * ST2];
#pragma unroll
    for (int j = 0; j < WAVES; ++j) {
      p[j * ST2] = run;
      run += c[j];
    }
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

// Write every record id of a wave quarter to its slots.  The next free slot
// of each of the 16 tiles (initially the quarter's base: tile start plus the
// prefix of earlier quarters) is wave-uniform; per 64-entry step the covering
// lanes of tile t take consecutive slots in lane order.  Waves run
// independently.
__global__ __launch_bounds__(B) void k_seg_write(const Hdr* __restrict__ hdr,
                                                  const uint4* __restrict__ seg_meta,
                                                  const uint32_t* __restrict__ ekeys,
                                                  const uint32_t* __restrict__ evals,
                                                  const uint32_t* __restrict__ seg_cnt,
                                                  const uint32_t* __restrict__ tile_start,
                                                  BinViews views, uint32_t* __restrict__ out) {
  const int w = threadIdx.x >> 6, lane = lane_id();
  const uint32_t nseg = hdr->n_seg;
  for (uint32_t seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
    const Quarter g = quarter(seg_meta[seg], w);
    if (g.a >= g.e) continue;  // uniform per wave
    uint32_t start = 0;
    if (lane < ST2) {
      const StLoc L = st_locate(views, g.st);
      const int ix = lane & 3, iy = lane >> 2;
      if (ix < L.nx && iy < L.ny)
        start = tile_start[L.tile0 + iy * L.grid_w + ix] +
                seg_cnt[((int64_t)seg * WAVES + w) * ST2 + lane];
    }
    uint32_t next[ST2];
#pragma unroll
    for (int t = 0; t < ST2; ++t) next[t] = __builtin_amdgcn_readlane(start, t);
    for (int32_t base = g.a; base < g.e; base += 64) {
      const int32_t i = base + lane;
      const bool valid = i < g.e;
      const uint32_t cov = valid ? clip_mask(ekeys[i] >> kClipShift) : 0u;
      const uint32_t id = valid ? evals[i] : 0u;
#pragma unroll
      for (int t = 0; t < ST2; ++t) {
        const bool c = (cov >> t) & 1u;
        const uint64_t bal = __ballot(c);
        if (c) {
          const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
              (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
          out[next[t] + rank] = id;
        }
        next[t] += (uint32_t)__popcll(bal);
      }
    }
  }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t nblocks_for(int64_t n) { return (n + TILE - 1) / TILE; }

int grid_for(int64_t nb) { return (int)std::max<int64_t>(1, std::min<int64_t>(nb, kMaxGrid)); }

// One radix pass over a device-side count of at most max_count items, or
// (span_cnt given, d_count null) over the live slots of a staged input of
// max_count slots; the staged pass also resets the header and sets n_vis.
template <int IT, int NT = kRadixThreads>
hipError_t radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                      const uint32_t* d_count, int64_t max_count, int shift, int bits,
                      uint32_t* hist, uint32_t* digits, hipStream_t stream,
                      const uint64_t* span_cnt = nullptr, Hdr* hdr = nullptr,
                      const uint32_t* pin = nullptr, uint32_t* pout = nullptr) {
  constexpr int BLK = NT * IT;
  const int64_t nb = (max_count + BLK - 1) / BLK;
  if (nb == 0) return hipSuccess;
  const int stride = (int)nb;
  const dim3 grid(grid_for(nb));
  const uint32_t nslots = span_cnt ? (uint32_t)max_count : 0u;
  hipLaunchKernelGGL((k_radix_hist<IT, NT>), grid, dim3(NT), 0, stream, kin, d_count, shift, bits,
                     hist, stride, span_cnt, nslots, hdr);
  hipLaunchKernelGGL(k_radix_rowscan, dim3(1 << bits), dim3(B), 0, stream, hist, stride, d_count,
                     BLK, digits, nslots);
  if (pin)
    hipLaunchKernelGGL((k_radix_scatter<IT, NT, true>), grid, dim3(NT), 0, stream, kin, vin, kout,
                       vout, d_count, shift, bits, hist, digits, stride, span_cnt, nslots, hdr,
                       pin, pout);
  else
    hipLaunchKernelGGL((k_radix_scatter<IT, NT, false>), grid, dim3(NT), 0, stream, kin, vin,
                       kout, vout, d_count, shift, bits, hist, digits, stride, span_cnt, nslots,
                       hdr, nullptr, nullptr);
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
  for (int pass = 0; pass < passes; ++pass) {
    const int src = pass & 1, dst = src ^ 1;
    const int pb = std::min(8, bits - 8 * pass);
    const hipError_t e = radix_pass<ITEMS, B>(k[src], v[src], k[dst], v[dst], d_count, n, 8 * pass,
                                           pb, hist, digits, stream);
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
  const int64_t nb_span = std::max<int64_t>((n_records + kSpanBlock - 1) / kSpanBlock, 1);
  const int64_t rblk = (int64_t)kRadixThreads * kRadixIT;
  // buffer 1 of the depth sort also holds the stage: 256 slots per span of
  // 256 records and view, so up to n_records + 256 * kMaxViewsBin; the first
  // staged pass runs over all of them
  const int64_t stage_slots = n_records + 256 * (int64_t)kMaxViewsBin;
  const int64_t nb_hist = std::max<int64_t>({(stage_slots + rblk - 1) / rblk,
                                             (capacity + rblk - 1) / rblk, 1});
  const int64_t nb_part = std::max<int64_t>(
      {WAVES * nb_span, nblocks_for(p.max_st), nblocks_for(n_tiles_total), 1});
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  p.off_hdr = take(sizeof(Hdr));
  p.off_partial = take(8 * (size_t)nb_part);
  p.off_partial2 = take(8 * WAVES * (size_t)nb_span);
  p.off_dkeys0 = take(4 * (size_t)n_records);
  p.off_dkeys1 = take(4 * (size_t)stage_slots);
  p.off_dvals0 = take(4 * (size_t)n_records);
  p.off_dvals1 = take(4 * (size_t)stage_slots);
  p.off_skeys0 = take(4 * (size_t)capacity);
  p.off_skeys1 = take(4 * (size_t)capacity);
  p.off_svals0 = take(4 * (size_t)capacity);
  p.off_svals1 = 0;  // the second value buffer is the caller's sorted_ids
  // the packed rectangles of the depth sort share rx / ry (the packed path
  // never writes those, the others only after the sort): ry holds the stage
  p.off_rx = take(4 * (size_t)n_records);
  p.off_ry = take(4 * (size_t)stage_slots);
  p.off_prect0 = p.off_rx;
  p.off_prect1 = p.off_ry;
  p.off_rid = take(8 * (size_t)n_records);
  p.off_span = take(8 * ((size_t)(n_records + 255) / 256 + kMaxViewsBin));
  const int64_t nb_emit = (n_records + kEmitBlock - 1) / kEmitBlock;
  p.off_hist = take(4 * std::max<size_t>(256 * (size_t)nb_hist, (size_t)kEmitMaxSt * nb_emit));
  p.off_digits = take(4 * (size_t)kEmitMaxSt);
  p.off_st_range = take(8 * (size_t)p.max_st);
  p.off_st_seg = take(4 * (size_t)p.max_st);
  p.off_seg_st = take(16 * (size_t)p.max_seg);  // per segment {super-tile, begin, end, 0}
  p.off_seg_cnt = take(4 * WAVES * ST2 * (size_t)p.max_seg);
  p.off_tile_cnt = take(4 * (size_t)std::max<int64_t>(n_tiles_total, 1));
  p.off_tile_start = take(4 * (size_t)std::max<int64_t>(n_tiles_total, 1));
  p.total = off;
  return p;
}

BinStage bin_stage_of(const BinSortPlan& p, void* ws, int64_t n) {
  char* base = static_cast<char*>(ws);
  BinStage s;
  s.keys = reinterpret_cast<uint32_t*>(base + p.off_dkeys1);
  s.ids = reinterpret_cast<uint32_t*>(base + p.off_dvals1);
  s.span_count = reinterpret_cast<uint64_t*>(base + p.off_span);
  s.rid = reinterpret_cast<uint2*>(base + p.off_rid);
  s.prect = reinterpret_cast<uint32_t*>(base + p.off_prect1);
  s.n_blocks = (n + 255) / 256;
  return s;
}

hipError_t launch_bin_sort(const BinSortPlan& p, const BinViews& views, const seele_splat* splats,
                           const int32_t* n_tiles, void* ws, uint32_t* sorted_ids,
                           int32_t* tile_ranges, int64_t* num_pairs, hipStream_t stream,
                           bool super, uint32_t* entry_keys, bool staged) {
  char* base = static_cast<char*>(ws);
  auto at = [&](size_t o) { return reinterpret_cast<uint32_t*>(base + o); };
  Hdr* hdr = reinterpret_cast<Hdr*>(base + p.off_hdr);
  uint64_t* partial = reinterpret_cast<uint64_t*>(base + p.off_partial);
  uint64_t* partial2 = reinterpret_cast<uint64_t*>(base + p.off_partial2);
  uint32_t* dk[2] = {at(p.off_dkeys0), at(p.off_dkeys1)};
  uint32_t* dv[2] = {at(p.off_dvals0), at(p.off_dvals1)};
  uint32_t* rx_s = at(p.off_rx);
  uint2* rid = reinterpret_cast<uint2*>(at(p.off_rid));
  uint32_t* ry_s = at(p.off_ry);
  uint32_t* hist = at(p.off_hist);
  uint32_t* digits = at(p.off_digits);
  // super-tile ranges: the caller's array for super-tile lists
  int32_t* st_range = super ? tile_ranges : reinterpret_cast<int32_t*>(base + p.off_st_range);
  uint32_t* st_seg = at(p.off_st_seg);
  uint4* seg_meta = reinterpret_cast<uint4*>(base + p.off_seg_st);
  uint32_t* seg_cnt = at(p.off_seg_cnt);
  uint32_t* tile_cnt = at(p.off_tile_cnt);
  uint32_t* tile_start = at(p.off_tile_start);
  const uint32_t* d_nvis = &hdr->n_vis;
  const uint32_t* d_nent = &hdr->n_ent;
  const int64_t n_st = views.n_st;
  const int64_t TT = p.n_tiles_total;
  hipError_t e;

  const int64_t R = p.n_records;
  const int nbR = (int)((R + kSpanBlock - 1) / kSpanBlock);  // record-span workgroups
  // one-pass super-tile bucketing when the frame has few enough super-tiles
  const bool emit1 = n_st <= kEmitMaxSt;
  // a staged depth sort resets the header in its first pass
  if (!(staged && nbR > 0)) hipLaunchKernelGGL(k_zero_hdr, dim3(1), dim3(64), 0, stream, hdr);
  if (!emit1 && n_st > 0)
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((2 * n_st + 255) / 256)), dim3(256), 0, stream,
                       st_range, 2 * n_st, 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint32_t* ids_sorted = dv[0];
  // The one-pass bucketing on grids of at most 256 x 256 tiles takes each
  // record's rectangle packed into 32 bits along the depth sort (a third
  // value per item) instead of gathering it by id afterwards.
  bool packed = emit1;
  for (int k = 0; k < views.n_views; ++k)
    packed = packed && views.v[k].grid_w <= 256 && views.v[k].grid_h <= 256;
  uint32_t* pr[2] = {at(p.off_prect0), at(p.off_prect1)};
  const uint32_t* prect_sorted = pr[0];
  if (nbR > 0) {
    // 1. visible records with their depth keys, stably sorted by float32
    //    depth bits (4 x 8-bit passes)
    if (staged) {
      // pass 0 reads the live slots of the stage (buffer 1) directly; the
      // passes end in buffer 1
      const BinStage bs = bin_stage_of(p, ws, views.n);
      const int64_t nslots = (int64_t)views.n_views * bs.n_blocks * 256;
      e = radix_pass<kRadixIT>(bs.keys, bs.ids, dk[0], dv[0], nullptr, nslots, 0, 8, hist, digits,
                               stream, bs.span_count, hdr, packed ? bs.prect : nullptr, pr[0]);
      if (e != hipSuccess) return e;
      for (int pass = 1; pass < 4; ++pass) {
        const int src = (pass + 1) & 1, dst = src ^ 1;
        e = radix_pass<kRadixIT>(dk[src], dv[src], dk[dst], dv[dst], d_nvis, R, 8 * pass, 8,
                                 hist, digits, stream, nullptr, nullptr,
                                 packed ? pr[src] : nullptr, pr[dst]);
        if (e != hipSuccess) return e;
      }
      ids_sorted = dv[1];
      prect_sorted = pr[1];
    } else {
      hipLaunchKernelGGL(k_vis_count, dim3(nbR), dim3(B), 0, stream, n_tiles, R, partial);
      hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, stream, partial,
                         WAVES * (int64_t)nbR, hdr, 0, p.capacity, num_pairs);
      hipLaunchKernelGGL(k_vis_compact, dim3(nbR), dim3(B), 0, stream, n_tiles, R, splats,
                         partial, dk[0], dv[0], rid, pr[0]);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      for (int pass = 0; pass < 4; ++pass) {
        const int src = pass & 1, dst = src ^ 1;
        e = radix_pass<kRadixIT>(dk[src], dv[src], dk[dst], dv[dst], d_nvis, R, 8 * pass, 8,
                                 hist, digits, stream, nullptr, nullptr,
                                 packed ? pr[src] : nullptr, pr[dst]);
        if (e != hipSuccess) return e;
      }
    }
  }
  const uint32_t* ekeys;
  const uint32_t* evals;
  if (emit1) {
    // 2. entries per (super-tile, record block), their slots, the emission
    uint32_t* ek = super ? entry_keys : at(p.off_skeys0);
    uint32_t* ev = super ? sorted_ids : at(p.off_svals0);
    const int64_t nbE = std::max<int64_t>((R + kEmitBlock - 1) / kEmitBlock, 1);
    const int stride = (int)nbE;
    const dim3 gridE(grid_for(nbE));
    constexpr int NT = kEmitWaves * 64;
    if (nbR > 0) {
      if (packed)
        hipLaunchKernelGGL((k_st_count<kEmitMaxSt, kEmitWaves, true>), gridE, dim3(NT), 0, stream,
                           ids_sorted, rid, prect_sorted, views, hdr, rx_s, ry_s, hist, stride,
                           partial);
      else
        hipLaunchKernelGGL((k_st_count<kEmitMaxSt, kEmitWaves, false>), gridE, dim3(NT), 0,
                           stream, ids_sorted, rid, nullptr, views, hdr, rx_s, ry_s, hist, stride,
                           partial);
    }
    hipLaunchKernelGGL(k_radix_rowscan, dim3((unsigned)std::max<int64_t>(n_st, 1)), dim3(B), 0,
                       stream, hist, stride, d_nvis, kEmitBlock, digits, 0u);
    if (packed)
      hipLaunchKernelGGL((k_st_emit<kEmitMaxSt, kEmitWaves, true>), gridE, dim3(NT), 0, stream,
                         ids_sorted, rx_s, ry_s, prect_sorted, views, hdr, hist, stride, digits,
                         p.capacity, ek, ev, st_range, num_pairs, super ? 1 : 0, partial);
    else
      hipLaunchKernelGGL((k_st_emit<kEmitMaxSt, kEmitWaves, false>), gridE, dim3(NT), 0, stream,
                         ids_sorted, rx_s, ry_s, nullptr, views, hdr, hist, stride, digits,
                         p.capacity, ek, ev, st_range, num_pairs, super ? 1 : 0, partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    ekeys = ek;
    evals = ev;
  } else {
    // 2. pair and entry totals (pairs -> num_pairs)
    if (nbR > 0)
      hipLaunchKernelGGL(k_pair_count, dim3(nbR), dim3(B), 0, stream, ids_sorted, rid, views, hdr,
                         rx_s, ry_s, partial, partial2);
    // pair partials, then entry partials (whose count depends on the pair
    // total), in one launch
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, stream, partial,
                       WAVES * (int64_t)nbR, hdr, 1, p.capacity, num_pairs, partial2,
                       super ? 1 : 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    //    entries, then sorted by super-tile id (balanced digit widths <= 8).
    //    Per-tile lists: the value buffers alternate between svals0 and
    //    sorted_ids so that the last pass ends in svals0.  Super-tile lists:
    //    keys and values end in the caller's entry_keys and sorted_ids.
    int st_bits = 0;
    while (st_bits < 24 && ((int64_t)1 << st_bits) < n_st) ++st_bits;
    const int passes = std::max(1, (st_bits + 7) / 8);
    const int per = (st_bits + passes - 1) / passes;
    const int fin = passes & 1;  // buffer index the last pass writes
    uint32_t* sk[2] = {at(p.off_skeys0), at(p.off_skeys1)};
    uint32_t* sv[2] = {(passes % 2 == 0) ? at(p.off_svals0) : sorted_ids,
                       (passes % 2 == 0) ? sorted_ids : at(p.off_svals0)};
    if (super) {
      sk[fin] = entry_keys;
      sk[fin ^ 1] = at(p.off_skeys0);
      sv[fin] = sorted_ids;
      sv[fin ^ 1] = at(p.off_svals0);
    }
    if (nbR > 0)
      hipLaunchKernelGGL(k_entry_emit, dim3(nbR), dim3(B), 0, stream, ids_sorted, rx_s, ry_s,
                         views, hdr, partial2, p.capacity, sk[0], sv[0]);
    int shift = 0;
    for (int pass = 0; pass < passes; ++pass) {
      const int src = pass & 1, dst = src ^ 1;
      const int bits = std::min(per, st_bits - shift);
      e = radix_pass<kRadixIT>(sk[src], sv[src], sk[dst], sv[dst], d_nent, p.capacity, shift,
                               bits, hist, digits, stream);
      if (e != hipSuccess) return e;
      shift += bits;
    }
    ekeys = sk[fin];
    evals = sv[fin];
    // 3. super-tile ranges
    if (p.capacity > 0)
      hipLaunchKernelGGL(k_st_ranges, dim3(grid_for((p.capacity + 255) / 256)), dim3(256), 0,
                         stream, ekeys, hdr, st_range);
  }
  // 3. per-tile lists: segments, per-tile counts, tile ranges, write
  if (super) return hipGetLastError();
  const int nbS = (int)nblocks_for(n_st);
  if (nbS > 0) {
    hipLaunchKernelGGL(k_seg_count, dim3(nbS), dim3(B), 0, stream, st_range, n_st, partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, stream, partial,
                       (int64_t)nbS, hdr, 3,
                       p.capacity, num_pairs);
    hipLaunchKernelGGL(k_seg_emit, dim3(nbS), dim3(B), 0, stream, st_range, n_st, partial, st_seg,
                       seg_meta);
  }
  const int seg_grid = grid_for(p.max_seg);
  hipLaunchKernelGGL(k_seg_tile_count, dim3(seg_grid), dim3(B), 0, stream, hdr, seg_meta, ekeys,
                     seg_cnt);
  if (n_st > 0)
    hipLaunchKernelGGL(k_st_tile_prefix, dim3((unsigned)((n_st * ST2 + 255) / 256)), dim3(256), 0,
                       stream, st_range, st_seg, n_st, views, seg_cnt, tile_cnt);
  const int nbT = (int)nblocks_for(TT);
  if (nbT > 0) {
    hipLaunchKernelGGL(k_tile_partials, dim3(nbT), dim3(B), 0, stream, tile_cnt, TT, partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, stream, partial,
                       (int64_t)nbT, hdr, 4,
                       p.capacity, num_pairs);
    hipLaunchKernelGGL(k_tile_ranges, dim3(nbT), dim3(B), 0, stream, tile_cnt, TT, partial, hdr,
                       tile_start, tile_ranges);
  }
  hipLaunchKernelGGL(k_seg_write, dim3(seg_grid), dim3(B), 0, stream, hdr, seg_meta, ekeys, evals,
                     seg_cnt, tile_start, views, sorted_ids);
  return hipGetLastError();
}

}  // namespace seele
