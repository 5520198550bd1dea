// Tile binning and per-tile depth order on gfx950 (Sec. 3.1 "Preprocessing"
// finds Gaussian-tile intersections, "Sorting" orders each tile's Gaussians
// from the closest to the furthest).
//
// The required order is lexicographic in (global tile, float32 depth bits,
// record id).  Instead of sorting 64-bit (tile, depth) keys for every pair,
// the visible records are first sorted by depth alone (4 stable 8-bit LSD
// passes over N_vis records, input in id order so ties stay in id order),
// then pairs are emitted in that order and stably sorted by tile id over only
// the ceil(log2(tiles)) bits it needs (2 passes for a 1080p frame).  Stability
// of both sorts makes the result exactly the lexicographic order.
//
// Every count (visible records, pairs) stays on the device: grids are sized
// for the maximum and blocks past the live count exit, so the whole stage can
// be captured in a graph and never synchronises with the host.
#include "seele_internal.h"

namespace seele {

namespace {

constexpr int B = kSortBlock;
constexpr int ITEMS = kSortItems;
constexpr int TILE = kSortTile;
constexpr int WAVES = B / 64;

struct Hdr {
  uint32_t n_vis;      // visible records
  uint32_t n_pairs;    // pairs to sort: P if P <= capacity, else 0
  uint64_t p_total;    // pairs the frame needs
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
  }
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

// Exclusive scan of nb partial sums in place by one block; writes the total.
// mode 0: total -> hdr->n_vis.  mode 1: total -> hdr->p_total, *num_pairs and
// hdr->n_pairs (zero when the total exceeds capacity).
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
    } else {
      hdr->p_total = carry;
      *num_pairs = (int64_t)carry;
      hdr->n_pairs = carry <= (uint64_t)capacity ? (uint32_t)carry : 0u;
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
// from arrays (LOAD) or are generated on the fly as the depth-ordered
// Gaussian-tile pairs [b*BLK, (b+1)*BLK) (GEN: the pair emission fused into
// the first tile pass, so the pairs are never written unsorted).
// hist layout: [digit][block].

constexpr int kGenIT = 8;                 // GEN blocks hold 2048 pairs
constexpr int kGenBlk = B * kGenIT;

struct GenSrc {
  const uint32_t* ids;          // depth-ordered visible records
  const seele_splat* splats;
  const uint32_t* goff;         // first pair of each depth-ordered record
  const uint32_t* block_first;  // record holding the first pair of each GEN block
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

// Stage the records covering pairs [S, S + BLK) in LDS (first pair, id, global
// tile of the rectangle's top-left corner, rectangle width | grid width << 16;
// W <= BLK + 1 records) and map every position of the block to its record:
// each record marks the block position of its first pair, and an inclusive
// max-scan spreads the marks over the record's pairs.
template <int IT>
__device__ __forceinline__ void gen_window(const GenSrc& g, const BinViews& views, uint32_t blk,
                                           uint32_t nblk, uint32_t* s_off, uint32_t* s_id,
                                           uint32_t* s_t0, uint32_t* s_wg, uint32_t* s_rec,
                                           uint32_t* s_tmp) {
  constexpr int BLK = B * IT;
  const uint32_t nv = g.hdr->n_vis;
  const uint32_t S = blk * (uint32_t)BLK;
  const uint32_t g_lo = g.block_first[blk];
  const uint32_t g_hi = blk + 1 < nblk ? g.block_first[blk + 1] : nv - 1;
  const int W = (int)(g_hi - g_lo + 1);
  const uint32_t n = (uint32_t)views.n;
  for (int j = threadIdx.x; j < BLK; j += B) s_rec[j] = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < W; j += B) {
    const uint32_t id = g.ids[g_lo + j];
    const uint32_t o = g.goff[g_lo + j];
    const uint32_t rx = g.splats[id].rect_x, ry = g.splats[id].rect_y;
    const BinView bv = views.v[id / n];
    const uint32_t x0 = rx & 0xffffu, y0 = ry & 0xffffu;
    s_off[j] = o;
    s_id[j] = id;
    s_t0[j] = (uint32_t)bv.tile_base + y0 * (uint32_t)bv.grid_w + x0;
    s_wg[j] = ((rx >> 16) - x0) | ((uint32_t)bv.grid_w << 16);
    if (j > 0 && o - S < (uint32_t)BLK) s_rec[o - S] = (uint32_t)j;
  }
  __syncthreads();
  block_inclusive_max<IT>(s_rec, s_tmp);
}

// Pair at block position p (global position q).
__device__ __forceinline__ void gen_pair(uint32_t q, uint32_t p, const uint32_t* s_off,
                                         const uint32_t* s_id, const uint32_t* s_t0,
                                         const uint32_t* s_wg, const uint32_t* s_rec,
                                         uint32_t& key, uint32_t& val) {
  const uint32_t j = s_rec[p];
  const uint32_t k = q - s_off[j];
  const uint32_t wg = s_wg[j];
  const uint32_t w = wg & 0xffffu;
  const uint32_t dy = div_small(k, w);
  key = s_t0[j] + dy * (wg >> 16) + (k - dy * w);
  val = s_id[j];
}

template <int IT, bool GEN>
__global__ __launch_bounds__(B) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ d_count,
                                                   GenSrc gs, BinViews views, int shift,
                                                   int bits, uint32_t* __restrict__ hist,
                                                   int nblocks) {
  constexpr int BLK = B * IT;
  constexpr int kWin = GEN ? 5 * (BLK + 1) : 1;
  __shared__ uint32_t h[WAVES][256];
  __shared__ uint32_t s_win[kWin];
  __shared__ uint32_t s_tmp[WAVES + 1];
  const int radix = 1 << bits;
  const int w = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < WAVES * 256; d += B) (&h[0][0])[d] = 0;
  const uint32_t count = *d_count;
  const int64_t begin = (int64_t)blockIdx.x * BLK;
  const uint32_t mask = (uint32_t)radix - 1u;
  uint32_t* s_off = s_win;
  uint32_t* s_id = s_win + (BLK + 1);
  uint32_t* s_t0 = s_win + 2 * (BLK + 1);
  uint32_t* s_wg = s_win + 3 * (BLK + 1);
  uint32_t* s_rec = s_win + 4 * (BLK + 1);
  if (GEN && begin < count) {
    const uint32_t nblk = (count + BLK - 1) / BLK;
    gen_window<IT>(gs, views, blockIdx.x, nblk, s_off, s_id, s_t0, s_wg, s_rec, s_tmp);
  }
  __syncthreads();
  if (begin < count) {
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const uint32_t p = it * B + threadIdx.x;
      const int64_t idx = begin + p;
      if (idx < count) {
        uint32_t k, v;
        if (GEN)
          gen_pair((uint32_t)idx, p, s_off, s_id, s_t0, s_wg, s_rec, k, v);
        else
          k = keys[idx];
        atomicAdd(&h[w][(k >> shift) & mask], 1u);
      }
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < radix; d += B) {
    uint32_t t = 0;
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) t += h[ww][d];
    hist[(int64_t)d * nblocks + blockIdx.x] = t;
  }
}

// One block per digit: exclusive scan of that digit's per-block counts in
// place (16 consecutive entries per thread); the digit total goes to
// digit_total[d].
__global__ __launch_bounds__(B) void k_radix_rowscan(uint32_t* __restrict__ hist, int nblocks,
                                                      uint32_t* __restrict__ digit_total) {
  constexpr int R = 16;
  __shared__ uint32_t s[WAVES + 1];
  uint32_t* row = hist + (int64_t)blockIdx.x * nblocks;
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
    const uint32_t* __restrict__ digit_total, int nblocks) {
  constexpr int BLK = B * IT;
  constexpr int kWords = GEN ? 5 * (BLK + 1) : 2 * BLK;
  __shared__ uint32_t s_mem[kWords];  // GEN window, then the staged (key, value) pairs
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_loc[256];
  __shared__ uint32_t s_w[WAVES][256];
  __shared__ uint32_t s_tmp[WAVES + 1];
  const uint32_t count = *d_count;
  const int64_t begin = (int64_t)blockIdx.x * BLK;
  if (begin >= count) return;  // uniform per block
  const int radix = 1 << bits;
  const uint32_t mask = (uint32_t)radix - 1u;
  const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();

  // digit bases: exclusive scan over digit totals (radix <= 256 == B)
  {
    const uint32_t t = tid < radix ? digit_total[tid] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t>(t, s_tmp, tot);
    if (tid < radix) s_base[tid] = ex + hist[(int64_t)tid * nblocks + blockIdx.x];
  }
  for (int d = tid; d < WAVES * 256; d += B) (&s_w[0][0])[d] = 0;
  if (GEN) {
    const uint32_t nblk = (count + BLK - 1) / BLK;
    gen_window<IT>(gs, views, blockIdx.x, nblk, s_mem, s_mem + (BLK + 1), s_mem + 2 * (BLK + 1),
                   s_mem + 3 * (BLK + 1), s_mem + 4 * (BLK + 1), s_tmp);
  }
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
        gen_pair((uint32_t)idx, (uint32_t)(idx - begin), s_mem, s_mem + (BLK + 1),
                 s_mem + 2 * (BLK + 1), s_mem + 3 * (BLK + 1), s_mem + 4 * (BLK + 1), k[it],
                 v[it]);
      else {
        k[it] = kin[idx];
        v[it] = vin[idx];
      }
    }
  }
  const uint64_t lt = lanemask_lt();
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
    if (kout) kout[pos] = kk;
    vout[pos] = s_v[j];
  }
}

// ---- pair emission in depth order
__global__ __launch_bounds__(B) void k_pair_count(const uint32_t* __restrict__ ids,
                                                   const int32_t* __restrict__ n_tiles,
                                                   const Hdr* __restrict__ hdr,
                                                   uint64_t* __restrict__ partial) {
  const uint32_t nv = hdr->n_vis;
  const int64_t begin = (int64_t)blockIdx.x * TILE;
  uint64_t c = 0;
  if (begin < nv) {
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const int64_t i = begin + it * B + threadIdx.x;
      if (i < nv) c += (uint64_t)n_tiles[ids[i]];
    }
  }
  __shared__ uint64_t s[WAVES];
  c = wave_sum(c);
  if (lane_id() == 0) s[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < WAVES; ++w) t += s[w];
    partial[blockIdx.x] = t;
  }
}

// Per-record pair offsets in depth order (exclusive scan of tile counts), and
// for every output block of kEmitBlock pairs the record holding its first
// pair.  Skipped when the frame overflows the pair capacity.
constexpr int kEmitBlock = kGenBlk;

__global__ __launch_bounds__(B) void k_pair_offsets(const uint32_t* __restrict__ ids,
                                                     const int32_t* __restrict__ n_tiles,
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
    const uint32_t c = i < nv ? (uint32_t)n_tiles[ids[i]] : 0u;
    uint64_t tot;
    const uint64_t off = carry + block_exclusive_scan<uint64_t>((uint64_t)c, s, tot);
    carry += tot;
    if (i < nv) {
      goff[i] = (uint32_t)off;
      // output blocks whose first pair belongs to this record
      for (uint64_t b = (off + kEmitBlock - 1) / kEmitBlock; b * kEmitBlock < off + c; ++b)
        block_first[b] = (uint32_t)i;
    }
  }
}

__global__ void k_tile_ranges(const uint32_t* __restrict__ keys, const Hdr* __restrict__ hdr,
                              int32_t* __restrict__ ranges) {
  const uint32_t cnt = hdr->n_pairs;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const uint32_t t = keys[i];
  if (i == 0 || keys[i - 1] != t) ranges[2 * (int64_t)t] = (int32_t)i;
  if (i == (int64_t)cnt - 1 || keys[i + 1] != t) ranges[2 * (int64_t)t + 1] = (int32_t)(i + 1);
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t nblocks_for(int64_t n) { return (n + TILE - 1) / TILE; }
int64_t gen_blocks_for(int64_t n) { return (n + kGenBlk - 1) / kGenBlk; }

template <int IT, bool GEN>
hipError_t radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                      const uint32_t* d_count, int64_t max_count, const GenSrc& gs,
                      const BinViews& views, int shift, int bits, uint32_t* hist,
                      uint32_t* digits, hipStream_t stream) {
  constexpr int BLK = B * IT;
  const int nb = (int)((max_count + BLK - 1) / BLK);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL((k_radix_hist<IT, GEN>), dim3(nb), dim3(B), 0, stream, kin, d_count, gs,
                     views, shift, bits, hist, nb);
  hipLaunchKernelGGL(k_radix_rowscan, dim3(1 << bits), dim3(B), 0, stream, hist, nb, digits);
  hipLaunchKernelGGL((k_radix_scatter<IT, GEN>), dim3(nb), dim3(B), 0, stream, kin, vin, kout,
                     vout, d_count, gs, views, shift, bits, hist, digits, nb);
  return hipGetLastError();
}

__global__ void k_set_count(uint32_t* d_count, uint32_t n) {
  if (threadIdx.x == 0) *d_count = n;
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
  int bits = 0;
  while (bits < 32 && ((int64_t)1 << bits) < n_tiles_total) ++bits;
  p.tile_bits = bits;
  const int64_t nb_max = std::max<int64_t>(nblocks_for(n_records), gen_blocks_for(capacity));
  size_t off = 0;
  p.off_hdr = off;
  off = align_up(off + sizeof(Hdr));
  p.off_partial = off;
  off = align_up(off + sizeof(uint64_t) * (size_t)std::max<int64_t>(nb_max, 1));
  p.off_dkeys0 = off;
  off = align_up(off + 4 * (size_t)n_records);
  p.off_dkeys1 = off;
  off = align_up(off + 4 * (size_t)n_records);
  p.off_dvals0 = off;
  off = align_up(off + 4 * (size_t)n_records);
  p.off_dvals1 = off;
  off = align_up(off + 4 * (size_t)n_records);
  p.off_tkeys0 = off;
  off = align_up(off + 4 * (size_t)capacity);
  p.off_tkeys1 = off;
  off = align_up(off + 4 * (size_t)capacity);
  p.off_tvals = off;
  off = align_up(off + 4 * (size_t)capacity);
  p.off_goff = off;
  off = align_up(off + 4 * (size_t)n_records);
  p.off_bfirst = off;
  off = align_up(off + 4 * (size_t)(capacity / kEmitBlock + 2));
  p.off_hist = off;
  off = align_up(off + 4 * (size_t)256 * (size_t)std::max<int64_t>(nb_max, 1));
  p.off_digits = off;
  off = align_up(off + 4 * 256);
  p.total = off;
  return p;
}

hipError_t launch_bin_sort(const BinSortPlan& p, const BinViews& views, const seele_splat* splats,
                           const int32_t* n_tiles, void* ws, uint32_t* sorted_ids,
                           int32_t* tile_ranges, int64_t* num_pairs, hipStream_t stream) {
  char* base = static_cast<char*>(ws);
  Hdr* hdr = reinterpret_cast<Hdr*>(base + p.off_hdr);
  uint64_t* partial = reinterpret_cast<uint64_t*>(base + p.off_partial);
  uint32_t* dk[2] = {reinterpret_cast<uint32_t*>(base + p.off_dkeys0),
                     reinterpret_cast<uint32_t*>(base + p.off_dkeys1)};
  uint32_t* dv[2] = {reinterpret_cast<uint32_t*>(base + p.off_dvals0),
                     reinterpret_cast<uint32_t*>(base + p.off_dvals1)};
  uint32_t* tk[2] = {reinterpret_cast<uint32_t*>(base + p.off_tkeys0),
                     reinterpret_cast<uint32_t*>(base + p.off_tkeys1)};
  uint32_t* tv_ws = reinterpret_cast<uint32_t*>(base + p.off_tvals);
  uint32_t* hist = reinterpret_cast<uint32_t*>(base + p.off_hist);
  uint32_t* goff = reinterpret_cast<uint32_t*>(base + p.off_goff);
  uint32_t* bfirst = reinterpret_cast<uint32_t*>(base + p.off_bfirst);
  uint32_t* digits = reinterpret_cast<uint32_t*>(base + p.off_digits);
  const uint32_t* d_nvis = &hdr->n_vis;
  const uint32_t* d_npairs = &hdr->n_pairs;

  hipLaunchKernelGGL(k_zero_hdr, dim3(1), dim3(64), 0, stream, hdr);
  const int64_t nr2 = 2 * p.n_tiles_total;
  if (nr2 > 0)
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((nr2 + 255) / 256)), dim3(256), 0, stream,
                       tile_ranges, nr2, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
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
    // 2. stable sort by float32 depth bits (4 x 8-bit passes, ends in buffer 0)
    for (int pass = 0; pass < 4; ++pass) {
      const int src = pass & 1, dst = src ^ 1;
      e = radix_pass<ITEMS, false>(dk[src], dv[src], dk[dst], dv[dst], d_nvis, R, GenSrc{}, views,
                                   8 * pass, 8, hist, digits, stream);
      if (e != hipSuccess) return e;
    }
  }
  // 3. pair offsets in depth order, total -> num_pairs
  if (nbR > 0) {
    hipLaunchKernelGGL(k_pair_count, dim3(nbR), dim3(B), 0, stream, dv[0], n_tiles, hdr, partial);
  }
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(B), 0, stream, partial, (int64_t)nbR, hdr, 1,
                     p.capacity, num_pairs);
  if (nbR > 0) {
    hipLaunchKernelGGL(k_pair_offsets, dim3(nbR), dim3(B), 0, stream, dv[0], n_tiles, hdr,
                       partial, p.capacity, goff, bfirst);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 4. stable sort by tile id over tile_bits (balanced digit widths <= 8); the
  //    first pass generates the pairs from the depth-ordered records
  const int tile_passes = std::max(1, (p.tile_bits + 7) / 8);
  const int per = (p.tile_bits + tile_passes - 1) / tile_passes;
  uint32_t* vcur = (tile_passes % 2 == 1) ? sorted_ids : tv_ws;
  int kcur = 0;
  int shift = std::min(per, p.tile_bits);
  {
    const GenSrc gs{dv[0], splats, goff, bfirst, hdr};
    e = radix_pass<kGenIT, true>(nullptr, nullptr, tk[0], vcur, d_npairs, p.capacity, gs, views, 0,
                                 shift, hist, digits, stream);
    if (e != hipSuccess) return e;
  }
  for (int pass = 1; pass < tile_passes; ++pass) {
    const int bits = std::min(per, p.tile_bits - shift);
    uint32_t* vdst = (vcur == sorted_ids) ? tv_ws : sorted_ids;
    e = radix_pass<ITEMS, false>(tk[kcur], vcur, tk[kcur ^ 1], vdst, d_npairs, p.capacity,
                                 GenSrc{}, views, shift, bits, hist, digits, stream);
    if (e != hipSuccess) return e;
    kcur ^= 1;
    vcur = vdst;
    shift += bits;
  }
  // 5. per-tile ranges
  if (p.capacity > 0)
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)((p.capacity + 255) / 256)), dim3(256), 0,
                       stream, tk[kcur], hdr, tile_ranges);
  return hipGetLastError();
}

}  // namespace seele
