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
// hist layout: [digit][block]
__global__ __launch_bounds__(B) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ d_count,
                                                   int shift, int bits,
                                                   uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t h[256];
  const int radix = 1 << bits;
  for (int d = threadIdx.x; d < radix; d += B) h[d] = 0;
  __syncthreads();
  const uint32_t count = *d_count;
  const int64_t begin = (int64_t)blockIdx.x * TILE;
  const uint32_t mask = (uint32_t)radix - 1u;
  if (begin < count) {
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const int64_t idx = begin + it * B + threadIdx.x;
      if (idx < count) atomicAdd(&h[(keys[idx] >> shift) & mask], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < radix; d += B) hist[(int64_t)d * nblocks + blockIdx.x] = h[d];
}

// One block per digit: exclusive scan of that digit's per-block counts in
// place; the digit total goes to digit_total[d].
__global__ __launch_bounds__(B) void k_radix_rowscan(uint32_t* __restrict__ hist, int nblocks,
                                                      uint32_t* __restrict__ digit_total) {
  __shared__ uint32_t s[WAVES + 1];
  uint32_t* row = hist + (int64_t)blockIdx.x * nblocks;
  uint32_t carry = 0;
  for (int base = 0; base < nblocks; base += B) {
    const int idx = base + threadIdx.x;
    const uint32_t x = idx < nblocks ? row[idx] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t>(x, s, tot);
    if (idx < nblocks) row[idx] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) digit_total[blockIdx.x] = carry;
}

// Stable scatter.  Block b owns items [b*TILE, (b+1)*TILE); wave w owns the
// contiguous quarter w, processed 64 items at a time in index order.  Within
// a 64-item step a lane's rank among equal digits comes from ballots over the
// digit bits; per-wave running counts in LDS order the steps; per-digit wave
// offsets order the waves.  Final position = digit base + block offset +
// wave offset + rank, which preserves input order among equal digits.
__global__ __launch_bounds__(B) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, const uint32_t* __restrict__ d_count,
    int shift, int bits, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ digit_total, int nblocks) {
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_w[WAVES][256];
  __shared__ uint32_t s_tmp[WAVES + 1];
  const uint32_t count = *d_count;
  const int64_t begin = (int64_t)blockIdx.x * TILE;
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
  __syncthreads();

  uint32_t k[ITEMS], v[ITEMS], rank[ITEMS];
  const int64_t wbase = begin + (int64_t)w * 64 * ITEMS;
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int64_t idx = wbase + it * 64 + lane;
    const bool valid = idx < count;
    k[it] = valid ? kin[idx] : 0u;
    v[it] = valid ? vin[idx] : 0u;
  }
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
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
  __syncthreads();
  if (tid < radix) {
    uint32_t run = 0;
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) {
      const uint32_t c = s_w[ww][tid];
      s_w[ww][tid] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int64_t idx = wbase + it * 64 + lane;
    if (idx < count) {
      const uint32_t d = (k[it] >> shift) & mask;
      const uint32_t pos = s_base[d] + s_w[w][d] + rank[it];
      kout[pos] = k[it];
      vout[pos] = v[it];
    }
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

__global__ __launch_bounds__(B) void k_pair_emit(const uint32_t* __restrict__ ids,
                                                  const int32_t* __restrict__ n_tiles,
                                                  const seele_splat* __restrict__ splats,
                                                  const Hdr* __restrict__ hdr,
                                                  const uint64_t* __restrict__ partial,
                                                  BinViews views, int64_t capacity,
                                                  uint32_t* __restrict__ tile_keys,
                                                  uint32_t* __restrict__ pair_vals) {
  __shared__ uint64_t s[WAVES + 1];
  const uint32_t nv = hdr->n_vis;
  const int64_t begin = (int64_t)blockIdx.x * TILE;
  if (begin >= nv || hdr->p_total > (uint64_t)capacity) return;  // uniform per block
  uint64_t carry = partial[blockIdx.x];
#pragma unroll 1
  for (int it = 0; it < ITEMS; ++it) {
    const int64_t i = begin + it * B + threadIdx.x;
    uint32_t id = 0;
    int32_t c = 0;
    if (i < nv) {
      id = ids[i];
      c = n_tiles[id];
    }
    uint64_t tot;
    const uint64_t off = carry + block_exclusive_scan<uint64_t>((uint64_t)c, s, tot);
    carry += tot;
    if (c > 0) {
      const int v = (int)((int64_t)id / views.n);
      const BinView bv = views.v[v];
      const seele_splat& sp = splats[id];
      const uint32_t x0 = sp.rect_x & 0xffffu, x1 = sp.rect_x >> 16;
      const uint32_t y0 = sp.rect_y & 0xffffu, y1 = sp.rect_y >> 16;
      uint64_t o = off;
      for (uint32_t ty = y0; ty < y1; ++ty) {
        const uint32_t row = (uint32_t)bv.tile_base + ty * (uint32_t)bv.grid_w;
        for (uint32_t tx = x0; tx < x1; ++tx, ++o) {
          tile_keys[o] = row + tx;
          pair_vals[o] = id;
        }
      }
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

hipError_t radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                      const uint32_t* d_count, int64_t max_count, int shift, int bits,
                      uint32_t* hist, uint32_t* digits, hipStream_t stream) {
  const int nb = (int)nblocks_for(max_count);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(B), 0, stream, kin, d_count, shift, bits, hist,
                     nb);
  hipLaunchKernelGGL(k_radix_rowscan, dim3(1 << bits), dim3(B), 0, stream, hist, nb, digits);
  hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(B), 0, stream, kin, vin, kout, vout, d_count,
                     shift, bits, hist, digits, nb);
  return hipGetLastError();
}

}  // namespace

BinSortPlan plan_bin_sort(int64_t n_records, int64_t capacity, int64_t n_tiles_total) {
  BinSortPlan p{};
  p.n_records = n_records;
  p.capacity = capacity;
  p.n_tiles_total = n_tiles_total;
  int bits = 0;
  while (bits < 32 && ((int64_t)1 << bits) < n_tiles_total) ++bits;
  p.tile_bits = bits;
  const int64_t nb_max = std::max<int64_t>(nblocks_for(n_records), nblocks_for(capacity));
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
      e = radix_pass(dk[src], dv[src], dk[dst], dv[dst], d_nvis, R, 8 * pass, 8, hist, digits,
                     stream);
      if (e != hipSuccess) return e;
    }
  }
  // 3. pair offsets in depth order, total -> num_pairs; emission
  const int tile_passes = (p.tile_bits + 7) / 8;
  uint32_t* emit_vals = (tile_passes % 2 == 0) ? sorted_ids : tv_ws;
  if (nbR > 0) {
    hipLaunchKernelGGL(k_pair_count, dim3(nbR), dim3(B), 0, stream, dv[0], n_tiles, hdr, partial);
  }
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(B), 0, stream, partial, (int64_t)nbR, hdr, 1,
                     p.capacity, num_pairs);
  if (nbR > 0) {
    hipLaunchKernelGGL(k_pair_emit, dim3(nbR), dim3(B), 0, stream, dv[0], n_tiles, splats, hdr,
                       partial, views, p.capacity, tk[0], emit_vals);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 4. stable sort by tile id over tile_bits, balanced digit widths <= 8
  int kcur = 0;
  uint32_t* vcur = emit_vals;
  if (tile_passes > 0) {
    const int per = (p.tile_bits + tile_passes - 1) / tile_passes;
    int shift = 0;
    for (int pass = 0; pass < tile_passes; ++pass) {
      const int bits = std::min(per, p.tile_bits - shift);
      uint32_t* vdst = (vcur == sorted_ids) ? tv_ws : sorted_ids;
      e = radix_pass(tk[kcur], vcur, tk[kcur ^ 1], vdst, d_npairs, p.capacity, shift, bits, hist,
                     digits, stream);
      if (e != hipSuccess) return e;
      kcur ^= 1;
      vcur = vdst;
      shift += bits;
    }
  }
  // 5. per-tile ranges
  if (p.capacity > 0)
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)((p.capacity + 255) / 256)), dim3(256), 0,
                       stream, tk[kcur], hdr, tile_ranges);
  return hipGetLastError();
}

}  // namespace seele
