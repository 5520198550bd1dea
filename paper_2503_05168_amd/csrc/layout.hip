// Storage order of a scene for memory locality: Gaussians sorted by the
// Morton code of their means.  Culling, binning and rasterization then read
// spatially coherent runs of the attribute arrays and of the per-record
// splats (a view culls whole regions; a tile's list holds neighbours), so
// fewer cache lines are fetched.  Not a step of the method: a one-time
// layout choice at scene load.
#include <cmath>

#include "layout_internal.h"

namespace seele {

namespace {

constexpr int kLB = 256, kLItems = 8;

__device__ __forceinline__ bool finite3(float x) { return isfinite(x); }

// per-block min / max of the finite mean coordinates
__global__ __launch_bounds__(kLB) void k_bbox_partial(const float* __restrict__ means, int64_t n,
                                                       float* __restrict__ part) {
  __shared__ float s[6][kLB / 64];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  const int64_t base = (int64_t)blockIdx.x * kLB * kLItems + threadIdx.x;
  for (int k = 0; k < kLItems; ++k) {
    const int64_t i = base + (int64_t)k * kLB;
    if (i >= n) break;
    for (int a = 0; a < 3; ++a) {
      const float x = means[a * n + i];
      if (finite3(x)) {
        lo[a] = fminf(lo[a], x);
        hi[a] = fmaxf(hi[a], x);
      }
    }
  }
  for (int a = 0; a < 3; ++a) {
    for (int d = 32; d >= 1; d >>= 1) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], d, 64));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], d, 64));
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 3; ++a) {
      s[a][w] = lo[a];
      s[3 + a][w] = hi[a];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    float v = s[a][0];
    for (int j = 1; j < kLB / 64; ++j) v = a < 3 ? fminf(v, s[a][j]) : fmaxf(v, s[a][j]);
    part[(int64_t)blockIdx.x * 6 + a] = v;
  }
}

// the box and the per-axis scale 1024 / (hi - lo) (0 for an empty or flat axis)
__global__ void k_bbox_final(const float* __restrict__ part, int nb, float* __restrict__ box) {
  if (threadIdx.x >= 3) return;
  const int a = threadIdx.x;
  float lo = INFINITY, hi = -INFINITY;
  for (int b = 0; b < nb; ++b) {
    lo = fminf(lo, part[b * 6 + a]);
    hi = fmaxf(hi, part[b * 6 + 3 + a]);
  }
  const float ext = hi - lo;
  box[a] = lo;
  box[3 + a] = (lo <= hi && ext > 0.0f && isfinite(ext)) ? 1024.0f / ext : 0.0f;
}

__device__ __forceinline__ uint32_t spread10(uint32_t x) {
  x &= 0x3FFu;
  x = (x | (x << 16)) & 0x30000FFu;
  x = (x | (x << 8)) & 0x300F00Fu;
  x = (x | (x << 4)) & 0x30C30C3u;
  x = (x | (x << 2)) & 0x9249249u;
  return x;
}

__global__ __launch_bounds__(kLB) void k_morton(const float* __restrict__ means, int64_t n,
                                                 const float* __restrict__ box,
                                                 uint32_t* __restrict__ keys,
                                                 uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kLB + threadIdx.x;
  if (i >= n) return;
  uint32_t code = 0;
  for (int a = 0; a < 3; ++a) {
    const float x = means[a * n + i];
    uint32_t q = 1023u;
    if (finite3(x)) {
      const float t = (x - box[a]) * box[3 + a];
      q = t >= 1023.0f ? 1023u : (uint32_t)t;  // t >= 0 for finite x
    }
    code |= spread10(q) << a;
  }
  keys[i] = code;
  vals[i] = (uint32_t)i;
}

__global__ __launch_bounds__(kLB) void k_perm_out(const uint32_t* __restrict__ vals, int64_t n,
                                                   int64_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * kLB + threadIdx.x;
  if (i < n) perm[i] = (int64_t)vals[i];
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t spatial_order_workspace_size(int64_t n) {
  const int64_t nb = (n + kLB * kLItems - 1) / (kLB * kLItems);
  return 2 * align256(4 * (size_t)std::max<int64_t>(n, 1)) + align256(24 * (size_t)std::max<int64_t>(nb, 1)) +
         align256(32) + radix_sort_workspace_size(n);
}

hipError_t launch_spatial_order(const float* means, int64_t n, void* ws, int64_t* perm,
                                hipStream_t stream) {
  char* b = static_cast<char*>(ws);
  const int64_t nb = (n + kLB * kLItems - 1) / (kLB * kLItems);
  uint32_t* keys = reinterpret_cast<uint32_t*>(b);
  b += align256(4 * (size_t)n);
  uint32_t* vals = reinterpret_cast<uint32_t*>(b);
  b += align256(4 * (size_t)n);
  float* part = reinterpret_cast<float*>(b);
  b += align256(24 * (size_t)nb);
  float* box = reinterpret_cast<float*>(b);
  b += align256(32);
  hipLaunchKernelGGL(k_bbox_partial, dim3((unsigned)nb), dim3(kLB), 0, stream, means, n, part);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, stream, part, (int)nb, box);
  const unsigned g = (unsigned)((n + kLB - 1) / kLB);
  hipLaunchKernelGGL(k_morton, dim3(g), dim3(kLB), 0, stream, means, n, box, keys, vals);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = radix_sort_pairs(keys, vals, n, 30, b, stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_perm_out, dim3(g), dim3(kLB), 0, stream, vals, n, perm);
  return hipGetLastError();
}

}  // namespace seele
