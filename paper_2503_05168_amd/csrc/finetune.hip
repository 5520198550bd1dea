// Fine-tuning kernels (Sec. 3.5): the photometric loss of 3DGS training,
// L = (1 - lambda) L1 + lambda (1 - SSIM), with its gradient with respect to
// the rendered image, and the Adam step over the Gaussian attribute arrays.
//
// SSIM is the mean over pixels and channels of the SSIM map with an 11 x 11
// Gaussian window (sigma 1.5, normalised) under zero padding.  Per pixel and
// channel, from the window moments of the render x and the target y
// (mu_x, mu_y, E[x^2], E[y^2], E[xy]):
//   S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x + s_y + C2)),
// s_x = E[x^2] - mu_x^2, s_y likewise, s_xy = E[xy] - mu_x mu_y.  With the
// partials of S at q with respect to (mu_x, E[x^2], E[xy]) written P1, P2, P3,
// the derivative of the SSIM sum with respect to x_p is
//   (w * P1)(p) + 2 x_p (w * P2)(p) + y_p (w * P3)(p),
// three more window sums (the window is symmetric).  Every window sum is a
// horizontal then a vertical 11-tap pass over a tile staged in LDS with its
// halo; elements of a view are laid out [3][H][W] as the rasterizer writes
// them.
#include <cmath>

#include "finetune_internal.h"

namespace seele {

namespace {

constexpr int kLossBlock = 256;
constexpr int kTap = 11, kHalf = 5;
// one workgroup per (view, channel, 32 x 16 output tile); the tile and its
// 5-pixel halo are staged in LDS and both window passes run there
constexpr int kTX = 32, kTY = 16;
constexpr int kIX = kTX + 2 * kHalf, kIY = kTY + 2 * kHalf;

struct Win {
  float w[kTap];
};

struct TileJob {
  int v, c, x0, y0, W, H;
  int64_t base;  // element index of (v, c, 0, 0)
};

__device__ __forceinline__ TileJob tile_job(const LossViews& lv) {
  TileJob j{};
  int v = 0;
  for (int q = 1; q < lv.n_views; ++q)
    if (lv.blk_off[q] <= (int)blockIdx.x) v = q;
  const int W = lv.w[v], H = lv.h[v];
  const int gx = (W + kTX - 1) / kTX, gy = (H + kTY - 1) / kTY;
  int b = (int)blockIdx.x - lv.blk_off[v];
  j.c = b / (gx * gy);
  b -= j.c * gx * gy;
  j.y0 = (b / gx) * kTY;
  j.x0 = (b % gx) * kTX;
  j.v = v;
  j.W = W;
  j.H = H;
  j.base = lv.elem_off[v] + (int64_t)j.c * W * H;
  return j;
}

// Stage NM maps of the tile plus halo into LDS (zero outside the image).
template <int NM>
__device__ __forceinline__ void stage(const TileJob& j, const float* const* src,
                                      float (*dst)[kIY][kIX]) {
  for (int i = threadIdx.x; i < kIY * kIX; i += kLossBlock) {
    const int r = i / kIX, c = i - r * kIX;
    const int y = j.y0 + r - kHalf, x = j.x0 + c - kHalf;
    float val[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) val[m] = 0.0f;
    if (x >= 0 && x < j.W && y >= 0 && y < j.H) {
      const int64_t o = j.base + (int64_t)y * j.W + x;
#pragma unroll
      for (int m = 0; m < NM; ++m) val[m] = src[m][o];
    }
#pragma unroll
    for (int m = 0; m < NM; ++m) dst[m][r][c] = val[m];
  }
}

// SSIM forward on a tile: the window moments of x and y, the SSIM map and
// its partials (P1, P2, P3) at every in-image pixel; per-block sums of S
// and |x - y|.
__global__ __launch_bounds__(kLossBlock) void k_ssim_fwd(LossViews lv, Win win,
                                                          const float* __restrict__ img,
                                                          const float* __restrict__ tgt,
                                                          float* __restrict__ part, int64_t stride,
                                                          float* __restrict__ blk) {
  __shared__ float s_in[2][kIY][kIX];
  __shared__ float s_h[5][kIY][kTX];
  __shared__ float s_red[2][kLossBlock / 64];
  const TileJob j = tile_job(lv);
  const float* src[2] = {img, tgt};
  stage<2>(j, src, s_in);
  __syncthreads();
  for (int i = threadIdx.x; i < kIY * kTX; i += kLossBlock) {
    const int r = i / kTX, c = i - r * kTX;
    float h0 = 0.f, h1 = 0.f, h2 = 0.f, h3 = 0.f, h4 = 0.f;
#pragma unroll
    for (int t = 0; t < kTap; ++t) {
      const float a = s_in[0][r][c + t], b = s_in[1][r][c + t], w = win.w[t];
      h0 = __builtin_fmaf(w, a, h0);
      h1 = __builtin_fmaf(w, b, h1);
      h2 = __builtin_fmaf(w, a * a, h2);
      h3 = __builtin_fmaf(w, b * b, h3);
      h4 = __builtin_fmaf(w, a * b, h4);
    }
    s_h[0][r][c] = h0;
    s_h[1][r][c] = h1;
    s_h[2][r][c] = h2;
    s_h[3][r][c] = h3;
    s_h[4][r][c] = h4;
  }
  __syncthreads();
  float ssum = 0.f, lsum = 0.f;
  for (int i = threadIdx.x; i < kTY * kTX; i += kLossBlock) {
    const int oy = i / kTX, ox = i - oy * kTX;
    const int y = j.y0 + oy, x = j.x0 + ox;
    if (y >= j.H || x >= j.W) continue;
    float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < kTap; ++t) {
      const float w = win.w[t];
#pragma unroll
      for (int k = 0; k < 5; ++k) m[k] = __builtin_fmaf(w, s_h[k][oy + t][ox], m[k]);
    }
    const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
    const float mx = m[0], my = m[1];
    const float sx = m[2] - mx * mx, sy = m[3] - my * my, sxy = m[4] - mx * my;
    const float a1 = 2.f * mx * my + C1, a2 = 2.f * sxy + C2;
    const float b1 = mx * mx + my * my + C1, b2 = sx + sy + C2;
    // hardware reciprocals (about 1 ulp)
    const float ib1 = __builtin_amdgcn_rcpf(b1), ib2 = __builtin_amdgcn_rcpf(b2);
    const float inv = ib1 * ib2;
    const float S = a1 * a2 * inv;
    const int64_t o = j.base + (int64_t)y * j.W + x;
    part[o] = 2.f * my * (a2 - a1) * inv - 2.f * mx * S * (ib1 - ib2);
    part[stride + o] = -S * ib2;
    part[2 * stride + o] = 2.f * a1 * inv;
    ssum += S;
    lsum += fabsf(s_in[0][oy + kHalf][ox + kHalf] - s_in[1][oy + kHalf][ox + kHalf]);
  }
  const float ws = wave_sum(ssum), wl = wave_sum(lsum);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_red[0][wv] = ws;
    s_red[1][wv] = wl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = 0.f, b = 0.f;
    for (int k = 0; k < kLossBlock / 64; ++k) {
      a += s_red[0][k];
      b += s_red[1][k];
    }
    blk[2 * blockIdx.x] = a;
    blk[2 * blockIdx.x + 1] = b;
  }
}

// SSIM backward on a tile: window sums of the partial maps, then dL/dx.
__global__ __launch_bounds__(kLossBlock) void k_ssim_bwd(LossViews lv, Win win,
                                                          const float* __restrict__ img,
                                                          const float* __restrict__ tgt,
                                                          const float* __restrict__ part,
                                                          int64_t stride, float lambda,
                                                          float inv_views,
                                                          float* __restrict__ grad) {
  __shared__ float s_in[3][kIY][kIX];
  __shared__ float s_h[3][kIY][kTX];
  const TileJob j = tile_job(lv);
  const float* src[3] = {part, part + stride, part + 2 * stride};
  stage<3>(j, src, s_in);
  __syncthreads();
  for (int i = threadIdx.x; i < kIY * kTX; i += kLossBlock) {
    const int r = i / kTX, c = i - r * kTX;
    float h[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < kTap; ++t) {
      const float w = win.w[t];
#pragma unroll
      for (int k = 0; k < 3; ++k) h[k] = __builtin_fmaf(w, s_in[k][r][c + t], h[k]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) s_h[k][r][c] = h[k];
  }
  __syncthreads();
  const float inv_n = inv_views / (3.f * (float)j.W * (float)j.H);
  for (int i = threadIdx.x; i < kTY * kTX; i += kLossBlock) {
    const int oy = i / kTX, ox = i - oy * kTX;
    const int y = j.y0 + oy, x = j.x0 + ox;
    if (y >= j.H || x >= j.W) continue;
    float g[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < kTap; ++t) {
      const float w = win.w[t];
#pragma unroll
      for (int k = 0; k < 3; ++k) g[k] = __builtin_fmaf(w, s_h[k][oy + t][ox], g[k]);
    }
    const int64_t o = j.base + (int64_t)y * j.W + x;
    const float xv = img[o], yv = tgt[o];
    const float d = xv - yv;
    const float sgn = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
    grad[o] = inv_n * ((1.f - lambda) * sgn - lambda * (g[0] + 2.f * xv * g[1] + yv * g[2]));
  }
}

// per view: loss = (1 - lambda) mean|x - y| + lambda (1 - mean S), the block
// sums added in block order
__global__ __launch_bounds__(kLossBlock) void k_loss_reduce(LossViews lv,
                                                             const float* __restrict__ blk,
                                                             float lambda,
                                                             float* __restrict__ loss) {
  __shared__ double s_r[2][kLossBlock / 64];
  const int v = blockIdx.x;
  double s = 0.0, l = 0.0;
  for (int b = lv.blk_off[v] + (int)threadIdx.x; b < lv.blk_off[v + 1]; b += kLossBlock) {
    s += (double)blk[2 * b];
    l += (double)blk[2 * b + 1];
  }
  s = wave_sum(s);
  l = wave_sum(l);
  if ((threadIdx.x & 63) == 0) {
    s_r[0][threadIdx.x >> 6] = s;
    s_r[1][threadIdx.x >> 6] = l;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s = 0.0;
    l = 0.0;
    for (int w = 0; w < kLossBlock / 64; ++w) {
      s += s_r[0][w];
      l += s_r[1][w];
    }
    const double n = 3.0 * (double)lv.w[v] * (double)lv.h[v];
    loss[v] = (float)((1.0 - (double)lambda) * l / n + (double)lambda * (1.0 - s / n));
  }
}

struct AdamSegs {
  float* p[6];
  const float* g[6];
  float* m[6];
  float* v[6];
  int64_t end[6];  // exclusive prefix ends of the segments in the flat index
  float lr[6];
};

__global__ __launch_bounds__(256) void k_adam(AdamSegs a, float b1, float b2, float eps,
                                               float step_scale_1, float inv_sqrt_bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.end[5]) return;
  int s = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) s += i >= a.end[k];
  const int64_t j = i - (s ? a.end[s - 1] : 0);
  const float g = a.g[s][j];
  const float m = b1 * a.m[s][j] + (1.f - b1) * g;
  const float v = b2 * a.v[s][j] + (1.f - b2) * (g * g);
  a.m[s][j] = m;
  a.v[s][j] = v;
  const float denom = sqrtf(v) * inv_sqrt_bc2 + eps;
  a.p[s][j] -= a.lr[s] * step_scale_1 * (m / denom);
}

// the same step four elements at a time (16-byte loads and stores), for
// segments whose lengths are multiples of four and whose arrays are 16-byte
// aligned; `end` counts float4 elements here
__global__ __launch_bounds__(256) void k_adam4(AdamSegs a, float b1, float b2, float eps,
                                                float step_scale_1, float inv_sqrt_bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.end[5]) return;
  int s = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) s += i >= a.end[k];
  const int64_t j = i - (s ? a.end[s - 1] : 0);
  const float4 g = reinterpret_cast<const float4*>(a.g[s])[j];
  float4 m = reinterpret_cast<const float4*>(a.m[s])[j];
  float4 v = reinterpret_cast<const float4*>(a.v[s])[j];
  float4 p = reinterpret_cast<const float4*>(a.p[s])[j];
  const float lr = a.lr[s] * step_scale_1;
  const float gg[4] = {g.x, g.y, g.z, g.w};
  float mm[4] = {m.x, m.y, m.z, m.w}, vv[4] = {v.x, v.y, v.z, v.w}, pp[4] = {p.x, p.y, p.z, p.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    mm[e] = b1 * mm[e] + (1.f - b1) * gg[e];
    vv[e] = b2 * vv[e] + (1.f - b2) * (gg[e] * gg[e]);
    pp[e] -= lr * (mm[e] / (sqrtf(vv[e]) * inv_sqrt_bc2 + eps));
  }
  reinterpret_cast<float4*>(a.m[s])[j] = make_float4(mm[0], mm[1], mm[2], mm[3]);
  reinterpret_cast<float4*>(a.v[s])[j] = make_float4(vv[0], vv[1], vv[2], vv[3]);
  reinterpret_cast<float4*>(a.p[s])[j] = make_float4(pp[0], pp[1], pp[2], pp[3]);
}

}  // namespace

void loss_window(float* w) {
  double g[kTap], s = 0.0;
  for (int k = 0; k < kTap; ++k) {
    const double d = (double)(k - kHalf);
    g[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    s += g[k];
  }
  for (int k = 0; k < kTap; ++k) w[k] = (float)(g[k] / s);
}

int64_t loss_blocks(int w, int h) {
  return 3 * (int64_t)((w + kTX - 1) / kTX) * ((h + kTY - 1) / kTY);
}

hipError_t launch_photometric_loss(const LossViews& lv, int n_blocks, const float* img,
                                   const float* tgt, float lambda, float inv_views, float* maps,
                                   int64_t stride, float* blk, float* loss, float* grad,
                                   hipStream_t stream) {
  Win win;
  loss_window(win.w);
  const dim3 grid((unsigned)n_blocks), block(kLossBlock);
  hipLaunchKernelGGL(k_ssim_fwd, grid, block, 0, stream, lv, win, img, tgt, maps, stride, blk);
  hipLaunchKernelGGL(k_ssim_bwd, grid, block, 0, stream, lv, win, img, tgt, maps, stride, lambda,
                     inv_views, grad);
  hipLaunchKernelGGL(k_loss_reduce, dim3((unsigned)lv.n_views), dim3(kLossBlock), 0, stream, lv,
                     blk, lambda, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* const* p, const float* const* g, float* const* m, float* const* v,
                       const int64_t* len, const float* lr, float b1, float b2, float eps,
                       int64_t step, hipStream_t stream) {
  AdamSegs a{};
  int64_t acc = 0;
  for (int s = 0; s < 6; ++s) {
    a.p[s] = p[s];
    a.g[s] = g[s];
    a.m[s] = m[s];
    a.v[s] = v[s];
    acc += len[s];
    a.end[s] = acc;
    a.lr[s] = lr[s];
  }
  if (acc == 0) return hipSuccess;
  const double bc1 = 1.0 - std::pow((double)b1, (double)step);
  const double bc2 = 1.0 - std::pow((double)b2, (double)step);
  bool vec = true;
  for (int s = 0; s < 6; ++s) {
    vec = vec && len[s] % 4 == 0;
    for (const void* q : {(const void*)p[s], (const void*)g[s], (const void*)m[s],
                          (const void*)v[s]})
      vec = vec && (len[s] == 0 || reinterpret_cast<uintptr_t>(q) % 16 == 0);
  }
  if (vec) {
    for (int s = 0; s < 6; ++s) a.end[s] /= 4;
    hipLaunchKernelGGL(k_adam4, dim3((unsigned)((acc / 4 + 255) / 256)), dim3(256), 0, stream, a,
                       b1, b2, eps, (float)(1.0 / bc1), (float)(1.0 / std::sqrt(bc2)));
  } else {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((acc + 255) / 256)), dim3(256), 0, stream, a, b1,
                       b2, eps, (float)(1.0 / bc1), (float)(1.0 / std::sqrt(bc2)));
  }
  return hipGetLastError();
}

}  // namespace seele
