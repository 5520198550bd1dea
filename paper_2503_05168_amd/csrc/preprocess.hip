// Per-view preprocessing on gfx950 (Sec. 3.1 "Preprocessing"; EWA screen-space
// covariance behind Eq. 2; opacity-aware extent of Sec. 3.3, Eqs. 3-5).
//
// One lane per Gaussian.  The SoA attribute arrays are read coalesced; the
// Gaussian's activations (3D covariance, opacity) are computed once and reused
// for every view of the launch, and the 48 SH coefficients are read only if the
// Gaussian is visible in some view.  Output is one 48-byte record per (view,
// Gaussian) plus its tile count.  HBM-bound: 44 B of geometry/opacity read and
// 4 B of tile count written per active Gaussian, plus 192 B of SH read and
// 48 B written per visible one.
#include "seele_internal.h"

namespace seele {

namespace {

// Real SH basis (Condon-Shortley phase), degree <= 3, index l*l + l + m.
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[0] = 0.28209479177387814f;
  Y[1] = -0.48860251190291987f * y;
  Y[2] = 0.48860251190291987f * z;
  Y[3] = -0.48860251190291987f * x;
  Y[4] = 1.0925484305920792f * x * y;
  Y[5] = -1.0925484305920792f * y * z;
  Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
  Y[7] = -1.0925484305920792f * x * z;
  Y[8] = 0.54627421529603959f * (xx - yy);
  Y[9] = -0.59004358992664352f * y * (3.0f * xx - yy);
  Y[10] = 2.8906114426405538f * x * y * z;
  Y[11] = -0.45704579946446572f * y * (4.0f * zz - xx - yy);
  Y[12] = 0.37317633259011540f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = -0.45704579946446572f * x * (4.0f * zz - xx - yy);
  Y[14] = 1.4453057213202769f * z * (xx - yy);
  Y[15] = -0.59004358992664352f * x * (xx - 3.0f * yy);
}

__device__ __forceinline__ bool finite(float v) { return __builtin_isfinite(v); }

__global__ __launch_bounds__(256) void k_preprocess(PreArgs a, const float* __restrict__ means,
                                                    const float* __restrict__ log_scales,
                                                    const float* __restrict__ quats,
                                                    const float* __restrict__ logits,
                                                    const float* __restrict__ sh,
                                                    seele_splat* __restrict__ splats,
                                                    int32_t* __restrict__ n_tiles) {
  const int64_t n = a.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;

  bool active = a.n_segs == 0;
  for (int s = 0; s < a.n_segs; ++s) active |= (i >= a.seg_begin[s]) & (i < a.seg_end[s]);
  if (!active) {
    for (int v = 0; v < a.n_views; ++v) n_tiles[(a.view0 + v) * n + i] = 0;
    return;
  }

  const float mx = means[i], my = means[n + i], mz = means[2 * n + i];
  const float l0 = log_scales[i], l1 = log_scales[n + i], l2 = log_scales[2 * n + i];
  const float qw = quats[i], qx = quats[n + i], qy = quats[2 * n + i], qz = quats[3 * n + i];
  const float lg = logits[i];
  const float qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
  const bool attrs_ok = finite(mx) && finite(my) && finite(mz) && finite(l0) && finite(l1) &&
                        finite(l2) && finite(qw) && finite(qx) && finite(qy) && finite(qz) &&
                        finite(lg) && qn2 > 0.0f && finite(qn2);
  if (!attrs_ok) {
    for (int v = 0; v < a.n_views; ++v) n_tiles[(a.view0 + v) * n + i] = 0;
    return;
  }

  // activations: Sigma = (R S)(R S)^T, o = sigmoid(logit)
  const float qinv = 1.0f / sqrtf(qn2);
  const float w = qw * qinv, x = qx * qinv, y = qy * qinv, z = qz * qinv;
  const float R00 = 1.0f - 2.0f * (y * y + z * z), R01 = 2.0f * (x * y - w * z),
              R02 = 2.0f * (x * z + w * y);
  const float R10 = 2.0f * (x * y + w * z), R11 = 1.0f - 2.0f * (x * x + z * z),
              R12 = 2.0f * (y * z - w * x);
  const float R20 = 2.0f * (x * z - w * y), R21 = 2.0f * (y * z + w * x),
              R22 = 1.0f - 2.0f * (x * x + y * y);
  const float s0 = expf(l0), s1 = expf(l1), s2 = expf(l2);
  const float M00 = R00 * s0, M01 = R01 * s1, M02 = R02 * s2;
  const float M10 = R10 * s0, M11 = R11 * s1, M12 = R12 * s2;
  const float M20 = R20 * s0, M21 = R21 * s1, M22 = R22 * s2;
  const float S00 = M00 * M00 + M01 * M01 + M02 * M02;
  const float S01 = M00 * M10 + M01 * M11 + M02 * M12;
  const float S02 = M00 * M20 + M01 * M21 + M02 * M22;
  const float S11 = M10 * M10 + M11 * M11 + M12 * M12;
  const float S12 = M10 * M20 + M11 * M21 + M12 * M22;
  const float S22 = M20 * M20 + M21 * M21 + M22 * M22;
  const float o = 1.0f / (1.0f + expf(-lg));

  const int nb = (a.sh_degree + 1) * (a.sh_degree + 1);
  float coef[48];
  bool have_sh = false;
  const float inv_tile = 1.0f / (float)a.tile;

  for (int v = 0; v < a.n_views; ++v) {
    const CamK& c = a.cam[v];
    const int64_t rec = (a.view0 + v) * n + i;
    int32_t nt = 0;
    // camera transform and near cull
    const float tx = c.R[0] * mx + c.R[1] * my + c.R[2] * mz + c.t[0];
    const float ty = c.R[3] * mx + c.R[4] * my + c.R[5] * mz + c.t[1];
    const float tz = c.R[6] * mx + c.R[7] * my + c.R[8] * mz + c.t[2];
    if (tz > a.z_near) {
      // EWA: T = J W with J the Jacobian of the perspective projection at t
      const float iz = 1.0f / tz;
      const float j00 = c.fx * iz, j02 = -c.fx * tx * iz * iz;
      const float j11 = c.fy * iz, j12 = -c.fy * ty * iz * iz;
      const float T00 = j00 * c.R[0] + j02 * c.R[6];
      const float T01 = j00 * c.R[1] + j02 * c.R[7];
      const float T02 = j00 * c.R[2] + j02 * c.R[8];
      const float T10 = j11 * c.R[3] + j12 * c.R[6];
      const float T11 = j11 * c.R[4] + j12 * c.R[7];
      const float T12 = j11 * c.R[5] + j12 * c.R[8];
      // U = T Sigma (2x3), Sigma' = U T^T + lowpass I
      const float U00 = T00 * S00 + T01 * S01 + T02 * S02;
      const float U01 = T00 * S01 + T01 * S11 + T02 * S12;
      const float U02 = T00 * S02 + T01 * S12 + T02 * S22;
      const float U10 = T10 * S00 + T11 * S01 + T12 * S02;
      const float U11 = T10 * S01 + T11 * S11 + T12 * S12;
      const float U12 = T10 * S02 + T11 * S12 + T12 * S22;
      const float ca = U00 * T00 + U01 * T01 + U02 * T02 + a.lowpass;
      const float cb = U00 * T10 + U01 * T11 + U02 * T12;
      const float cc = U10 * T10 + U11 * T11 + U12 * T12 + a.lowpass;
      const float det = ca * cc - cb * cb;
      const float px = c.fx * tx * iz + c.cx;
      const float py = c.fy * ty * iz + c.cy;
      float ex, ey;
      bool op_ok;
      if (a.extent == SEELE_EXTENT_OPACITY) {
        const float tau = fminf(2.0f * logf(o / a.alpha_min), 9.0f);
        op_ok = tau > 0.0f;
        ex = sqrtf(tau * ca);
        ey = sqrtf(tau * cc);
      } else {
        // lambda_max = mid + sqrt(mid^2 - det), with mid^2 - det = ((a-c)/2)^2 + b^2
        const float mid = 0.5f * (ca + cc), hd = 0.5f * (ca - cc);
        const float lam = mid + sqrtf(hd * hd + cb * cb);
        const float r = 3.0f * sqrtf(lam);
        op_ok = o >= a.alpha_min;
        ex = r;
        ey = r;
      }
      const float ia = cc / det, ib = -cb / det, ic = ca / det;
      bool ok = op_ok && det > 0.0f && finite(det) && finite(ia) && finite(ib) && finite(ic) &&
                finite(px) && finite(py) && finite(ex) && finite(ey);
      if (ok) {
        const float gw = (float)c.gridW, gh = (float)c.gridH;
        const int x0 = (int)fminf(fmaxf(floorf((px - ex) * inv_tile), 0.0f), gw);
        const int x1 = (int)fminf(fmaxf(floorf((px + ex) * inv_tile) + 1.0f, 0.0f), gw);
        const int y0 = (int)fminf(fmaxf(floorf((py - ey) * inv_tile), 0.0f), gh);
        const int y1 = (int)fminf(fmaxf(floorf((py + ey) * inv_tile) + 1.0f, 0.0f), gh);
        if (x1 > x0 && y1 > y0) {
          // colour toward the camera
          if (!have_sh) {
#pragma unroll
            for (int k = 0; k < 16; ++k)
#pragma unroll
              for (int ch = 0; ch < 3; ++ch)
                coef[k * 3 + ch] = k < nb ? sh[(int64_t)(k * 3 + ch) * n + i] : 0.0f;
            have_sh = true;
          }
          float dx = mx - c.C[0], dy = my - c.C[1], dz = mz - c.C[2];
          const float dinv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
          dx *= dinv;
          dy *= dinv;
          dz *= dinv;
          float Y[16];
          sh_basis(dx, dy, dz, Y);
          float rgb[3];
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < 16; ++k) acc += Y[k] * coef[k * 3 + ch];
            rgb[ch] = 0.5f + acc;
          }
          if (finite(rgb[0]) && finite(rgb[1]) && finite(rgb[2])) {
            nt = (x1 - x0) * (y1 - y0);
            float4* dst = reinterpret_cast<float4*>(splats + rec);
            dst[0] = make_float4(px, py, ia, ib);
            dst[1] = make_float4(ic, o, fmaxf(rgb[0], 0.0f), fmaxf(rgb[1], 0.0f));
            dst[2] = make_float4(fmaxf(rgb[2], 0.0f), tz,
                                 __uint_as_float((uint32_t)x0 | ((uint32_t)x1 << 16)),
                                 __uint_as_float((uint32_t)y0 | ((uint32_t)y1 << 16)));
          }
        }
      }
    }
    n_tiles[rec] = nt;
  }
}

}  // namespace

hipError_t launch_preprocess(const PreArgs& a, const seele_gaussians& g, seele_splat* splats,
                             int32_t* n_tiles, hipStream_t stream) {
  if (a.n == 0) return hipSuccess;
  const int block = 256;
  const int64_t grid = (a.n + block - 1) / block;
  hipLaunchKernelGGL(k_preprocess, dim3((unsigned)grid), dim3(block), 0, stream, a, g.means,
                     g.log_scales, g.quats, g.opacity_logits, g.sh, splats, n_tiles);
  return hipGetLastError();
}

}  // namespace seele
