// Per-view preprocessing on gfx950 (Sec. 3.1 "Preprocessing"; EWA screen-space
// covariance behind Eq. 2; opacity-aware extent of Sec. 3.3, Eqs. 3-5) and its
// backward pass (Sec. 3.5: gradients of the unchanged pipeline).
//
// One lane per Gaussian.  The SoA attribute arrays are read coalesced; the
// Gaussian's activations (3D covariance, opacity) are computed once and reused
// for every view of the launch, and the 48 SH coefficients are read only if the
// Gaussian is visible in some view.  Output is one 48-byte record per (view,
// Gaussian) plus its tile count.  HBM-bound: 44 B of geometry/opacity read and
// 4 B of tile count written per active Gaussian, plus 192 B of SH read and
// 48 B written per visible one.
//
// The forward and backward kernels share the activation and projection code
// below, so the backward recomputes exactly the forward's float32 values.
#include "seele_internal.h"

namespace seele {

namespace {

__device__ __forceinline__ bool finite(float v) { return __builtin_isfinite(v); }

// Real SH basis (Condon-Shortley phase), degree <= 3, index l*l + l + m.
constexpr float C0 = 0.28209479177387814f;
constexpr float C1 = 0.48860251190291987f;
constexpr float C2a = 1.0925484305920792f;
constexpr float C2b = 0.31539156525252005f;
constexpr float C2c = 0.54627421529603959f;
constexpr float C3a = 0.59004358992664352f;
constexpr float C3b = 2.8906114426405538f;
constexpr float C3c = 0.45704579946446572f;
constexpr float C3d = 0.37317633259011540f;
constexpr float C3e = 1.4453057213202769f;

__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[0] = C0;
  Y[1] = -C1 * y;
  Y[2] = C1 * z;
  Y[3] = -C1 * x;
  Y[4] = C2a * x * y;
  Y[5] = -C2a * y * z;
  Y[6] = C2b * (2.0f * zz - xx - yy);
  Y[7] = -C2a * x * z;
  Y[8] = C2c * (xx - yy);
  Y[9] = -C3a * y * (3.0f * xx - yy);
  Y[10] = C3b * x * y * z;
  Y[11] = -C3c * y * (4.0f * zz - xx - yy);
  Y[12] = C3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = -C3c * x * (4.0f * zz - xx - yy);
  Y[14] = C3e * z * (xx - yy);
  Y[15] = -C3a * x * (xx - 3.0f * yy);
}

// d Y_k / d(x, y, z) of the polynomials above (only the part tangent to the
// sphere matters; the caller projects through the normalisation).
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, float* gx, float* gy,
                                              float* gz) {
  const float xx = x * x, yy = y * y, zz = z * z;
  gx[0] = 0.0f; gy[0] = 0.0f; gz[0] = 0.0f;
  gx[1] = 0.0f; gy[1] = -C1; gz[1] = 0.0f;
  gx[2] = 0.0f; gy[2] = 0.0f; gz[2] = C1;
  gx[3] = -C1; gy[3] = 0.0f; gz[3] = 0.0f;
  gx[4] = C2a * y; gy[4] = C2a * x; gz[4] = 0.0f;
  gx[5] = 0.0f; gy[5] = -C2a * z; gz[5] = -C2a * y;
  gx[6] = -2.0f * C2b * x; gy[6] = -2.0f * C2b * y; gz[6] = 4.0f * C2b * z;
  gx[7] = -C2a * z; gy[7] = 0.0f; gz[7] = -C2a * x;
  gx[8] = 2.0f * C2c * x; gy[8] = -2.0f * C2c * y; gz[8] = 0.0f;
  gx[9] = -6.0f * C3a * x * y; gy[9] = -3.0f * C3a * (xx - yy); gz[9] = 0.0f;
  gx[10] = C3b * y * z; gy[10] = C3b * x * z; gz[10] = C3b * x * y;
  gx[11] = 2.0f * C3c * x * y; gy[11] = -C3c * (4.0f * zz - xx - 3.0f * yy);
  gz[11] = -8.0f * C3c * y * z;
  gx[12] = -6.0f * C3d * x * z; gy[12] = -6.0f * C3d * y * z;
  gz[12] = C3d * (6.0f * zz - 3.0f * xx - 3.0f * yy);
  gx[13] = -C3c * (4.0f * zz - 3.0f * xx - yy); gy[13] = 2.0f * C3c * x * y;
  gz[13] = -8.0f * C3c * x * z;
  gx[14] = 2.0f * C3e * x * z; gy[14] = -2.0f * C3e * y * z; gz[14] = C3e * (xx - yy);
  gx[15] = -3.0f * C3a * (xx - yy); gy[15] = 6.0f * C3a * x * y; gz[15] = 0.0f;
}

// Activations of one Gaussian: Sigma = (R S)(R S)^T, o = sigmoid(logit).
struct Act {
  float mx, my, mz;
  float w, x, y, z, qinv;  // unit quaternion and 1/|q|
  float R[9], s[3], M[9];
  float S00, S01, S02, S11, S12, S22;
  float o;
};

__device__ __forceinline__ bool activate(int64_t i, int64_t n, const float* __restrict__ means,
                                         const float* __restrict__ log_scales,
                                         const float* __restrict__ quats,
                                         const float* __restrict__ logits, Act& g) {
  g.mx = means[i];
  g.my = means[n + i];
  g.mz = means[2 * n + i];
  const float l0 = log_scales[i], l1 = log_scales[n + i], l2 = log_scales[2 * n + i];
  const float qw = quats[i], qx = quats[n + i], qy = quats[2 * n + i], qz = quats[3 * n + i];
  const float lg = logits[i];
  const float qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
  const bool ok = finite(g.mx) && finite(g.my) && finite(g.mz) && finite(l0) && finite(l1) &&
                  finite(l2) && finite(qw) && finite(qx) && finite(qy) && finite(qz) &&
                  finite(lg) && qn2 > 0.0f && finite(qn2);
  if (!ok) return false;
  g.qinv = 1.0f / sqrtf(qn2);
  const float w = qw * g.qinv, x = qx * g.qinv, y = qy * g.qinv, z = qz * g.qinv;
  g.w = w;
  g.x = x;
  g.y = y;
  g.z = z;
  g.R[0] = 1.0f - 2.0f * (y * y + z * z);
  g.R[1] = 2.0f * (x * y - w * z);
  g.R[2] = 2.0f * (x * z + w * y);
  g.R[3] = 2.0f * (x * y + w * z);
  g.R[4] = 1.0f - 2.0f * (x * x + z * z);
  g.R[5] = 2.0f * (y * z - w * x);
  g.R[6] = 2.0f * (x * z - w * y);
  g.R[7] = 2.0f * (y * z + w * x);
  g.R[8] = 1.0f - 2.0f * (x * x + y * y);
  g.s[0] = expf(l0);
  g.s[1] = expf(l1);
  g.s[2] = expf(l2);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) g.M[r * 3 + c] = g.R[r * 3 + c] * g.s[c];
  const float* M = g.M;
  g.S00 = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  g.S01 = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  g.S02 = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  g.S11 = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  g.S12 = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  g.S22 = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
  g.o = 1.0f / (1.0f + expf(-lg));
  return true;
}

// Projection of one Gaussian into one view (EWA, Eq. 2's x' and Sigma').
struct Proj {
  float tx, ty, tz, iz;
  float j00, j02, j11, j12;      // Jacobian of the perspective projection
  float T[6];                    // T = J W (2x3, row-major)
  float U[6];                    // U = T Sigma (2x3)
  float ca, cb, cc, det;         // Sigma' (with low-pass) and its determinant
  float ia, ib, ic;              // conic = Sigma'^-1
  float px, py;                  // x'
};

__device__ __forceinline__ void project(const CamK& c, const Act& g, float lowpass, Proj& p) {
  p.tx = c.R[0] * g.mx + c.R[1] * g.my + c.R[2] * g.mz + c.t[0];
  p.ty = c.R[3] * g.mx + c.R[4] * g.my + c.R[5] * g.mz + c.t[1];
  p.tz = c.R[6] * g.mx + c.R[7] * g.my + c.R[8] * g.mz + c.t[2];
  p.iz = 1.0f / p.tz;
  p.j00 = c.fx * p.iz;
  p.j02 = -c.fx * p.tx * p.iz * p.iz;
  p.j11 = c.fy * p.iz;
  p.j12 = -c.fy * p.ty * p.iz * p.iz;
  p.T[0] = p.j00 * c.R[0] + p.j02 * c.R[6];
  p.T[1] = p.j00 * c.R[1] + p.j02 * c.R[7];
  p.T[2] = p.j00 * c.R[2] + p.j02 * c.R[8];
  p.T[3] = p.j11 * c.R[3] + p.j12 * c.R[6];
  p.T[4] = p.j11 * c.R[4] + p.j12 * c.R[7];
  p.T[5] = p.j11 * c.R[5] + p.j12 * c.R[8];
  p.U[0] = p.T[0] * g.S00 + p.T[1] * g.S01 + p.T[2] * g.S02;
  p.U[1] = p.T[0] * g.S01 + p.T[1] * g.S11 + p.T[2] * g.S12;
  p.U[2] = p.T[0] * g.S02 + p.T[1] * g.S12 + p.T[2] * g.S22;
  p.U[3] = p.T[3] * g.S00 + p.T[4] * g.S01 + p.T[5] * g.S02;
  p.U[4] = p.T[3] * g.S01 + p.T[4] * g.S11 + p.T[5] * g.S12;
  p.U[5] = p.T[3] * g.S02 + p.T[4] * g.S12 + p.T[5] * g.S22;
  p.ca = p.U[0] * p.T[0] + p.U[1] * p.T[1] + p.U[2] * p.T[2] + lowpass;
  p.cb = p.U[0] * p.T[3] + p.U[1] * p.T[4] + p.U[2] * p.T[5];
  p.cc = p.U[3] * p.T[3] + p.U[4] * p.T[4] + p.U[5] * p.T[5] + lowpass;
  p.det = p.ca * p.cc - p.cb * p.cb;
  p.ia = p.cc / p.det;
  p.ib = -p.cb / p.det;
  p.ic = p.ca / p.det;
  p.px = c.fx * p.tx * p.iz + c.cx;
  p.py = c.fy * p.ty * p.iz + c.cy;
}

// NB = (sh_degree + 1)^2 is a template argument so that the coefficient
// loads carry no per-coefficient branch and are all in flight together.  ONE
// compiles the single-view launch without the view loop: nothing of the
// Gaussian has to stay live across views, which halves the registers.
//
// STAGE also does the binning's first step for each view: the workgroup's
// visible records (n_tiles > 0) are compacted in record order into their
// span (view, workgroup) of the stage arrays -- float32 depth bits and record
// id, and its tile rectangle packed into 32 bits (for grids of at most 256 x
// 256 tiles) -- with the span's count, and every record's tile rectangle
// (zero if not visible) goes to the dense id-indexed array rid.  The binning then
// starts from a scan of the span counts instead of re-reading the records.
template <int NB, bool ONE, bool STAGE>
__global__ __launch_bounds__(256) void k_preprocess(PreArgs a, const float* __restrict__ means,
                                                    const float* __restrict__ log_scales,
                                                    const float* __restrict__ quats,
                                                    const float* __restrict__ logits,
                                                    const float* __restrict__ sh,
                                                    seele_splat* __restrict__ splats,
                                                    int32_t* __restrict__ n_tiles, BinStage bs) {
  const int64_t n = a.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < n;
  if (!STAGE && !in) return;

  bool live = false;
  Act g;
  if (in) {
    bool active = a.n_segs == 0;
    for (int s = 0; s < a.n_segs; ++s) active |= (i >= a.seg_begin[s]) & (i < a.seg_end[s]);
    live = active && activate(i, n, means, log_scales, quats, logits, g);
  }
  if (!live) {
    if (in)
      for (int v = 0; v < a.n_views; ++v) n_tiles[(a.view0 + v) * n + i] = 0;
    if (!STAGE) return;  // (the staging below needs every thread of the block)
  }

  const float inv_tile = 1.0f / (float)a.tile;
  const int nviews = ONE ? 1 : a.n_views;
  __shared__ uint32_t s_wc[4];

  for (int v = 0; v < nviews; ++v) {
    const CamK& c = a.cam[v];
    const int64_t rec = (a.view0 + v) * n + i;
    int32_t nt = 0;
    uint32_t dkey = 0, srx = 0, sry = 0;
    if (live) {
      Proj p;
      project(c, g, a.lowpass, p);
      if (p.tz > a.z_near) {
        float ex, ey;
        bool op_ok;
        if (a.extent == SEELE_EXTENT_OPACITY) {
          const float tau = fminf(2.0f * logf(g.o / a.alpha_min), 9.0f);
          op_ok = tau > 0.0f;
          ex = sqrtf(tau * p.ca);
          ey = sqrtf(tau * p.cc);
        } else {
          // lambda_max = mid + sqrt(mid^2 - det), with mid^2 - det = ((a-c)/2)^2 + b^2
          const float mid = 0.5f * (p.ca + p.cc), hd = 0.5f * (p.ca - p.cc);
          const float lam = mid + sqrtf(hd * hd + p.cb * p.cb);
          const float r = 3.0f * sqrtf(lam);
          op_ok = g.o >= a.alpha_min;
          ex = r;
          ey = r;
        }
        const bool ok = op_ok && p.det > 0.0f && finite(p.det) && finite(p.ia) && finite(p.ib) &&
                        finite(p.ic) && finite(p.px) && finite(p.py) && finite(ex) && finite(ey);
        if (ok) {
          const float gw = (float)c.gridW, gh = (float)c.gridH;
          const int x0 = (int)fminf(fmaxf(floorf((p.px - ex) * inv_tile), 0.0f), gw);
          const int x1 = (int)fminf(fmaxf(floorf((p.px + ex) * inv_tile) + 1.0f, 0.0f), gw);
          const int y0 = (int)fminf(fmaxf(floorf((p.py - ey) * inv_tile), 0.0f), gh);
          const int y1 = (int)fminf(fmaxf(floorf((p.py + ey) * inv_tile) + 1.0f, 0.0f), gh);
          if (x1 > x0 && y1 > y0) {
            // colour toward the camera; coefficients streamed from the SoA array
            float dx = g.mx - c.C[0], dy = g.my - c.C[1], dz = g.mz - c.C[2];
            const float dinv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
            dx *= dinv;
            dy *= dinv;
            dz *= dinv;
            float coef[NB * 3];
  #pragma unroll
            for (int k = 0; k < NB * 3; ++k) coef[k] = sh[(int64_t)k * n + i];
            float Y[16];
            sh_basis(dx, dy, dz, Y);
            float acc[3] = {0.0f, 0.0f, 0.0f};
  #pragma unroll
            for (int k = 0; k < NB; ++k) {
  #pragma unroll
              for (int ch = 0; ch < 3; ++ch) acc[ch] += Y[k] * coef[k * 3 + ch];
            }
            const float rgb[3] = {0.5f + acc[0], 0.5f + acc[1], 0.5f + acc[2]};
            if (finite(rgb[0]) && finite(rgb[1]) && finite(rgb[2])) {
              nt = (x1 - x0) * (y1 - y0);
              const Chol L = conic_factor(p.ia, p.ib, p.ic);
              dkey = __float_as_uint(p.tz);
              srx = (uint32_t)x0 | ((uint32_t)x1 << 16);
              sry = (uint32_t)y0 | ((uint32_t)y1 << 16);
              float4* dst = reinterpret_cast<float4*>(splats + rec);
              dst[0] = make_float4(p.px, p.py, L.l11, L.l21);
              dst[1] = make_float4(L.l22, g.o, fmaxf(rgb[0], 0.0f), fmaxf(rgb[1], 0.0f));
              dst[2] = make_float4(fmaxf(rgb[2], 0.0f), p.ia, p.ib, p.ic);
              dst[3] = make_float4(p.tz, __uint_as_float(srx), __uint_as_float(sry), 0.0f);
            }
          }
        }
      }
      n_tiles[rec] = nt;
    }
    if (STAGE) {
      const bool vis = nt > 0;
      const int w = threadIdx.x >> 6;
      const uint64_t b = __ballot(vis);
      if ((threadIdx.x & 63) == 0) s_wc[w] = (uint32_t)__popcll(b);
      __syncthreads();
      uint32_t off = 0, tot = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t cw = s_wc[k];
        off += k < w ? cw : 0u;
        tot += cw;
      }
      const int64_t span = (a.view0 + v) * bs.n_blocks + blockIdx.x;
      if (vis) {
        const uint32_t pos =
            off + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
        bs.keys[span * 256 + pos] = dkey;
        bs.ids[span * 256 + pos] = (uint32_t)rec;
        bs.prect[span * 256 + pos] = pack_rect8(srx, sry);
      }
      if (threadIdx.x == 0) bs.span_count[span] = tot;
      if (in) bs.rid[rec] = make_uint2(srx, sry);
      __syncthreads();  // s_wc is rewritten for the next view
    }
  }
}

// ------------------------------------------------------------------ backward
// For every view in which Gaussian i was visible (n_tiles > 0), its 2D
// gradient dL/d(x', conic, o, rgb) is chained back in two kernels:
//  * colour (float32): rgb = max(0, 0.5 + sum_k Y_k(d) k_k) -> SH coefficients
//    and, through the unit view direction d = (x - C)/|x - C|, the mean;
//  * geometry (float64, recomputed from the raw parameters): conic -> Sigma'
//    (dSigma' = -A dA A); x' and Sigma' = T Sigma T^T with T = J(t) W ->
//    t = W x + t_w -> mean and Sigma; sigmoid -> logit; the Sigma gradients
//    of all views are summed before the chain through Sigma = M M^T,
//    M = R(q) diag(exp(s)), to log-scales and the quaternion.
// The geometric chain multiplies Jacobians of magnitude f/z ~ 1e3 into
// scale-sized covariances and cancels strongly for small Gaussians; double
// precision (half the float32 vector rate on this GPU, on per-Gaussian work)
// keeps its relative error at the float32 input's.

// NB = (sh_degree + 1)^2: the coefficients are loaded once, for all views.
template <int NB>
__global__ __launch_bounds__(256) void k_preprocess_bwd_color(
    PreArgs a, const float* __restrict__ means, const float* __restrict__ sh,
    const int32_t* __restrict__ n_tiles, const float* __restrict__ grad2d,
    float* __restrict__ g_means, float* __restrict__ g_sh, int accumulate) {
  const int64_t n = a.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gsh[NB * 3];
#pragma unroll
  for (int k = 0; k < NB * 3; ++k) gsh[k] = 0.0f;
  float gm0 = 0.0f, gm1 = 0.0f, gm2 = 0.0f;
  bool any = false;
  for (int v = 0; v < a.n_views; ++v) any |= n_tiles[(a.view0 + v) * n + i] > 0;
  if (any) {
    float coef[NB * 3];
#pragma unroll
    for (int k = 0; k < NB * 3; ++k) coef[k] = sh[(int64_t)k * n + i];
    const float mx = means[i], my = means[n + i], mz = means[2 * n + i];
    for (int v = 0; v < a.n_views; ++v) {
      const int64_t rec = (a.view0 + v) * n + i;
      if (n_tiles[rec] <= 0) continue;
      const CamK& c = a.cam[v];
      const float* G = grad2d + rec * 9;
      const float gcol[3] = {G[6], G[7], G[8]};
      const float vx = mx - c.C[0], vy = my - c.C[1], vz = mz - c.C[2];
      const float dinv = 1.0f / sqrtf(vx * vx + vy * vy + vz * vz);
      const float dx = vx * dinv, dy = vy * dinv, dz = vz * dinv;
      float Y[16], Gx[16], Gy[16], Gz[16];
      sh_basis(dx, dy, dz, Y);
      sh_basis_grad(dx, dy, dz, Gx, Gy, Gz);
      float acc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) acc[ch] += Y[k] * coef[k * 3 + ch];
      float graw[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) graw[ch] = (0.5f + acc[ch]) > 0.0f ? gcol[ch] : 0.0f;
      float gdx = 0.0f, gdy = 0.0f, gdz = 0.0f;
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        float t = 0.0f;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          gsh[k * 3 + ch] += Y[k] * graw[ch];
          t += graw[ch] * coef[k * 3 + ch];
        }
        gdx += t * Gx[k];
        gdy += t * Gy[k];
        gdz += t * Gz[k];
      }
      const float dotd = dx * gdx + dy * gdy + dz * gdz;
      gm0 += (gdx - dx * dotd) * dinv;
      gm1 += (gdy - dy * dotd) * dinv;
      gm2 += (gdz - dz * dotd) * dinv;
    }
  }
  const float outm[3] = {gm0, gm1, gm2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float* pm = g_means + k * n + i;
    *pm = accumulate ? *pm + outm[k] : outm[k];
  }
  // coefficients above the degree get no gradient
#pragma unroll
  for (int k = 0; k < 48; ++k) {
    float* ps = g_sh + (int64_t)k * n + i;
    const float gk = k < NB * 3 ? gsh[k < NB * 3 ? k : 0] : 0.0f;
    *ps = accumulate ? *ps + gk : gk;
  }
}

__global__ __launch_bounds__(256) void k_preprocess_bwd_geom(
    PreArgs a, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits,
    const int32_t* __restrict__ n_tiles, const float* __restrict__ grad2d,
    float* __restrict__ g_means, float* __restrict__ g_ls, float* __restrict__ g_quats,
    float* __restrict__ g_logits, int accumulate) {
  const int64_t n = a.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double gm0 = 0.0, gm1 = 0.0, gm2 = 0.0, glg = 0.0;
  double GS00 = 0.0, GS01 = 0.0, GS02 = 0.0, GS11 = 0.0, GS12 = 0.0, GS22 = 0.0;
  double gl[3] = {0.0, 0.0, 0.0}, gq[4] = {0.0, 0.0, 0.0, 0.0};
  bool any = false;
  const double mx = means[i], my = means[n + i], mz = means[2 * n + i];
  const double qw0 = quats[i], qx0 = quats[n + i], qy0 = quats[2 * n + i], qz0 = quats[3 * n + i];
  const double qinv = 1.0 / sqrt(qw0 * qw0 + qx0 * qx0 + qy0 * qy0 + qz0 * qz0);
  const double w = qw0 * qinv, x = qx0 * qinv, y = qy0 * qinv, z = qz0 * qinv;
  double R[9];
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
  const double sc[3] = {exp((double)log_scales[i]), exp((double)log_scales[n + i]),
                        exp((double)log_scales[2 * n + i])};
  double M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) M[r * 3 + c] = R[r * 3 + c] * sc[c];
  const double S00 = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  const double S01 = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  const double S02 = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  const double S11 = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  const double S12 = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  const double S22 = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
  const double o = 1.0 / (1.0 + exp(-(double)logits[i]));

  for (int v = 0; v < a.n_views; ++v) {
    const int64_t rec = (a.view0 + v) * n + i;
    if (n_tiles[rec] <= 0) continue;
    any = true;
    const CamK& c = a.cam[v];
    const float* G = grad2d + rec * 9;
    const double gmx = G[0], gmy = G[1], ga = G[2], gb = G[3], gc = G[4], go = G[5];
    const double W[9] = {c.R[0], c.R[1], c.R[2], c.R[3], c.R[4], c.R[5], c.R[6], c.R[7], c.R[8]};
    const double fx = c.fx, fy = c.fy;
    const double tx = W[0] * mx + W[1] * my + W[2] * mz + (double)c.t[0];
    const double ty = W[3] * mx + W[4] * my + W[5] * mz + (double)c.t[1];
    const double tz = W[6] * mx + W[7] * my + W[8] * mz + (double)c.t[2];
    const double iz = 1.0 / tz;
    const double j00 = fx * iz, j02 = -fx * tx * iz * iz, j11 = fy * iz, j12 = -fy * ty * iz * iz;
    const double T[6] = {j00 * W[0] + j02 * W[6], j00 * W[1] + j02 * W[7], j00 * W[2] + j02 * W[8],
                         j11 * W[3] + j12 * W[6], j11 * W[4] + j12 * W[7], j11 * W[5] + j12 * W[8]};
    const double U[6] = {T[0] * S00 + T[1] * S01 + T[2] * S02, T[0] * S01 + T[1] * S11 + T[2] * S12,
                         T[0] * S02 + T[1] * S12 + T[2] * S22, T[3] * S00 + T[4] * S01 + T[5] * S02,
                         T[3] * S01 + T[4] * S11 + T[5] * S12, T[3] * S02 + T[4] * S12 + T[5] * S22};
    const double ca = U[0] * T[0] + U[1] * T[1] + U[2] * T[2] + (double)a.lowpass;
    const double cb = U[0] * T[3] + U[1] * T[4] + U[2] * T[5];
    const double cc = U[3] * T[3] + U[4] * T[4] + U[5] * T[5] + (double)a.lowpass;
    const double det = ca * cc - cb * cb;
    const double ia = cc / det, ib = -cb / det, ic = ca / det;
    glg += go * o * (1.0 - o);
    // conic -> Sigma':  GS' = -A GA A, GA = [[ga, gb/2], [gb/2, gc]]
    const double hb = 0.5 * gb;
    const double X00 = ga * ia + hb * ib, X01 = ga * ib + hb * ic;
    const double X10 = hb * ia + gc * ib, X11 = hb * ib + gc * ic;
    const double P00 = -(ia * X00 + ib * X10);
    const double P01 = -(ia * X01 + ib * X11);
    const double P11 = -(ib * X01 + ic * X11);
    // GSigma += T^T GS' T
    const double Q0 = P00 * T[0] + P01 * T[3], Q1 = P00 * T[1] + P01 * T[4],
                 Q2 = P00 * T[2] + P01 * T[5];
    const double Q3 = P01 * T[0] + P11 * T[3], Q4 = P01 * T[1] + P11 * T[4],
                 Q5 = P01 * T[2] + P11 * T[5];
    GS00 += T[0] * Q0 + T[3] * Q3;
    GS01 += T[0] * Q1 + T[3] * Q4;
    GS02 += T[0] * Q2 + T[3] * Q5;
    GS11 += T[1] * Q1 + T[4] * Q4;
    GS12 += T[1] * Q2 + T[4] * Q5;
    GS22 += T[2] * Q2 + T[5] * Q5;
    // GT = 2 GS' U;  GJ = GT W^T (only J00, J02, J11, J12 vary with t)
    const double GT0 = 2.0 * (P00 * U[0] + P01 * U[3]), GT1 = 2.0 * (P00 * U[1] + P01 * U[4]),
                 GT2 = 2.0 * (P00 * U[2] + P01 * U[5]);
    const double GT3 = 2.0 * (P01 * U[0] + P11 * U[3]), GT4 = 2.0 * (P01 * U[1] + P11 * U[4]),
                 GT5 = 2.0 * (P01 * U[2] + P11 * U[5]);
    const double GJ00 = GT0 * W[0] + GT1 * W[1] + GT2 * W[2];
    const double GJ02 = GT0 * W[6] + GT1 * W[7] + GT2 * W[8];
    const double GJ11 = GT3 * W[3] + GT4 * W[4] + GT5 * W[5];
    const double GJ12 = GT3 * W[6] + GT4 * W[7] + GT5 * W[8];
    const double iz2 = iz * iz, iz3 = iz2 * iz;
    // x' has Jacobian J with respect to t
    double gtx = j00 * gmx, gty = j11 * gmy, gtz = j02 * gmx + j12 * gmy;
    gtx += GJ02 * (-fx * iz2);
    gty += GJ12 * (-fy * iz2);
    gtz += GJ00 * (-fx * iz2) + GJ02 * (2.0 * fx * tx * iz3) + GJ11 * (-fy * iz2) +
           GJ12 * (2.0 * fy * ty * iz3);
    // t = W x + t_w
    gm0 += W[0] * gtx + W[3] * gty + W[6] * gtz;
    gm1 += W[1] * gtx + W[4] * gty + W[7] * gtz;
    gm2 += W[2] * gtx + W[5] * gty + W[8] * gtz;
  }
  if (any) {
    // Sigma = M M^T: GM = 2 GSigma M;  M = R diag(s)
    const double GSm[9] = {GS00, GS01, GS02, GS01, GS11, GS12, GS02, GS12, GS22};
    double GR[9];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      double gs = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double gmrc = 2.0 * (GSm[r * 3 + 0] * M[0 * 3 + cc] + GSm[r * 3 + 1] * M[1 * 3 + cc] +
                                   GSm[r * 3 + 2] * M[2 * 3 + cc]);
        gs += gmrc * R[r * 3 + cc];
        GR[r * 3 + cc] = gmrc * sc[cc];
      }
      gl[cc] = gs * sc[cc];
    }
    // R(qhat): derivatives of each entry with respect to (w, x, y, z)
    const double gw = GR[1] * (-2.0 * z) + GR[2] * (2.0 * y) + GR[3] * (2.0 * z) +
                      GR[5] * (-2.0 * x) + GR[6] * (-2.0 * y) + GR[7] * (2.0 * x);
    const double gx = GR[1] * (2.0 * y) + GR[2] * (2.0 * z) + GR[3] * (2.0 * y) +
                      GR[4] * (-4.0 * x) + GR[5] * (-2.0 * w) + GR[6] * (2.0 * z) +
                      GR[7] * (2.0 * w) + GR[8] * (-4.0 * x);
    const double gy = GR[0] * (-4.0 * y) + GR[1] * (2.0 * x) + GR[2] * (2.0 * w) +
                      GR[3] * (2.0 * x) + GR[5] * (2.0 * z) + GR[6] * (-2.0 * w) +
                      GR[7] * (2.0 * z) + GR[8] * (-4.0 * y);
    const double gz = GR[0] * (-4.0 * z) + GR[1] * (-2.0 * w) + GR[2] * (2.0 * x) +
                      GR[3] * (2.0 * w) + GR[4] * (-4.0 * z) + GR[5] * (2.0 * y) +
                      GR[6] * (2.0 * x) + GR[7] * (2.0 * y);
    // through the normalisation q / |q|
    const double dq = w * gw + x * gx + y * gy + z * gz;
    gq[0] = (gw - w * dq) * qinv;
    gq[1] = (gx - x * dq) * qinv;
    gq[2] = (gy - y * dq) * qinv;
    gq[3] = (gz - z * dq) * qinv;
  }
  // the colour kernel wrote its share of the mean gradient first
  const double outm[3] = {gm0, gm1, gm2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g_means[k * n + i] += (float)outm[k];
    float* pl = g_ls + k * n + i;
    *pl = accumulate ? *pl + (float)gl[k] : (float)gl[k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float* pq = g_quats + k * n + i;
    *pq = accumulate ? *pq + (float)gq[k] : (float)gq[k];
  }
  g_logits[i] = accumulate ? g_logits[i] + (float)glg : (float)glg;
}

}  // namespace

hipError_t launch_preprocess(const PreArgs& a, const seele_gaussians& g, seele_splat* splats,
                             int32_t* n_tiles, hipStream_t stream, const BinStage* stage) {
  if (a.n == 0) return hipSuccess;
  const int block = 256;
  const int64_t grid = (a.n + block - 1) / block;
  const dim3 g3((unsigned)grid), b3(block);
  const bool one = a.n_views == 1;
  const BinStage bs = stage ? *stage : BinStage{};
#define SEELE_PRE_ONE(NB, ONE)                                                                  \
  if (stage)                                                                                    \
    hipLaunchKernelGGL((k_preprocess<NB, ONE, true>), g3, b3, 0, stream, a, g.means,            \
                       g.log_scales, g.quats, g.opacity_logits, g.sh, splats, n_tiles, bs);     \
  else                                                                                          \
    hipLaunchKernelGGL((k_preprocess<NB, ONE, false>), g3, b3, 0, stream, a, g.means,           \
                       g.log_scales, g.quats, g.opacity_logits, g.sh, splats, n_tiles, bs);
#define SEELE_PRE(NB)                                                                           \
  if (one) {                                                                                    \
    SEELE_PRE_ONE(NB, true)                                                                     \
  } else {                                                                                      \
    SEELE_PRE_ONE(NB, false)                                                                    \
  }
  switch (a.sh_degree) {
    case 0:
      SEELE_PRE(1);
      break;
    case 1:
      SEELE_PRE(4);
      break;
    case 2:
      SEELE_PRE(9);
      break;
    default:
      SEELE_PRE(16);
  }
#undef SEELE_PRE
#undef SEELE_PRE_ONE
  return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const PreArgs& a, const seele_gaussians& g,
                                 const int32_t* n_tiles, const float* grad2d,
                                 const seele_gaussian_grads& out, bool accumulate,
                                 hipStream_t stream) {
  if (a.n == 0) return hipSuccess;
  const int block = 256;
  const int64_t grid = (a.n + block - 1) / block;
  const int acc = accumulate ? 1 : 0;
  switch (a.sh_degree) {
    case 0:
      hipLaunchKernelGGL(k_preprocess_bwd_color<1>, dim3((unsigned)grid), dim3(block), 0, stream,
                         a, g.means, g.sh, n_tiles, grad2d, out.means, out.sh, acc);
      break;
    case 1:
      hipLaunchKernelGGL(k_preprocess_bwd_color<4>, dim3((unsigned)grid), dim3(block), 0, stream,
                         a, g.means, g.sh, n_tiles, grad2d, out.means, out.sh, acc);
      break;
    case 2:
      hipLaunchKernelGGL(k_preprocess_bwd_color<9>, dim3((unsigned)grid), dim3(block), 0, stream,
                         a, g.means, g.sh, n_tiles, grad2d, out.means, out.sh, acc);
      break;
    default:
      hipLaunchKernelGGL(k_preprocess_bwd_color<16>, dim3((unsigned)grid), dim3(block), 0, stream,
                         a, g.means, g.sh, n_tiles, grad2d, out.means, out.sh, acc);
  }
  hipLaunchKernelGGL(k_preprocess_bwd_geom, dim3((unsigned)grid), dim3(block), 0, stream, a,
                     g.means, g.log_scales, g.quats, g.opacity_logits, n_tiles, grad2d, out.means,
                     out.log_scales, out.quats, out.opacity_logits, accumulate ? 1 : 0);
  return hipGetLastError();
}

}  // namespace seele
