// FLIP (LDR) image difference and its gradient with respect to the test
// image, for the view-consistency term of the fine-tuning loss (Sec. 3.5).
//
// Per pixel of each view ([3][H][W] sRGB, clamped to [0, 1]):
//   colour: sRGB -> linear -> XYZ -> YCxCz; each opponent channel filtered
//     with its contrast-sensitivity kernel (separable: one Gaussian for Y
//     and Cx, two for Cz), edges replicated; -> linear RGB clamped to
//     [0, 1] -> CIELAB -> Hunt-adjusted; HyAB distance to the reference's,
//     to the power qc, mapped piecewise linearly onto [0, 1] (cmax: the
//     same for green against blue);
//   features: edge and point detectors (separable derivative-of-Gaussian
//     kernels, positive and negative weights normalised to +-1) along x and
//     y on the normalised luminance; dF = (max of the magnitude
//     differences, floored at eps, / sqrt 2)^qf;
//   value dE_c^(1 - dF); a view's score is its mean.
// The gradient runs the same chain backwards: per-pixel seeds for the
// filtered channels and the four feature responses, the adjoints of the
// vertical and horizontal passes (edge replication adds the weights of
// every padded tap to the border pixel), then the colour transforms.
#include <cmath>

#include "finetune_internal.h"

namespace seele {

namespace {

constexpr int kFB = 256;

// x^y for x > 0 through the hardware base-2 logarithm and exponential
// (about 1 ulp each); x = 0 gives 0 for y > 0
__device__ __forceinline__ float fpow(float x, float y) {
  return x > 0.0f ? __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x)) : 0.0f;
}

// 1 / x through the hardware reciprocal (about 1 ulp)
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ int flip_view(const FlipViews& fv) {
  int v = 0;
  for (int q = 1; q < fv.n_views; ++q)
    if (fv.blk_off[q] <= (int)blockIdx.x) v = q;
  return v;
}

struct Px {
  int v, x, y, W, H;
  int64_t p;     // pixel index (view offset + y W + x) in the maps
  int64_t e0;    // element index of channel 0 of this pixel in the images
  int64_t plane;
  bool ok;
};

__device__ __forceinline__ Px px_of(const FlipViews& fv) {
  Px q{};
  const int v = flip_view(fv);
  const int W = fv.w[v], H = fv.h[v];
  const int64_t i = (int64_t)(blockIdx.x - fv.blk_off[v]) * kFB + threadIdx.x;
  q.plane = (int64_t)W * H;
  q.ok = i < q.plane;
  const int64_t ii = q.ok ? i : 0;
  q.v = v;
  q.y = (int)(ii / W);
  q.x = (int)(ii - (int64_t)q.y * W);
  q.W = W;
  q.H = H;
  q.p = fv.pix_off[v] + ii;
  q.e0 = 3 * fv.pix_off[v] + ii;
  return q;
}

__device__ __forceinline__ float srgb_lin(float c) {
  return c > 0.04045f ? fpow((c + 0.055f) * (1.0f / 1.055f), 2.4f) : c * (1.0f / 12.92f);
}
__device__ __forceinline__ float srgb_lin_d(float c) {
  return c > 0.04045f ? (2.4f / 1.055f) * fpow((c + 0.055f) * (1.0f / 1.055f), 1.4f)
                      : 1.0f / 12.92f;
}

// sRGB (clamped) -> YCxCz
__device__ __forceinline__ void to_ycxcz(const FlipConst& k, const float* rgb, float* o) {
  float l[3];
  for (int c = 0; c < 3; ++c) l[c] = srgb_lin(fminf(fmaxf(rgb[c], 0.f), 1.f));
  float n[3];
  for (int i = 0; i < 3; ++i)
    n[i] = (k.m[i][0] * l[0] + k.m[i][1] * l[1] + k.m[i][2] * l[2]) * k.inv_white[i];
  o[0] = 116.f * n[1] - 16.f;
  o[1] = 500.f * (n[0] - n[1]);
  o[2] = 200.f * (n[1] - n[2]);
}

__global__ __launch_bounds__(kFB) void k_flip_prep(FlipViews fv, FlipConst k,
                                                    const float* __restrict__ test,
                                                    const float* __restrict__ ref,
                                                    float* __restrict__ o, int64_t P) {
  const Px q = px_of(fv);
  if (!q.ok) return;
  float a[3], b[3], ot[3], orf[3];
  for (int c = 0; c < 3; ++c) {
    a[c] = test[q.e0 + c * q.plane];
    b[c] = ref[q.e0 + c * q.plane];
  }
  to_ycxcz(k, a, ot);
  to_ycxcz(k, b, orf);
  for (int c = 0; c < 3; ++c) {
    o[c * P + q.p] = ot[c];
    o[(3 + c) * P + q.p] = orf[c];
  }
}

// horizontal passes (x clamped to the row) of both images:
// maps per image: Y*gA, Cx*gRG, Cz*u1, Cz*u2, yn*fe, yn*gn, yn*fp
__global__ __launch_bounds__(kFB) void k_flip_h(FlipViews fv, FlipFilt f,
                                                 const float* __restrict__ o, int64_t P,
                                                 float* __restrict__ h) {
  const Px q = px_of(fv);
  if (!q.ok) return;
  const int64_t row = q.p - q.x;
  for (int im = 0; im < 2; ++im) {
    const float* Y = o + (3 * im) * P + row;
    const float* Cx = Y + P;
    const float* Cz = Y + 2 * P;
    float s[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int t = -f.rc; t <= f.rc; ++t) {
      const int xx = min(max(q.x + t, 0), q.W - 1);
      const int j = t + f.rc;
      s[0] += f.gA[j] * Y[xx];
      s[1] += f.gRG[j] * Cx[xx];
      s[2] += f.u1[j] * Cz[xx];
      s[3] += f.u2[j] * Cz[xx];
    }
    for (int t = -f.rf; t <= f.rf; ++t) {
      const int xx = min(max(q.x + t, 0), q.W - 1);
      const int j = t + f.rf;
      const float yn = (Y[xx] + 16.f) * (1.f / 116.f);
      s[4] += f.fe[j] * yn;
      s[5] += f.gn[j] * yn;
      s[6] += f.fp[j] * yn;
    }
    for (int m = 0; m < 7; ++m) h[(7 * im + m) * P + q.p] = s[m];
  }
}

// vertical pass of map `src` (column of pixel q, y clamped) with weights w[2r+1]
__device__ __forceinline__ float vpass(const float* src, const Px& q, const float* w, int r) {
  const int64_t col = q.p - (int64_t)q.y * q.W;
  float s = 0.f;
  for (int t = -r; t <= r; ++t) {
    const int yy = min(max(q.y + t, 0), q.H - 1);
    s += w[t + r] * src[col + (int64_t)yy * q.W];
  }
  return s;
}

struct Colour {
  float L, a, b;     // Hunt-adjusted CIELAB
  float Lr, ar, br;  // CIELAB before the Hunt adjustment
  float rgb[3];      // linear RGB before the clamp
  float n[3];        // XYZ / white after the clamp
};

__device__ __forceinline__ float lab_f(float t) {
  const float d = 6.f / 29.f;
  return t > d * d * d ? fpow(t, 1.f / 3.f) : t * (1.f / (3.f * d * d)) + 4.f / 29.f;
}
__device__ __forceinline__ float lab_fd(float t) {
  const float d = 6.f / 29.f;
  return t > d * d * d ? (1.f / 3.f) * fpow(t, -2.f / 3.f) : 1.f / (3.f * d * d);
}

__device__ __forceinline__ Colour colour_of(const FlipConst& k, float Y, float Cx, float Cz) {
  Colour c{};
  const float yy = (Y + 16.f) * (1.f / 116.f);
  const float xyz[3] = {k.white[0] * (Cx * (1.f / 500.f) + yy), k.white[1] * yy,
                        k.white[2] * (yy - Cz * (1.f / 200.f))};
  float l[3];
  for (int i = 0; i < 3; ++i) {
    c.rgb[i] = k.mi[i][0] * xyz[0] + k.mi[i][1] * xyz[1] + k.mi[i][2] * xyz[2];
    l[i] = fminf(fmaxf(c.rgb[i], 0.f), 1.f);
  }
  for (int i = 0; i < 3; ++i)
    c.n[i] = (k.m[i][0] * l[0] + k.m[i][1] * l[1] + k.m[i][2] * l[2]) * k.inv_white[i];
  const float fx = lab_f(c.n[0]), fy = lab_f(c.n[1]), fz = lab_f(c.n[2]);
  c.Lr = 116.f * fy - 16.f;
  c.ar = 500.f * (fx - fy);
  c.br = 200.f * (fy - fz);
  c.L = c.Lr;
  c.a = 0.01f * c.Lr * c.ar;
  c.b = 0.01f * c.Lr * c.br;
  return c;
}

// Per-pixel FLIP from the filtered colour (cf[image][Y, Cx, Cz]) and the
// feature responses (fe[image][ex, ey, px, py]) of test (0) and reference
// (1); sd receives the value's derivatives with respect to the test's
// filtered Y, Cx, Cz and its ex, ey, px, py.
__device__ __forceinline__ float flip_pixel(const FlipConst& k, const float (*cf)[3],
                                            const float (*fe)[4], float* sd) {
  // colour error
  const Colour t = colour_of(k, cf[0][0], cf[0][1], cf[0][2]);
  const Colour r = colour_of(k, cf[1][0], cf[1][1], cf[1][2]);
  const float dL = r.L - t.L, da = r.a - t.a, db = r.b - t.b;
  const float rr = da * da + db * db;
  const float root = sqrtf(fmaxf(rr, k.eps));
  const float hy = fabsf(dL) + root;
  const float e = fpow(hy, k.qc);
  const float pcc = k.pc * k.cmax;
  const bool low = e < pcc;
  const float dEc = low ? k.lo_slope * e : k.pt + (e - pcc) * k.hi_slope;
  // feature error
  const float et = sqrtf(fe[0][0] * fe[0][0] + fe[0][1] * fe[0][1]);
  const float er = sqrtf(fe[1][0] * fe[1][0] + fe[1][1] * fe[1][1]);
  const float pt = sqrtf(fe[0][2] * fe[0][2] + fe[0][3] * fe[0][3]);
  const float pr = sqrtf(fe[1][2] * fe[1][2] + fe[1][3] * fe[1][3]);
  const float d1 = fabsf(er - et), d2 = fabsf(pr - pt);
  const float mraw = fmaxf(d1, d2);
  const float m = fmaxf(mraw, k.eps);
  const float dF = fpow(m * 0.70710678118654752f, k.qf);
  const float val = fpow(dEc, 1.f - dF);
  // seeds: dval/d(filtered Y, Cx, Cz of the test), dval/d(ex, ey, px, py)
  const float g_dEc = (1.f - dF) * fpow(dEc, -dF);
  const float g_dF = -val * (0.69314718055994531f * __builtin_amdgcn_logf(dEc));
  const float g_e = g_dEc * (low ? k.lo_slope : k.hi_slope);
  const float g_hy = g_e * k.qc * fpow(hy, k.qc - 1.f);
  // d hy / d (test L, a, b) (Hunt-adjusted); the root is floored at eps
  const float sgn = dL > 0.f ? 1.f : (dL < 0.f ? -1.f : 0.f);
  float gL = -g_hy * sgn;
  const float ir = frcp(root);
  float ga = rr > k.eps ? -g_hy * da * ir : 0.f;
  float gb = rr > k.eps ? -g_hy * db * ir : 0.f;
  // Hunt: a' = L a / 100, b' = L b / 100
  const float gLr = gL + 0.01f * (t.ar * ga + t.br * gb);
  const float gar = 0.01f * t.Lr * ga, gbr = 0.01f * t.Lr * gb;
  // CIELAB from XYZ / white
  const float gfx = 500.f * gar, gfy = 116.f * gLr - 500.f * gar + 200.f * gbr,
              gfz = -200.f * gbr;
  const float gn[3] = {gfx * lab_fd(t.n[0]), gfy * lab_fd(t.n[1]), gfz * lab_fd(t.n[2])};
  // XYZ = M clamp(rgb); n = XYZ / white
  float grgb[3];
  for (int j = 0; j < 3; ++j) {
    float s = 0.f;
    for (int i = 0; i < 3; ++i) s += k.m[i][j] * gn[i] * k.inv_white[i];
    grgb[j] = (t.rgb[j] >= 0.f && t.rgb[j] <= 1.f) ? s : 0.f;
  }
  // rgb = Mi xyz(Y, Cx, Cz)
  float gxyz[3];
  for (int j = 0; j < 3; ++j)
    gxyz[j] = k.mi[0][j] * grgb[0] + k.mi[1][j] * grgb[1] + k.mi[2][j] * grgb[2];
  // xyz = white * (Cx/500 + yy, yy, yy - Cz/200), yy = (Y + 16)/116
  const float gyy = k.white[0] * gxyz[0] + k.white[1] * gxyz[1] + k.white[2] * gxyz[2];
  sd[0] = gyy * (1.f / 116.f);
  sd[1] = k.white[0] * gxyz[0] * (1.f / 500.f);
  sd[2] = -k.white[2] * gxyz[2] * (1.f / 200.f);
  // features
  const float g_m = mraw > k.eps ? g_dF * k.qf * dF * frcp(m) : 0.f;
  float gex = 0.f, gey = 0.f, gpx = 0.f, gpy = 0.f;
  if (d1 >= d2) {
    const float g_et = -g_m * ((er - et) > 0.f ? 1.f : ((er - et) < 0.f ? -1.f : 0.f));
    if (et > 0.f) {
      const float ie = frcp(et);
      gex = g_et * fe[0][0] * ie;
      gey = g_et * fe[0][1] * ie;
    }
  } else {
    const float g_pt = -g_m * ((pr - pt) > 0.f ? 1.f : ((pr - pt) < 0.f ? -1.f : 0.f));
    if (pt > 0.f) {
      const float ip = frcp(pt);
      gpx = g_pt * fe[0][2] * ip;
      gpy = g_pt * fe[0][3] * ip;
    }
  }
  sd[3] = gex;
  sd[4] = gey;
  sd[5] = gpx;
  sd[6] = gpy;
  return val;
}

// vertical passes -> per-pixel FLIP and the seeds of its gradient
__global__ __launch_bounds__(kFB) void k_flip_eval(FlipViews fv, FlipFilt f, FlipConst k,
                                                    const float* __restrict__ h, int64_t P,
                                                    float* __restrict__ seed,
                                                    float* __restrict__ blk) {
  __shared__ float s_red[kFB / 64];
  const Px q = px_of(fv);
  float val = 0.f;
  if (q.ok) {
    float cf[2][3], fe[2][4];
    for (int im = 0; im < 2; ++im) {
      const float* hm = h + (int64_t)(7 * im) * P;
      cf[im][0] = vpass(hm, q, f.gA, f.rc);
      cf[im][1] = vpass(hm + P, q, f.gRG, f.rc);
      cf[im][2] = f.c1 * vpass(hm + 2 * P, q, f.u1, f.rc) + f.c2 * vpass(hm + 3 * P, q, f.u2, f.rc);
      fe[im][0] = vpass(hm + 4 * P, q, f.gn, f.rf);  // edge x
      fe[im][1] = vpass(hm + 5 * P, q, f.fe, f.rf);  // edge y
      fe[im][2] = vpass(hm + 6 * P, q, f.gn, f.rf);  // point x
      fe[im][3] = vpass(hm + 5 * P, q, f.fp, f.rf);  // point y
    }
    float sd[7];
    val = flip_pixel(k, cf, fe, sd);
    for (int m = 0; m < 7; ++m) seed[m * P + q.p] = sd[m];
  }
  const float ws = wave_sum(val);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = ws;
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = 0.f;
    for (int i = 0; i < kFB / 64; ++i) a += s_red[i];
    blk[blockIdx.x] = a;
  }
}

// adjoint of an edge-replicated correlation along one axis: the weight that
// carries output position p onto input position i (0 <= i < n)
__device__ __forceinline__ float adj_weight(const float* w, int r, int i, int p, int n) {
  const bool lo = i == 0, hi = i == n - 1;
  if (!lo && !hi) return w[i - p + r];
  float s = 0.f;
  for (int t = -r; t <= r; ++t) {
    const int j = p + t;
    const int c = j < 0 ? 0 : (j > n - 1 ? n - 1 : j);
    if (c == i) s += w[t + r];
  }
  return s;
}

__device__ __forceinline__ float vadj(const float* src, const Px& q, const float* w, int r) {
  const int64_t col = q.p - (int64_t)q.y * q.W;
  float s = 0.f;
  const int p0 = max(q.y - r, 0), p1 = min(q.y + r, q.H - 1);
  for (int p = p0; p <= p1; ++p) s += adj_weight(w, r, q.y, p, q.H) * src[col + (int64_t)p * q.W];
  return s;
}

__device__ __forceinline__ float hadj(const float* src, const Px& q, const float* w, int r) {
  const int64_t row = q.p - q.x;
  float s = 0.f;
  const int p0 = max(q.x - r, 0), p1 = min(q.x + r, q.W - 1);
  for (int p = p0; p <= p1; ++p) s += adj_weight(w, r, q.x, p, q.W) * src[row + p];
  return s;
}

// adjoint vertical passes of the seeds
__global__ __launch_bounds__(kFB) void k_flip_vadj(FlipViews fv, FlipFilt f,
                                                    const float* __restrict__ seed, int64_t P,
                                                    float* __restrict__ t) {
  const Px q = px_of(fv);
  if (!q.ok) return;
  const int64_t o = q.p;
  t[o] = vadj(seed, q, f.gA, f.rc);
  t[P + o] = vadj(seed + P, q, f.gRG, f.rc);
  t[2 * P + o] = f.c1 * vadj(seed + 2 * P, q, f.u1, f.rc);
  t[3 * P + o] = f.c2 * vadj(seed + 2 * P, q, f.u2, f.rc);
  t[4 * P + o] = vadj(seed + 3 * P, q, f.gn, f.rf);                                   // -> fe
  t[5 * P + o] = vadj(seed + 4 * P, q, f.fe, f.rf) + vadj(seed + 6 * P, q, f.fp, f.rf);  // -> gn
  t[6 * P + o] = vadj(seed + 5 * P, q, f.gn, f.rf);                                   // -> fp
}

// adjoint horizontal passes, then the colour transforms of the test back to
// its sRGB values
__global__ __launch_bounds__(kFB) void k_flip_grad(FlipViews fv, FlipFilt f, FlipConst k,
                                                    const float* __restrict__ test,
                                                    const float* __restrict__ t, int64_t P,
                                                    float scale, int accumulate,
                                                    float* __restrict__ grad) {
  const Px q = px_of(fv);
  if (!q.ok) return;
  const float gY = hadj(t, q, f.gA, f.rc) +
                   (hadj(t + 4 * P, q, f.fe, f.rf) + hadj(t + 5 * P, q, f.gn, f.rf) +
                    hadj(t + 6 * P, q, f.fp, f.rf)) * (1.f / 116.f);
  const float gCx = hadj(t + P, q, f.gRG, f.rc);
  const float gCz = hadj(t + 2 * P, q, f.u1, f.rc) + hadj(t + 3 * P, q, f.u2, f.rc);
  // YCxCz = (116 ny - 16, 500 (nx - ny), 200 (ny - nz)), n = M lin / white
  const float gn[3] = {500.f * gCx, 116.f * gY - 500.f * gCx + 200.f * gCz, -200.f * gCz};
  const float sc = scale / (float)q.plane;
  for (int j = 0; j < 3; ++j) {
    float s = 0.f;
    for (int i = 0; i < 3; ++i) s += k.m[i][j] * gn[i] * k.inv_white[i];
    const int64_t e = q.e0 + j * q.plane;
    const float x = test[e];
    const float g = (x >= 0.f && x <= 1.f) ? s * srgb_lin_d(x) : 0.f;
    grad[e] = accumulate ? grad[e] + sc * g : sc * g;
  }
}

__global__ __launch_bounds__(kFB) void k_flip_reduce(FlipViews fv, const float* __restrict__ blk,
                                                      float* __restrict__ out) {
  __shared__ double s_r[kFB / 64];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int b = fv.blk_off[v] + (int)threadIdx.x; b < fv.blk_off[v + 1]; b += kFB) s += blk[b];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) s_r[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    s = 0.0;
    for (int w = 0; w < kFB / 64; ++w) s += s_r[w];
    out[v] = (float)(s / ((double)fv.w[v] * (double)fv.h[v]));
  }
}

// ---- tiled path (filter radii <= kFlipHalo): one workgroup per 32 x 8
// output tile of one view; the tile and its halo are staged in LDS, both
// window passes run there

constexpr int kFTX = 32, kFTY = 8, kFlipHalo = 10;
constexpr int kFRX = kFTX + 2 * kFlipHalo, kFRY = kFTY + 2 * kFlipHalo;
// row pitch of the staged forward input: = 1 mod 4, so the horizontal
// pass's items (four adjacent columns each, eight per row) hit distinct banks
constexpr int kFRXP = kFRX + 1;

struct FTile {
  int v, x0, y0, W, H;
  int64_t pix0;  // first pixel of the view in the maps
};

__device__ __forceinline__ FTile ftile(const FlipViews& fv) {
  FTile t{};
  const int v = flip_view(fv);
  const int W = fv.w[v], H = fv.h[v];
  const int gx = (W + kFTX - 1) / kFTX;
  const int b = (int)blockIdx.x - fv.blk_off[v];
  t.v = v;
  t.W = W;
  t.H = H;
  t.x0 = (b % gx) * kFTX;
  t.y0 = (b / gx) * kFTY;
  t.pix0 = fv.pix_off[v];
  return t;
}

constexpr int kFTap = 2 * kFlipHalo + 1;

// the seven 1D filters, zero-padded to kFTap taps (centre at kFlipHalo):
// 0 gA, 1 gRG, 2 u1, 3 u2 (radius rc); 4 gn, 5 fe, 6 fp (radius rf)
__device__ __forceinline__ void load_weights(const FlipFilt& f, float (*w)[kFTap]) {
  for (int i = threadIdx.x; i < 7 * kFTap; i += kFB) {
    const int m = i / kFTap, t = i - m * kFTap - kFlipHalo;
    const int r = m < 4 ? f.rc : f.rf;
    const float* src = m == 0 ? f.gA : m == 1 ? f.gRG : m == 2 ? f.u1 : m == 3 ? f.u2
                     : m == 4 ? f.gn : m == 5 ? f.fe : f.fp;
    w[m][t + kFlipHalo] = (t >= -r && t <= r) ? src[t + r] : 0.0f;
  }
}

// Per filter, the sums of its zero-padded taps up to and from each index:
// cs[m][0][t] = w[0] + ... + w[t] and cs[m][1][t] = w[t] + ... + w[kFTap-1],
// both added in increasing tap order.
__device__ __forceinline__ void load_tap_sums(const FlipFilt& f, float (*cs)[2][kFTap]) {
  for (int i = threadIdx.x; i < 7 * kFTap; i += kFB) {
    const int m = i / kFTap, t = i - m * kFTap;
    const int r = m < 4 ? f.rc : f.rf;
    const float* src = m == 0 ? f.gA : m == 1 ? f.gRG : m == 2 ? f.u1 : m == 3 ? f.u2
                     : m == 4 ? f.gn : m == 5 ? f.fe : f.fp;
    float pre = 0.f, suf = 0.f;
    for (int j = 0; j < kFTap; ++j) {
      const int d = j - kFlipHalo;
      const float wj = (d >= -r && d <= r) ? src[d + r] : 0.0f;
      if (j <= t) pre += wj;
      if (j >= t) suf += wj;
    }
    cs[m][0][t] = pre;
    cs[m][1][t] = suf;
  }
}

// At most 168 VGPRs (3 waves per SIMD), the occupancy the kernel's LDS
// allows; without the bound the compiler takes 182 and runs 2 (with it, 6
// VGPRs spill, which costs less).
__global__ __launch_bounds__(kFB) __attribute__((amdgpu_waves_per_eu(3))) void k_flip_fwd_tile(FlipViews fv, FlipFilt f, FlipConst k,
                                                        const float* __restrict__ o,
                                                        float* __restrict__ seed, int64_t P,
                                                        float* __restrict__ blk) {
  __shared__ float s_w[7][kFTap];
  __shared__ float s_in[3][kFRY][kFRXP];
  __shared__ float s_h[7][kFRY][kFTX];
  __shared__ float s_red[kFB / 64];
  const FTile T = ftile(fv);
  load_weights(f, s_w);
  const int oy = threadIdx.x / kFTX, ox = threadIdx.x % kFTX;
  const int x = T.x0 + ox, y = T.y0 + oy;
  float cf[2][3], fe[2][4];
  for (int im = 1; im >= 0; --im) {  // reference first, then the test
    const float* src = o + (int64_t)(3 * im) * P + T.pix0;
    for (int i = threadIdx.x; i < kFRY * kFRX; i += kFB) {
      const int r = i / kFRX, c = i - r * kFRX;
      const int yy = min(max(T.y0 + r - kFlipHalo, 0), T.H - 1);
      const int xx = min(max(T.x0 + c - kFlipHalo, 0), T.W - 1);
      const int64_t e = (int64_t)yy * T.W + xx;
      s_in[0][r][c] = src[e];
      s_in[1][r][c] = src[P + e];
      s_in[2][r][c] = src[2 * P + e];
    }
    __syncthreads();
    // horizontal passes, four adjacent outputs per item sharing their taps
    for (int i = threadIdx.x; i < kFRY * (kFTX / 4); i += kFB) {
      const int r = i / (kFTX / 4), c0 = (i - r * (kFTX / 4)) * 4;
      float dY[kFTap + 3], dX[kFTap + 3], dZ[kFTap + 3];
#pragma unroll
      for (int j = 0; j < kFTap + 3; ++j) {
        dY[j] = s_in[0][r][c0 + j];
        dX[j] = s_in[1][r][c0 + j];
        dZ[j] = s_in[2][r][c0 + j];
      }
      float a[4][7];
#pragma unroll
      for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int m = 0; m < 7; ++m) a[o][m] = 0.f;
#pragma unroll
      for (int j = 0; j < kFTap; ++j) {
        const float w0 = s_w[0][j], w1 = s_w[1][j], w2 = s_w[2][j], w3 = s_w[3][j];
        const float w4 = s_w[4][j], w5 = s_w[5][j], w6 = s_w[6][j];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
          // the feature passes run on Y: every feature kernel sums to zero,
          // so on the normalised luminance (Y + 16) / 116 they give the
          // same responses divided by 116 (applied after the vertical pass)
          const float Y = dY[j + o], cz = dZ[j + o];
          a[o][0] = __builtin_fmaf(w0, Y, a[o][0]);
          a[o][1] = __builtin_fmaf(w1, dX[j + o], a[o][1]);
          a[o][2] = __builtin_fmaf(w2, cz, a[o][2]);
          a[o][3] = __builtin_fmaf(w3, cz, a[o][3]);
          a[o][4] = __builtin_fmaf(w5, Y, a[o][4]);  // edge profile along x
          a[o][5] = __builtin_fmaf(w4, Y, a[o][5]);  // Gaussian along x
          a[o][6] = __builtin_fmaf(w6, Y, a[o][6]);  // point profile along x
        }
      }
#pragma unroll
      for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int m = 0; m < 7; ++m) s_h[m][r][c0 + o] = a[o][m];
    }
    __syncthreads();
    // vertical passes: thread (k, column) gives filter output k of all kFTY
    // rows of its column from a register window of the column (taps in
    // increasing order, as per pixel); the outputs go through LDS (the staged
    // input is dead by now) to their pixels' threads
    static_assert(8 * kFTX == kFB && 8 * kFTY * kFTX <= 3 * kFRY * kFRXP, "vertical items");
    {
      const int vk = threadIdx.x / kFTX, vc = threadIdx.x % kFTX;
      // (filter, horizontal map) of output k: 0..5 as is, 6 = px, 7 = py
      const int wk = vk == 6 ? 4 : vk == 7 ? 6 : vk;
      const int hm = vk == 7 ? 5 : vk;
      float acc[kFTY];
#pragma unroll
      for (int oy2 = 0; oy2 < kFTY; ++oy2) acc[oy2] = 0.f;
#pragma unroll
      for (int j = 0; j < kFTap; ++j) {
        const float w = s_w[wk][j];
#pragma unroll
        for (int oy2 = 0; oy2 < kFTY; ++oy2)
          acc[oy2] = __builtin_fmaf(w, s_h[hm][oy2 + j][vc], acc[oy2]);
      }
      float* s_vo = &s_in[0][0][0];  // [8][kFTY][kFTX]
#pragma unroll
      for (int oy2 = 0; oy2 < kFTY; ++oy2) s_vo[(vk * kFTY + oy2) * kFTX + vc] = acc[oy2];
    }
    __syncthreads();
    float v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = (&s_in[0][0][0])[(m * kFTY + oy) * kFTX + ox];
    cf[im][0] = v[0];
    cf[im][1] = v[1];
    cf[im][2] = f.c1 * v[2] + f.c2 * v[3];
    fe[im][0] = v[4] * (1.f / 116.f);
    fe[im][1] = v[5] * (1.f / 116.f);
    fe[im][2] = v[6] * (1.f / 116.f);
    fe[im][3] = v[7] * (1.f / 116.f);
    __syncthreads();
  }
  float val = 0.f;
  if (x < T.W && y < T.H) {
    float sd[7];
    val = flip_pixel(k, cf, fe, sd);
    const int64_t oo = T.pix0 + (int64_t)y * T.W + x;
    for (int m = 0; m < 7; ++m) seed[m * P + oo] = sd[m];
  }
  const float ws = wave_sum(val);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = ws;
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = 0.f;
    for (int i = 0; i < kFB / 64; ++i) a += s_red[i];
    blk[blockIdx.x] = a;
  }
}

// Adjoint of an edge-replicated 1D correlation at input position i of n,
// from the outputs g(p) at LDS positions (base + p) * stride, which hold
// zero for p outside the image: interior positions take sum_t w[t] g(i - t)
// over the whole staged window.  A border position also takes every tap that
// the replication folded onto it: output p reaches input 0 through its taps
// t <= halo - p and input n - 1 through its taps t >= halo + n - 1 - p (a
// one-pixel line: all taps), so its weight is a prefix or suffix sum `cs` of
// the filter's taps.
__device__ __forceinline__ float adj1d(const float* w, const float (*cs)[kFTap], int i, int n,
                                       const float* g, int base, int stride) {
  float s = 0.f;
  if (i > 0 && i < n - 1) {
    const float* gi = g + (base + i + kFlipHalo) * stride;
#pragma unroll
    for (int j = 0; j < kFTap; ++j) s = __builtin_fmaf(w[j], gi[-j * stride], s);
    return s;
  }
  const int p0 = max(i - kFlipHalo, 0), p1 = min(i + kFlipHalo, n - 1);
  for (int p = p0; p <= p1; ++p) {
    const float wt = n == 1   ? cs[0][kFTap - 1]
                     : i == 0 ? cs[0][kFlipHalo - p]
                              : cs[1][kFlipHalo + n - 1 - p];
    s += wt * g[(base + p) * stride];
  }
  return s;
}

__global__ __launch_bounds__(kFB) void k_flip_bwd_tile(FlipViews fv, FlipFilt f, FlipConst k,
                                                        const float* __restrict__ test,
                                                        const float* __restrict__ seed, int64_t P,
                                                        float scale, int accumulate,
                                                        float* __restrict__ grad) {
  __shared__ float s_w[7][kFTap];
  __shared__ float s_cs[7][2][kFTap];
  __shared__ float s_s[7][kFRY][kFRX];
  __shared__ float s_v[7][kFTY][kFRX];
  const FTile T = ftile(fv);
  load_weights(f, s_w);
  load_tap_sums(f, s_cs);
  // seeds of the tile and its halo (zero outside the image)
  for (int i = threadIdx.x; i < kFRY * kFRX; i += kFB) {
    const int r = i / kFRX, c = i - r * kFRX;
    const int yy = T.y0 + r - kFlipHalo, xx = T.x0 + c - kFlipHalo;
    float val[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (yy >= 0 && yy < T.H && xx >= 0 && xx < T.W) {
      const int64_t oo = T.pix0 + (int64_t)yy * T.W + xx;
      for (int m = 0; m < 7; ++m) val[m] = seed[m * P + oo];
    }
    for (int m = 0; m < 7; ++m) s_s[m][r][c] = val[m];
  }
  __syncthreads();
  // adjoint vertical passes at the tile's rows, every in-image halo column;
  // row p of the image sits at LDS row p - y0 + halo.  One item per (output
  // map, column): when every tile row is an interior row of the image, the
  // column's kFRY staged seeds are read once into registers and give all
  // kFTY rows (taps added in the order adj1d adds them); otherwise each row
  // takes adj1d.  Output map 5 sums two filters (ey and py).
  const int rbase = kFlipHalo - T.y0;
  const bool rows_inside = T.y0 > 0 && T.y0 + kFTY < T.H;  // 0 < y < H - 1 for every row
  for (int i = threadIdx.x; i < 7 * kFRX; i += kFB) {
    const int dm = i / kFRX, c = i - dm * kFRX;
    const int xx = T.x0 + c - kFlipHalo;
    // (filter, seed map) of the output map's terms and its colour weight
    const int wk = dm == 6 ? 4 : dm, sm = dm <= 2 ? dm : dm - 1;
    const float sc = dm == 2 ? f.c1 : dm == 3 ? f.c2 : 1.f;
    const int sm2 = dm == 3 ? 2 : sm;
    float acc[kFTY];
#pragma unroll
    for (int oy = 0; oy < kFTY; ++oy) acc[oy] = 0.f;
    if (xx >= 0 && xx < T.W) {
      if (rows_inside) {
        float wv[kFTap], col[kFRY];
#pragma unroll
        for (int j = 0; j < kFTap; ++j) wv[j] = s_w[wk][j];
#pragma unroll
        for (int r = 0; r < kFRY; ++r) col[r] = s_s[sm2][r][c];
#pragma unroll
        for (int oy = 0; oy < kFTY; ++oy) {
          float s = 0.f;
#pragma unroll
          for (int j = 0; j < kFTap; ++j) s = __builtin_fmaf(wv[j], col[oy + 2 * kFlipHalo - j], s);
          acc[oy] = s;
        }
        if (dm == 5) {
#pragma unroll
          for (int j = 0; j < kFTap; ++j) wv[j] = s_w[6][j];
#pragma unroll
          for (int r = 0; r < kFRY; ++r) col[r] = s_s[6][r][c];
#pragma unroll
          for (int oy = 0; oy < kFTY; ++oy) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < kFTap; ++j)
              s = __builtin_fmaf(wv[j], col[oy + 2 * kFlipHalo - j], s);
            acc[oy] = acc[oy] + s;
          }
        }
      } else {
        for (int oy = 0; oy < kFTY; ++oy) {
          const int y = T.y0 + oy;
          if (y >= T.H) break;
          float s = adj1d(s_w[wk], s_cs[wk], y, T.H, &s_s[sm2][0][c], rbase, kFRX);
          if (dm == 5) s = s + adj1d(s_w[6], s_cs[6], y, T.H, &s_s[6][0][c], rbase, kFRX);
          acc[oy] = s;
        }
      }
    }
#pragma unroll
    for (int oy = 0; oy < kFTY; ++oy) s_v[dm][oy][c] = sc * acc[oy];
  }
  __syncthreads();
  // adjoint horizontal passes: item (filter term, row, 4 adjacent columns)
  // gives its 4 outputs from one register window of the row when all 4 are
  // interior columns of the image (taps in the order adj1d adds them), else
  // per column through adj1d; the terms go through LDS (the staged seeds are
  // dead by now) and each pixel sums its own
  const int cbase = kFlipHalo - T.x0;
  float* s_p = &s_s[0][0][0];  // [7][kFTY][kFTX]
  static_assert(7 * kFTY * kFTX <= 7 * kFRY * kFRX, "horizontal terms");
  for (int i = threadIdx.x; i < 7 * kFTY * (kFTX / 4); i += kFB) {
    const int hk = i / (kFTY * (kFTX / 4));
    const int rem = i - hk * (kFTY * (kFTX / 4));
    const int hy = rem / (kFTX / 4), c0 = (rem - hy * (kFTX / 4)) * 4;
    // (filter, vertical map) of term hk: A, RG, B1, B2, ex, px, py
    const int wk = hk == 4 ? 5 : hk == 5 ? 4 : hk;
    const float* row = s_v[hk][hy];
    float out[4];
    const int xa = T.x0 + c0;
    if (xa > 0 && xa + 3 < T.W - 1) {
      float win[kFTap + 3];
#pragma unroll
      for (int j = 0; j < kFTap + 3; ++j) win[j] = row[c0 + j];
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < kFTap; ++j) s = __builtin_fmaf(s_w[wk][j], win[o + 2 * kFlipHalo - j], s);
        out[o] = s;
      }
    } else {
      for (int o = 0; o < 4; ++o)
        out[o] = xa + o < T.W ? adj1d(s_w[wk], s_cs[wk], xa + o, T.W, row, cbase, 1) : 0.f;
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) s_p[(hk * kFTY + hy) * kFTX + c0 + o] = out[o];
  }
  __syncthreads();
  const int oy = threadIdx.x / kFTX, ox = threadIdx.x % kFTX;
  const int x = T.x0 + ox, y = T.y0 + oy;
  if (x >= T.W || y >= T.H) return;
  const int pp = oy * kFTX + ox, ps = kFTY * kFTX;
  const float gA = s_p[pp];
  const float gRG = s_p[ps + pp];
  const float gB = s_p[2 * ps + pp] + s_p[3 * ps + pp];
  const float gF = s_p[4 * ps + pp] + s_p[5 * ps + pp] + s_p[6 * ps + pp];
  const float gY = gA + gF * (1.f / 116.f);
  const float gn[3] = {500.f * gRG, 116.f * gY - 500.f * gRG + 200.f * gB, -200.f * gB};
  const int64_t plane = (int64_t)T.W * T.H;
  const float sc = scale / (float)plane;
  const int64_t e0 = 3 * T.pix0 + (int64_t)y * T.W + x;
  for (int j = 0; j < 3; ++j) {
    float s = 0.f;
    for (int i = 0; i < 3; ++i) s += k.m[i][j] * gn[i] * k.inv_white[i];
    const int64_t e = e0 + j * plane;
    const float xv = test[e];
    const float g = (xv >= 0.f && xv <= 1.f) ? s * srgb_lin_d(xv) : 0.f;
    grad[e] = accumulate ? grad[e] + sc * g : sc * g;
  }
}

}  // namespace

int64_t flip_blocks(int w, int h) { return ((int64_t)w * h + kFB - 1) / kFB; }

int flip_tile_halo() { return kFlipHalo; }

int64_t flip_tile_blocks(int w, int h) {
  return (int64_t)((w + kFTX - 1) / kFTX) * ((h + kFTY - 1) / kFTY);
}

hipError_t launch_flip_tiled(const FlipViews& fv, int n_blocks, const FlipFilt& f,
                             const FlipConst& k, const float* test, const float* ref,
                             float* maps, int64_t P, float* blk, float scale, bool accumulate,
                             float* out, float* grad, hipStream_t stream) {
  // YCxCz of both images once per pixel (6 maps), then the tiles
  float* o = maps;
  float* seed = maps + 6 * P;
  unsigned pix_blocks = 0;
  for (int v = 0; v < fv.n_views; ++v) pix_blocks += (unsigned)flip_blocks(fv.w[v], fv.h[v]);
  FlipViews pv = fv;
  for (int v = 0, b = 0; v <= fv.n_views; ++v) {
    pv.blk_off[v] = b;
    if (v < fv.n_views) b += (int)flip_blocks(fv.w[v], fv.h[v]);
  }
  hipLaunchKernelGGL(k_flip_prep, dim3(pix_blocks), dim3(kFB), 0, stream, pv, k, test, ref, o, P);
  const dim3 grid((unsigned)n_blocks), block(kFB);
  hipLaunchKernelGGL(k_flip_fwd_tile, grid, block, 0, stream, fv, f, k, o, seed, P, blk);
  hipLaunchKernelGGL(k_flip_bwd_tile, grid, block, 0, stream, fv, f, k, test, seed, P, scale,
                     accumulate ? 1 : 0, grad);
  hipLaunchKernelGGL(k_flip_reduce, dim3((unsigned)fv.n_views), dim3(kFB), 0, stream, fv, blk, out);
  return hipGetLastError();
}

hipError_t launch_flip(const FlipViews& fv, int n_blocks, const FlipFilt& f, const FlipConst& k,
                       const float* test, const float* ref, float* maps, int64_t P, float* blk,
                       float scale, bool accumulate, float* out, float* grad,
                       hipStream_t stream) {
  float* o = maps;            // 6 maps: YCxCz of test and reference
  float* h = maps + 6 * P;    // 14 maps: horizontal passes; later 7 adjoint maps
  float* seed = maps + 20 * P;  // 7 maps
  const dim3 grid((unsigned)n_blocks), block(kFB);
  hipLaunchKernelGGL(k_flip_prep, grid, block, 0, stream, fv, k, test, ref, o, P);
  hipLaunchKernelGGL(k_flip_h, grid, block, 0, stream, fv, f, o, P, h);
  hipLaunchKernelGGL(k_flip_eval, grid, block, 0, stream, fv, f, k, h, P, seed, blk);
  hipLaunchKernelGGL(k_flip_vadj, grid, block, 0, stream, fv, f, seed, P, h);
  hipLaunchKernelGGL(k_flip_grad, grid, block, 0, stream, fv, f, k, test, h, P, scale,
                     accumulate ? 1 : 0, grad);
  hipLaunchKernelGGL(k_flip_reduce, dim3((unsigned)fv.n_views), dim3(kFB), 0, stream, fv, blk, out);
  return hipGetLastError();
}

}  // namespace seele
