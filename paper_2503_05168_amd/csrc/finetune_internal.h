// Fine-tuning kernels (loss and optimizer) shared between finetune.hip and
// the C ABI.
#pragma once

#include "seele_internal.h"

namespace seele {

// Photometric loss (fine-tuning): one launch covers up to kMaxViewsLoss
// views; a workgroup (one view, channel and 32 x 16 tile) never straddles
// two views, and blk_off counts workgroups.
constexpr int kMaxViewsLoss = 64;
struct LossViews {
  int n_views;
  int64_t elem_off[kMaxViewsLoss + 1];  // first element of view v ([3][H][W] per view)
  int32_t blk_off[kMaxViewsLoss + 1];   // first block of view v
  int32_t w[kMaxViewsLoss], h[kMaxViewsLoss];
};

int64_t loss_blocks(int w, int h);
hipError_t launch_photometric_loss(const LossViews& lv, int n_blocks, const float* img,
                                   const float* tgt, float lambda, float inv_views, float* maps,
                                   int64_t stride, float* blk, float* loss, float* grad,
                                   hipStream_t stream);
hipError_t launch_adam(float* const* p, const float* const* g, float* const* m, float* const* v,
                       const int64_t* len, const float* lr, float b1, float b2, float eps,
                       int64_t step, hipStream_t stream);

// FLIP (view-consistency term): pixel blocks of 256 never straddle a view.
constexpr int kMaxViewsFlip = 64;
constexpr int kMaxFlipRadius = 24;
struct FlipViews {
  int n_views;
  int64_t pix_off[kMaxViewsFlip + 1];  // first pixel of view v in the maps
  int32_t blk_off[kMaxViewsFlip + 1];
  int32_t w[kMaxViewsFlip], h[kMaxViewsFlip];
};
// separable filters: CSF (radius rc) for Y (gA), Cx (gRG) and Cz
// (c1 u1 + c2 u2 in both axes); feature (radius rf): normalised Gaussian gn,
// edge fe and point fp profiles
struct FlipFilt {
  int rc, rf;
  float c1, c2;
  float gA[2 * kMaxFlipRadius + 1], gRG[2 * kMaxFlipRadius + 1];
  float u1[2 * kMaxFlipRadius + 1], u2[2 * kMaxFlipRadius + 1];
  float gn[2 * kMaxFlipRadius + 1], fe[2 * kMaxFlipRadius + 1], fp[2 * kMaxFlipRadius + 1];
};
struct FlipConst {
  float m[3][3], mi[3][3], white[3], inv_white[3];
  float qc, qf, pc, pt, eps, cmax;
  float lo_slope, hi_slope;  // pt / (pc cmax) and (1 - pt) / (cmax - pc cmax)
};

int64_t flip_blocks(int w, int h);
// tiled path: filter radii up to flip_tile_halo(), one block per 32 x 8 tile
int flip_tile_halo();
int64_t flip_tile_blocks(int w, int h);
hipError_t launch_flip_tiled(const FlipViews& fv, int n_blocks, const FlipFilt& f,
                             const FlipConst& k, const float* test, const float* ref,
                             float* maps, int64_t P, float* blk, float scale, bool accumulate,
                             float* out, float* grad, hipStream_t stream);
hipError_t launch_flip(const FlipViews& fv, int n_blocks, const FlipFilt& f, const FlipConst& k,
                       const float* test, const float* ref, float* maps, int64_t P, float* blk,
                       float scale, bool accumulate, float* out, float* grad,
                       hipStream_t stream);

}  // namespace seele
