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

}  // namespace seele
