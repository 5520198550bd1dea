// Scene storage order (Morton order of the means) shared between layout.hip
// and the C ABI.
#pragma once

#include "seele_internal.h"

namespace seele {

size_t spatial_order_workspace_size(int64_t n);
hipError_t launch_spatial_order(const float* means, int64_t n, void* ws, int64_t* perm,
                                hipStream_t stream);

}  // namespace seele
