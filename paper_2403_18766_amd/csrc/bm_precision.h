// Declarations of the reduced-precision kernels (bm_wide.hip); the shared
// argument structures are in bm_internal.h.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

#include "bm_internal.h"

namespace bm {

// Wide-point assignment (cp > kMaxRegDim) with the dot products on the BF16
// matrix cores: FP32 rows and centroids are split into BF16 high parts and
// residuals while they are staged, and x.c = xh.ch + xh.cl + xl.ch accumulates
// in FP32.  Same arguments, outputs and decision rules as launch_assign_wide;
// tile_pts must be a multiple of 256.
hipError_t launch_assign_wide_bf16(hipStream_t st, const AssignArgs& a, int32_t ntiles, bool sums);

}  // namespace bm
