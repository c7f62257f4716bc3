// Declarations of kernels of bm_wide.hip that bm_kernels.hip does not share
// (matrix-core precisions, staged K-means++ potentials); the argument
// structures are in bm_internal.h.
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

// K-means++ potentials with the rows staged through LDS by coalesced loads
// (same results as launch_kpp_pot; the faster one for rows of 32 floats or
// more).
hipError_t launch_kpp_pot_staged(hipStream_t st, const KppArgs& a, int32_t njobs, int64_t max_s);

}  // namespace bm
