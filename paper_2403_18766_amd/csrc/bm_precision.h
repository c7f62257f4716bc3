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

// Greedy K-means++ initial D of the wide points of every job whose K-means++
// has centroids to fill and kept centroids: D_i = min over the kept centroids
// (deg[j] == 0) of ||S_i - c_j||^2, found on the FP32 matrix cores with the
// assignment's certification (the winner's distance in the block-wise direct
// form), written to D (slot 0) with the FP64 sum of every 256-point tile.
struct KppInitOut {
  const KppState* ks;       // [job]: jobs with ntodo == 0 or has_d == 0 are skipped
  const uint8_t* deg;       // [job][k]
  float* D;                 // job j's D at D + j * D_job_stride
  int64_t D_job_stride;
  double* Dt;               // job j's tile sums at Dt + j * Dt_job_stride
  int64_t Dt_job_stride;
};
// a: as for launch_assign_wide with labels, st and tnear null (objective mode);
// the norms cn must be those of Cp.
hipError_t launch_kpp_init_wide(hipStream_t st, const AssignArgs& a, int32_t ntiles,
                                const KppInitOut& kp);

// K-means++ potentials with the rows staged through LDS by coalesced loads
// (same results as launch_kpp_pot; the faster one for rows of 32 floats or
// more).
hipError_t launch_kpp_pot_staged(hipStream_t st, const KppArgs& a, int32_t njobs, int64_t max_s);

}  // namespace bm
