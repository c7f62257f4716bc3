// Static workspace of bm_objective_noalloc: one device array per GPU that
// holds the objective's tile map, padded centroids and norms, per-chunk
// partials and results, so that the call allocates nothing.
//
// The array's name is a host-side stand-in in host code: its device address
// is looked up once per device (noalloc_scratch, with that device current)
// and only that address is ever handed to kernels or copies.

#include <mutex>

#include <hip/hip_runtime.h>

#include "bm_internal.h"

namespace bm {

namespace {

__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Tile map of one job of m points (tile t covers points [t * tile_pts, ...))
// and its size.
__global__ __launch_bounds__(kWG) void k_noalloc_tiles(int32_t* __restrict__ tile_job,
                                                        int32_t* __restrict__ tile_idx,
                                                        int32_t ntiles, int64_t* __restrict__ sizes,
                                                        int64_t m) {
  const int t = blockIdx.x * kWG + threadIdx.x;
  if (t < ntiles) {
    tile_job[t] = 0;
    tile_idx[t] = t;
  }
  if (t == 0) sizes[0] = m;
}

}  // namespace

hipError_t noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

hipError_t launch_noalloc_tiles(hipStream_t st, int32_t* tile_job, int32_t* tile_idx,
                                int32_t ntiles, int64_t* sizes, int64_t m) {
  const int blocks = (ntiles + kWG - 1) / kWG;
  hipLaunchKernelGGL(k_noalloc_tiles, dim3(blocks > 0 ? blocks : 1), dim3(kWG), 0, st, tile_job,
                     tile_idx, ntiles, sizes, m);
  return hipGetLastError();
}

}  // namespace bm
