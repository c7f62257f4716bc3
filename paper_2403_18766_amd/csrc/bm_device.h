// Device helpers shared by the kernel sources (gfx950, wave64).
#pragma once

#include <math.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace bm {
namespace {

constexpr float kU = 5.9604644775390625e-8f;  // 2^-24, unit roundoff of FP32

// Butterfly sums over a wave: every lane ends with the same total, and the
// order of the additions depends only on the lane positions.
__device__ inline double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline int wave_sum_i32(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Value of v in lane l (l uniform), broadcast through SGPRs.
__device__ inline double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned int lo = (unsigned int)__builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const unsigned int hi = (unsigned int)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum of the 64 lane values in lane order, the same in every lane.
__device__ inline double wave_ordered_sum(double v) {
  double total = 0.0;
#pragma unroll 8
  for (int l = 0; l < 64; ++l) total += lane_value(v, l);
  return total;
}

// Deterministic sum of v[0..cnt) by one wave: lane l adds a contiguous chunk
// in order, then the 64 chunk totals are added in lane order.  The result is
// the same in every lane and depends only on cnt and the values.
__device__ inline double wave_chunked_sum(const double* __restrict__ v, int64_t cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t cs = (cnt + 63) / 64;
  const int64_t lo = min(cnt, (int64_t)lane * cs), hi = min(cnt, lo + cs);
  double tot = 0.0;
  // eight loads issued together, added in index order
  for (int64_t q0 = lo; q0 < hi; q0 += 8) {
    double t[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) t[q] = q0 + q < hi ? v[q0 + q] : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (q0 + q < hi) tot += t[q];
  }
  return wave_ordered_sum(tot);
}

// Fixed-point value of one coordinate: trunc(x * 2^shift_d), exact in int64
// for the scales the library derives from the data.
__device__ inline long long quantize(float x, double scale) {
  return (long long)((double)x * scale);
}

}  // namespace
}  // namespace bm
