// Counter-based randomness of the library (device and host).
//
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128 multiplications with Weyl-sequence key bumps.  The SplitMix64
// finaliser (Steele, Lea, Flood, OOPSLA'14) is the Feistel round function
// of the sampler.  The sampler permutes [0, 4^h) with a 4-round balanced
// Feistel network and walks each value into [0, m) (cycle walking), which
// gives s distinct rows for s <= m: the paper's uniform random sample
// without repetition (Section 4.1, Algorithm 1).
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace bm {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;
constexpr uint64_t kMixC1 = 0xBF58476D1CE4E5B9ull;
constexpr uint64_t kMixC2 = 0x94D049BB133111EBull;

struct U64x4 {
  uint64_t w[4];
};

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
#endif
}

__host__ __device__ inline U64x4 philox4x64_10(U64x4 x, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t hi0 = mulhi64(kPhiloxM0, x.w[0]);
    const uint64_t lo0 = kPhiloxM0 * x.w[0];
    const uint64_t hi1 = mulhi64(kPhiloxM1, x.w[2]);
    const uint64_t lo1 = kPhiloxM1 * x.w[2];
    U64x4 y;
    y.w[0] = hi1 ^ x.w[1] ^ k0;
    y.w[1] = lo1;
    y.w[2] = hi0 ^ x.w[3] ^ k1;
    y.w[3] = lo0;
    x = y;
  }
  return x;
}

// Key of the stream (seed, worker, purpose).
__host__ __device__ inline void stream_key(uint64_t seed, uint32_t worker, uint32_t purpose,
                                           uint64_t* k0, uint64_t* k1) {
  *k0 = seed;
  *k1 = ((uint64_t)worker << 8) | (uint64_t)purpose;
}

__host__ __device__ inline U64x4 philox_ctr(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                            uint64_t k0, uint64_t k1) {
  U64x4 c;
  c.w[0] = c0;
  c.w[1] = c1;
  c.w[2] = c2;
  c.w[3] = c3;
  return philox4x64_10(c, k0, k1);
}

// u(w) = (w >> 11) * 2^-53 in [0, 1).
__host__ __device__ inline double u01(uint64_t w) {
  return (double)(w >> 11) * 1.1102230246251565404236316680908203125e-16;
}

// floor(w * n / 2^64), in [0, n).
__host__ __device__ inline uint64_t bounded(uint64_t w, uint64_t n) { return mulhi64(w, n); }

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * kMixC1;
  z = (z ^ (z >> 27)) * kMixC2;
  return z ^ (z >> 31);
}

// h = max(1, ceil(ceil(log2 m) / 2)): the Feistel domain [0, 4^h) covers [0, m).
__host__ __device__ inline int feistel_half_bits(uint64_t m) {
  int lg = 0;
  while (lg < 64 && (1ull << lg) < m) ++lg;  // ceil(log2 m) for m >= 1
  const int h = (lg + 1) / 2;
  return h < 1 ? 1 : h;
}

struct FeistelKey {
  uint64_t rk[4];
  uint64_t m;
  int h;
};

__host__ __device__ inline FeistelKey feistel_key(uint64_t m, uint64_t seed, uint32_t worker,
                                                  uint32_t purpose, uint64_t g) {
  uint64_t k0, k1;
  stream_key(seed, worker, purpose, &k0, &k1);
  const U64x4 b = philox_ctr(g, 0, 0, 0, k0, k1);
  FeistelKey fk;
  for (int r = 0; r < 4; ++r) fk.rk[r] = b.w[r];
  fk.m = m;
  fk.h = feistel_half_bits(m);
  return fk;
}

__host__ __device__ inline uint64_t feistel_permute(uint64_t x, const FeistelKey& fk) {
  const uint64_t mask = (1ull << fk.h) - 1ull;
  uint64_t left = x >> fk.h;
  uint64_t right = x & mask;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint64_t f = mix64(right ^ fk.rk[r]) & mask;
    const uint64_t nl = right;
    right = left ^ f;
    left = nl;
  }
  return (left << fk.h) | right;
}

// Row index of sample element i (i < m).  The walk ends because the
// permutation's cycle through i returns to i < m; the expected number of
// steps is below 4 since 4^h < 4 m.  The step cap only guards memory safety
// (a result >= m is never returned): a walk of 2^20 steps has probability
// far below 2^-400.
__host__ __device__ inline uint64_t feistel_index(uint64_t i, const FeistelKey& fk) {
  uint64_t y = feistel_permute(i, fk);
  for (int step = 0; y >= fk.m && step < (1 << 20); ++step) y = feistel_permute(y, fk);
  return y < fk.m ? y : fk.m - 1;
}

}  // namespace bm
