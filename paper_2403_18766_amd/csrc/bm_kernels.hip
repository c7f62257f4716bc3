// gfx950 kernels of the Big-means hot path.
//
//   k_sample          sample without replacement + row gather (Section 4.1)
//   k_assign_small    nearest-centre assignment, FP64 objective partials and
//                     fixed-point per-cluster sums for one Lloyd iteration, or
//                     the objective of Eq. (1) alone (dimension <= 64)
//   k_finalize        cluster means, convergence test, Lloyd job state
//   k_kpp_*           greedy K-means++ steps (Section 3, Section 5)
//   k_accept          strict-improvement acceptance (Algorithm 1)
//
// Layout: samples are row-major with a padded row stride cp (a multiple of 4,
// zero-filled), so a point is NP/4 16-byte loads and sits in NP registers of
// its lane; centroids are padded the same way and are uniform across a wave,
// so the compiler reads them with scalar loads (SGPR operands of the FMAs).
//
// Numerics: the argmin runs on e_j = ||c_j||^2 - 2 x.c_j (one FMA per
// dimension).  Its rounding error is bounded per point by
// B = 2(2 gamma + 2u)(|x| cmax + cmax^2), gamma = (NP/2+1)u/(1-(NP/2+1)u),
// u = 2^-24 (two interleaved partial sums).  A point whose two best e
// differ by more than 2B plus 2.5e-5 (e2 + |x|^2) keeps its winner; any other
// point is decided again in the direct form sum_d (x_d - c_d)^2 over all
// centres (lowest index on ties), which also counts the near ties
// d2 - d1 < 1e-5 d2.  The winner's distance entering f is always the direct
// form.  f is summed in FP64 in a fixed order (wave butterfly, waves, tiles),
// and the per-cluster sums are exact 64-bit fixed-point integers, so every
// result is bitwise reproducible and independent of scheduling.

#include <math.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "bm_device.h"
#include "bm_internal.h"
#include "bm_rng.h"

namespace bm {

namespace {




// Deterministic sum over a 256-thread workgroup; result valid in thread 0.
__device__ inline double block_sum_f64(double v, double* sh4) {
  v = wave_sum_f64(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh4[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
  __syncthreads();
  return r;
}

__device__ inline int block_sum_i32(int v, int* sh4) {
  v = wave_sum_i32(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh4[w] = v;
  __syncthreads();
  int r = 0;
  if (threadIdx.x == 0) r = (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
  __syncthreads();
  return r;
}


// min that propagates NaN from either operand.
__device__ inline float min_nan(float a, float b) {
  const float r = b < a ? b : a;
  return (a != a || b != b) ? __builtin_nanf("") : r;
}

// Squared distance in the direct form with four interleaved partial sums;
// x and c are read from memory (any n).
__device__ inline float dist_direct_mem(const float* __restrict__ x, const float* __restrict__ c,
                                        int n) {
  float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
  int d = 0;
  for (; d + 4 <= n; d += 4) {
    const float t0 = x[d] - c[d], t1 = x[d + 1] - c[d + 1];
    const float t2 = x[d + 2] - c[d + 2], t3 = x[d + 3] - c[d + 3];
    p0 = fmaf(t0, t0, p0);
    p1 = fmaf(t1, t1, p1);
    p2 = fmaf(t2, t2, p2);
    p3 = fmaf(t3, t3, p3);
  }
  for (; d < n; ++d) {
    const float t = x[d] - c[d];
    p0 = fmaf(t, t, p0);
  }
  return (p0 + p1) + (p2 + p3);
}

// dist_direct_reg with the point's row in LDS (same operation order).
template <int NP>
__device__ inline float dist_direct_lds(const float* x, const float* __restrict__ c) {
  float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
  for (int d = 0; d < NP; d += 4) {
    const float t0 = x[d] - c[d], t1 = x[d + 1] - c[d + 1];
    const float t2 = x[d + 2] - c[d + 2], t3 = x[d + 3] - c[d + 3];
    p0 = fmaf(t0, t0, p0);
    p1 = fmaf(t1, t1, p1);
    p2 = fmaf(t2, t2, p2);
    p3 = fmaf(t3, t3, p3);
  }
  return (p0 + p1) + (p2 + p3);
}

template <int NP>
__device__ inline float dist_direct_reg(const float (&x)[NP], const float* __restrict__ c) {
  float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
  for (int d = 0; d < NP; d += 4) {
    const float t0 = x[d] - c[d], t1 = x[d + 1] - c[d + 1];
    const float t2 = x[d + 2] - c[d + 2], t3 = x[d + 3] - c[d + 3];
    p0 = fmaf(t0, t0, p0);
    p1 = fmaf(t1, t1, p1);
    p2 = fmaf(t2, t2, p2);
    p3 = fmaf(t3, t3, p3);
  }
  return (p0 + p1) + (p2 + p3);
}

// ---------------------------------------------------------------------------
// Sampling: grid (ceil(max_s / 256), jobs).  Phase 1: one Feistel index per
// thread.  Phase 2: the workgroup copies its 256 rows with consecutive
// threads on consecutive 16-byte pieces of a row.
// ---------------------------------------------------------------------------
// One block of up to 256 sample elements starting at `base`: Feistel index
// per thread, then the workgroup copies the rows (consecutive threads on
// consecutive 16-byte pieces of a row when vec).  Sj points at row 0 of the
// job's sample; idxj (nullable) at its index 0.
__device__ inline void sample_block(const float* __restrict__ X, int n, const FeistelKey& fk,
                                    int64_t sj, int64_t base, int32_t* __restrict__ idxj,
                                    float* __restrict__ Sj, int ld, bool vec) {
  __shared__ int64_t rows[kWG];
  const int64_t i = base + threadIdx.x;
  if (i < sj) {
    const uint64_t y = feistel_index((uint64_t)i, fk);
    rows[threadIdx.x] = (int64_t)y;
    if (idxj) idxj[i] = (int32_t)y;
  }
  __syncthreads();
  if (Sj != nullptr) {
    const int nrows = (int)min((int64_t)kWG, sj - base);
    float* __restrict__ Sb = Sj + base * ld;
    if (vec) {
      const int nv = n >> 2, lv = ld >> 2;
      for (int e = threadIdx.x; e < nrows * lv; e += kWG) {
        const int r = e / lv, c = e - r * lv;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (c < nv) v = reinterpret_cast<const float4*>(X + rows[r] * (int64_t)n)[c];
        reinterpret_cast<float4*>(Sb + (int64_t)r * ld)[c] = v;
      }
    } else {
      for (int e = threadIdx.x; e < nrows * ld; e += kWG) {
        const int r = e / ld, c = e - r * ld;
        Sb[(int64_t)r * ld + c] = c < n ? X[rows[r] * (int64_t)n + c] : 0.f;
      }
    }
  }
  __syncthreads();  // rows[] is reused by the next block
}

__global__ __launch_bounds__(kWG) void k_sample(const float* __restrict__ X, int64_t m, int n,
                                                 const int64_t* __restrict__ sizes,
                                                 const uint64_t* __restrict__ rkeys,
                                                 int32_t* __restrict__ idx, int64_t idx_stride,
                                                 float* __restrict__ S, int64_t S_stride, int ld,
                                                 int vec) {
  const int job = blockIdx.y;
  const int64_t sj = sizes[job];
  const int64_t base = (int64_t)blockIdx.x * kWG;
  if (base >= sj) return;
  FeistelKey fk;
#pragma unroll
  for (int r = 0; r < 4; ++r) fk.rk[r] = rkeys[job * 4 + r];
  fk.m = (uint64_t)m;
  fk.h = feistel_half_bits((uint64_t)m);
  sample_block(X, n, fk, sj, base, idx ? idx + job * idx_stride : nullptr,
               S ? S + job * S_stride : nullptr, ld, vec != 0);
}

// Per-dimension max |x| as float bits (non-negative floats order like uints).
__global__ __launch_bounds__(kWG) void k_absmax(const float* __restrict__ X, int64_t rows, int n,
                                                 int ld, unsigned int* __restrict__ out) {
  extern __shared__ unsigned int smax[];
  for (int d = threadIdx.x; d < n; d += kWG) smax[d] = 0u;
  __syncthreads();
  const int64_t total = rows * (int64_t)n;
  for (int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kWG) {
    const int64_t r = e / n;
    const int d = (int)(e - r * n);
    const unsigned int b = __float_as_uint(X[r * ld + d]) & 0x7fffffffu;
    atomicMax(&smax[d], b);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < n; d += kWG) atomicMax(&out[d], smax[d]);
}

// Fixed-point scales: every |x_d| < 2^e_d, so each of at most 2^L points
// contributes less than 2^(62-L) in magnitude and a cluster sum stays below
// 2^62: scale_d = 2^(62 - e_d - L).
__global__ void k_scales(const unsigned int* __restrict__ absmax_bits, int n, int cp,
                         int64_t max_s, double* __restrict__ scale,
                         double* __restrict__ inv_scale) {
  const int d = threadIdx.x + blockIdx.x * blockDim.x;
  if (d >= cp) return;
  int L = 0;
  while (L < 62 && (1ll << L) < max_s) ++L;
  int shift = 62 - L;
  if (d < n) {
    const float a = __uint_as_float(absmax_bits[d]);
    if (a > 0.f && a <= 3.4028234663852886e38f) {
      int e;
      frexp((double)a, &e);  // a = f 2^e, f in [0.5, 1): a < 2^e
      shift = 62 - e - L;
    }
  }
  scale[d] = ldexp(1.0, shift);
  inv_scale[d] = ldexp(1.0, -shift);
}

// Pad k x n centroids into k x cp rows (zero fill) and compute ||c||^2 in FP64.
__global__ __launch_bounds__(kWG) void k_pad_centroids(const float* __restrict__ C,
                                                        int64_t C_stride, int n, int cp, int k,
                                                        float* __restrict__ Cp,
                                                        int64_t Cp_stride,
                                                        float* __restrict__ cn,
                                                        int64_t cn_stride) {
  const int job = blockIdx.x;
  const float* Cj = C + job * C_stride;
  float* Cpj = Cp + job * Cp_stride;
  for (int e = threadIdx.x; e < k * cp; e += kWG) {
    const int r = e / cp, d = e - r * cp;
    Cpj[e] = d < n ? Cj[(int64_t)r * n + d] : 0.f;
  }
  for (int r = threadIdx.x; r < k; r += kWG) {
    double acc = 0.0;
    for (int d = 0; d < n; ++d) {
      const double v = Cj[(int64_t)r * n + d];
      acc += v * v;
    }
    cn[job * cn_stride + r] = (float)acc;
  }
}

__global__ __launch_bounds__(kWG) void k_centroid_norms(const float* __restrict__ Cp, int cp,
                                                         int k, float* __restrict__ cn) {
  const int job = blockIdx.x;
  for (int r = threadIdx.x; r < k; r += kWG) {
    const float* c = Cp + ((int64_t)job * k + r) * cp;
    double acc = 0.0;
    for (int d = 0; d < cp; ++d) acc += (double)c[d] * (double)c[d];
    cn[(int64_t)job * k + r] = (float)acc;
  }
}

__global__ __launch_bounds__(kWG) void k_unpad(const float* __restrict__ Cp, int cp, int n, int k,
                                               float* __restrict__ C, int64_t C_stride) {
  const int job = blockIdx.x;
  for (int e = threadIdx.x; e < k * n; e += kWG) {
    const int r = e / n, d = e - r * n;
    C[job * C_stride + e] = Cp[((int64_t)job * k + r) * cp + d];
  }
}

// ---------------------------------------------------------------------------
// Ranking on the FP32 matrix cores (from kMfmaMinK centres on).  The wave's
// 64 points (lane l: point l, its row in registers) form two 32-point blocks;
// v_mfma_f32_32x32x2f32 takes, per step of two dimensions, the centres of a
// 32-centre tile as operand A (lane (h, c): centre c of the tile, dimension
// 2q + h) and a block's points as operand B (lane (h, c): point c of the block,
// dimension 2q + h).  One v_permlane32_swap of the rows' dimensions 2q and
// 2q + 1 gives the B operands of both blocks.  Lane (h, c) then holds, for
// point c of each block, the dot products with the tile's centres
// 8 (v / 4) + 4 h + v % 4 (v < 16), keeps a running best and second best, and
// the two halves of every point's centre set merge with one lane exchange
// (lowest index on equal values).  The products are summed in an order the
// hardware chooses, so the certification bound takes gamma for NP + 1 terms.
// ---------------------------------------------------------------------------
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline void top2_merge_narrow(float& e1, int& j1, float& e2, float oe1, int oj1,
                                         float oe2) {
  if (oe1 < e1 || (oe1 == e1 && oj1 < j1)) {
    e2 = fminf(e1, oe2);
    e1 = oe1;
    j1 = oj1;
  } else {
    e2 = fminf(e2, oe1);
  }
}

// Best and second-best e_j = ||c_j||^2 - 2 x.c_j over the k centres in LDS
// (sC rows of NP floats, norms sCn) for this lane's point x, best index j1.
template <int NP>
__device__ inline void mfma_rank(const float (&x)[NP], const float* sC, const float* sCn, int k,
                                 float& e1o, float& e2o, int& j1o) {
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5, col = lane & 31;
  float e1[2] = {__builtin_inff(), __builtin_inff()};
  float e2[2] = {__builtin_inff(), __builtin_inff()};
  int j1[2] = {0, 0};
  for (int t0 = 0; t0 < k; t0 += 32) {  // one tile of 32 centres per pass
    f32x16 acc[2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[b][v] = 0.f;
    // rows past the last centre repeat it (their products are never ranked)
    const float* a0 = sC + min(t0 + col, k - 1) * NP + h;
#pragma unroll
    for (int q = 0; q < NP / 2; ++q) {
      const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[2 * q]),
                                                       __float_as_uint(x[2 * q + 1]), false, false);
      const float av = a0[2 * q];
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, __uint_as_float(sw[0]), acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, __uint_as_float(sw[1]), acc[1], 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int c = t0 + 8 * (v >> 2) + 4 * h + (v & 3);
      if (c < k) {
        const float cnc = sCn[c];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const float e = fmaf(-2.f, acc[b][v], cnc);
          e2[b] = __builtin_amdgcn_fmed3f(e1[b], e, e2[b]);
          j1[b] = e < e1[b] ? c : j1[b];
          e1[b] = fminf(e1[b], e);
        }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const float oe1 = __shfl_xor(e1[b], 32, 64);
    const int oj1 = __shfl_xor(j1[b], 32, 64);
    const float oe2 = __shfl_xor(e2[b], 32, 64);
    top2_merge_narrow(e1[b], j1[b], e2[b], oe1, oj1, oe2);
  }
  // lane l's own point is point (l & 31) of block (l >> 5)
  e1o = h ? e1[1] : e1[0];
  e2o = h ? e2[1] : e2[0];
  j1o = h ? j1[1] : j1[0];
}

// ---------------------------------------------------------------------------
// Assignment.  Grid = flattened tiles of the active jobs; each workgroup
// handles tile_pts points of one job in chunks of 256 (one point per lane).
//
// With SUMS (a Lloyd iteration) the per-cluster coordinate sums and counts
// are maintained incrementally: only a point whose label changed since the
// previous assignment of this Lloyd run contributes, +q to its new cluster
// and -q to its old one, where q = x * 2^shift_d rounded to an integer.
// The first assignment of a run counts every point.  The sums are exact
// 64-bit integers, so the order of the atomic additions (LDS within the
// workgroup, global across workgroups) cannot change the result.
// ---------------------------------------------------------------------------
typedef const double __attribute__((address_space(4)))* cdouble_p;


// PPL points per lane: the workgroup covers 256*PPL consecutive points per
// step, lane t taking points base + t + 256 p.  The job's centroids and norms
// are first copied into LDS with one coalesced load (they were just written
// by the previous kernel, so per-centroid fetches from memory would leave
// every wave waiting on a chain of cache misses); the distance loop then
// reads each centroid row as LDS broadcasts and feeds it to PPL*NP FMAs.
template <int NP, int PPL, bool SUMS, bool COOP = false, bool MF = false>
__device__ inline void assign_range(const AssignArgs& a, int job, int64_t p_begin, int64_t p_end,
                                    int first_assign, unsigned char* smem, bool staged = false,
                                    double* tfj = nullptr, unsigned long long* accj = nullptr,
                                    int32_t* cntj = nullptr, unsigned int* claim = nullptr,
                                    int first_unit = 0, int claim_base = 0) {
  if (tfj == nullptr) tfj = a.tf + (int64_t)job * a.max_chunks;
  if (SUMS && accj == nullptr) {
    accj = a.acc + (int64_t)job * a.k * NP;
    cntj = a.cnt + (int64_t)job * a.k;
  }
  const float* __restrict__ S = a.S + job * a.S_stride;
  const float* __restrict__ Cg = a.Cp + job * a.C_stride;
  const float* __restrict__ cng = a.cn + job * a.cn_stride;
  const cdouble_p scale = (cdouble_p)a.scale;
  int32_t* __restrict__ lab = a.labels ? a.labels + job * a.lab_stride : nullptr;
  const int k = a.k;
  const int n = a.n;
  const int ld = a.ld;

  // LDS: [k][NP] centroids, [k] norms, then (SUMS) [k][NP] int64 sums, [k] counts
  float* sC = reinterpret_cast<float*>(smem);
  float* sCn = sC + k * NP;
  unsigned long long* lds_acc =
      reinterpret_cast<unsigned long long*>(smem + (((size_t)k * NP + k) * 4 + 15) / 16 * 16);
  int* lds_cnt = reinterpret_cast<int*>(lds_acc + k * NP);
  // per-wave chunk partials, double-buffered over loop iterations
  __shared__ double red_f[2][PPL][4];
  __shared__ int red_i[2][PPL][4];

  if (!staged) {
    // centroids not yet in LDS: one coalesced copy; LDS sums start at zero
    for (int e = threadIdx.x; e < k * NP / 4; e += kWG)
      reinterpret_cast<float4*>(sC)[e] = reinterpret_cast<const float4*>(Cg)[e];
    for (int e = threadIdx.x; e < k; e += kWG) sCn[e] = cng[e];
    if (SUMS) {
      for (int e = threadIdx.x; e < k * NP; e += kWG) lds_acc[e] = 0ull;
      for (int e = threadIdx.x; e < k; e += kWG) lds_cnt[e] = 0;
    }
    __syncthreads();
  }
  // staged: the caller has placed centroids and norms in LDS, synchronised,
  // and keeps the LDS sums at zero between calls (the flush below clears them)

  float cmax2 = 0.f;  // max_j ||c_j||^2 (max is exact in any order)
  for (int j = threadIdx.x & 63; j < k; j += 64) cmax2 = fmaxf(cmax2, sCn[j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) cmax2 = fmaxf(cmax2, __shfl_xor(cmax2, off, 64));
  const float cmax = sqrtf(cmax2) * 1.0000002f;
  // two interleaved FMA chains of NP/2 terms per dot product, then one add;
  // on the matrix cores, NP products summed in any order
  constexpr float kTerms = MF ? (float)(NP + 1) : (float)(NP / 2 + 1);
  const float gam = kTerms * kU / (1.f - kTerms * kU);
  const float kB = 2.f * (2.f * gam + 2.f * kU);
  const bool vec = a.vec != 0;
  const bool want_near = a.tnear != nullptr;
  const int wv = threadIdx.x >> 6;

  int changed = 0;
  int par = 0;
  // With a claim counter the workgroups of a job share its units of kWG * PPL
  // points dynamically: a workgroup starts with unit first_unit, and while it
  // works on a unit thread 0 claims the next one (claim_base + the counter's
  // value), which the end-of-unit barrier hands over.  Which workgroup takes
  // a unit changes no result (per-chunk partials, exact integer sums,
  // per-point labels); labels written by other workgroups are read with
  // device-scope loads, never from L1.
  constexpr int64_t kUnit = (int64_t)kWG * PPL;
  __shared__ int64_t sh_next[2];
  int64_t base = claim ? p_begin + (int64_t)first_unit * kUnit : p_begin;
  while (base < p_end) {
    if (claim && threadIdx.x == 0)
      sh_next[par] = p_begin + ((int64_t)claim_base + atomicAdd(claim, 1u)) * kUnit;
    float x[PPL][NP];
    bool valid[PPL];
    int jold[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      const int64_t i = base + threadIdx.x + kWG * p;
      valid[p] = i < p_end;
      // previous label, loaded up front so its latency overlaps the distances
      jold[p] = -1;
      if (SUMS && lab && valid[p] && !first_assign)
        jold[p] = claim ? __hip_atomic_load(lab + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                        : lab[i];
      if (valid[p] && vec) {
        const float4* src = reinterpret_cast<const float4*>(S + i * (int64_t)NP);
#pragma unroll
        for (int q = 0; q < NP / 4; ++q) {
          const float4 v = src[q];
          x[p][4 * q] = v.x;
          x[p][4 * q + 1] = v.y;
          x[p][4 * q + 2] = v.z;
          x[p][4 * q + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int d = 0; d < NP; ++d) x[p][d] = (valid[p] && d < n) ? S[i * (int64_t)ld + d] : 0.f;
      }
    }

    // best and second-best expanded-form values e_j = ||c_j||^2 - 2 x.c_j
    float e1[PPL], e2[PPL];
    int j1[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      e1[p] = __builtin_inff();
      e2[p] = __builtin_inff();
      j1[p] = 0;
    }
    if constexpr (MF) {
#pragma unroll
      for (int p = 0; p < PPL; ++p) mfma_rank<NP>(x[p], sC, sCn, k, e1[p], e2[p], j1[p]);
    } else
    for (int j = 0; j < k; ++j) {
      const float4* c4 = reinterpret_cast<const float4*>(sC + j * NP);
      float q0[PPL], q1[PPL];
#pragma unroll
      for (int p = 0; p < PPL; ++p) q0[p] = q1[p] = 0.f;
#pragma unroll
      for (int q = 0; q < NP / 4; ++q) {
        const float4 c = c4[q];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          q0[p] = fmaf(x[p][4 * q], c.x, q0[p]);
          q1[p] = fmaf(x[p][4 * q + 1], c.y, q1[p]);
          q0[p] = fmaf(x[p][4 * q + 2], c.z, q0[p]);
          q1[p] = fmaf(x[p][4 * q + 3], c.w, q1[p]);
        }
      }
      const float cnj = sCn[j];
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        const float e = fmaf(-2.f, q0[p] + q1[p], cnj);
        // new second best is the median of (best, e, second best)
        e2[p] = __builtin_amdgcn_fmed3f(e1[p], e, e2[p]);
        j1[p] = e < e1[p] ? j : j1[p];
        e1[p] = fminf(e1[p], e);
      }
    }

#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      double fpart = 0.0;
      int near = 0;
      const int64_t i = base + threadIdx.x + kWG * p;
      float xx = 0.f;
#pragma unroll
      for (int d = 0; d < NP; ++d) xx = fmaf(x[p][d], x[p][d], xx);
      const float B = kB * (sqrtf(xx) * cmax + cmax2);
      const bool recheck = valid[p] && !((e2[p] - e1[p]) > 2.f * B + 2.5e-5f * fabsf(e2[p] + xx));
      int jw = j1[p];
      if constexpr (COOP) {
        // the wave re-decides its flagged points one at a time: the point's
        // row goes to LDS, lane l ranks the centres l, l + 64, ... and the
        // lanes' best two merge (lowest index on equal distances) -- the
        // same values and choice as one lane ranking all centres in order
        __shared__ float xrow[kWG / 64][NP];
        const int lane = threadIdx.x & 63;
        unsigned long long pending = __ballot(recheck);
        while (pending) {
          const int src = __ffsll(pending) - 1;
          pending &= pending - 1;
          if (lane == src) {
#pragma unroll
            for (int d = 0; d < NP; ++d) xrow[wv][d] = x[p][d];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          float b1 = __builtin_inff(), b2 = __builtin_inff();
          int jb = 0;
          for (int j = lane; j < k; j += 64) {
            // the row is read from LDS for every centre rather than held in
            // registers (the kernel's registers already hold its points)
            __asm__ volatile("" ::: "memory");
            const float dd = dist_direct_lds<NP>(xrow[wv], sC + j * NP);
            if (dd < b1) {
              b2 = b1;
              b1 = dd;
              jb = j;
            } else if (dd < b2) {
              b2 = dd;
            }
          }
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) {
            const float o1 = __shfl_xor(b1, off, 64);
            const int oj = __shfl_xor(jb, off, 64);
            const float o2 = __shfl_xor(b2, off, 64);
            if (o1 < b1 || (o1 == b1 && oj < jb)) {
              b2 = fminf(b1, o2);
              b1 = o1;
              jb = oj;
            } else {
              b2 = fminf(b2, o1);
            }
          }
          if (lane == src) {
            jw = jb;
            if (b2 - b1 < 1e-5f * b2) ++near;
          }
          // every lane has read the row before the next point replaces it
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      } else if (recheck) {
        float b1 = __builtin_inff(), b2 = __builtin_inff();
        int jb = 0;
        for (int j = 0; j < k; ++j) {
          const float dd = dist_direct_reg<NP>(x[p], sC + j * NP);
          if (dd < b1) {
            b2 = b1;
            b1 = dd;
            jb = j;
          } else if (dd < b2) {
            b2 = dd;
          }
        }
        jw = jb;
        if (b2 - b1 < 1e-5f * b2) ++near;
      }
      if (valid[p]) {
        // the winner's distance in the direct form
        const float d1 = dist_direct_reg<NP>(x[p], sC + jw * NP);
        fpart += (double)d1;
        const int jo = jold[p];
        if (lab) lab[i] = jw;
        if (SUMS && jo != jw) {
          changed = 1;
#pragma unroll
          for (int d = 0; d < NP; ++d) {
            if (d < n) {
              const long long q = quantize(x[p][d], scale[d]);
              atomicAdd(&lds_acc[jw * NP + d], (unsigned long long)q);
              if (jo >= 0) atomicAdd(&lds_acc[jo * NP + d], (unsigned long long)(-q));
            }
          }
          atomicAdd(&lds_cnt[jw], 1);
          if (jo >= 0) atomicAdd(&lds_cnt[jo], -1);
        }
      }
      // wave partials of this 256-point chunk's objective and near-tie count
      fpart = wave_sum_f64(fpart);
      if ((threadIdx.x & 63) == 0) red_f[par][p][wv] = fpart;
      if (want_near) {
        near = wave_sum_i32(near);
        if ((threadIdx.x & 63) == 0) red_i[par][p][wv] = near;
      }
    }
    // one synchronisation for all chunks of this iteration; the buffers of
    // the other parity are rewritten only after the next one
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        const int64_t cbase = base + kWG * p;
        if (cbase < p_end) {
          const double* r4 = red_f[par][p];
          tfj[cbase / kWG] = (r4[0] + r4[1]) + (r4[2] + r4[3]);
          if (want_near) {
            const int* q4 = red_i[par][p];
            a.tnear[(int64_t)job * a.max_chunks + cbase / kWG] = (q4[0] + q4[1]) + (q4[2] + q4[3]);
          }
        }
      }
    }
    base = claim ? sh_next[par] : base + kUnit;
    par ^= 1;
  }

  if (SUMS) {
    const int any = __syncthreads_or(changed);
    if (any) {
      for (int e = threadIdx.x; e < k * NP; e += kWG) {
        const unsigned long long v = lds_acc[e];
        if (v) {
          atomicAdd(&accj[e], v);
          if (staged) lds_acc[e] = 0ull;
        }
      }
      for (int e = threadIdx.x; e < k; e += kWG) {
        const int v = lds_cnt[e];
        if (v) {
          atomicAdd(&cntj[e], v);
          if (staged) lds_cnt[e] = 0;
        }
      }
    }
  }
  __syncthreads();  // the LDS is reused by whatever the workgroup does next
}

// Multi-launch form: one workgroup per tile of the flattened tile map.
template <int NP, int PPL, bool SUMS, bool COOP, bool MF>
__global__ __launch_bounds__(kWG) void k_assign_small(AssignArgs a) {
  const int job = a.tile_job[blockIdx.x];
  const int t = a.tile_idx[blockIdx.x];
  int first_assign = 0;
  if (a.st) {
    const JobState st = a.st[job];
    if (!st.active) return;
    first_assign = st.iter == 0;
  }
  const int64_t s = a.s[job];
  const int64_t p_begin = (int64_t)t * a.tile_pts;
  const int64_t p_end = min(s, p_begin + a.tile_pts);
  extern __shared__ __align__(16) unsigned char smem[];
  assign_range<NP, PPL, SUMS, COOP, MF>(a, job, p_begin, p_end, first_assign, smem);
}

// ---------------------------------------------------------------------------
// Lloyd finalize: one workgroup per job.  f = fixed-order sum of the chunk
// partials; stop (f_prev - f <= tol f, f not finite, or max_iter updates) or
// move every non-empty centroid to fp32(sum / count) and recompute its norm.
// ---------------------------------------------------------------------------
__device__ __noinline__ void finalize_job(const FinalizeArgs& a, int job, double* sh_sq /* [k][cp] LDS */) {
  JobState st = a.st[job];
  if (!st.active) return;
  const int k = a.k, cp = a.cp;
  __shared__ double sh_f;
  __shared__ int sh_upd;
  __shared__ int sh_acc;
  __shared__ int sh_empty;
  if (threadIdx.x < 64) {
    const double f = wave_chunked_sum(a.tf + (int64_t)job * a.max_chunks, st.nchunks);
    const bool stop = (st.iter > 0 && st.f_prev - f <= a.tol * f) || !isfinite(f) ||
                      st.iter >= a.max_iter;
    if (threadIdx.x == 0) {
      sh_f = f;
      sh_upd = stop ? 0 : 1;
      // Acceptance (Algorithm 1): the run replaces the incumbent only if its
      // objective is strictly smaller (a NaN never is).
      sh_acc = (stop && a.Cinc != nullptr && f < a.fhat[job]) ? 1 : 0;
      sh_empty = 0;
    }
  }
  __syncthreads();
  const int upd = sh_upd;
  const unsigned long long* acc = a.acc + (int64_t)job * k * cp;
  const int32_t* cnt = a.cnt + (int64_t)job * k;
  float* C = a.Cp + (int64_t)job * k * cp;
  if (upd) {
    // eight means per thread at a time, their loads issued together (an
    // empty cluster keeps its centroid)
    const int kcp = k * cp;
    for (int e0 = threadIdx.x; e0 < kcp; e0 += kWG * 8) {
      long long av[8];
      int cv[8];
      double sv[8];
      float co[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kWG;
        const int j = e / cp, d = e - j * cp;
        const bool in = e < kcp;
        av[u] = in ? (long long)acc[e] : 0;
        cv[u] = in ? cnt[j] : 0;
        sv[u] = in ? a.inv_scale[d] : 0.0;
        co[u] = in ? C[e] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kWG;
        if (e < kcp) {
          float c = co[u];
          if (cv[u] > 0) {
            c = (float)(((double)av[u] * sv[u]) / (double)cv[u]);
            C[e] = c;
          }
          const double x = c;
          sh_sq[e] = x * x;
        }
      }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += kWG) {
      double q = 0.0;
      for (int d = 0; d < cp; ++d) q += sh_sq[j * cp + d];
      a.cn[(int64_t)job * k + j] = (float)q;
    }
  } else {
    int empty = 0;
    for (int j = threadIdx.x; j < k; j += kWG) {
      const int e0 = cnt[j] == 0 ? 1 : 0;
      a.deg[(int64_t)job * k + j] = (uint8_t)e0;
      empty += e0;
    }
    if (empty) atomicAdd(&sh_empty, empty);
  }
  __syncthreads();
  const bool accept = sh_acc != 0;
  if (accept) {
    const int n = a.n;
    for (int e = threadIdx.x; e < k * n; e += kWG) {
      const int j = e / n, d = e - j * n;
      a.Cinc[(int64_t)job * k * n + e] = C[j * cp + d];
    }
    for (int j = threadIdx.x; j < k; j += kWG)
      a.deg_inc[(int64_t)job * k + j] = a.deg[(int64_t)job * k + j];
  }
  if (threadIdx.x == 0) {
    st.f = sh_f;
    if (upd) {
      st.f_prev = sh_f;
      st.iter += 1;
    } else {
      st.active = 0;
      st.ndeg = sh_empty;
      st.accepted = accept ? 1 : 0;
      if (accept) a.fhat[job] = sh_f;
    }
    a.st[job] = st;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kWG) void k_finalize(FinalizeArgs a) {
  extern __shared__ double sh_sq[];
  finalize_job(a, blockIdx.x, sh_sq);
}

// Start of a Lloyd run: job state, zero cluster sums and counts, and the
// norms ||c_j||^2 (FP64, rounded once) of the starting centroids.
__device__ __noinline__ void job_init_one(JobState* js, const int64_t* sizes, int k, int cp,
                             unsigned long long* acc, int32_t* cnt, const float* __restrict__ Cp,
                             float* __restrict__ cn, int j) {
  for (int e = threadIdx.x; e < k * cp; e += kWG) acc[(int64_t)j * k * cp + e] = 0ull;
  for (int e = threadIdx.x; e < k; e += kWG) cnt[(int64_t)j * k + e] = 0;
  for (int r = threadIdx.x; r < k; r += kWG) {
    const float* c = Cp + ((int64_t)j * k + r) * cp;
    double q = 0.0;
    for (int d = 0; d < cp; ++d) q += (double)c[d] * (double)c[d];
    cn[(int64_t)j * k + r] = (float)q;
  }
  if (threadIdx.x == 0) {
    JobState st;
    st.f = 0.0;
    st.f_prev = 0.0;
    st.iter = 0;
    st.active = 1;
    st.ndeg = 0;
    st.accepted = 0;
    st.nchunks = (int32_t)((sizes[j] + kWG - 1) / kWG);
    st.pad_ = 0;
    js[j] = st;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kWG) void k_job_init(JobState* js, const int64_t* sizes, int k, int cp,
                                                  unsigned long long* acc, int32_t* cnt,
                                                  const float* __restrict__ Cp,
                                                  float* __restrict__ cn) {
  job_init_one(js, sizes, k, cp, acc, cnt, Cp, cn, blockIdx.x);
}

// Objective of each job: fixed-order sum of its chunk partials (one wave per job).
__global__ __launch_bounds__(64) void k_reduce_f(const double* __restrict__ tf,
                                                 const int32_t* __restrict__ tnear,
                                                 const int64_t* __restrict__ sizes, int max_chunks,
                                                 double* __restrict__ f,
                                                 long long* __restrict__ near) {
  const int j = blockIdx.x;
  const int64_t nch = (sizes[j] + kWG - 1) / kWG;
  const double acc = wave_chunked_sum(tf + (int64_t)j * max_chunks, nch);
  long long nn = 0;
  if (tnear) {
    for (int64_t q = threadIdx.x; q < nch; q += 64) nn += tnear[(int64_t)j * max_chunks + q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nn += __shfl_xor(nn, off, 64);
  }
  if (threadIdx.x == 0) {
    f[j] = acc;
    if (near) near[j] = nn;
  }
}

// Start of a pass: working centroids and degenerate flags from the incumbent.
__device__ __noinline__ void copy_incumbent_one(const float* __restrict__ Cinc,
                                   const uint8_t* __restrict__ deg_inc, int n, int cp, int k,
                                   float* __restrict__ Cp, uint8_t* __restrict__ deg_work,
                                   int job) {
  for (int e = threadIdx.x; e < k * cp; e += kWG) {
    const int r = e / cp, d = e - r * cp;
    Cp[(int64_t)job * k * cp + e] = d < n ? Cinc[((int64_t)job * k + r) * n + d] : 0.f;
  }
  for (int e = threadIdx.x; e < k; e += kWG) deg_work[(int64_t)job * k + e] = deg_inc[(int64_t)job * k + e];
}

__global__ __launch_bounds__(kWG) void k_copy_incumbent(const float* __restrict__ Cinc,
                                                         const uint8_t* __restrict__ deg_inc,
                                                         int n, int cp, int k,
                                                         float* __restrict__ Cp,
                                                         uint8_t* __restrict__ deg_work) {
  copy_incumbent_one(Cinc, deg_inc, n, cp, k, Cp, deg_work, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Greedy K-means++.  D lives in one of four slots; a step writes the three
// candidates' updated D into the other three slots together with per-tile
// FP64 sums, and the next step keeps the slot of the winning candidate.
// ---------------------------------------------------------------------------
__device__ inline int other_slot(int dcur, int c) { return c < dcur ? c : c + 1; }

// A job's K-means++ state.  Callers read it after a kernel boundary or after
// a barrier that invalidated L1; global loads are never scalarised in this
// library (build flag), so the scalar cache cannot hold a stale copy.
__device__ inline KppState load_ks(const KppState* p) { return *p; }


__device__ __noinline__ void kpp_setup_job(const KppArgs& a, int job) {
  const int k = a.k;
  if (a.picks) {
    for (int e = threadIdx.x; e < 4 * k; e += kWG) a.picks[(int64_t)job * 4 * k + e] = -1;
  }
  if (threadIdx.x == 0) {
    int nt = 0;
    for (int j = 0; j < k; ++j)
      if (a.deg[(int64_t)job * k + j]) a.todo[(int64_t)job * k + nt++] = j;
    KppState ks;
    ks.T = 0.0;
    ks.pot[0] = ks.pot[1] = ks.pot[2] = 0.0;
    ks.cand[0] = ks.cand[1] = ks.cand[2] = -1;
    ks.ncand = 0;
    ks.dcur = 0;
    ks.ntodo = nt;
    ks.has_d = nt < k ? 1 : 0;
    ks.step = 0;
    ks.uniform = 0;
    a.ks[job] = ks;
  }
  __syncthreads();
}

// Job index of launch job j (a batch may cover any set of workspace slots).
__device__ inline int kpp_job(const KppArgs& a, int j) { return a.job_slot ? a.job_slot[j] : j; }

__global__ __launch_bounds__(kWG) void k_kpp_setup(KppArgs a) { kpp_setup_job(a, kpp_job(a, blockIdx.x)); }

// D_i = min over kept centroids of ||S_i - c_j||^2 (slot 0) and the tile's sum.
__device__ __noinline__ void kpp_init_tile(const KppArgs& a, int job, int64_t tile) {
  const KppState ks = load_ks(a.ks + job);
  if (ks.ntodo == 0 || !ks.has_d) return;
  const int64_t s = a.s[job];
  const int64_t i = tile * kDTile + threadIdx.x;
  if (tile * kDTile >= s) return;
  const float* S = a.S + job * a.S_stride;
  const float* C = a.Cp + job * a.C_stride;
  const uint8_t* deg = a.deg + (int64_t)job * a.k;
  float dmin = __builtin_inff();
  if (i < s) {
    for (int j = 0; j < a.k; ++j)
      if (!deg[j]) dmin = min_nan(dmin, dist_direct_mem(S + i * a.ld, C + (int64_t)j * a.cp, a.n));
    a.D[0 * a.D_slot_stride + job * a.D_job_stride + i] = dmin;
  }
  __shared__ double red[4];
  const double ts = block_sum_f64(i < s ? (double)dmin : 0.0, red);
  if (threadIdx.x == 0) a.Dt[(0 * (int64_t)a.njobs + job) * a.ndt_max + tile] = ts;
}

__global__ __launch_bounds__(kWG) void k_kpp_init(KppArgs a) {
  kpp_init_tile(a, kpp_job(a, blockIdx.y), blockIdx.x);
}

// Wave-level monotone prefix over v[0..cnt): lane l sums the contiguous chunk
// [l * cs, (l + 1) * cs) in index order (cs = ceil(cnt / 64)); the lane
// carries are a sequential sum of the chunk totals in lane order.  Returns the
// total (the same in every lane).  For each of the first nt thresholds
// tau[0..2], first[t] receives the first index whose running prefix exceeds
// tau[t] (or -1) and before[t] the prefix just before it.  A chunk of at most
// PRE values is loaded at once and kept in registers for every threshold;
// longer chunks are read PRE values at a time, once per pass.
template <typename T, int PRE>
__device__ inline double wave_prefix_multi(const T* v, int64_t cnt, int nt, const double (&tau)[3],
                                           int64_t (&first)[3], double (&before)[3]) {
  const int lane = threadIdx.x & 63;
  const int64_t cs = (cnt + 63) / 64;
  const int64_t lo = min(cnt, (int64_t)lane * cs), hi = min(cnt, lo + cs);
  const bool held = cs <= PRE;
  T pre[PRE];
  double tot = 0.0;
  if (held) {
#pragma unroll
    for (int q = 0; q < PRE; ++q) pre[q] = lo + q < hi ? v[lo + q] : (T)0;
#pragma unroll
    for (int q = 0; q < PRE; ++q)
      if (lo + q < hi) tot += (double)pre[q];
  } else {
    for (int64_t q0 = lo; q0 < hi; q0 += PRE) {
      T b[PRE];
#pragma unroll
      for (int u = 0; u < PRE; ++u) b[u] = q0 + u < hi ? v[q0 + u] : (T)0;
#pragma unroll
      for (int u = 0; u < PRE; ++u)
        if (q0 + u < hi) tot += (double)b[u];
    }
  }
  double carry = 0.0, total = 0.0;
#pragma unroll 8
  for (int l = 0; l < 64; ++l) {
    const double tl = lane_value(tot, l);
    if (l == lane) carry = total;
    total += tl;
  }
  if (nt <= 0) return total;
  // one running prefix, compared with every threshold
  int64_t found[3] = {-1, -1, -1};
  double bef[3] = {0.0, 0.0, 0.0};
  double r = carry;
  if (held) {
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
      if (lo + q < hi) {
        const double prev = r;
        r += (double)pre[q];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          if (t < nt && found[t] < 0 && r > tau[t]) {
            found[t] = lo + q;
            bef[t] = prev;
          }
        }
      }
    }
  } else {
    for (int64_t q0 = lo; q0 < hi; q0 += PRE) {
      T b[PRE];
#pragma unroll
      for (int u = 0; u < PRE; ++u) b[u] = q0 + u < hi ? v[q0 + u] : (T)0;
#pragma unroll
      for (int u = 0; u < PRE; ++u) {
        if (q0 + u < hi) {
          const double prev = r;
          r += (double)b[u];
#pragma unroll
          for (int t = 0; t < 3; ++t) {
            if (t < nt && found[t] < 0 && r > tau[t]) {
              found[t] = q0 + u;
              bef[t] = prev;
            }
          }
        }
      }
    }
  }
  // per threshold, the smallest index found by any lane
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (t < nt) {
      int64_t best = found[t] >= 0 ? found[t] : INT64_MAX;
      double bbef = bef[t];
      for (int off = 32; off > 0; off >>= 1) {
        const int64_t ob = __shfl_xor(best, off, 64);
        const double obf = __shfl_xor(bbef, off, 64);
        if (ob < best) {
          best = ob;
          bbef = obf;
        }
      }
      first[t] = best == INT64_MAX ? -1 : best;
      before[t] = bbef;
    }
  }
  return total;
}

// Total of v[0..cnt) in the order of wave_prefix_multi.
template <typename T, int PRE>
__device__ inline double wave_prefix_total(const T* v, int64_t cnt) {
  const double none[3] = {0.0, 0.0, 0.0};
  int64_t f[3];
  double b[3];
  return wave_prefix_multi<T, PRE>(v, cnt, 0, none, f, b);
}

// One wave per job: commit the pending step, then draw the next one (scans
// and searches are wave-level; lane = threadIdx.x, which must be < 64).
// PRE values per lane of a tile-sum scan are held in registers (see
// wave_prefix_multi): the scan then costs one round trip to memory.
template <int PRE>
__device__ __noinline__ void kpp_step_job(const KppArgs& a, int job) {
  KppState ks = a.ks[job];
  const int64_t s = a.s[job];
  const int k = a.k;
  const int64_t ndt = (s + kDTile - 1) / kDTile;
  const float* S = a.S + job * a.S_stride;
  const int lane = threadIdx.x;
  if (ks.ncand > 0) {
    // the state's arrays are indexed by constants only (selects), so that it
    // stays in registers instead of scratch memory
    double pot0 = 0.0, pot1 = 0.0, pot2 = 0.0;
    for (int c = 0; c < ks.ncand; ++c) {
      const int sl = other_slot(ks.dcur, c);
      const double pc = wave_prefix_total<double, PRE>(a.Dt + ((int64_t)sl * a.njobs + job) * a.ndt_max, ndt);
      pot0 = c == 0 ? pc : pot0;
      pot1 = c == 1 ? pc : pot1;
      pot2 = c == 2 ? pc : pot2;
    }
    ks.pot[0] = pot0;
    ks.pot[1] = pot1;
    ks.pot[2] = pot2;
    int best = 0;
    double pbest = pot0;
    if (ks.ncand > 1 && pot1 < pbest) {
      best = 1;
      pbest = pot1;
    }
    if (ks.ncand > 2 && pot2 < pbest) {
      best = 2;
      pbest = pot2;
    }
    const int j = a.todo[(int64_t)job * k + ks.step - 1];
    const int64_t istar = best == 0 ? ks.cand[0] : (best == 1 ? ks.cand[1] : ks.cand[2]);
    float* cj = a.Cp + job * a.C_stride + (int64_t)j * a.cp;
    for (int d = lane; d < a.cp; d += 64) cj[d] = d < a.n ? S[istar * a.ld + d] : 0.f;
    if (lane == 0) {
      a.deg[(int64_t)job * k + j] = 0;
      if (a.picks) {
        int32_t* p = a.picks + ((int64_t)job * k + j) * 4;
        p[0] = (int32_t)istar;
        for (int c = 0; c < 3; ++c) p[1 + c] = (!ks.uniform && c < ks.ncand) ? ks.cand[c] : -1;
      }
    }
    ks.dcur = other_slot(ks.dcur, best);
    ks.T = pbest;
    ks.has_d = 1;
    ks.ncand = 0;
  }
  if (ks.step < ks.ntodo) {
    uint64_t k0, k1;
    stream_key(a.seed_worker[job * 2], (uint32_t)a.seed_worker[job * 2 + 1], 3u, &k0, &k1);
    const uint64_t g = a.gs ? a.gs[job] : a.g;
    const U64x4 w = philox_ctr((uint64_t)ks.step, g, 0, 0, k0, k1);
    const double* dt = a.Dt + ((int64_t)ks.dcur * a.njobs + job) * a.ndt_max;
    if (ks.has_d && ks.step == 0) ks.T = wave_prefix_total<double, PRE>(dt, ndt);
    if (!ks.has_d || !(ks.T > 0.0 && ks.T < __builtin_inf())) {
      ks.ncand = 1;
      ks.uniform = 1;
      ks.cand[0] = (int32_t)bounded(w.w[3], (uint64_t)s);
      ks.cand[1] = ks.cand[2] = -1;
    } else {
      const int nc = a.n_cand;
      ks.ncand = nc;
      ks.uniform = 0;
      const float* Dj = a.D + (int64_t)ks.dcur * a.D_slot_stride + job * a.D_job_stride;
      // the tiles of all candidates in one scan of the tile sums
      const double tau[3] = {u01(w.w[0]) * ks.T, u01(w.w[1]) * ks.T, u01(w.w[2]) * ks.T};
      int64_t tile[3];
      double base[3];
      wave_prefix_multi<double, PRE>(dt, ndt, nc, tau, tile, base);
      // then the points inside those tiles (at most 256 each: four per lane),
      // all loaded before the searches
      int64_t lo[3], cnt[3];
      double tin[3];
      float held[3][4];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        lo[c] = 0;
        cnt[c] = 0;
        tin[c] = 0.0;
        if (c < nc) {
          if (tile[c] < 0) {  // rounding put tau at the very end: last tile with
            int64_t t = ndt - 1;  // mass, whose first point with D > 0 is taken below
            while (t > 0 && !(dt[t] > 0.0)) --t;
            tile[c] = t;
            base[c] = tau[c];
          }
          lo[c] = tile[c] * kDTile;
          cnt[c] = min((int64_t)kDTile, s - lo[c]);
          // running prefix inside the tile, started at the tile's base
          tin[c] = tau[c] - base[c];
        }
        const int64_t cs = (cnt[c] + 63) / 64;
        const int64_t l0 = min(cnt[c], (int64_t)lane * cs), l1 = min(cnt[c], l0 + cs);
#pragma unroll
        for (int q = 0; q < 4; ++q) held[c][q] = l0 + q < l1 ? Dj[lo[c] + l0 + q] : 0.f;
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (c < nc) {
          const int64_t cs = (cnt[c] + 63) / 64;
          const int64_t l0 = min(cnt[c], (int64_t)lane * cs), l1 = min(cnt[c], l0 + cs);
          double tot = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (l0 + q < l1) tot += (double)held[c][q];
          double carry = 0.0, total = 0.0;
#pragma unroll 8
          for (int l = 0; l < 64; ++l) {
            const double tl = lane_value(tot, l);
            if (l == lane) carry = total;
            total += tl;
          }
          int64_t found = -1;
          double r = carry;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (found < 0 && l0 + q < l1) {
              r += (double)held[c][q];
              if (r > tin[c]) found = l0 + q;
            }
          }
          int64_t within = found >= 0 ? found : INT64_MAX;
          for (int off = 32; off > 0; off >>= 1) within = min(within, __shfl_xor(within, off, 64));
          if (within == INT64_MAX) {  // fallback: last point of the tile with D > 0
            within = cnt[c] - 1;
            while (within > 0 && !(Dj[lo[c] + within] > 0.f)) --within;
          }
          ks.cand[c] = (int32_t)(lo[c] + within);
        } else {
          ks.cand[c] = -1;
        }
      }
    }
    ks.step += 1;
  }
  if (lane == 0) a.ks[job] = ks;
}

__global__ __launch_bounds__(64) void k_kpp_step(KppArgs a) {
  kpp_step_job<16>(a, kpp_job(a, blockIdx.x));
}

// Potentials of the pending candidates: new D per candidate into the other
// slots, with per-tile sums.
__device__ __noinline__ void kpp_pot_tile(const KppArgs& a, int job, int64_t tile) {
  const KppState ks = load_ks(a.ks + job);
  if (ks.ncand == 0) return;
  const int64_t s = a.s[job];
  if (tile * kDTile >= s) return;
  const int64_t i = tile * kDTile + threadIdx.x;
  const float* S = a.S + job * a.S_stride;
  const int n = a.n, nc = ks.ncand;
  // the candidates' rows in LDS; every point's row is read once for all of them
  extern __shared__ float cand_rows[];  // [3][n]
  for (int e = threadIdx.x; e < nc * n; e += kWG) {
    const int c = e / n, d = e - c * n;
    cand_rows[e] = S[(int64_t)ks.cand[c] * a.ld + d];
  }
  __syncthreads();
  __shared__ double red[12];
  float dcur = 0.f;
  if (i < s && ks.has_d) dcur = a.D[(int64_t)ks.dcur * a.D_slot_stride + job * a.D_job_stride + i];
  // direct-form distances with the operation order of dist_direct_mem
  float p[3][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
  if (i < s) {
    const float* x = S + i * a.ld;
    const int n4 = n & ~3;
    const bool vec = (a.ld % 4) == 0 && (((uintptr_t)S & 15) == 0);
    for (int d = 0; d < n4; d += 4) {
      float4 xv;
      if (vec) {
        xv = *reinterpret_cast<const float4*>(x + d);
      } else {
        xv = make_float4(x[d], x[d + 1], x[d + 2], x[d + 3]);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (c < nc) {
          const float* cr = cand_rows + c * n + d;
          const float t0 = xv.x - cr[0], t1 = xv.y - cr[1], t2 = xv.z - cr[2], t3 = xv.w - cr[3];
          p[c][0] = fmaf(t0, t0, p[c][0]);
          p[c][1] = fmaf(t1, t1, p[c][1]);
          p[c][2] = fmaf(t2, t2, p[c][2]);
          p[c][3] = fmaf(t3, t3, p[c][3]);
        }
      }
    }
    for (int d = n4; d < n; ++d) {
      const float xd = x[d];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (c < nc) {
          const float t = xd - cand_rows[c * n + d];
          p[c][0] = fmaf(t, t, p[c][0]);
        }
      }
    }
  }
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c < nc) {
      float m = 0.f;
      if (i < s) {
        const float dc = (p[c][0] + p[c][1]) + (p[c][2] + p[c][3]);
        m = ks.has_d ? min_nan(dcur, dc) : dc;
        a.D[(int64_t)other_slot(ks.dcur, c) * a.D_slot_stride + job * a.D_job_stride + i] = m;
      }
      const double part = wave_sum_f64(i < s ? (double)m : 0.0);
      if ((threadIdx.x & 63) == 0) red[c * 4 + wv] = part;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int c = 0; c < nc; ++c)
      a.Dt[((int64_t)other_slot(ks.dcur, c) * a.njobs + job) * a.ndt_max + tile] =
          (red[c * 4] + red[c * 4 + 1]) + (red[c * 4 + 2] + red[c * 4 + 3]);
}

__global__ __launch_bounds__(kWG) void k_kpp_pot(KppArgs a) {
  kpp_pot_tile(a, kpp_job(a, blockIdx.y), blockIdx.x);
}

// ---------------------------------------------------------------------------
// Persistent round kernel (cooperative launch: all workgroups co-resident).
//
// Each workgroup reads the id of the XCD it runs on and registers there; after
// one device-wide barrier every workgroup knows how many workgroups each XCD
// holds, and splits its XCD's workgroups among the workers the host placed on
// that XCD (in proportion to their sample sizes, at least one each).  A worker
// therefore lives inside one XCD: its workgroups share that XCD's L2, so its
// group barrier needs no L2 write-back or invalidation — only completed
// stores, L2 atomics and an L1 invalidation.  Buffers updated by atomics
// (fixed-point deltas, counts, barrier words) are only ever accessed through
// atomics.  Workers never wait for each other.
//
// Lloyd needs one barrier per iteration: every workgroup adds the iteration's
// fixed-point deltas (triple-buffered) to its own copy of the cluster sums in
// LDS and computes the same new centroids and the same convergence decision.
// Every loop is bounded, and a barrier that waits longer than two seconds sets
// the error flag, after which no barrier waits again.
// ---------------------------------------------------------------------------
constexpr uint64_t kBarrierTimeoutTicks = 200000000ull;  // 2 s of the 100 MHz wall clock

__device__ inline bool timed_out(uint64_t t0) { return wall_clock64() - t0 > kBarrierTimeoutTicks; }

// Device-wide barrier (agent-scope fences); used once per launch.
__device__ inline void grid_barrier(GroupBar* b, unsigned int nwg, int32_t* err) {
  __syncthreads();
  if (threadIdx.x == 0 && nwg > 1 &&
      __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
    const unsigned int g = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned int arrived =
        __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nwg - 1) {
      __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const uint64_t t0 = wall_clock64();
      while (__hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(2);
        if (timed_out(t0)) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Wait until this wave's stores and atomics (flat ones count on both
// counters) have completed; the compiler keeps memory accesses on their side.
__device__ inline void drain_vm() { asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory"); }

// Barrier of one worker's workgroups, all on one XCD.  The arrival counter
// only grows: the e-th barrier of a launch waits until it reaches e * nwg
// (the host zeroes it before the launch).  A wait ends after two seconds and
// sets the error flag; once the flag is set no wait lasts longer than 64 polls,
// so a launch always ends.  Arrival is a non-returning L2
// atomic issued after this workgroup's stores have completed; the wait polls
// the counter in L2.  With inv, every wave then invalidates at device scope,
// so no later load is served from a line its CU's L1 kept from before
// (another workgroup may have rewritten it since).  Without inv the caller
// reads what other workgroups wrote only through device-scope loads
// (load_dev), which are never served from L1.
__device__ inline void xcd_barrier(unsigned int* count, unsigned int nwg, unsigned int& epoch,
                                   int32_t* err, bool inv = true) {
  drain_vm();
  __syncthreads();
  epoch += 1;
  if (threadIdx.x == 0 && nwg > 1) {
    __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned int target = epoch * nwg;
    const uint64_t t0 = wall_clock64();
    // every 64 polls: give up after the time limit, or at once when an
    // earlier barrier already timed out (the flag is set)
    for (unsigned int polls = 1;
         (int)(__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0;
         ++polls) {
      __builtin_amdgcn_s_sleep(1);
      if ((polls & 63) == 0 &&
          (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || timed_out(t0))) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
  if (inv) asm volatile("buffer_inv sc1" ::: "memory");
}

// Device-scope loads (never served from L1).
__device__ inline unsigned long long load_dev(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int load_dev(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double load_dev(const double* p) {
  return __longlong_as_double((long long)load_dev(reinterpret_cast<const unsigned long long*>(p)));
}

// wave_chunked_sum through device-scope loads (same order, same result):
// eight values per lane are loaded together before they are added.
__device__ inline double wave_chunked_sum_dev(const double* v, int64_t cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t cs = (cnt + 63) / 64;
  const int64_t lo = min(cnt, (int64_t)lane * cs), hi = min(cnt, lo + cs);
  double tot = 0.0;
  for (int64_t q0 = lo; q0 < hi; q0 += 8) {
    double t[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) t[q] = q0 + q < hi ? load_dev(v + q0 + q) : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (q0 + q < hi) tot += t[q];
  }
  return wave_ordered_sum(tot);
}

__device__ inline void sample_range(const RoundArgs& r, int w, uint32_t purpose, uint64_t g,
                                    int64_t sj, int64_t p0, int64_t p1, bool vec) {
  const FeistelKey fk = feistel_key((uint64_t)r.m, r.seed, (uint32_t)w, purpose, g);
  float* Sj = const_cast<float*>(r.as.S) + w * r.as.S_stride;
  for (int64_t base = p0; base < p1; base += kWG)
    sample_block(r.X, r.n, fk, sj, base, nullptr, Sj, r.cp, vec);
}

// Norm of every centroid row in LDS (FP64, one rounding): same arithmetic as
// job_init_one / finalize_job.
template <int NP>
__device__ inline void lds_norms(const float* sC, float* sCn, int k) {
  for (int j = threadIdx.x; j < k; j += kWG) {
    double q = 0.0;
    for (int d = 0; d < NP; ++d) q += (double)sC[j * NP + d] * (double)sC[j * NP + d];
    sCn[j] = (float)q;
  }
}

// Direct-form distance of a register-resident point, with the operation
// order of dist_direct_mem over the first n dimensions (partial sum d mod 4
// for the first floor(n/4)*4 dimensions, the rest into the first partial).
template <int NP>
__device__ inline float dist_direct_regn(const float (&x)[NP], const float* __restrict__ c, int n) {
  float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
  const int n4 = n & ~3;
#pragma unroll
  for (int d = 0; d < NP; d += 4) {
    if (d < n4) {
      const float t0 = x[d] - c[d], t1 = x[d + 1] - c[d + 1];
      const float t2 = x[d + 2] - c[d + 2], t3 = x[d + 3] - c[d + 3];
      p0 = fmaf(t0, t0, p0);
      p1 = fmaf(t1, t1, p1);
      p2 = fmaf(t2, t2, p2);
      p3 = fmaf(t3, t3, p3);
    }
  }
#pragma unroll
  for (int d = 0; d < NP; ++d) {
    if (d >= n4 && d < n) {
      const float t = x[d] - c[d];
      p0 = fmaf(t, t, p0);
    }
  }
  return (p0 + p1) + (p2 + p3);
}

// The rows [i0, i0 + 256) of a worker's padded sample, one per thread.
template <int NP>
__device__ inline void load_row(const float* S, int64_t i, bool valid, float (&x)[NP]) {
  if (valid) {
    const float4* src = reinterpret_cast<const float4*>(S + i * (int64_t)NP);
#pragma unroll
    for (int q = 0; q < NP / 4; ++q) {
      const float4 v = src[q];
      x[4 * q] = v.x;
      x[4 * q + 1] = v.y;
      x[4 * q + 2] = v.z;
      x[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int d = 0; d < NP; ++d) x[d] = 0.f;
  }
}

// kpp_init_tile with the point's row read once into registers (NP = the
// padded width): the distances keep dist_direct_mem's operation order, so D
// and the tile sums are the same.  The row used to be re-read for every kept
// centroid, which with many centroids and many waves per compute unit missed
// L1.
template <int NP>
__global__ __launch_bounds__(kWG) void k_kpp_init_np(KppArgs a) {
  const int job = kpp_job(a, blockIdx.y);
  const int64_t tile = blockIdx.x;
  const KppState ks = load_ks(a.ks + job);
  if (ks.ntodo == 0 || !ks.has_d) return;
  const int64_t s = a.s[job];
  if (tile * kDTile >= s) return;
  const int64_t i = tile * kDTile + threadIdx.x;
  const bool valid = i < s;
  const float* S = a.S + job * a.S_stride;
  const float* C = a.Cp + job * a.C_stride;
  const uint8_t* deg = a.deg + (int64_t)job * a.k;
  const int n = a.n, ld = a.ld;
  // whole 16-byte groups when every row holds NP floats at a 16-byte boundary;
  // otherwise the first n values one by one (the others are not read below)
  const bool vec = (ld % 4 == 0) && ld >= NP && (((uintptr_t)S & 15) == 0);
  float x[NP];
  if (vec) {
    const float4* src = reinterpret_cast<const float4*>(S + (valid ? i : 0) * (int64_t)ld);
#pragma unroll
    for (int q = 0; q < NP / 4; ++q) {
      const float4 v = src[q];
      x[4 * q] = v.x;
      x[4 * q + 1] = v.y;
      x[4 * q + 2] = v.z;
      x[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int d = 0; d < NP; ++d) x[d] = (valid && d < n) ? S[i * (int64_t)ld + d] : 0.f;
  }
  float dmin = __builtin_inff();
  if (valid) {
    for (int j = 0; j < a.k; ++j)
      if (!deg[j]) dmin = min_nan(dmin, dist_direct_regn<NP>(x, C + (int64_t)j * a.cp, n));
    a.D[0 * a.D_slot_stride + job * a.D_job_stride + i] = dmin;
  }
  __shared__ double red[4];
  const double ts = block_sum_f64(valid ? (double)dmin : 0.0, red);
  if (threadIdx.x == 0) a.Dt[(0 * (int64_t)a.njobs + job) * a.ndt_max + tile] = ts;
}

// K-means++ in the persistent kernel: the same values as kpp_init_tile and
// kpp_pot_tile for the tiles [c0, c1) of one worker, with the workgroup's
// points in registers, the centres (the incumbent in LDS) or the candidate
// rows (staged in LDS) as broadcasts, and one synchronisation per tile.
template <int NP>
__device__ void kpp_init_range(const KppArgs& a, int job, int64_t c0, int64_t c1,
                               const float* sI, const uint8_t* sIdeg, double* red) {
  const KppState ks = load_ks(a.ks + job);
  if (ks.ntodo == 0 || !ks.has_d) return;
  const int64_t s = a.s[job];
  const float* S = a.S + job * a.S_stride;
  const int k = a.k, n = a.n, wv = threadIdx.x >> 6;
  for (int64_t tile = c0; tile < c1; ++tile) {
    if (tile * kDTile >= s) break;
    const int64_t i = tile * kDTile + threadIdx.x;
    const bool valid = i < s;
    float x[NP];
    load_row<NP>(S, i, valid, x);
    float dmin = __builtin_inff();
    if (valid) {
      for (int j = 0; j < k; ++j)
        if (!sIdeg[j]) dmin = min_nan(dmin, dist_direct_regn<NP>(x, sI + j * NP, n));
      a.D[0 * a.D_slot_stride + job * a.D_job_stride + i] = dmin;
    }
    const double part = wave_sum_f64(valid ? (double)dmin : 0.0);
    if ((threadIdx.x & 63) == 0) red[wv] = part;
    __syncthreads();
    if (threadIdx.x == 0)
      a.Dt[(0 * (int64_t)a.njobs + job) * a.ndt_max + tile] = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
  }
}

template <int NP>
__device__ void kpp_pot_range(const KppArgs& a, int job, int64_t c0, int64_t c1, float* rows,
                              double* red) {
  const KppState ks = load_ks(a.ks + job);
  if (ks.ncand == 0) return;
  const int64_t s = a.s[job];
  const float* S = a.S + job * a.S_stride;
  const int n = a.n, wv = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < ks.ncand * NP; e += kWG) {
    const int c = e / NP, d = e - c * NP;
    rows[e] = S[(int64_t)ks.cand[c] * NP + d];
  }
  __syncthreads();
  for (int64_t tile = c0; tile < c1; ++tile) {
    if (tile * kDTile >= s) break;
    const int64_t i = tile * kDTile + threadIdx.x;
    const bool valid = i < s;
    float x[NP];
    load_row<NP>(S, i, valid, x);
    float dcur = 0.f;
    if (valid && ks.has_d) dcur = a.D[(int64_t)ks.dcur * a.D_slot_stride + job * a.D_job_stride + i];
    for (int c = 0; c < ks.ncand; ++c) {
      float m = 0.f;
      if (valid) {
        const float dc = dist_direct_regn<NP>(x, rows + c * NP, n);
        m = ks.has_d ? min_nan(dcur, dc) : dc;
        a.D[(int64_t)other_slot(ks.dcur, c) * a.D_slot_stride + job * a.D_job_stride + i] = m;
      }
      const double part = wave_sum_f64(valid ? (double)m : 0.0);
      if ((threadIdx.x & 63) == 0) red[c * 4 + wv] = part;
    }
    __syncthreads();
    if (threadIdx.x == 0)
      for (int c = 0; c < ks.ncand; ++c)
        a.Dt[((int64_t)other_slot(ks.dcur, c) * a.njobs + job) * a.ndt_max + tile] =
            (red[c * 4] + red[c * 4 + 1]) + (red[c * 4 + 2] + red[c * 4 + 3]);
    __syncthreads();
  }
}

size_t __host__ __device__ inline round_assign_bytes(int cp, int k) {
  const size_t base = (((size_t)k * cp + k) * 4 + 15) / 16 * 16;
  return base + (size_t)k * cp * 8 + ((size_t)k * 4 + 15) / 16 * 16;
}

// Fewest Lloyd units per workgroup at which a worker's workgroups share them
// dynamically (fewer, or one workgroup: each keeps its own range).
constexpr int kShareUnits = 4;

template <int NP, bool MF>
__global__ __launch_bounds__(kWG, 4) void k_round(const RoundArgs* __restrict__ rp) {
  constexpr int PPL = (NP <= 32 && !MF) ? 2 : 1;
  // the arguments, read many times by every phase, live in LDS
  __shared__ RoundArgs r_lds;
  if (threadIdx.x == 0) r_lds = *rp;
  __syncthreads();
  const RoundArgs& r = r_lds;
  extern __shared__ __align__(16) unsigned char smem[];
  const int k = r.k, n = r.n;
  // LDS: [assign region: centroids sC, norms sCn, delta sums, counts]
  //      [tot: k*NP int64][tcnt: k int32][sI: k*NP incumbent][sIdeg: k]
  float* sC = reinterpret_cast<float*>(smem);
  float* sCn = sC + k * NP;
  long long* tot = reinterpret_cast<long long*>(smem + round_assign_bytes(NP, k));
  int* tcnt = reinterpret_cast<int*>(tot + k * NP);
  float* sI = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(tcnt) + ((size_t)k * 4 + 15) / 16 * 16);
  uint8_t* sIdeg = reinterpret_cast<uint8_t*>(sI + k * NP);
  __shared__ unsigned int sh_slot;
  __shared__ double sh_f;
  __shared__ float krows[3 * NP];  // K-means++ candidate rows
  __shared__ double kred[12];      // K-means++ per-wave partial sums

  // ---- registration on this workgroup's XCD, one device-wide barrier ----
  unsigned int xcc;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
  xcc &= (kMaxXcd - 1);
  if (threadIdx.x == 0)
    sh_slot = __hip_atomic_fetch_add(&r.reg[xcc], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  grid_barrier(r.gbar, gridDim.x, r.err);
  const unsigned int slot = sh_slot;
  // every workgroup checks the whole placement, so all of them agree to stop
  for (int x = 0; x < kMaxXcd; ++x) {
    const int got = (int)__hip_atomic_load(&r.reg[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int need = 0;
    for (int i = 0; i < r.xcd_nw[x]; ++i) need += r.xcd_g[x * r.W + i];
    if (got < need) {
      if (threadIdx.x == 0) __hip_atomic_store(r.err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
  }
  // this XCD's workgroups, in registration order, go to its workers in list
  // order, r.xcd_g of them each; surplus workgroups leave at once
  int w = -1, rank = 0, nwg = 0;
  {
    int cum = 0;
    for (int i = 0; i < r.xcd_nw[xcc]; ++i) {
      const int gi = r.xcd_g[xcc * r.W + i];
      if ((int)slot >= cum && (int)slot < cum + gi) {
        w = r.xcd_workers[xcc * r.W + i];
        rank = (int)slot - cum;
        nwg = gi;
      }
      cum += gi;
    }
  }
  if (w < 0) return;
  const bool leader = rank == 0;
  const int64_t sj = r.s[w];
  const int64_t nch = (sj + kWG - 1) / kWG;
  // contiguous chunk ranges in units of PPL chunks (one assignment loop
  // step), the units spread as evenly as possible
  const int64_t units = (nch + PPL - 1) / PPL;
  const int64_t ubase = units / nwg, urem = units % nwg;
  const int64_t u0 = rank * ubase + min((int64_t)rank, urem);
  const int64_t u1 = u0 + ubase + (rank < urem ? 1 : 0);
  const int64_t c0 = min(nch, u0 * PPL), c1 = min(nch, u1 * PPL);
  const int64_t p0 = c0 * kWG, p1 = min(sj, c1 * kWG);
  unsigned int* bar = &r.bar[w].count;
  unsigned int epoch = 0;
  const bool vec = (((uintptr_t)r.X & 15) == 0) && (n % 4 == 0);
  const int64_t mc = r.as.max_chunks;
  double* tf3 = r.tf3 + (int64_t)w * 3 * mc;
  unsigned long long* dl3 = r.delta + (int64_t)w * 3 * k * NP;
  int32_t* dc3 = r.dcnt + (int64_t)w * 3 * k;
  unsigned int* claim3 = r.claim + (int64_t)w * 3;
  // the same for every workgroup of the worker
  const bool share = nwg > 1 && units >= (int64_t)kShareUnits * nwg;

  // the incumbent, kept in this workgroup's LDS
  for (int e = threadIdx.x; e < k * NP; e += kWG) {
    const int j = e / NP, d = e - j * NP;
    sI[e] = d < n ? r.Cinc[((int64_t)w * k + j) * n + d] : 0.f;
  }
  for (int j = threadIdx.x; j < k; j += kWG) sIdeg[j] = r.deg_inc[(int64_t)w * k + j];
  {  // the assignment's LDS sums start at zero and are left at zero by every flush
    unsigned long long* lacc =
        reinterpret_cast<unsigned long long*>(smem + (((size_t)k * NP + k) * 4 + 15) / 16 * 16);
    for (int e = threadIdx.x; e < k * NP; e += kWG) lacc[e] = 0ull;
    int* lcnt = reinterpret_cast<int*>(lacc + k * NP);
    for (int j = threadIdx.x; j < k; j += kWG) lcnt[j] = 0;
  }
  double fhat = r.fhat[w];
  __syncthreads();

  // ---- re-evaluation after a size change (Algorithm 1; Section 4.2) ----
  if (r.recalc[w]) {
    sample_range(r, w, 4u /* RECALC */, (uint64_t)r.t, sj, p0, p1, vec);
    for (int e = threadIdx.x; e < k * NP; e += kWG) sC[e] = sI[e];
    __syncthreads();
    lds_norms<NP>(sC, sCn, k);
    __syncthreads();
    assign_range<NP, PPL, false, false, MF>(r.as, w, p0, p1, 0, smem, true, tf3 + 2 * mc);
    xcd_barrier(bar, nwg, epoch, r.err);
    if (threadIdx.x < 64) {
      const double f = wave_chunked_sum(tf3 + 2 * mc, nch);
      if (threadIdx.x == 0) sh_f = f;
    }
    __syncthreads();
    fhat = sh_f;
    if (leader && threadIdx.x == 0) {
      r.fhat[w] = fhat;
      r.recalc_f[w] = fhat;
    }
  }

  int ig = 0;  // Lloyd iterations of this launch (selects the triple buffers)
  for (int q = 0; q < r.passes_p; ++q) {
    const uint64_t g = (uint64_t)r.t * r.passes_p + q;
    sample_range(r, w, 2u /* SAMPLE */, g, sj, p0, p1, vec);
    int ntodo = 0;
    for (int j = 0; j < k; ++j) ntodo += sIdeg[j] ? 1 : 0;
    if (ntodo > 0) {
      // K-means++ for the degenerate centroids, on the global working copy
      const KppArgs& ka = r.ka;
      if (leader) {
        float* Cp = r.Cp + (int64_t)w * k * NP;
        for (int e = threadIdx.x; e < k * NP; e += kWG) Cp[e] = sI[e];
        for (int j = threadIdx.x; j < k; j += kWG) r.deg_work[(int64_t)w * k + j] = sIdeg[j];
        if (threadIdx.x == 0) const_cast<uint64_t*>(ka.gs)[w] = g;
        drain_vm();
        __syncthreads();
        kpp_setup_job(ka, w);
      }
      xcd_barrier(bar, nwg, epoch, r.err);
      kpp_init_range<NP>(ka, w, c0, c1, sI, sIdeg, kred);
      xcd_barrier(bar, nwg, epoch, r.err);
      for (int step = 0; step < ntodo; ++step) {
        if (leader && threadIdx.x < 64) kpp_step_job<4>(ka, w);
        xcd_barrier(bar, nwg, epoch, r.err);
        kpp_pot_range<NP>(ka, w, c0, c1, krows, kred);
        xcd_barrier(bar, nwg, epoch, r.err);
      }
      if (leader && threadIdx.x < 64) kpp_step_job<4>(ka, w);  // commits the last step
      xcd_barrier(bar, nwg, epoch, r.err);
      const float* Cp = r.Cp + (int64_t)w * k * NP;
      for (int e = threadIdx.x; e < k * NP; e += kWG) sC[e] = Cp[e];
    } else {
      for (int e = threadIdx.x; e < k * NP; e += kWG) sC[e] = sI[e];
      // shared units: rows gathered by the worker's other workgroups are read
      // from here on (the barrier invalidates L1)
      if (share) xcd_barrier(bar, nwg, epoch, r.err);
    }
    for (int e = threadIdx.x; e < k * NP; e += kWG) tot[e] = 0;
    for (int j = threadIdx.x; j < k; j += kWG) tcnt[j] = 0;
    __syncthreads();
    lds_norms<NP>(sC, sCn, k);
    __syncthreads();

    // ---- Lloyd ----
    double f_prev = 0.0;
    for (int it = 0; it <= r.max_iter; ++it, ++ig) {
      const int b = ig % 3;
      // the first assignment of a pass takes the points this workgroup
      // gathered; later ones share the worker's units dynamically (rows
      // gathered by other workgroups, read after the first barrier, which
      // invalidates L1)
      assign_range<NP, PPL, true, false, MF>(r.as, w, share ? 0 : p0, share ? sj : p1,
                                             it == 0 ? 1 : 0, smem, true, tf3 + b * mc,
                                             dl3 + (int64_t)b * k * NP, dc3 + b * k,
                                             share ? claim3 + b : nullptr, rank, nwg);
      {  // clear the buffers of the next iteration (last read two barriers ago),
         // each workgroup its share
        const int bn = (b + 1) % 3;
        if (leader && threadIdx.x == 0)
          __hip_atomic_store(claim3 + bn, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int tot_e = k * NP + k;
        const int share = (tot_e + nwg - 1) / nwg;
        const int e1 = min(tot_e, (rank + 1) * share);
        for (int e = rank * share + threadIdx.x; e < e1; e += kWG) {
          if (e < k * NP)
            __hip_atomic_store(dl3 + (int64_t)bn * k * NP + e, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          else
            __hip_atomic_store(dc3 + bn * k + (e - k * NP), 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      xcd_barrier(bar, nwg, epoch, r.err, false);
      // every arrival's atomics and stores are complete in L2
      // the iteration's deltas on the first three waves, the counts and the
      // objective's chunk partials on the last, so that every wave waits for
      // about one round trip (integer sums: any order; f in its fixed order)
      constexpr int kDW = kWG - 64;
      if (threadIdx.x < kDW) {  // eight loads in flight per thread
        const unsigned long long* src = dl3 + (int64_t)b * k * NP;
        const int tot_e = k * NP;
        for (int e0 = threadIdx.x; e0 < tot_e; e0 += 8 * kDW) {
          unsigned long long t8[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) t8[u] = e0 + u * kDW < tot_e ? load_dev(src + e0 + u * kDW) : 0ull;
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (e0 + u * kDW < tot_e) tot[e0 + u * kDW] += (long long)t8[u];
        }
      } else {
        const int l = threadIdx.x - kDW;
        for (int j = l; j < k; j += 64) tcnt[j] += load_dev(dc3 + b * k + j);
        const double f = wave_chunked_sum_dev(tf3 + b * mc, nch);
        if (l == 0) sh_f = f;
      }
      __syncthreads();
      const double f = sh_f;
      const bool stop = (it > 0 && f_prev - f <= r.tol * f) || !isfinite(f) || it >= r.max_iter;
      if (!stop) {
        for (int e = threadIdx.x; e < k * NP; e += kWG) {
          const int j = e / NP, d = e - j * NP;
          if (tcnt[j] > 0) sC[e] = (float)(((double)tot[e] * r.inv_scale[d]) / (double)tcnt[j]);
        }
        __syncthreads();
        lds_norms<NP>(sC, sCn, k);
        __syncthreads();
        f_prev = f;
        continue;
      }
      // stop: degenerate flags; acceptance on a strict improvement
      const bool accept = f < fhat;
      int nd = 0;
      for (int j = 0; j < k; ++j) nd += tcnt[j] == 0 ? 1 : 0;
      if (accept) {
        for (int e = threadIdx.x; e < k * NP; e += kWG) sI[e] = sC[e];
        for (int j = threadIdx.x; j < k; j += kWG) sIdeg[j] = tcnt[j] == 0 ? 1 : 0;
        if (leader) {
          for (int e = threadIdx.x; e < k * n; e += kWG) {
            const int j = e / n, d = e - j * n;
            r.Cinc[(int64_t)w * k * n + e] = sC[j * NP + d];
          }
          for (int j = threadIdx.x; j < k; j += kWG)
            r.deg_inc[(int64_t)w * k + j] = tcnt[j] == 0 ? 1 : 0;
          if (threadIdx.x == 0) r.fhat[w] = f;
        }
        fhat = f;
      }
      if (leader && threadIdx.x == 0) {
        PassOut o;
        o.accepted = accept ? 1 : 0;
        o.iters = it;
        o.ndeg = nd;
        o.pad_ = 1;  // marks the pass as run
        o.f = f;
        r.out[(int64_t)w * r.passes_p + q] = o;
      }
      __syncthreads();
      ++ig;
      break;
    }
  }
}

// XCD id of each workgroup of a grid (the hardware's workgroup placement).
__global__ __launch_bounds__(64) void k_xcd_probe(uint32_t* __restrict__ out) {
  unsigned int x;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
  if (threadIdx.x == 0) out[blockIdx.x] = x & (kMaxXcd - 1);
}

template <int NP, bool MF>
hipError_t round_capacity_np(size_t lds, int* blocks) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_round<NP, MF>, kWG, lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  *blocks = per_cu * cus;
  return hipSuccess;
}

template <int NP, bool MF>
hipError_t launch_round_np(hipStream_t st, const RoundArgs* r_dev, int grid, size_t lds) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_round<NP, MF>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const RoundArgs* p = r_dev;
  void* args[] = {&p};
  return hipLaunchCooperativeKernel((const void*)k_round<NP, MF>, dim3(grid), dim3(kWG), args,
                                    (unsigned int)lds, st);
}

template <int NP, bool SUMS, bool COOP, bool MF>
hipError_t launch_assign_v(hipStream_t st, const AssignArgs& a, int ntiles, size_t lds) {
  // two points per lane while both fit comfortably in registers (one on the
  // matrix cores, whose accumulators take the room)
  constexpr int PPL = (NP <= 32 && !MF) ? 2 : 1;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_assign_small<NP, PPL, SUMS, COOP, MF>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_assign_small<NP, PPL, SUMS, COOP, MF>), dim3(ntiles), dim3(kWG), lds, st, a);
  return hipGetLastError();
}

// The wave re-decides its flagged points together: the sequential form
// costs k distances per lane whenever one lane of the wave needs it, and on
// clustered data with background noise most waves hold such a point (the
// objective over 10,000,000 x 28 points with k = 50: 1.18 -> 0.85 ms).  Up to
// 32 dimensions the per-step kernels rank on the FP32 FMAs, two points per
// lane (measured faster than the matrix-core ranking there, whose looser
// bound flags more points).  Wider rows hold one point per lane either way;
// with many centres they rank on the matrix cores (n = 64: a Lloyd step with
// k = 200 5 % faster, k = 50 2 % slower, so from one full group of 128 on).
constexpr int kMfmaStepMinK = 128;

template <int NP>
hipError_t launch_assign_np(hipStream_t st, const AssignArgs& a, int ntiles, bool sums) {
  const size_t base = (((size_t)a.k * NP + a.k) * 4 + 15) / 16 * 16;
  const size_t lds = sums ? base + (size_t)a.k * NP * 8 + (size_t)a.k * 4 : base;
  if constexpr (NP > 32) {
    if (a.k >= kMfmaStepMinK)
      return sums ? launch_assign_v<NP, true, true, true>(st, a, ntiles, lds)
                  : launch_assign_v<NP, false, true, true>(st, a, ntiles, lds);
  }
  return sums ? launch_assign_v<NP, true, true, false>(st, a, ntiles, lds)
              : launch_assign_v<NP, false, true, false>(st, a, ntiles, lds);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_sample(hipStream_t st, const float* X, int64_t m, int32_t n, int32_t njobs,
                         int64_t max_s, const int64_t* s, const uint64_t* rkeys, int32_t* idx,
                         int64_t idx_stride, float* S, int64_t S_stride, int32_t ld) {
  const dim3 grid((unsigned)((max_s + kWG - 1) / kWG), (unsigned)njobs);
  const int vec = ((n % 4 == 0) && (ld % 4 == 0) && (((uintptr_t)X & 15) == 0) &&
                   (S == nullptr || ((uintptr_t)S & 15) == 0) && (S_stride % 4 == 0)) ? 1 : 0;
  hipLaunchKernelGGL(k_sample, grid, dim3(kWG), 0, st, X, m, n, s, rkeys, idx, idx_stride, S,
                     S_stride, ld, vec);
  return hipGetLastError();
}

hipError_t launch_absmax(hipStream_t st, const float* X, int64_t rows, int32_t n, int32_t ld,
                         unsigned int* absmax_bits) {
  const int64_t total = rows * n;
  int64_t blocks = (total + kWG - 1) / kWG;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_absmax, dim3((unsigned)blocks), dim3(kWG), (size_t)n * 4, st, X, rows, n,
                     ld, absmax_bits);
  return hipGetLastError();
}

hipError_t launch_scales(hipStream_t st, const unsigned int* absmax_bits, int32_t n, int32_t cp,
                         int64_t max_s, double* scale, double* inv_scale) {
  hipLaunchKernelGGL(k_scales, dim3((cp + 255) / 256), dim3(256), 0, st, absmax_bits, n, cp,
                     max_s, scale, inv_scale);
  return hipGetLastError();
}

hipError_t launch_pad_centroids(hipStream_t st, const float* C, int64_t C_stride, int32_t n,
                                int32_t cp, int32_t k, int32_t njobs, float* Cp, int64_t Cp_stride,
                                float* cn, int64_t cn_stride) {
  hipLaunchKernelGGL(k_pad_centroids, dim3(njobs), dim3(kWG), 0, st, C, C_stride, n, cp, k, Cp,
                     Cp_stride, cn, cn_stride);
  return hipGetLastError();
}

hipError_t launch_centroid_norms(hipStream_t st, const float* Cp, int32_t cp, int32_t k,
                                 int32_t njobs, float* cn) {
  hipLaunchKernelGGL(k_centroid_norms, dim3(njobs), dim3(kWG), 0, st, Cp, cp, k, cn);
  return hipGetLastError();
}

hipError_t launch_assign(hipStream_t st, const AssignArgs& a, int32_t ntiles, bool sums) {
  switch (a.cp) {
#define BM_CASE(NPV) \
  case NPV:          \
    return launch_assign_np<NPV>(st, a, ntiles, sums);
    BM_CASE(4)
    BM_CASE(8)
    BM_CASE(12)
    BM_CASE(16)
    BM_CASE(20)
    BM_CASE(24)
    BM_CASE(28)
    BM_CASE(32)
    BM_CASE(36)
    BM_CASE(40)
    BM_CASE(44)
    BM_CASE(48)
    BM_CASE(52)
    BM_CASE(56)
    BM_CASE(60)
    BM_CASE(64)
#undef BM_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_finalize(hipStream_t st, const FinalizeArgs& a, int32_t njobs) {
  const size_t lds = (size_t)a.k * a.cp * sizeof(double);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_finalize,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_finalize, dim3(njobs), dim3(kWG), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_job_init(hipStream_t st, JobState* js, const int64_t* sizes, int32_t njobs,
                           int32_t k, int32_t cp, unsigned long long* acc, int32_t* cnt,
                           const float* Cp, float* cn) {
  hipLaunchKernelGGL(k_job_init, dim3(njobs), dim3(kWG), 0, st, js, sizes, k, cp, acc, cnt, Cp,
                     cn);
  return hipGetLastError();
}

hipError_t launch_reduce_f(hipStream_t st, const double* tf, const int32_t* tnear,
                           const int64_t* sizes, int32_t max_chunks, int32_t njobs, double* f,
                           long long* near) {
  hipLaunchKernelGGL(k_reduce_f, dim3(njobs), dim3(64), 0, st, tf, tnear, sizes, max_chunks, f,
                     near);
  return hipGetLastError();
}

hipError_t launch_unpad(hipStream_t st, const float* Cp, int32_t cp, int32_t n, int32_t k,
                        int32_t njobs, float* C, int64_t C_stride) {
  hipLaunchKernelGGL(k_unpad, dim3(njobs), dim3(kWG), 0, st, Cp, cp, n, k, C, C_stride);
  return hipGetLastError();
}

hipError_t launch_copy_incumbent(hipStream_t st, const float* Cinc, const uint8_t* deg_inc,
                                 int32_t n, int32_t cp, int32_t k, int32_t njobs, float* Cp,
                                 uint8_t* deg_work) {
  hipLaunchKernelGGL(k_copy_incumbent, dim3(njobs), dim3(kWG), 0, st, Cinc, deg_inc, n, cp, k, Cp,
                     deg_work);
  return hipGetLastError();
}

size_t round_lds_bytes(int32_t cp, int32_t k) {
  return round_assign_bytes(cp, k) + (size_t)k * cp * 8 + ((size_t)k * 4 + 15) / 16 * 16 +
         (size_t)k * cp * 4 + ((size_t)k + 15) / 16 * 16;
}

#define BM_ROUND_SWITCH(CALL)      \
  switch (cp) {                    \
    case 4: return CALL(4);        \
    case 8: return CALL(8);        \
    case 12: return CALL(12);      \
    case 16: return CALL(16);      \
    case 20: return CALL(20);      \
    case 24: return CALL(24);      \
    case 28: return CALL(28);      \
    case 32: return CALL(32);      \
    case 36: return CALL(36);      \
    case 40: return CALL(40);      \
    case 44: return CALL(44);      \
    case 48: return CALL(48);      \
    case 52: return CALL(52);      \
    case 56: return CALL(56);      \
    case 60: return CALL(60);      \
    case 64: return CALL(64);      \
    default: return hipErrorInvalidValue; \
  }

template <int NP>
hipError_t assign_static_lds_np(size_t* out) {
  // the variants launched for a Lloyd step (FMA and, above 32 dimensions,
  // matrix-core ranking): the larger static LDS
  constexpr int PPL = NP <= 32 ? 2 : 1;
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, (const void*)k_assign_small<NP, PPL, true, true, false>);
  if (e != hipSuccess) return e;
  *out = fa.sharedSizeBytes;
  if constexpr (NP > 32) {
    e = hipFuncGetAttributes(&fa, (const void*)k_assign_small<NP, 1, true, true, true>);
    if (e == hipSuccess && fa.sharedSizeBytes > *out) *out = fa.sharedSizeBytes;
  }
  return e;
}

hipError_t assign_static_lds(int32_t cp, size_t* out) {
#define BM_SL(NPV) assign_static_lds_np<NPV>(out)
  BM_ROUND_SWITCH(BM_SL)
#undef BM_SL
}

hipError_t launch_xcd_probe(hipStream_t st, uint32_t* out, int32_t grid) {
  hipLaunchKernelGGL(k_xcd_probe, dim3(grid), dim3(64), 0, st, out);
  return hipGetLastError();
}

hipError_t round_capacity(int32_t cp, int32_t k, size_t lds, int* blocks) {
#define BM_CAP(NPV) (k >= kMfmaMinK ? round_capacity_np<NPV, true>(lds, blocks) \
                                    : round_capacity_np<NPV, false>(lds, blocks))
  BM_ROUND_SWITCH(BM_CAP)
#undef BM_CAP
}

hipError_t launch_round(hipStream_t st, const RoundArgs* r_dev, int32_t cp, int32_t k,
                        int32_t grid, size_t lds) {
#define BM_LR(NPV) (k >= kMfmaMinK ? launch_round_np<NPV, true>(st, r_dev, grid, lds) \
                                   : launch_round_np<NPV, false>(st, r_dev, grid, lds))
  BM_ROUND_SWITCH(BM_LR)
#undef BM_LR
}

hipError_t launch_kpp_setup(hipStream_t st, const KppArgs& a, int32_t njobs) {
  hipLaunchKernelGGL(k_kpp_setup, dim3(njobs), dim3(kWG), 0, st, a);
  return hipGetLastError();
}

template <int NP>
hipError_t launch_kpp_init_np(hipStream_t st, const KppArgs& a, dim3 grid) {
  hipLaunchKernelGGL(k_kpp_init_np<NP>, grid, dim3(kWG), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_kpp_init(hipStream_t st, const KppArgs& a, int32_t njobs, int64_t max_s) {
  const dim3 grid((unsigned)((max_s + kDTile - 1) / kDTile), (unsigned)njobs);
  const int cp = a.cp;
  if (cp >= 4 && cp <= kMaxRegDim && cp % 4 == 0) {
#define BM_KI(NPV) launch_kpp_init_np<NPV>(st, a, grid)
    BM_ROUND_SWITCH(BM_KI)
#undef BM_KI
  }
  hipLaunchKernelGGL(k_kpp_init, grid, dim3(kWG), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_kpp_step(hipStream_t st, const KppArgs& a, int32_t njobs) {
  hipLaunchKernelGGL(k_kpp_step, dim3(njobs), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_kpp_pot(hipStream_t st, const KppArgs& a, int32_t njobs, int64_t max_s) {
  const dim3 grid((unsigned)((max_s + kDTile - 1) / kDTile), (unsigned)njobs);
  const size_t lds = (size_t)3 * a.n * sizeof(float);  // candidate rows
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_kpp_pot,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_kpp_pot, grid, dim3(kWG), lds, st, a);
  return hipGetLastError();
}

}  // namespace bm
