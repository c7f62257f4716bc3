// gfx950 kernels of the Big-means hot path for wide points (padded dimension
// cp > 64), where a point no longer fits in one lane's registers.
//
//   k_assign_wide    nearest centre of every point of a tile (Eq. (1)), FP64
//                    objective partials of its 256-point chunks, labels
//   k_update_wide    exact fixed-point per-cluster sums of the points whose
//                    label changed (Lloyd centroid update)
//   k_finalize_wide  cluster means, norms, convergence and acceptance
//
// The dot products x.c_j of a 256-point chunk against up to 128 centres at a
// time run on the matrix cores (v_mfma_f32_32x32x2f32): the chunk's rows and
// the centres are staged through LDS 32 dimensions at a time, each wave owns
// 64 points (two 32-point blocks) and keeps 2 x 4 accumulator tiles.  The
// argmin then follows the same rules as the narrow path: e_j = ||c_j||^2 -
// 2 x.c_j, a rigorous bound on its FP32 rounding error (any summation order
// of cp terms), a direct-form re-decision of every point whose best two e are
// closer than that bound (the whole wave evaluates one such point's centres
// together; for k <= 256 only the centres inside the bound's band, marked
// in per-lane masks), lowest index on ties, and the
// winner's distance in the direct form sum_d (x_d - c_d)^2 (block by block,
// see stage_total), which each thread accumulates from the LDS stages while
// the rows pass for the matrix cores (for the previous label of its point),
// or the whole wave computes for a point whose label changed.
//
// Lloyd labels ping-pong between two arrays (assignment q writes array q mod
// 2), so the update kernel sees the old and the new label of every point.
//
// BF16 variant (k_assign_wide<SUMS, true>): the dot products run on the BF16
// matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation).  Every FP32
// coordinate is split while it is staged into a BF16 high part h = bf16(v)
// and a BF16 residual l = bf16(v - h), and x.c is taken as
// xh.ch + xh.cl + xl.ch: the dropped terms are below 3.01 u_b^2 |x_d||c_d|
// per coordinate (u_b = 2^-8), so the error bound stays near the FP32 one
// and so does the share of points the FP32 direct form re-decides.  With a
// single BF16 product the bound would be about 2^-7 ||x|| ||c||, and on
// unit-norm data with 100 clusters in 768-D about two thirds of the points
// would need the re-decision.  Re-decisions, the winner's distance and the
// objective are the FP32 direct form of the FP32 rows, as in the FP32 path.

#include <math.h>
#include <stdint.h>

#include <type_traits>

#include <hip/hip_runtime.h>

#include "bm_device.h"
#include "bm_internal.h"
#include "bm_precision.h"

namespace bm {
namespace {

constexpr int kDK = 32;            // dimensions per LDS stage
constexpr int kCG = 128;           // centres per group (four 32-wide MFMA tiles)
constexpr int kChunk = 256;        // points per chunk (one per thread in the per-point phase)
constexpr int kPotDK = 32;         // dimensions per LDS stage of the K-means++ potentials
constexpr int kUpdDims = 64;       // dimensions per update workgroup
constexpr int kUpdPts = 4096;      // points per update workgroup
constexpr int kUpdBatch = 16;      // changed points whose slices load together

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr float kUB2 = 1.52587890625e-5f;  // u_b^2 = 2^-16 (u_b = 2^-8, unit roundoff of BF16)

// High parts and residuals of four FP32 values (round to nearest even; the
// difference v - h is exact in FP32).
__device__ inline void split_bf16(const float4 v, bf16x4& h, bf16x4& l) {
  h[0] = (__bf16)v.x;
  h[1] = (__bf16)v.y;
  h[2] = (__bf16)v.z;
  h[3] = (__bf16)v.w;
  l[0] = (__bf16)(v.x - (float)h[0]);
  l[1] = (__bf16)(v.y - (float)h[1]);
  l[2] = (__bf16)(v.z - (float)h[2]);
  l[3] = (__bf16)(v.w - (float)h[3]);
}

// Direct-form squared distance over the padded width: partial sum d mod 4,
// then (p0 + p1) + (p2 + p3).  Padding is zero on both sides, so the value
// equals the same sum over the n real dimensions.
__device__ inline float dist_wide(const float* __restrict__ x, const float* __restrict__ c, int n,
                                  int ld_is_vec) {
  float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
  if (ld_is_vec) {
    const float4* x4 = reinterpret_cast<const float4*>(x);
    const float4* c4 = reinterpret_cast<const float4*>(c);
    const int n4 = (n + 3) / 4;
    for (int q = 0; q < n4; ++q) {
      const float4 a = x4[q], b = c4[q];
      const float t0 = a.x - b.x, t1 = a.y - b.y, t2 = a.z - b.z, t3 = a.w - b.w;
      p0 = fmaf(t0, t0, p0);
      p1 = fmaf(t1, t1, p1);
      p2 = fmaf(t2, t2, p2);
      p3 = fmaf(t3, t3, p3);
    }
  } else {
    for (int d = 0; d < n; ++d) {
      const float t = x[d] - c[d];
      const int r = d & 3;
      if (r == 0) p0 = fmaf(t, t, p0);
      else if (r == 1) p1 = fmaf(t, t, p1);
      else if (r == 2) p2 = fmaf(t, t, p2);
      else p3 = fmaf(t, t, p3);
    }
  }
  return (p0 + p1) + (p2 + p3);
}

// Squared distance by a whole wave (x and c uniform): lane l takes the
// 4-float groups l, l + 64, ... (the dimensions l, l + 64, ... when rows are
// not 16-byte aligned), then a butterfly adds the 64 partial sums, so every
// lane ends with the same value; the reads are coalesced.
__device__ inline float dist_wave(const float* __restrict__ x, const float* __restrict__ c, int n,
                                  int cp, int ld_is_vec) {
  const int lane = threadIdx.x & 63;
  float p = 0.f;
  if (ld_is_vec) {
    const float4* x4 = reinterpret_cast<const float4*>(x);
    const float4* c4 = reinterpret_cast<const float4*>(c);
    for (int q = lane; q < cp / 4; q += 64) {
      const float4 a = x4[q], b = c4[q];
      const float t0 = a.x - b.x, t1 = a.y - b.y, t2 = a.z - b.z, t3 = a.w - b.w;
      p = fmaf(t0, t0, p);
      p = fmaf(t1, t1, p);
      p = fmaf(t2, t2, p);
      p = fmaf(t3, t3, p);
    }
  } else {
    for (int d = lane; d < n; d += 64) {
      const float t = x[d] - c[d];
      p = fmaf(t, t, p);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off, 64);
  return p;
}

// min that propagates NaN from either operand.
__device__ inline float kpp_min_nan(float a, float b) {
  const float r = b < a ? b : a;
  return (a != a || b != b) ? __builtin_nanf("") : r;
}

// Best and second-best (value, index) merge; on equal values the lower index
// wins, so the result is the first minimum in index order.
__device__ inline void top2_merge(float& e1, int& j1, float& e2, float oe1, int oj1, float oe2) {
  if (oe1 < e1 || (oe1 == e1 && oj1 < j1)) {
    e2 = fminf(e1, oe2);
    e1 = oe1;
    j1 = oj1;
  } else {
    e2 = fminf(e2, oe1);
  }
}

// LDS of one assignment workgroup: the chunk's rows and the centre group,
// 32 dimensions of each (FP32).  Row strides: 33 floats for the FP32 matrix
// cores (one float per lane and column reads hit distinct banks), 36 for the
// BF16 ones (8 floats per lane read as two 16-byte words).
template <bool BF>
struct __align__(16) WideShared {
  static constexpr int kR = BF ? 36 : 33;
  float S[kChunk * kR];
  float C[kCG * kR];
  double red_f[4];
  int red_i[4];
  // candidate masks of the first centre group when there are two groups
  // ([wave][point block][lane], lane layout of the matrix-core results)
  unsigned long long m0[4][2][64];
};

// Row of the staging loops: 4 consecutive dimensions d .. d + 3 of row r of
// the chunk (zero past the point count, past n and past cp).
__device__ inline float4 stage_point(const float* __restrict__ S, int64_t row, int ld, int d, int n,
                                     int cp, int vec, bool in) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (in) {
    const float* src = S + row * (int64_t)ld + d;
    if (vec) {
      if (d < cp) v = *reinterpret_cast<const float4*>(src);
    } else {
      v.x = d < n ? src[0] : 0.f;
      v.y = d + 1 < n ? src[1] : 0.f;
      v.z = d + 2 < n ? src[2] : 0.f;
      v.w = d + 3 < n ? src[3] : 0.f;
    }
  }
  return v;
}

// 4 consecutive dimensions d .. d + 3 of a row for a staging loop: all loads
// of a stage are issued before the first LDS store.  Out-of-range slots read
// row 0 / dimension 0 of the same array (always valid) and are zeroed.
__device__ inline float4 stage_load(const float* __restrict__ S, int64_t row, int ld, int d, int n,
                                    int cp, int vec, bool in) {
  if (vec) {
    const bool ok = in && d < cp;
    const float4 v = *reinterpret_cast<const float4*>(S + (ok ? row * (int64_t)ld + d : 0));
    return ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  return stage_point(S, row, ld, d, n, cp, vec, in);
}

// One 32-dimension stage of the chunk's rows (256 x 32) and of the centre
// group g0 (ng rows, zero past k) into LDS: all loads of the stage are
// issued before the first store.
template <bool BF>
__device__ inline void stage_store(float* dst, const float4 v) {
  if constexpr (BF) {
    *reinterpret_cast<float4*>(dst) = v;
  } else {
    dst[0] = v.x;
    dst[1] = v.y;
    dst[2] = v.z;
    dst[3] = v.w;
  }
}

template <bool BF>
__device__ inline void stage_rows(WideShared<BF>& sh, const float* __restrict__ S, int64_t cb,
                                  int np, const float* __restrict__ C, int g0, int ng, int d0,
                                  int ld, int n, int cp, int vec, bool centres) {
  constexpr int R = WideShared<BF>::kR;
  constexpr int kPt = kChunk * (kDK / 4) / 256;  // float4 per thread: rows
  constexpr int kCt = kCG * (kDK / 4) / 256;     // float4 per thread: centres
  const int tid = threadIdx.x;
  // thread tid takes dimensions d0 + 4 (tid % 8) .. + 3 of rows tid / 8 + 32 u
  const int r0 = tid / (kDK / 4), q = tid - r0 * (kDK / 4);
  float4 v[kPt], w[kCt];
#pragma unroll
  for (int u = 0; u < kPt; ++u)
    v[u] = stage_load(S, cb + r0 + 32 * u, ld, d0 + 4 * q, n, cp, vec, r0 + 32 * u < np);
  if (centres) {
#pragma unroll
    for (int u = 0; u < kCt; ++u)
      w[u] = stage_load(C, g0 + r0 + 32 * u, cp, d0 + 4 * q, cp, cp, 1, r0 + 32 * u < ng);
  }
#pragma unroll
  for (int u = 0; u < kPt; ++u) stage_store<BF>(sh.S + (r0 + 32 * u) * R + 4 * q, v[u]);
  if (!centres) return;
#pragma unroll
  for (int u = 0; u < kCt; ++u) stage_store<BF>(sh.C + (r0 + 32 * u) * R + 4 * q, w[u]);
}

// The winner's squared distance is defined stage by stage: for every
// 32-dimension block s (dimensions 32 s .. 32 s + 31 of the padded row) four
// partial sums by d mod 4 (increasing d, fused multiply-adds) give
// T_s = (p0 + p1) + (p2 + p3), and the blocks add in order,
// ((T_0 + T_1) + T_2) + ...  A thread computes T_s of its row against centre
// row cr while the block sits in LDS (stage_total); a wave computes the whole
// sum of one point with one block per lane (dist_blocks).  Both give the same
// bits.
template <bool BF>
__device__ inline float stage_total(const WideShared<BF>& sh, int cr) {
  constexpr int R = WideShared<BF>::kR;
  const float* x = sh.S + threadIdx.x * R;
  const float* c = sh.C + cr * R;
  float p[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int d = 0; d < kDK; d += 4) {
    float xv[4], cv[4];
    if constexpr (BF) {
      const float4 a = *reinterpret_cast<const float4*>(x + d);
      const float4 b = *reinterpret_cast<const float4*>(c + d);
      xv[0] = a.x; xv[1] = a.y; xv[2] = a.z; xv[3] = a.w;
      cv[0] = b.x; cv[1] = b.y; cv[2] = b.z; cv[3] = b.w;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        xv[q] = x[d + q];
        cv[q] = c[d + q];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float t = xv[q] - cv[q];
      p[q] = fmaf(t, t, p[q]);
    }
  }
  return (p[0] + p[1]) + (p[2] + p[3]);
}

// T_s of block s of row x against row c (zero past n, and past cp).
__device__ inline float block_total(const float* __restrict__ x, const float* __restrict__ c,
                                    int s, int n, int cp, int vec) {
  float p[4] = {0.f, 0.f, 0.f, 0.f};
  const int d0 = s * kDK;
  if (vec) {
#pragma unroll
    for (int g = 0; g < kDK / 4; ++g) {
      const int d = d0 + 4 * g;
      if (d < cp) {
        const float4 a = *reinterpret_cast<const float4*>(x + d);
        const float4 b = *reinterpret_cast<const float4*>(c + d);
        const float t0 = a.x - b.x, t1 = a.y - b.y, t2 = a.z - b.z, t3 = a.w - b.w;
        p[0] = fmaf(t0, t0, p[0]);
        p[1] = fmaf(t1, t1, p[1]);
        p[2] = fmaf(t2, t2, p[2]);
        p[3] = fmaf(t3, t3, p[3]);
      }
    }
  } else {
    for (int dd = 0; dd < kDK; ++dd) {
      const int d = d0 + dd;
      const float t = d < n ? x[d] - c[d] : 0.f;
      p[dd & 3] = fmaf(t, t, p[dd & 3]);
    }
  }
  return (p[0] + p[1]) + (p[2] + p[3]);
}

__device__ inline float dist_blocks(const float* __restrict__ x, const float* __restrict__ c, int n,
                                    int cp, int vec) {
  const int lane = threadIdx.x & 63;
  const int nb = (cp + kDK - 1) / kDK;
  float total = 0.f;
  for (int s0 = 0; s0 < nb; s0 += 64) {
    const float t = s0 + lane < nb ? block_total(x, c, s0 + lane, n, cp, vec) : 0.f;
    const int m = min(64, nb - s0);
    for (int q = 0; q < m; ++q) total += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), q));
  }
  return total;
}

// Eight consecutive FP32 values as BF16 high parts and residuals.
__device__ inline void split8(const float* v, bf16x8& h, bf16x8& l) {
  const float4 a = *reinterpret_cast<const float4*>(v);
  const float4 b = *reinterpret_cast<const float4*>(v + 4);
  bf16x4 h0, l0, h1, l1;
  split_bf16(a, h0, l0);
  split_bf16(b, h1, l1);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    h[q] = h0[q];
    h[4 + q] = h1[q];
    l[q] = l0[q];
    l[4 + q] = l1[q];
  }
}

template <bool SUMS, bool BF, bool KPP, bool G2>
__global__ __launch_bounds__(256, 2) void k_assign_wide(AssignArgs a, KppInitOut kp) {
  constexpr int R = WideShared<BF>::kR;
  const int job = a.tile_job[blockIdx.x];
  const uint8_t* dg = nullptr;  // K-means++ initial D: centroids to leave out
  if (KPP) {
    const KppState kst = kp.ks[job];
    if (kst.ntodo == 0 || !kst.has_d) return;
    dg = kp.deg + (int64_t)job * a.k;
  }
  int parity = 0, iter = 0;
  if (a.st) {
    const JobState st = a.st[job];
    if (!st.active) return;
    parity = st.iter & 1;
    iter = st.iter;
  }
  const int64_t s = a.s[job];
  const int64_t t0 = (int64_t)a.tile_idx[blockIdx.x] * a.tile_pts;
  const int64_t t1 = min(s, t0 + (int64_t)a.tile_pts);
  const int k = a.k, n = a.n, cp = a.cp, ld = a.ld;
  // two centre groups, both re-decided through candidate masks (G2 builds
  // only: the masks of the first group take registers the others keep)
  const bool two = G2 && k > kCG && k <= 2 * kCG;
  const float* __restrict__ S = a.S + job * a.S_stride;
  const float* __restrict__ C = a.Cp + job * a.C_stride;
  const float* __restrict__ cn = a.cn + job * a.cn_stride;
  int32_t* const lbase = (parity && a.labels2) ? a.labels2 : a.labels;
  int32_t* __restrict__ lab = lbase ? lbase + job * a.lab_stride : nullptr;
  // Lloyd step q >= 1 of a wide job: step q - 1 wrote the other label array;
  // each point's previous label predicts its winner, whose distance is then
  // accumulated while the rows pass through LDS
  const int32_t* prev = nullptr;
  if (a.st && a.labels2 && iter >= 1) prev = (parity ? a.labels : a.labels2) + job * a.lab_stride;
  double* tfj = a.tf + (int64_t)job * a.max_chunks;
  const bool want_near = a.tnear != nullptr;
  const int vec = a.vec;

  __shared__ WideShared<BF> sh;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int half = lane >> 5, col = lane & 31;

  float cmax2 = 0.f;
  for (int j = lane; j < k; j += 64)
    if (!KPP || !dg[j]) cmax2 = fmaxf(cmax2, cn[j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) cmax2 = fmaxf(cmax2, __shfl_xor(cmax2, off, 64));
  const float cmax = sqrtf(cmax2) * 1.0000002f;
  // any summation order of the products: gamma_{cp+1} (FP32), gamma_{3cp+1}
  // (three split products per dimension, whose magnitudes add up to at most
  // 1.02 |x_d||c_d|) plus the dropped split terms (BF16)
  const float terms = BF ? (float)(3 * cp + 1) : (float)(cp + 1);
  const float gam = terms * kU / (1.f - terms * kU);
  const float kB = BF ? 2.f * (2.f * (3.2f * kUB2 + 1.02f * gam) + 2.1f * kU)
                      : 2.f * (2.f * gam + 2.f * kU);

  for (int64_t cb = t0; cb < t1; cb += kChunk) {
    const int np = (int)min((int64_t)kChunk, t1 - cb);  // valid points of the chunk
    const int64_t i = cb + tid;
    const bool valid = tid < np;
    int pl = -1;  // predicted winner
    if (prev && valid) {
      pl = prev[i];
      if (pl < 0 || pl >= k) pl = -1;
    }
    float wacc = 0.f;  // winner's distance to pl, block by block
    float e1[2], e2[2];
    int j1[2];
    float xxp[2] = {0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      e1[b] = __builtin_inff();
      e2[b] = __builtin_inff();
      j1[b] = 0;
    }
    f32x16 acc[2][4];  // after the loop: the products of the last centre group
    for (int g0 = 0; g0 < k; g0 += kCG) {
      const int ng = min(kCG, k - g0);
      const bool mine = pl >= g0 && pl < g0 + ng;
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[b][t][v] = 0.f;
      for (int d0 = 0; d0 < cp; d0 += kDK) {
        __syncthreads();  // the previous stage has been consumed
        stage_rows<BF>(sh, S, cb, np, C, g0, ng, d0, ld, n, cp, vec, true);
        __syncthreads();
        if (mine) wacc += stage_total<BF>(sh, pl - g0);
        if constexpr (!BF) {
          // lane (half, col): A = centre (tile*32 + col) at dim kk + half,
          //                   B = point (wv*64 + b*32 + col) at dim kk + half
          for (int kk = 0; kk < kDK; kk += 2) {
            float bv[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              bv[b] = sh.S[(wv * 64 + b * 32 + col) * R + kk + half];
              if (g0 == 0) xxp[b] = fmaf(bv[b], bv[b], xxp[b]);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const float av = sh.C[(t * 32 + col) * R + kk + half];
#pragma unroll
              for (int b = 0; b < 2; ++b)
                acc[b][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[b], acc[b][t], 0, 0, 0);
            }
          }
        } else {
          // lane (half, col): A = centre (tile*32 + col), B = point
          // (wv*64 + b*32 + col), both at dims ks + 8 half .. ks + 8 half + 7,
          // split into high parts and residuals as they are read
          for (int ks = 0; ks < kDK; ks += 16) {
            bf16x8 xh[2], xl[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              const float* p = sh.S + (wv * 64 + b * 32 + col) * R + ks + 8 * half;
              split8(p, xh[b], xl[b]);
              if (g0 == 0) {
#pragma unroll
                for (int q = 0; q < 8; ++q) xxp[b] = fmaf(p[q], p[q], xxp[b]);
              }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              bf16x8 ch, cl;
              split8(sh.C + (t * 32 + col) * R + ks + 8 * half, ch, cl);
#pragma unroll
              for (int b = 0; b < 2; ++b) {
                acc[b][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cl, xh[b], acc[b][t], 0, 0, 0);
                acc[b][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ch, xl[b], acc[b][t], 0, 0, 0);
                acc[b][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ch, xh[b], acc[b][t], 0, 0, 0);
              }
            }
          }
        }
      }
      // this lane holds, for point col of block b, the centres
      // g0 + 32 t + 8 (v / 4) + 4 half + v % 4, in increasing order
#pragma unroll
      for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int c = g0 + t * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
            if (c < k && (!KPP || !dg[c])) {
              const float e = fmaf(-2.f, acc[b][t][v], cn[c]);
              e2[b] = __builtin_amdgcn_fmed3f(e1[b], e, e2[b]);
              j1[b] = e < e1[b] ? c : j1[b];
              e1[b] = fminf(e1[b], e);
            }
          }
        }
      }
      if (two && g0 == 0) {
        // candidates of the first group against the running best: a later
        // group can only lower the best, so these masks (with a 0.1 % wider
        // band) hold every centre of the group that the final band admits
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const float XX = xxp[b] + __shfl_xor(xxp[b], 32, 64);
          const float E1 = fminf(e1[b], __shfl_xor(e1[b], 32, 64));
          const float Bb = kB * (sqrtf(XX) * cmax + cmax2);
          unsigned long long m = 0ull;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int c = t * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
              if (!KPP || !dg[c]) {
                const float e = fmaf(-2.f, acc[b][t][v], cn[c]);
                if (!((e - E1) > (2.f * Bb + 2.5e-5f * fabsf(e + XX)) * 1.001f)) m |= 1ull << (t * 16 + v);
              }
            }
          }
          sh.m0[wv][b][lane] = m;
        }
      }
    }
    // combine the two halves of every point's centre set
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const float oe1 = __shfl_xor(e1[b], 32, 64);
      const int oj1 = __shfl_xor(j1[b], 32, 64);
      const float oe2 = __shfl_xor(e2[b], 32, 64);
      top2_merge(e1[b], j1[b], e2[b], oe1, oj1, oe2);
    }
    // per-point phase: thread tid <-> point cb + tid (block = half, position col)
    const float xo = __shfl_xor(half ? xxp[0] : xxp[1], 32, 64);
    const float xx = (half ? xxp[1] : xxp[0]) + xo;
    const float pe1 = half ? e1[1] : e1[0];
    const float pe2 = half ? e2[1] : e2[0];
    const int pj1 = half ? j1[1] : j1[0];
    double fpart = 0.0;
    int near = 0;
    const float B = kB * (sqrtf(xx) * cmax + cmax2);
    const bool recheck = valid && !((pe2 - pe1) > 2.f * B + 2.5e-5f * fabsf(pe2 + xx));
    int jw = pj1;
    if (k <= kCG || two) {
      // Re-decision among the candidates only: a centre j whose e_j exceeds
      // the point's best e by more than 2 B + 2.5e-5 |e_j + ||x||^2| is
      // certified farther than the winner and not within the near-tie band.
      // Lane (half, col) marks, for point col of each block, the candidates
      // among its centres of the last group (bit 16 t + v for centre
      // gl + 32 t + 8 (v / 4) + 4 half + v % 4; the first group's masks, if
      // there are two groups, are in LDS); then the wave takes the flagged
      // points one at a time and their candidates one at a time (lanes over
      // the dimensions).
      const int gl = two ? kCG : 0;
      unsigned long long cmask[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int owner = b * 32 + col;
        const float E1 = __shfl(pe1, owner, 64);
        const float Bb = __shfl(B, owner, 64);
        const float XX = __shfl(xx, owner, 64);
        unsigned long long m = 0ull;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int c = gl + t * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
            if (c < k && (!KPP || !dg[c])) {
              const float e = fmaf(-2.f, acc[b][t][v], cn[c]);
              if (!((e - E1) > 2.f * Bb + 2.5e-5f * fabsf(e + XX))) m |= 1ull << (t * 16 + v);
            }
          }
        }
        cmask[b] = m;
      }
      unsigned long long pending = __ballot(recheck);
      while (pending) {
        const int src = __ffsll(pending) - 1;
        pending &= pending - 1;
        const int sb = src >> 5, sc = src & 31;
        const unsigned long long mb = sb ? cmask[1] : cmask[0];
        unsigned long long mh[2];
        mh[0] = ((unsigned long long)__builtin_amdgcn_readlane((int)(mb >> 32), sc) << 32) |
                (unsigned int)__builtin_amdgcn_readlane((int)(mb & 0xffffffffull), sc);
        mh[1] = ((unsigned long long)__builtin_amdgcn_readlane((int)(mb >> 32), sc + 32) << 32) |
                (unsigned int)__builtin_amdgcn_readlane((int)(mb & 0xffffffffull), sc + 32);
        const float* xs = S + (cb + wv * 64 + src) * (int64_t)ld;
        float b1 = __builtin_inff(), b2 = __builtin_inff();
        int jb = 0;
        for (int q = two ? 0 : 2; q < 4; ++q) {
          const int h = q & 1;
          unsigned long long mm = q < 2 ? sh.m0[wv][sb][sc + 32 * h] : mh[h];
          const int go = q < 2 ? 0 : gl;
          while (mm) {
            const int bit = __ffsll(mm) - 1;
            mm &= mm - 1;
            const int c = go + (bit >> 4) * 32 + 8 * ((bit & 15) >> 2) + 4 * h + (bit & 3);
            const float dd = dist_wave(xs, C + (int64_t)c * cp, n, cp, vec);
            top2_merge(b1, jb, b2, dd, c, __builtin_inff());
          }
        }
        if (lane == src) {
          jw = jb;
          if (b2 - b1 < 1e-5f * b2) near = 1;
        }
      }
    } else {
    // direct-form re-decision, one flagged point at a time by the whole wave:
    // lane l takes the centres l, l + 64, ... in order, then the best and
    // second best merge across lanes (lowest index on equal distances)
    unsigned long long pending = __ballot(recheck);
    while (pending) {
      const int src = __ffsll(pending) - 1;
      pending &= pending - 1;
      const float* xs = S + (cb + wv * 64 + src) * (int64_t)ld;
      float b1 = __builtin_inff(), b2 = __builtin_inff();
      int jb = 0;
      for (int j = lane; j < k; j += 64) {
        if (KPP && dg[j]) continue;
        const float dd = dist_wide(xs, C + (int64_t)j * cp, n, vec);
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
        top2_merge(b1, jb, b2, o1, oj, o2);
      }
      if (lane == src) {
        jw = jb;
        if (b2 - b1 < 1e-5f * b2) near = 1;
      }
    }
    }
    // winner's distance: the accumulated one when the prediction holds, else
    // the whole wave computes it for each such point (same bits)
    unsigned long long missed = __ballot(valid && jw != pl);
    while (missed) {
      const int src = __ffsll(missed) - 1;
      missed &= missed - 1;
      const int jq = __builtin_amdgcn_readlane(jw, src);
      const float dq = dist_blocks(S + (cb + wv * 64 + src) * (int64_t)ld, C + (int64_t)jq * cp, n, cp, vec);
      if (lane == src) wacc = dq;
    }
    if (valid) {
      fpart = (double)wacc;
      if (lab) lab[i] = jw;
      if (KPP) kp.D[(int64_t)job * kp.D_job_stride + i] = wacc;
    }
    fpart = wave_sum_f64(fpart);
    if (lane == 0) sh.red_f[wv] = fpart;
    if (want_near) {
      near = wave_sum_i32(near);
      if (lane == 0) sh.red_i[wv] = near;
    }
    __syncthreads();
    if (tid == 0) {
      const double tot = (sh.red_f[0] + sh.red_f[1]) + (sh.red_f[2] + sh.red_f[3]);
      if (KPP)
        kp.Dt[(int64_t)job * kp.Dt_job_stride + cb / kChunk] = tot;
      else
        tfj[cb / kChunk] = tot;
      if (want_near)
        a.tnear[(int64_t)job * a.max_chunks + cb / kChunk] =
            (sh.red_i[0] + sh.red_i[1]) + (sh.red_i[2] + sh.red_i[3]);
    }
  }
}

// Greedy K-means++ potentials, rows staged through LDS: for every pending candidate
// c of a job, the new D_i = min(D_i, ||S_i - S_cand_c||^2) into the D slot of
// that candidate and the sum of every 256-point tile (the four wave sums
// added in a fixed order).  The tile's rows pass through LDS 32 dimensions at
// a time with coalesced loads, the candidates' rows sit in LDS whole, and each
// thread keeps its point's distances in four partial sums by d mod 4 (the
// dimensions past the last multiple of 4 in the first one), so D is the same
// as from a thread reading its row directly.
__global__ __launch_bounds__(256) void k_kpp_pot_staged(KppArgs a) {
  const int job = a.job_slot ? a.job_slot[blockIdx.y] : (int)blockIdx.y;
  const KppState ks = a.ks[job];
  if (ks.ncand == 0) return;
  const int64_t s = a.s[job];
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  if (base >= s) return;
  const int tid = threadIdx.x;
  const int64_t i = base + tid;
  const float* S = a.S + job * a.S_stride;
  const int n = a.n, cp = a.cp, ld = a.ld, nc = ks.ncand;
  const int n4 = n & ~3;
  const int np = (int)min((int64_t)kChunk, s - base);
  const int vec = (ld % 4 == 0 && (((uintptr_t)S & 15) == 0)) ? 1 : 0;
  extern __shared__ __align__(16) float kpp_lds[];
  float* cand = kpp_lds;              // [3][cp]
  float* rows = kpp_lds + 3 * cp;     // [256][kPotDK + 1]
  __shared__ double red[12];
  for (int e = tid; e < 3 * cp; e += 256) {  // rows of absent candidates are zero
    const int c = e / cp, d = e - c * cp;
    const int64_t row = c == 0 ? ks.cand[0] : (c == 1 ? ks.cand[1] : ks.cand[2]);
    cand[e] = (c < nc && d < n) ? S[row * ld + d] : 0.f;
  }
  const int dslot = ks.dcur;
  float dcur = 0.f;
  if (i < s && ks.has_d) dcur = a.D[(int64_t)dslot * a.D_slot_stride + job * a.D_job_stride + i];
  float p[3][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
  // the loads of stage d0 + 32 are issued before stage d0 is computed, so they
  // are in flight behind this workgroup's own arithmetic
  constexpr int kPt = kChunk * (kPotDK / 4) / 256;
  float4 v[kPt];
#pragma unroll
  for (int u = 0; u < kPt; ++u) {
    const int e = tid + u * 256, r = e / (kPotDK / 4), q = e - r * (kPotDK / 4);
    v[u] = stage_load(S, base + r, ld, 4 * q, n, cp, vec, r < np);
  }
  for (int d0 = 0; d0 < cp; d0 += kPotDK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPt; ++u) {
      const int e = tid + u * 256, r = e / (kPotDK / 4), q = e - r * (kPotDK / 4);
      float* dst = rows + r * (kPotDK + 1) + 4 * q;
      dst[0] = v[u].x;
      dst[1] = v[u].y;
      dst[2] = v[u].z;
      dst[3] = v[u].w;
    }
    __syncthreads();
    if (d0 + kPotDK < cp) {
#pragma unroll
      for (int u = 0; u < kPt; ++u) {
        const int e = tid + u * 256, r = e / (kPotDK / 4), q = e - r * (kPotDK / 4);
        v[u] = stage_load(S, base + r, ld, d0 + kPotDK + 4 * q, n, cp, vec, r < np);
      }
    }
    const int dn = min(kPotDK, n - d0);  // real dimensions of this stage
    const float* xr = rows + tid * (kPotDK + 1);
    for (int dd = 0; dd < dn; dd += 4) {
      const int d = d0 + dd;
      if (d + 4 <= n4) {
        const float x0 = xr[dd], x1 = xr[dd + 1], x2 = xr[dd + 2], x3 = xr[dd + 3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float* cr = cand + c * cp + d;
          const float u0 = x0 - cr[0], u1 = x1 - cr[1], u2 = x2 - cr[2], u3 = x3 - cr[3];
          p[c][0] = fmaf(u0, u0, p[c][0]);
          p[c][1] = fmaf(u1, u1, p[c][1]);
          p[c][2] = fmaf(u2, u2, p[c][2]);
          p[c][3] = fmaf(u3, u3, p[c][3]);
        }
      } else {  // dimensions past the last multiple of 4, in order, into the first sum
        const int nq = min(4, dn - dd);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (q < nq) {
            const float xq = xr[dd + q];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const float u = xq - cand[c * cp + d + q];
              p[c][0] = fmaf(u, u, p[c][0]);
            }
          }
        }
      }
    }
  }
  const int wv = tid >> 6;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c < nc) {
      float m = 0.f;
      if (i < s) {
        const float dc = (p[c][0] + p[c][1]) + (p[c][2] + p[c][3]);
        m = ks.has_d ? kpp_min_nan(dcur, dc) : dc;
        const int sl = c < dslot ? c : c + 1;
        a.D[(int64_t)sl * a.D_slot_stride + job * a.D_job_stride + i] = m;
      }
      const double part = wave_sum_f64(i < s ? (double)m : 0.0);
      if ((tid & 63) == 0) red[c * 4 + wv] = part;
    }
  }
  __syncthreads();
  if (tid == 0)
    for (int c = 0; c < nc; ++c) {
      const int sl = c < dslot ? c : c + 1;
      a.Dt[((int64_t)sl * a.njobs + job) * a.ndt_max + blockIdx.x] =
          (red[c * 4] + red[c * 4 + 1]) + (red[c * 4 + 2] + red[c * 4 + 3]);
    }
}

// Fixed-point sums of the label changes: grid (cp / 64 dimension slices,
// point ranges of kUpdPts, jobs).  A point whose label went from jo to jn adds
// its coordinates to cluster jn and removes them from jo (jo < 0 on the first
// assignment).  The workgroup first sorts the changes of its range by cluster
// in LDS (a counting sort: one entry per (point, cluster, sign)), then each of
// its eight waves walks an eighth of the sorted entries, one dimension of the
// slice per lane, keeps the current cluster's sum in a register and adds it to memory
// with one integer atomic per lane when the cluster changes.  Integer sums:
// the result does not depend on the order.
struct UpdateArgs {
  const float* S;
  int64_t S_stride;
  int32_t ld, n, cp, k;
  const int64_t* s;
  const JobState* st;
  const int32_t* lab0;     // assignment q of a job (q = its iter) wrote lab[q % 2]
  const int32_t* lab1;
  int64_t lab_stride;
  unsigned long long* acc;  // [job][k][cp]
  int32_t* cnt;             // [job][k]
  const double* scale;      // [cp]
};

// entry of the sorted changes: cluster << 13 | point in range << 1 | removal
static_assert(kUpdPts <= 4096, "an entry holds the point's place in the range in 12 bits");
constexpr int kUpdThreads = 512;                 // eight waves
constexpr int kUpdWaves = kUpdThreads / 64;
constexpr int kUpdPerThread = kUpdPts / kUpdThreads;

__global__ __launch_bounds__(kUpdThreads) void k_update_wide(UpdateArgs u) {
  const int job = blockIdx.z;
  const JobState st = u.st[job];
  if (!st.active) return;
  const int q = st.iter;
  const int64_t s = u.s[job];
  const int64_t r0 = (int64_t)blockIdx.y * kUpdPts;
  if (r0 >= s) return;
  const int np = (int)min((int64_t)kUpdPts, s - r0);
  const int k = u.k, d0 = blockIdx.x * kUpdDims;
  const int nd = min(kUpdDims, u.n - d0);  // real dimensions of this slice
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* ent = reinterpret_cast<uint32_t*>(smem);  // [2 kUpdPts]
  int* off = reinterpret_cast<int*>(ent + 2 * kUpdPts);  // [k + 1] counts, then offsets
  int* cur = off + (k + 1);                                // [k] scatter cursors
  int* dcn = cur + k;                                      // [k] count changes
  const bool counts = blockIdx.x == 0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int e = tid; e <= k; e += kUpdThreads) off[e] = 0;
  for (int e = tid; e < k; e += kUpdThreads) dcn[e] = 0;
  // the labels of this thread's points, loaded together
  const int32_t* ln = ((q & 1) ? u.lab1 : u.lab0) + job * u.lab_stride + r0;
  const int32_t* lo = q == 0 ? nullptr : ((q & 1) ? u.lab0 : u.lab1) + job * u.lab_stride + r0;
  int jn[kUpdPerThread], jo[kUpdPerThread];
#pragma unroll
  for (int t = 0; t < kUpdPerThread; ++t) {
    const int i = tid + t * kUpdThreads;
    jn[t] = i < np ? ln[i] : -1;
    jo[t] = (i < np && lo) ? lo[i] : -1;
  }
  __syncthreads();
  // entries per cluster
#pragma unroll
  for (int t = 0; t < kUpdPerThread; ++t) {
    if (jn[t] != jo[t]) {
      atomicAdd(&off[jn[t]], 1);
      if (jo[t] >= 0) atomicAdd(&off[jo[t]], 1);
      if (counts) {
        atomicAdd(&dcn[jn[t]], 1);
        if (jo[t] >= 0) atomicAdd(&dcn[jo[t]], -1);
      }
    }
  }
  __syncthreads();
  // exclusive prefix over the clusters (wave 0), off[k] = number of entries
  if (wv == 0) {
    int carry = 0;
    for (int c0 = 0; c0 < k; c0 += 64) {
      const int c = c0 + lane;
      const int v = c < k ? off[c] : 0;
      int x = v;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
      }
      if (c < k) {
        off[c] = carry + x - v;
        cur[c] = carry + x - v;
      }
      carry += __shfl(x, 63);
    }
    if (lane == 0) off[k] = carry;
  }
  __syncthreads();
  const int ne = off[k];
  if (ne == 0) return;
  if (counts) {
    int32_t* cntj = u.cnt + (int64_t)job * k;
    for (int e = tid; e < k; e += kUpdThreads)
      if (dcn[e]) atomicAdd(&cntj[e], dcn[e]);
  }
#pragma unroll
  for (int t = 0; t < kUpdPerThread; ++t) {
    if (jn[t] != jo[t]) {
      const uint32_t pr = (uint32_t)(tid + t * kUpdThreads) << 1;
      ent[atomicAdd(&cur[jn[t]], 1)] = ((uint32_t)jn[t] << 13) | pr;
      if (jo[t] >= 0) ent[atomicAdd(&cur[jo[t]], 1)] = ((uint32_t)jo[t] << 13) | pr | 1u;
    }
  }
  __syncthreads();
  // this wave's share of the entries; lane l adds dimension d0 + l
  const int per = (ne + kUpdWaves - 1) / kUpdWaves;
  const int e0 = min(ne, wv * per), e1 = min(ne, e0 + per);
  const float* S = u.S + job * u.S_stride + r0 * (int64_t)u.ld + d0 + lane;
  unsigned long long* accj = u.acc + (int64_t)job * k * u.cp + d0 + lane;
  const double sc = lane < nd ? u.scale[d0 + lane] : 0.0;
  unsigned long long a = 0ull;
  int cl = -1;
  for (int b = e0; b < e1; b += 64) {
    const uint32_t mine = b + lane < e1 ? ent[b + lane] : 0u;
    const int nb = min(64, e1 - b);
    for (int t0 = 0; t0 < nb; t0 += kUpdBatch) {
      // the slices of up to kUpdBatch entries load together
      float xv[kUpdBatch];
#pragma unroll
      for (int t = 0; t < kUpdBatch; ++t) {
        const uint32_t e = __builtin_amdgcn_readlane(mine, min(t0 + t, 63));
        xv[t] = (t0 + t < nb && lane < nd) ? S[(int64_t)((e >> 1) & 4095u) * u.ld] : 0.f;
      }
      unsigned long long qv[kUpdBatch];
#pragma unroll
      for (int t = 0; t < kUpdBatch; ++t) qv[t] = (unsigned long long)quantize(xv[t], sc);
#pragma unroll
      for (int t = 0; t < kUpdBatch; ++t) {
        if (t0 + t >= nb) break;
        const uint32_t e = __builtin_amdgcn_readlane(mine, t0 + t);
        const int c = (int)(e >> 13);
        if (c != cl) {
          if (cl >= 0 && a != 0ull) atomicAdd(&accj[(int64_t)cl * u.cp], a);
          a = 0ull;
          cl = c;
        }
        a += (e & 1u) ? 0ull - qv[t] : qv[t];
      }
    }
  }
  if (cl >= 0 && a != 0ull) atomicAdd(&accj[(int64_t)cl * u.cp], a);
}

// Lloyd finalize for wide points: one workgroup per job.  Same decisions and
// arithmetic as the narrow finalize (means fp32(sum * 2^-shift / count),
// norms as the FP64 sum of c_d^2 in dimension order), with the norms read
// back from memory instead of LDS.
constexpr int kFinThreads = 512;

__global__ __launch_bounds__(kFinThreads) void k_finalize_wide(FinalizeArgs a) {
  const int job = blockIdx.x;
  JobState st = a.st[job];
  if (!st.active) return;
  const int k = a.k, cp = a.cp;
  __shared__ double sh_f;
  __shared__ int sh_upd, sh_acc, sh_empty;
  if (threadIdx.x < 64) {
    const double f = wave_chunked_sum(a.tf + (int64_t)job * a.max_chunks, st.nchunks);
    const bool stop = (st.iter > 0 && st.f_prev - f <= a.tol * f) || !isfinite(f) ||
                      st.iter >= a.max_iter;
    if (threadIdx.x == 0) {
      sh_f = f;
      sh_upd = stop ? 0 : 1;
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
    // eight means per thread at a time, their loads issued together
    const int kcp = k * cp;
    for (int e0 = threadIdx.x; e0 < kcp; e0 += kFinThreads * 8) {
      long long av[8];
      int cv[8];
      double sv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kFinThreads;
        const int j = e / cp, d = e - j * cp;
        av[u] = e < kcp ? (long long)acc[e] : 0;
        cv[u] = e < kcp ? cnt[j] : 0;
        sv[u] = e < kcp ? a.inv_scale[d] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kFinThreads;
        if (e < kcp && cv[u] > 0) C[e] = (float)(((double)av[u] * sv[u]) / (double)cv[u]);
      }
    }
    __syncthreads();
    // the row's squares added in dimension order; its values are read 64 at
    // a time (the additions form one dependent chain, so the loads must not)
    for (int j = threadIdx.x; j < k; j += kFinThreads) {
      const float4* c4 = reinterpret_cast<const float4*>(C + (int64_t)j * cp);
      const int n4 = cp / 4;
      double q = 0.0;
      for (int b = 0; b < n4; b += 16) {
        float4 v[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) v[t] = b + t < n4 ? c4[b + t] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          q += (double)v[t].x * (double)v[t].x;
          q += (double)v[t].y * (double)v[t].y;
          q += (double)v[t].z * (double)v[t].z;
          q += (double)v[t].w * (double)v[t].w;
        }
      }
      a.cn[(int64_t)job * k + j] = (float)q;
    }
  } else {
    int empty = 0;
    for (int j = threadIdx.x; j < k; j += kFinThreads) {
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
    for (int e = threadIdx.x; e < k * n; e += kFinThreads) {
      const int j = e / n, d = e - j * n;
      a.Cinc[(int64_t)job * k * n + e] = C[(int64_t)j * cp + d];
    }
    for (int j = threadIdx.x; j < k; j += kFinThreads) a.deg_inc[(int64_t)job * k + j] = a.deg[(int64_t)job * k + j];
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
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_assign_wide(hipStream_t st, const AssignArgs& a, int32_t ntiles, bool sums) {
  if (a.tile_pts % kChunk != 0) return hipErrorInvalidValue;
  const KppInitOut none{};
  const bool g2 = a.k > kCG && a.k <= 2 * kCG;
  if (sums && g2)
    hipLaunchKernelGGL((k_assign_wide<true, false, false, true>), dim3(ntiles), dim3(256), 0, st, a, none);
  else if (sums)
    hipLaunchKernelGGL((k_assign_wide<true, false, false, false>), dim3(ntiles), dim3(256), 0, st, a, none);
  else if (g2)
    hipLaunchKernelGGL((k_assign_wide<false, false, false, true>), dim3(ntiles), dim3(256), 0, st, a, none);
  else
    hipLaunchKernelGGL((k_assign_wide<false, false, false, false>), dim3(ntiles), dim3(256), 0, st, a, none);
  return hipGetLastError();
}

// (one BF16 build serves every k: its register allocation with the two-group
// masks was measured no slower at k <= 128)
hipError_t launch_assign_wide_bf16(hipStream_t st, const AssignArgs& a, int32_t ntiles, bool sums) {
  if (a.tile_pts % kChunk != 0) return hipErrorInvalidValue;
  const KppInitOut none{};
  if (sums)
    hipLaunchKernelGGL((k_assign_wide<true, true, false, true>), dim3(ntiles), dim3(256), 0, st, a, none);
  else
    hipLaunchKernelGGL((k_assign_wide<false, true, false, true>), dim3(ntiles), dim3(256), 0, st, a, none);
  return hipGetLastError();
}

hipError_t launch_kpp_init_wide(hipStream_t st, const AssignArgs& a, int32_t ntiles,
                                const KppInitOut& kp) {
  if (a.tile_pts % kChunk != 0 || a.labels || a.st || a.tnear) return hipErrorInvalidValue;
  if (a.k > kCG && a.k <= 2 * kCG)
    hipLaunchKernelGGL((k_assign_wide<false, false, true, true>), dim3(ntiles), dim3(256), 0, st, a, kp);
  else
    hipLaunchKernelGGL((k_assign_wide<false, false, true, false>), dim3(ntiles), dim3(256), 0, st, a, kp);
  return hipGetLastError();
}

hipError_t launch_kpp_pot_staged(hipStream_t st, const KppArgs& a, int32_t njobs, int64_t max_s) {
  const dim3 grid((unsigned)((max_s + kChunk - 1) / kChunk), (unsigned)njobs);
  const size_t lds = ((size_t)3 * a.cp + (size_t)kChunk * (kPotDK + 1)) * sizeof(float);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_kpp_pot_staged,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_kpp_pot_staged, grid, dim3(256), lds, st, a);
  return hipGetLastError();
}

hipError_t update_wide_static_lds(size_t* out) {
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, (const void*)k_update_wide);
  if (e == hipSuccess) *out = fa.sharedSizeBytes;
  return e;
}

size_t update_wide_lds(int32_t k) {
  return (size_t)2 * kUpdPts * sizeof(uint32_t) + ((size_t)3 * k + 1) * sizeof(int);
}

hipError_t launch_update_wide(hipStream_t st, const float* S, int64_t S_stride, int32_t ld,
                              int32_t n, int32_t cp, int32_t k, const int64_t* s,
                              const JobState* js, int32_t njobs, int64_t max_s,
                              const int32_t* lab0, const int32_t* lab1, int64_t lab_stride,
                              unsigned long long* acc, int32_t* cnt, const double* scale) {
  UpdateArgs u;
  u.S = S;
  u.S_stride = S_stride;
  u.ld = ld;
  u.n = n;
  u.cp = cp;
  u.k = k;
  u.s = s;
  u.st = js;
  u.lab0 = lab0;
  u.lab1 = lab1;
  u.lab_stride = lab_stride;
  u.acc = acc;
  u.cnt = cnt;
  u.scale = scale;
  const size_t lds = update_wide_lds(k);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_update_wide,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const dim3 grid((unsigned)((n + kUpdDims - 1) / kUpdDims),
                  (unsigned)((max_s + kUpdPts - 1) / kUpdPts), (unsigned)njobs);
  hipLaunchKernelGGL(k_update_wide, grid, dim3(kUpdThreads), lds, st, u);
  return hipGetLastError();
}

hipError_t launch_finalize_wide(hipStream_t st, const FinalizeArgs& a, int32_t njobs) {
  hipLaunchKernelGGL(k_finalize_wide, dim3(njobs), dim3(kFinThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace bm
