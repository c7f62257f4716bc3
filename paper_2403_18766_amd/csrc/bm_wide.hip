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
// together), lowest index on ties, and the winner's distance in the direct
// form sum_d (x_d - c_d)^2 (four partial sums by d mod 4).
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
constexpr int kRow = kDK + 1;      // LDS row stride in floats (column reads hit distinct banks)
constexpr int kCG = 128;           // centres per group (four 32-wide MFMA tiles)
constexpr int kChunk = 256;        // points per chunk (one per thread in the per-point phase)
constexpr int kUpdDims = 64;       // dimensions per update workgroup
constexpr int kUpdPts = 8192;      // points per update workgroup

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int kRowB = 2 * kDK + 8;  // BF16 LDS row: 32 high parts, 32 residuals, 8 pad (144 B)
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

struct WideShared {
  float S[kChunk * kRow];
  float C[kCG * kRow];
  double red_f[4];
  int red_i[4];
};

struct __align__(16) WideSharedB {
  __bf16 S[kChunk * kRowB];  // row r: high parts of its 32 dimensions, then their residuals
  __bf16 C[kCG * kRowB];
  double red_f[4];
  int red_i[4];
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

template <bool SUMS, bool BF>
__global__ __launch_bounds__(256, 2) void k_assign_wide(AssignArgs a) {
  const int job = a.tile_job[blockIdx.x];
  int parity = 0;
  if (a.st) {
    const JobState st = a.st[job];
    if (!st.active) return;
    parity = st.iter & 1;
  }
  const int64_t s = a.s[job];
  const int64_t t0 = (int64_t)a.tile_idx[blockIdx.x] * a.tile_pts;
  const int64_t t1 = min(s, t0 + (int64_t)a.tile_pts);
  const int k = a.k, n = a.n, cp = a.cp, ld = a.ld;
  const float* __restrict__ S = a.S + job * a.S_stride;
  const float* __restrict__ C = a.Cp + job * a.C_stride;
  const float* __restrict__ cn = a.cn + job * a.cn_stride;
  int32_t* const lbase = (parity && a.labels2) ? a.labels2 : a.labels;
  int32_t* __restrict__ lab = lbase ? lbase + job * a.lab_stride : nullptr;
  double* tfj = a.tf + (int64_t)job * a.max_chunks;
  const bool want_near = a.tnear != nullptr;
  const int vec = a.vec;

  __shared__ typename std::conditional<BF, WideSharedB, WideShared>::type sh;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int half = lane >> 5, col = lane & 31;

  float cmax2 = 0.f;
  for (int j = lane; j < k; j += 64) cmax2 = fmaxf(cmax2, cn[j]);
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
    float e1[2], e2[2];
    int j1[2];
    float xxp[2] = {0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      e1[b] = __builtin_inff();
      e2[b] = __builtin_inff();
      j1[b] = 0;
    }
    for (int g0 = 0; g0 < k; g0 += kCG) {
      const int ng = min(kCG, k - g0);
      f32x16 acc[2][4];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[b][t][v] = 0.f;
      for (int d0 = 0; d0 < cp; d0 += kDK) {
        __syncthreads();  // the previous stage has been consumed
        if constexpr (!BF) {
          // stage the chunk's rows: 256 x 32 floats, 8 consecutive dims per load group
          for (int e = tid; e < kChunk * (kDK / 4); e += 256) {
            const int r = e / (kDK / 4), q = e - r * (kDK / 4);
            const float4 v = stage_point(S, cb + r, ld, d0 + 4 * q, n, cp, vec, r < np);
            float* dst = sh.S + r * kRow + 4 * q;
            dst[0] = v.x;
            dst[1] = v.y;
            dst[2] = v.z;
            dst[3] = v.w;
          }
          // stage the group's centres: 128 x 32 floats (rows past k are zero)
          for (int e = tid; e < kCG * (kDK / 4); e += 256) {
            const int r = e / (kDK / 4), q = e - r * (kDK / 4);
            const int d = d0 + 4 * q;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < ng && d < cp) v = *reinterpret_cast<const float4*>(C + (int64_t)(g0 + r) * cp + d);
            float* dst = sh.C + r * kRow + 4 * q;
            dst[0] = v.x;
            dst[1] = v.y;
            dst[2] = v.z;
            dst[3] = v.w;
          }
          __syncthreads();
          // lane (half, col): A = centre (tile*32 + col) at dim kk + half,
          //                   B = point (wv*64 + b*32 + col) at dim kk + half
          for (int kk = 0; kk < kDK; kk += 2) {
            float bv[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              bv[b] = sh.S[(wv * 64 + b * 32 + col) * kRow + kk + half];
              if (g0 == 0) xxp[b] = fmaf(bv[b], bv[b], xxp[b]);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const float av = sh.C[(t * 32 + col) * kRow + kk + half];
#pragma unroll
              for (int b = 0; b < 2; ++b)
                acc[b][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[b], acc[b][t], 0, 0, 0);
            }
          }
        } else {
          // stage the chunk's rows split into high parts and residuals
          for (int e = tid; e < kChunk * (kDK / 4); e += 256) {
            const int r = e / (kDK / 4), q = e - r * (kDK / 4);
            const float4 v = stage_point(S, cb + r, ld, d0 + 4 * q, n, cp, vec, r < np);
            bf16x4 h, l;
            split_bf16(v, h, l);
            __bf16* dst = sh.S + r * kRowB + 4 * q;
            *reinterpret_cast<bf16x4*>(dst) = h;
            *reinterpret_cast<bf16x4*>(dst + kDK) = l;
          }
          for (int e = tid; e < kCG * (kDK / 4); e += 256) {
            const int r = e / (kDK / 4), q = e - r * (kDK / 4);
            const int d = d0 + 4 * q;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < ng && d < cp) v = *reinterpret_cast<const float4*>(C + (int64_t)(g0 + r) * cp + d);
            bf16x4 h, l;
            split_bf16(v, h, l);
            __bf16* dst = sh.C + r * kRowB + 4 * q;
            *reinterpret_cast<bf16x4*>(dst) = h;
            *reinterpret_cast<bf16x4*>(dst + kDK) = l;
          }
          __syncthreads();
          // lane (half, col): A = centre (tile*32 + col), B = point
          // (wv*64 + b*32 + col), both at dims ks + 8 half .. ks + 8 half + 7
          for (int ks = 0; ks < kDK; ks += 16) {
            bf16x8 xh[2], xl[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              const __bf16* p = sh.S + (wv * 64 + b * 32 + col) * kRowB + ks + 8 * half;
              xh[b] = *reinterpret_cast<const bf16x8*>(p);
              xl[b] = *reinterpret_cast<const bf16x8*>(p + kDK);
              if (g0 == 0) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                  const float v = (float)xh[b][q] + (float)xl[b][q];  // exact
                  xxp[b] = fmaf(v, v, xxp[b]);
                }
              }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const __bf16* p = sh.C + (t * 32 + col) * kRowB + ks + 8 * half;
              const bf16x8 ch = *reinterpret_cast<const bf16x8*>(p);
              const bf16x8 cl = *reinterpret_cast<const bf16x8*>(p + kDK);
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
            if (c < k) {
              const float e = fmaf(-2.f, acc[b][t][v], cn[c]);
              e2[b] = __builtin_amdgcn_fmed3f(e1[b], e, e2[b]);
              j1[b] = e < e1[b] ? c : j1[b];
              e1[b] = fminf(e1[b], e);
            }
          }
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
    const int64_t i = cb + tid;
    const bool valid = tid < np;
    double fpart = 0.0;
    int near = 0;
    const float* x = S + i * (int64_t)ld;
    const float B = kB * (sqrtf(xx) * cmax + cmax2);
    const bool recheck = valid && !((pe2 - pe1) > 2.f * B + 2.5e-5f * fabsf(pe2 + xx));
    int jw = pj1;
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
    if (valid) {
      fpart = (double)dist_wide(x, C + (int64_t)jw * cp, n, vec);
      if (lab) lab[i] = jw;
    }
    fpart = wave_sum_f64(fpart);
    if (lane == 0) sh.red_f[wv] = fpart;
    if (want_near) {
      near = wave_sum_i32(near);
      if (lane == 0) sh.red_i[wv] = near;
    }
    __syncthreads();
    if (tid == 0) {
      tfj[cb / kChunk] = (sh.red_f[0] + sh.red_f[1]) + (sh.red_f[2] + sh.red_f[3]);
      if (want_near)
        a.tnear[(int64_t)job * a.max_chunks + cb / kChunk] =
            (sh.red_i[0] + sh.red_i[1]) + (sh.red_i[2] + sh.red_i[3]);
    }
  }
}

// Fixed-point sums of the label changes: grid (cp / 64 dimension slices,
// point ranges of 8,192, jobs).  A point whose label went from jo to jn adds
// its coordinates to cluster jn and removes them from jo (jo < 0 on the first
// assignment).  The slice's sums gather in LDS, then go to memory with
// integer atomics, so the result does not depend on the order.
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

__global__ __launch_bounds__(256) void k_update_wide(UpdateArgs u) {
  const int job = blockIdx.z;
  const JobState st = u.st[job];
  if (!st.active) return;
  const int q = st.iter;
  const int64_t s = u.s[job];
  const int64_t r0 = (int64_t)blockIdx.y * kUpdPts;
  if (r0 >= s) return;
  const int64_t r1 = min(s, r0 + kUpdPts);
  const int k = u.k, d0 = blockIdx.x * kUpdDims;
  const int nd = min(kUpdDims, u.n - d0);  // real dimensions of this slice
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned long long* lacc = reinterpret_cast<unsigned long long*>(smem);
  int* lcnt = reinterpret_cast<int*>(lacc + (size_t)k * kUpdDims);
  for (int e = threadIdx.x; e < k * kUpdDims; e += 256) lacc[e] = 0ull;
  for (int e = threadIdx.x; e < k; e += 256) lcnt[e] = 0;
  __syncthreads();
  const float* S = u.S + job * u.S_stride;
  const int32_t* ln = ((q & 1) ? u.lab1 : u.lab0) + job * u.lab_stride;
  const int32_t* lo = q == 0 ? nullptr : ((q & 1) ? u.lab0 : u.lab1) + job * u.lab_stride;
  const bool counts = blockIdx.x == 0;
  int changed = 0;
  // one thread per point, the slice's dimensions in order
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) {
    const int jn = ln[i];
    const int jo = lo ? lo[i] : -1;
    if (jn == jo) continue;
    changed = 1;
    const float* x = S + i * (int64_t)u.ld + d0;
    for (int dd = 0; dd < nd; ++dd) {
      const long long q = quantize(x[dd], u.scale[d0 + dd]);
      if (q == 0) continue;
      atomicAdd(&lacc[jn * kUpdDims + dd], (unsigned long long)q);
      if (jo >= 0) atomicAdd(&lacc[jo * kUpdDims + dd], (unsigned long long)(-q));
    }
    if (counts) {
      atomicAdd(&lcnt[jn], 1);
      if (jo >= 0) atomicAdd(&lcnt[jo], -1);
    }
  }
  if (!__syncthreads_or(changed)) return;
  unsigned long long* accj = u.acc + (int64_t)job * k * u.cp;
  for (int e = threadIdx.x; e < k * kUpdDims; e += 256) {
    const int j = e / kUpdDims, dd = e - j * kUpdDims;
    const unsigned long long v = lacc[e];
    if (v && dd < nd) atomicAdd(&accj[(int64_t)j * u.cp + d0 + dd], v);
  }
  if (counts) {
    int32_t* cntj = u.cnt + (int64_t)job * k;
    for (int e = threadIdx.x; e < k; e += 256)
      if (lcnt[e]) atomicAdd(&cntj[e], lcnt[e]);
  }
}

// Lloyd finalize for wide points: one workgroup per job.  Same decisions and
// arithmetic as the narrow finalize (means fp32(sum * 2^-shift / count),
// norms as the FP64 sum of c_d^2 in dimension order), with the norms read
// back from memory instead of LDS.
__global__ __launch_bounds__(256) void k_finalize_wide(FinalizeArgs a) {
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
    for (int e = threadIdx.x; e < k * cp; e += 256) {
      const int j = e / cp, d = e - j * cp;
      const int cj = cnt[j];
      if (cj > 0) C[e] = (float)(((double)(long long)acc[e] * a.inv_scale[d]) / (double)cj);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += 256) {
      const float* c = C + (int64_t)j * cp;
      double q = 0.0;
      for (int d = 0; d < cp; ++d) q += (double)c[d] * (double)c[d];
      a.cn[(int64_t)job * k + j] = (float)q;
    }
  } else {
    int empty = 0;
    for (int j = threadIdx.x; j < k; j += 256) {
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
    for (int e = threadIdx.x; e < k * n; e += 256) {
      const int j = e / n, d = e - j * n;
      a.Cinc[(int64_t)job * k * n + e] = C[(int64_t)j * cp + d];
    }
    for (int j = threadIdx.x; j < k; j += 256) a.deg_inc[(int64_t)job * k + j] = a.deg[(int64_t)job * k + j];
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
  if (sums)
    hipLaunchKernelGGL((k_assign_wide<true, false>), dim3(ntiles), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_assign_wide<false, false>), dim3(ntiles), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_assign_wide_bf16(hipStream_t st, const AssignArgs& a, int32_t ntiles, bool sums) {
  if (a.tile_pts % kChunk != 0) return hipErrorInvalidValue;
  if (sums)
    hipLaunchKernelGGL((k_assign_wide<true, true>), dim3(ntiles), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_assign_wide<false, true>), dim3(ntiles), dim3(256), 0, st, a);
  return hipGetLastError();
}

size_t update_wide_lds(int32_t k) {
  return (size_t)k * kUpdDims * sizeof(unsigned long long) + (size_t)k * sizeof(int);
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
  hipLaunchKernelGGL(k_update_wide, grid, dim3(256), lds, st, u);
  return hipGetLastError();
}

hipError_t launch_finalize_wide(hipStream_t st, const FinalizeArgs& a, int32_t njobs) {
  hipLaunchKernelGGL(k_finalize_wide, dim3(njobs), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace bm
