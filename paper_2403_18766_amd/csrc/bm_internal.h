// Shared declarations of the kernels (bm_kernels.hip) and the host library
// (bm_host.cpp).  Everything here is internal; the public interface is
// include/bigmeans.h.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace bm {

constexpr int kWG = 256;         // threads per workgroup (4 wave64s)
constexpr int kMaxRegDim = 64;   // largest padded dimension kept in registers
constexpr int kDTile = 256;      // points per K-means++ tile

// Lloyd state of one job (one sample with its centroids).
struct JobState {
  double f;        // objective of the latest assignment
  double f_prev;   // objective before the latest centroid update
  int32_t iter;    // centroid updates made so far
  int32_t active;  // 1 while the job still iterates
  int32_t ndeg;    // empty clusters under the final assignment
  int32_t accepted;// the run replaced the incumbent (Algorithm 1 acceptance)
  int32_t nchunks; // 256-point chunks of this job (objective partials)
  int32_t pad_;
};

// K-means++ state of one job.
struct KppState {
  double T;          // total of D (scan of the current slot's tile sums)
  double pot[3];     // potentials of the candidates of the pending step
  int32_t cand[3];   // candidates of the pending step
  int32_t ncand;     // 0: nothing pending; 1: uniform pick; else D^2 candidates
  int32_t dcur;      // slot of the D buffers that holds D
  int32_t ntodo;     // degenerate centroids to fill
  int32_t has_d;     // D is defined (at least one centroid exists)
  int32_t step;      // next step number
  int32_t uniform;   // the pending pick is a uniform draw (no D^2 candidates)
};

// Arguments of the assignment kernels.  Job j reads its sample rows at
// S + j*S_stride (row i at + i*ld) and its padded centroids at
// Cp + j*C_stride (row r at + r*cp), norms at cn + j*cn_stride.
struct AssignArgs {
  const float* S;
  int64_t S_stride;
  int32_t ld;
  int32_t n;
  int32_t cp;
  int32_t k;
  int32_t tile_pts;
  int32_t max_chunks;
  int32_t vec;               // 1: rows are 16-byte aligned with ld == cp (vector loads)
  const int64_t* s;          // [job] sample sizes
  const int32_t* tile_job;   // [tile] job of each workgroup
  const int32_t* tile_idx;   // [tile] tile index inside its job
  const float* Cp;
  int64_t C_stride;
  const float* cn;
  int64_t cn_stride;
  int32_t* labels;           // nullable; job j at labels + j*lab_stride
  int64_t lab_stride;
  double* tf;                // [job][max_chunks] objective partial of each 256-point chunk
  int32_t* tnear;            // [job][max_chunks] near-tie count of each chunk (nullable)
  unsigned long long* acc;   // [job][k][cp] fixed-point cluster sums (Lloyd only)
  int32_t* cnt;              // [job][k] cluster counts (Lloyd only)
  const double* scale;       // [cp] fixed-point scales 2^shift_d
  const JobState* st;        // nullable: jobs with active == 0 are skipped; iter == 0 marks
                             // the first assignment of a Lloyd run
};

struct FinalizeArgs {
  int32_t n, cp, k, max_chunks, max_iter;
  double tol;
  const unsigned long long* acc;  // [job][k][cp]
  const int32_t* cnt;             // [job][k]
  const double* tf;               // [job][max_chunks]
  const double* inv_scale;        // [cp] 2^-shift_d
  float* Cp;
  float* cn;
  JobState* st;
  uint8_t* deg;                   // [job][k], written when the job stops
  // Acceptance (optional, Cinc == nullptr skips it): when a job stops with
  // f < fhat[job], its centroids, flags and f become the incumbent.
  float* Cinc;                    // [job][k][n]
  uint8_t* deg_inc;               // [job][k]
  double* fhat;                   // [job]
};

// ---- launchers (bm_kernels.hip) ----
hipError_t launch_sample(hipStream_t st, const float* X, int64_t m, int32_t n, int32_t njobs,
                         int64_t max_s, const int64_t* s, const uint64_t* rkeys, int32_t* idx,
                         int64_t idx_stride, float* S, int64_t S_stride, int32_t ld);
hipError_t launch_absmax(hipStream_t st, const float* X, int64_t rows, int32_t n, int32_t ld,
                         unsigned int* absmax_bits);
hipError_t launch_scales(hipStream_t st, const unsigned int* absmax_bits, int32_t n, int32_t cp,
                         int64_t max_s, double* scale, double* inv_scale);
hipError_t launch_pad_centroids(hipStream_t st, const float* C, int64_t C_stride, int32_t n,
                                int32_t cp, int32_t k, int32_t njobs, float* Cp, int64_t Cp_stride,
                                float* cn, int64_t cn_stride);
hipError_t launch_centroid_norms(hipStream_t st, const float* Cp, int32_t cp, int32_t k,
                                 int32_t njobs, float* cn);
hipError_t launch_assign(hipStream_t st, const AssignArgs& a, int32_t ntiles_total, bool sums);
hipError_t launch_finalize(hipStream_t st, const FinalizeArgs& a, int32_t njobs);
hipError_t launch_job_init(hipStream_t st, JobState* js, const int64_t* sizes, int32_t njobs,
                           int32_t k, int32_t cp, unsigned long long* acc, int32_t* cnt,
                           const float* Cp, float* cn);
hipError_t launch_reduce_f(hipStream_t st, const double* tf, const int32_t* tnear,
                           const int64_t* sizes, int32_t max_chunks, int32_t njobs, double* f,
                           long long* near);
hipError_t launch_unpad(hipStream_t st, const float* Cp, int32_t cp, int32_t n, int32_t k,
                        int32_t njobs, float* C, int64_t C_stride);
hipError_t launch_copy_incumbent(hipStream_t st, const float* Cinc, const uint8_t* deg_inc,
                                 int32_t n, int32_t cp, int32_t k, int32_t njobs, float* Cp,
                                 uint8_t* deg_work);

// K-means++ (greedy, batched over jobs)
struct KppArgs {
  const float* S;
  int64_t S_stride;
  int32_t ld, n, cp, k, ndt_max, njobs;
  const int64_t* s;
  float* Cp;
  int64_t C_stride;
  uint8_t* deg;          // [job][k]
  float* D;              // [slot 0..3][job][max_s]
  int64_t D_slot_stride; // floats between slots
  int64_t D_job_stride;  // floats between jobs
  double* Dt;            // [slot][job][ndt_max] tile sums
  KppState* ks;
  int32_t* todo;         // [job][k]
  int32_t* picks;        // [job][k][4] or nullptr
  const uint64_t* seed_worker;  // [job][2]: seed, worker
  uint64_t g;
  int32_t n_cand;
};
hipError_t launch_kpp_setup(hipStream_t st, const KppArgs& a, int32_t njobs);
hipError_t launch_kpp_init(hipStream_t st, const KppArgs& a, int32_t njobs, int64_t max_s);
hipError_t launch_kpp_step(hipStream_t st, const KppArgs& a, int32_t njobs);
hipError_t launch_kpp_pot(hipStream_t st, const KppArgs& a, int32_t njobs, int64_t max_s);

}  // namespace bm
