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
// From this many centres on, the persistent round kernel ranks centres on the
// FP32 matrix cores with one point per lane; below, with FP32 FMAs and two
// points per lane up to 32 dimensions.
constexpr int kMfmaMinK = 16;

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
  int32_t* labels2;          // wide-point Lloyd only (nullable): assignment q of a job writes
                             // labels when q is even, labels2 when q is odd (q = its iter)
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

// ---- static workspace of the no-allocation objective (bm_noalloc.hip) ----
constexpr size_t kNoallocScratchBytes = (size_t)16 << 20;
// Device address of the static workspace on `device`, which must be the
// current device; looked up on the first call per device, then cached.
hipError_t noalloc_scratch(int device, void** out);
// Tile map (tile t -> job 0, tile index t) and size m of a one-job launch.
hipError_t launch_noalloc_tiles(hipStream_t st, int32_t* tile_job, int32_t* tile_idx,
                                int32_t ntiles, int64_t* sizes, int64_t m);

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

// ---- wide points, cp > kMaxRegDim (bm_wide.hip) ----
// tile_pts must be a multiple of 256.
hipError_t launch_assign_wide(hipStream_t st, const AssignArgs& a, int32_t ntiles, bool sums);
// Fixed-point sums of the label changes of every active job: its assignment
// q = iter wrote lab[q % 2]; the previous one (none when q = 0) lab[(q+1) % 2].
hipError_t launch_update_wide(hipStream_t st, const float* S, int64_t S_stride, int32_t ld,
                              int32_t n, int32_t cp, int32_t k, const int64_t* s,
                              const JobState* js, int32_t njobs, int64_t max_s,
                              const int32_t* lab0, const int32_t* lab1, int64_t lab_stride,
                              unsigned long long* acc, int32_t* cnt, const double* scale);
hipError_t launch_finalize_wide(hipStream_t st, const FinalizeArgs& a, int32_t njobs);
// LDS bytes of the wide update kernel for k clusters.
size_t update_wide_lds(int32_t k);
// Static LDS of the Lloyd-step assignment kernel of padded dimension cp and of
// the wide update kernel; the dynamic LDS comes on top.
hipError_t assign_static_lds(int32_t cp, size_t* out);
hipError_t update_wide_static_lds(size_t* out);
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
  uint64_t g;            // global pass index of the draws (when gs is null)
  const uint64_t* gs;    // [job] global pass index per job (persistent rounds), or null
  int32_t n_cand;
  const int32_t* job_slot;  // nullable: launch job j works on job index job_slot[j]
};
// Persistent round kernel: every worker runs its (optional) re-evaluation
// and passes_p passes of Algorithm 1 on its own group of workgroups.
struct PassOut {
  int32_t accepted;  // the pass replaced the incumbent
  int32_t iters;     // centroid updates of its Lloyd run
  int32_t ndeg;      // empty clusters of the Lloyd result
  int32_t pad_;
  double f;          // objective of the Lloyd result on the pass's sample
};

struct GroupBar {
  unsigned int count;
  unsigned int gen;
  unsigned int pad_[14];  // one 64-byte line per worker
};

constexpr int kMaxXcd = 16;  // XCD ids are taken modulo this

struct RoundArgs {
  const float* X;
  int64_t m;
  int32_t n, cp, k, W, passes_p, max_iter, n_cand, t;
  uint64_t seed;
  double tol;
  const int64_t* s;            // [W] sample size of each worker this round
  const int32_t* recalc;       // [W] re-evaluate the incumbent on a fresh sample first
  const int32_t* xcd_nw;       // [kMaxXcd] number of workers placed on each XCD
  const int32_t* xcd_workers;  // [kMaxXcd][W] the workers placed on each XCD
  const int32_t* xcd_g;        // [kMaxXcd][W] workgroups of each of those workers
  unsigned int* reg;           // [kMaxXcd] registration counters (zero at launch)
  GroupBar* gbar;              // device-wide barrier (zero at launch)
  GroupBar* bar;               // [W] worker barriers (zero at launch)
  AssignArgs as;               // job = worker (S, labels, scale, layout)
  KppArgs ka;                  // job = worker
  unsigned long long* delta;   // [W][3][k*cp] fixed-point sum deltas (zero at launch)
  int32_t* dcnt;               // [W][3][k] count deltas (zero at launch)
  unsigned int* claim;         // [W][3] Lloyd assignment units claimed (zero at launch)
  double* tf3;                 // [W][3][max_chunks] chunk objective partials
  const double* inv_scale;     // [cp]
  float* Cinc;                 // [W][k][n] incumbents
  uint8_t* deg_inc;            // [W][k]
  double* fhat;                // [W]
  float* Cp;                   // [W][k][cp] working copy for K-means++
  uint8_t* deg_work;           // [W][k]
  PassOut* out;                // [W][passes_p]
  double* recalc_f;            // [W]
  int32_t* err;                // 1: a barrier timed out; 2: an XCD holds fewer workgroups than workers
};

// XCD id of every workgroup of a grid-sized launch: out[grid].
hipError_t launch_xcd_probe(hipStream_t st, uint32_t* out, int32_t grid);
// Largest grid of k_round<cp> that is co-resident on the device.
hipError_t round_capacity(int32_t cp, int32_t k, size_t lds, int* blocks);
size_t round_lds_bytes(int32_t cp, int32_t k);
// r_dev: the RoundArgs in device memory (read by every workgroup).
hipError_t launch_round(hipStream_t st, const RoundArgs* r_dev, int32_t cp, int32_t k,
                        int32_t grid, size_t lds);

hipError_t launch_kpp_setup(hipStream_t st, const KppArgs& a, int32_t njobs);
hipError_t launch_kpp_init(hipStream_t st, const KppArgs& a, int32_t njobs, int64_t max_s);
hipError_t launch_kpp_step(hipStream_t st, const KppArgs& a, int32_t njobs);
hipError_t launch_kpp_pot(hipStream_t st, const KppArgs& a, int32_t njobs, int64_t max_s);

}  // namespace bm
