/*
 * bigmeans.h - C ABI of the MI355X (gfx950) implementation of the hot path of
 * competitive stochastic-sample-size Big-means (Mussabayev & Mussabayev,
 * arXiv 2403.18766).
 *
 * The library computes, on one GPU:
 *   - uniform random samples of the data without replacement (Section 4.1,
 *     "shaking"; Algorithm 1, the sample S_w of each pass);
 *   - greedy K-means++ seeding of degenerate centroids on a sample
 *     (Section 3; Section 4.1; Section 5: three candidate points);
 *   - Lloyd K-means iterations on a sample (Algorithm 1; Section 5: at most
 *     300 iterations, relative tolerance 1e-4);
 *   - the MSSC objective f(C, X) of Eq. (1) with nearest-centre labels;
 *   - Algorithm 1 end to end (bm_bigmeans_run);
 *   - a serving loop of single-pass jobs of competing workers (bm_serve).
 *
 * Conventions for every call
 *   - Point, sample, centroid, label, index and flag arrays are DEVICE
 *     pointers on the context's device, row-major and densely packed
 *     (row stride = n floats), owned by the caller; the library never frees
 *     them.  Float arrays must be 4-byte aligned (16-byte alignment enables
 *     vector loads).
 *   - Scalar outputs (double f, iteration counts, result structs) are HOST
 *     pointers.  Calls with a host scalar output synchronise the context's
 *     stream before returning; calls without one only enqueue work.
 *   - All work is enqueued on the stream given to bm_create (0 = the legacy
 *     default stream).  The library owns only the workspace it allocates.
 *     Device memory is allocated in bm_create/bm_reserve; a call whose sizes
 *     exceed the reservation first grows it (bm_reserve's rule, before it
 *     enqueues work); bm_serve allocates its serving state at its start and
 *     frees it before returning (see there).  Nothing is allocated inside a
 *     Lloyd iteration or a serving loop.
 *   - Return value: BM_OK (0) or a negative bm_status.  bm_strerror(ctx)
 *     describes the last error of that context.  No call aborts and no C++
 *     exception crosses this interface.
 *   - A context is used by one host thread at a time.
 *   - Sizes: 1 <= n <= 4096.  Points whose dimension rounded up to 4 is at
 *     most 64 are assigned with the point in registers and the centroids in
 *     LDS; wider points with FP32 matrix-core dot products.  k is limited by
 *     the LDS of one compute unit: for narrow points the centroids and
 *     fixed-point cluster sums, 12 k cp + 8 k bytes (cp = n rounded up to 4)
 *     plus the assignment kernel's own LDS (at most about 1.4 KB) within
 *     160 KiB; for wide ones the centroid update's label changes sorted by
 *     cluster, 32,772 + 12 k bytes within 160 KiB (k <= 10,922); larger k
 *     returns BM_E_ARG.
 *
 * Randomness (the paper fixes none).  Every random draw comes from the
 * Philox4x64-10 block function B(ctr, key) of Salmon et al. (SC'11) with
 * key = (seed, (worker << 8) | purpose).  Sample element i is the i-th output
 * of a 4-round Feistel permutation of [0, 4^h) (h = max(1, ceil(ceil(log2 m)/2)))
 * walked into [0, m), with round keys B((g,0,0,0), key) and round function
 * SplitMix64-finaliser(R xor K_r).  K-means++ step t of global pass g uses
 * B((t, g, 0, 0), key); the size draw of round t uses B((t, 0, 0, 0), key).
 */
#ifndef BIGMEANS_H
#define BIGMEANS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define BM_API __attribute__((visibility("default")))
#else
#define BM_API
#endif

#define BM_VERSION 2

typedef struct bm_ctx bm_ctx;

typedef enum bm_status {
  BM_OK = 0,
  BM_E_ARG = -1,       /* invalid argument (sizes, null pointer, alignment) */
  BM_E_NOMEM = -2,     /* workspace allocation failed, or call exceeds reserved sizes */
  BM_E_HIP = -3,       /* a HIP runtime call failed */
  BM_E_NONFINITE = -4, /* the objective is NaN or infinite; outputs are still written */
  BM_E_STATE = -5      /* context not usable (no device, destroyed workspace) */
} bm_status;

/* Arithmetic of the distance products on the matrix-core path (padded
 * dimension above 64; narrower points use FP32 vector arithmetic whatever the
 * precision).  BM_FP32: FP32 matrix cores.  BM_BF16: BF16 matrix cores with
 * FP32 accumulation; every FP32 coordinate is split into a BF16 high part
 * and a BF16 residual, and x.c is taken as xh.ch + xh.cl + xl.ch.  In both,
 * a point whose two best centres are closer than the rigorous error bound of
 * that arithmetic is re-decided with FP32 direct-form distances of the FP32
 * rows, and every winner's distance (hence f) is the FP32 direct form, so
 * labels and f agree with the FP32 path except at such near ties. */
typedef enum bm_precision { BM_FP32 = 0, BM_BF16 = 1 } bm_precision;

typedef enum bm_size_policy {
  BM_SIZE_UNIFORM = 0,    /* s uniform integer in [s_min, s_max] (Algorithm 1) */
  BM_SIZE_FIXED = 1,      /* s = s_min (s_min == s_max) */
  BM_SIZE_LOGUNIFORM = 2, /* floor(exp(ln a + u (ln(b+1) - ln a))), clamped to [a, b] */
  BM_SIZE_BINS = 3,       /* round 0 log-uniform; later rounds pick one of 5 log-width bins
                             with weight (acc_i + 1)/(passes_i + 2), then log-uniform inside */
  BM_SIZE_SHRINK = 4      /* exploration narrowing to exploitation (Section 7, future work):
                             round 0, or while L is empty, log-uniform; round t log-uniform in
                             [mu / r_t, mu r_t] clamped to [a, b + 1), mu = round-half-up mean
                             of L over earlier rounds, ln r_t = (ln(b+1) - ln a) / 2 * 2^-t */
} bm_size_policy;

typedef enum bm_purpose {
  BM_PURPOSE_SIZE = 1,
  BM_PURPOSE_SAMPLE = 2,
  BM_PURPOSE_KMPP = 3,
  BM_PURPOSE_RECALC = 4,
  BM_PURPOSE_FINAL = 5
} bm_purpose;

#define BM_FINAL_WORKER 0xFFFFFFu

/* Library version (BM_VERSION).  Needs no device. */
BM_API int bm_version(void);

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t, or NULL for the default stream).  *out receives the
 * context.  Returns BM_E_STATE if the device cannot be used. */
BM_API int bm_create(int device, void* hip_stream, bm_ctx** out);

/* Release the context and its workspace.  NULL is ignored. */
BM_API void bm_destroy(bm_ctx* ctx);

/* Message of the last error of ctx (never NULL; "" if none). */
BM_API const char* bm_strerror(const bm_ctx* ctx);

/* Allocate workspace for up to max_jobs concurrent samples of at most max_s
 * points in max_n dimensions with max_k centroids.  Later calls with larger
 * sizes grow it; calls with sizes within the reservation never allocate.
 * Calls that need more than the reservation reserve it themselves first
 * (allocation happens there, not in the kernels' hot loop). */
BM_API int bm_reserve(bm_ctx* ctx, int64_t max_s, int32_t max_n, int32_t max_k,
                      int32_t max_jobs);

/* Random sample without replacement (Section 4.1; Algorithm 1, "random
 * sample of size s_w from X").
 *   X       device, m x n FP32 rows.
 *   idx_out device, s int32: idx_out[i] = row of X taken as sample element i.
 *   S_out   device, s x n FP32 (may be NULL): S_out[i] = X[idx_out[i]].
 * Requires 1 <= s <= m < 2^31, n >= 1.  Enqueue only. */
BM_API int bm_sample(bm_ctx* ctx, const float* X, int64_t m, int32_t n, int64_t s,
                     uint64_t seed, uint32_t worker, uint32_t purpose, uint64_t g,
                     int32_t* idx_out, float* S_out);

/* Greedy K-means++ (Section 3; Section 4.1: only centroids of degenerate
 * clusters are re-initialised; Section 5: three candidates).  Every centroid
 * j with degenerate[j] != 0 is replaced, in ascending j, by a point of S; the
 * others are kept and define the initial D^2 weights.  With no kept centroid
 * the first pick is uniform.  Each later pick draws n_candidates points with
 * probability proportional to D^2 and keeps the one with the smallest
 * potential sum_i min(D_i, ||S_i - cand||^2).
 *   S          device, s x n FP32.
 *   C          device, k x n FP32, in/out.
 *   degenerate device, k uint8, in/out (all cleared on return).
 *   picks_out  device, k x 4 int32 or NULL: for re-seeded centroid j,
 *              {chosen sample index, candidate 0, 1, 2} (-1 where unused);
 *              rows of kept centroids are -1.
 * Requires 1 <= k <= s, 1 <= n_candidates <= 3.  Enqueue only. */
BM_API int bm_seed(bm_ctx* ctx, const float* S, int64_t s, int32_t n, int32_t k,
                   float* C, uint8_t* degenerate, int32_t n_candidates,
                   uint64_t seed, uint32_t worker, uint64_t g, int32_t* picks_out);

/* Lloyd K-means on sample S from the centroids in C (Algorithm 1, "K-means
 * clustering on S_w with initial centroids C_w").  Each iteration labels
 * every point with its nearest centre (lowest index on ties) and evaluates
 * f = f(C, S) in FP64 accumulation; it stops when f_prev - f <= tol * f,
 * when f is not finite, or after max_iter centroid updates; otherwise each
 * centroid moves to the mean of its cluster (an empty cluster keeps its
 * centre).
 *   S              device, s x n FP32.
 *   C              device, k x n FP32, in: initial, out: final centroids.
 *   f_out          host: f(C_out, S).
 *   iters_out      host (or NULL): number of centroid updates made.
 *   degenerate_out device, k uint8 (or NULL): 1 if cluster j is empty under
 *                  the final assignment.
 *   labels_out     device, s int32 (or NULL): final labels.
 * prec: bm_precision.  Returns BM_E_NONFINITE if f is not finite.
 * Synchronises the stream. */
BM_API int bm_lloyd(bm_ctx* ctx, const float* S, int64_t s, int32_t n, int32_t k, float* C,
                    int32_t max_iter, double tol, int32_t prec, double* f_out,
                    int32_t* iters_out, uint8_t* degenerate_out, int32_t* labels_out);

/* MSSC objective, Eq. (1): f(C, X) = sum_i min_j ||x_i - c_j||^2 with FP32
 * distances and FP64 accumulation; labels_out[i] = argmin_j (lowest j on ties).
 *   X             device, m x n FP32.     C device, k x n FP32.
 *   f_out         host.
 *   labels_out    device, m int32, or NULL.
 *   near_ties_out host, or NULL: number of points whose two smallest squared
 *                 distances d1 <= d2 satisfy d2 - d1 < 1e-5 d2.
 * prec: bm_precision.  Returns BM_E_NONFINITE if f is not finite.
 * Synchronises the stream. */
BM_API int bm_objective(bm_ctx* ctx, const float* X, int64_t m, int32_t n, const float* C,
                        int32_t k, int32_t prec, double* f_out, int32_t* labels_out,
                        int64_t* near_ties_out);

/* bm_objective for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same
 * arguments, results and errors as bm_objective (same kernels, same bits),
 * but the call allocates nothing: its workspace (tile map, padded centroids
 * and norms, one FP64 partial and near-tie count per 256 points, the results)
 * is a static device array of 16 MiB per GPU that the library holds until
 * the process ends, and its scalar results are copied straight into f_out
 * and near_ties_out.  Sizes whose workspace exceeds the array (about
 * 12 bytes per 256 points + 4 k (cp + 1) bytes, cp = n rounded up to 4, e.g.
 * m up to about 300 million points at small k) return BM_E_ARG.  Every call
 * on one GPU shares that array, which keeps the last call's contents: calls
 * that overlap on one GPU (other streams or host threads) race and must be
 * serialised by the caller.  Synchronises the stream. */
BM_API int bm_objective_noalloc(bm_ctx* ctx, const float* X, int64_t m, int32_t n,
                                const float* C, int32_t k, int32_t prec, double* f_out,
                                int32_t* labels_out, int64_t* near_ties_out);

/* Parameters of Algorithm 1. */
typedef struct bm_params {
  int64_t m;           /* rows of X */
  int64_t s_min;       /* sample-size range; Section 5 uses 0.5 s and min(2 s, m) */
  int64_t s_max;
  int32_t n;           /* dimension */
  int32_t k;           /* clusters, 1 <= k <= s_min */
  int32_t workers;     /* competing workers W */
  int32_t rounds_T;    /* rounds (size draws) per worker */
  int32_t passes_p;    /* passes per size draw (Section 5: 10) */
  int32_t max_iter;    /* Lloyd update cap (Section 5: 300) */
  int32_t n_candidates;/* K-means++ candidates (Section 5: 3) */
  int32_t size_policy; /* bm_size_policy */
  int32_t prec;        /* bm_precision of the Lloyd and objective distances */
  int32_t batched;     /* 1: one persistent cooperative launch per round, each worker on
                             its own group of workgroups inside one XCD (default; wide
                             points, or a device placement that cannot hold every
                             worker, run as 2);
                          2: all workers' passes together, one launch per Lloyd step;
                          0: one worker's sample per launch (reference plain path).
                          All three give bitwise identical results. */
  double tol;          /* Lloyd relative tolerance (Section 5: 1e-4) */
  uint64_t seed;
} bm_params;

typedef struct bm_result {
  double f_full;        /* f(C_best, X) */
  double f_best_sample; /* winner's objective on the shared final sample */
  int64_t s_opt;        /* round-half-up mean of the list L of improving sizes */
  int64_t improvements; /* |L| */
  int64_t lloyd_dists;  /* sum over Lloyd runs of s * k * (assignment steps) */
  int64_t lloyd_iters;  /* total assignment steps */
  int32_t best_worker;
  int32_t pad_;
  double gpu_seconds;   /* device time of the whole run */
  double lloyd_seconds; /* device time of the Lloyd phases */
} bm_result;

/* Per-round snapshot callback: after round `round` (0-based), C_all_dev holds
 * the W incumbents (W x k x n FP32, device, valid during the call),
 * fhat_host the W incumbent objectives, s_host the W sample sizes, l_sum and
 * l_count the sum and number of the sizes in the list L so far (so the final
 * stage of Algorithm 1 after this round would draw its shared sample of size
 * s_opt = (l_sum + l_count / 2) / l_count, or s_max if L is empty), and
 * t_seconds the device time elapsed since the start of the run. */
typedef void (*bm_trace_cb)(void* user, int32_t round, const float* C_all_dev,
                            const double* fhat_host, const int64_t* s_host, int64_t l_sum,
                            int64_t l_count, double t_seconds);

/* Algorithm 1 end to end on X (device, m x n FP32): per round and worker a
 * size draw and, on a size change, re-evaluation of the incumbent on a fresh
 * sample; p passes of sample -> K-means++ for degenerate centroids -> Lloyd
 * -> strict-improvement acceptance (appending s_w to L); then
 * s_opt = mean of L, a shared sample of size s_opt, the worker with the
 * smallest objective on it, and the full assignment of X.
 *   C_best_out device, k x n FP32.   Y_out device, m int32 (or NULL).
 *   out        host.   cb/user optional.
 * Synchronises the stream. */
BM_API int bm_bigmeans_run(bm_ctx* ctx, const float* X, const bm_params* params,
                           float* C_best_out, int32_t* Y_out, bm_result* out,
                           bm_trace_cb cb, void* user);

/* ---- Serving: sample-solve jobs of competing workers, continuously batched ----
 *
 * One job is one pass of Algorithm 1 for one competing worker: a fresh sample
 * of size s (re-evaluating the worker's incumbent first when s differs from
 * its previous job's size), K-means++ for the incumbent's degenerate
 * centroids, Lloyd, and strict-improvement acceptance.  Jobs of one
 * (dataset, k, worker) share that worker's incumbent, which stays on the
 * device for the whole call, and run one after another in arrival order;
 * all other jobs are independent.  Jobs join the running set as soon as they
 * have arrived, their worker is idle, a workspace slot of their (dataset, k)
 * is free and the in-flight bytes stay within the budget; every Lloyd
 * iteration advances all running jobs together, and a finished job leaves
 * at once.  Each job's result is bitwise the same alone and in any mix.
 *
 * Randomness: the job's worker key is w' = (dataset << 20) | (k << 10) | worker
 * (dataset < 16, k < 1024, worker < 1024) in the key convention above; the
 * g-th job of a worker (g = 0, 1, ...) samples with purpose SAMPLE and
 * counter g, seeds with K-means++ counter g, and re-evaluates with purpose
 * RECALC and counter g. */
typedef struct bm_dataset {
  const float* X;  /* device, m x n FP32 rows, resident for the call */
  int64_t m;
  int32_t n;
  int32_t pad_;
} bm_dataset;

typedef struct bm_job {
  double arrival;  /* seconds after the start of bm_serve (0 for all: no pacing) */
  int64_t s;       /* sample size, 1 <= k <= s <= m */
  int32_t dataset; /* index into the dataset array */
  int32_t k;
  int32_t worker;
  int32_t prec;    /* bm_precision (jobs of one data set and k run in one launch per
                      precision) */
} bm_job;

typedef struct bm_job_result {
  double f;            /* objective of the job's Lloyd result on its sample */
  double f_incumbent;  /* the worker's incumbent objective after the job */
  double admitted;     /* seconds after the start: joined the running set */
  double finished;     /* seconds after the start: result final */
  int32_t iters;       /* Lloyd centroid updates */
  int32_t accepted;    /* the result replaced the incumbent */
  int32_t ndeg;        /* empty clusters of the result */
  int32_t pad_;
} bm_job_result;

typedef struct bm_serve_params {
  uint64_t seed;
  int64_t budget_bytes; /* device memory for job slots (samples, labels, sums): bounds both
                           the reserved slots and the bytes of the jobs running together */
  int32_t max_slots;    /* running jobs per (dataset, k) at most */
  int32_t max_iter;     /* Lloyd update cap (Section 5: 300) */
  int32_t n_candidates; /* K-means++ candidates (Section 5: 3) */
  int32_t paced;        /* 1: a job cannot start before its arrival time (wall clock) */
  double tol;           /* Lloyd relative tolerance (Section 5: 1e-4) */
} bm_serve_params;

typedef struct bm_serve_stats {
  double seconds;        /* wall time of the call */
  int64_t steps;         /* Lloyd iterations of the running set */
  int64_t peak_running;  /* most jobs running together */
  int64_t peak_bytes;    /* most in-flight workspace bytes */
  int64_t slot_bytes;    /* workspace reserved for all slots */
} bm_serve_stats;

/* Run the job list (any order of arrival times) to completion.
 *   datasets  host array of nds datasets (device rows).
 *   jobs      host array of njobs jobs.   results  host, njobs entries.
 *   stats     host (may be NULL).
 * Allocation: at its start, before any job runs, the call allocates the
 * incumbent store (k x n floats and k flags per worker the jobs name) and,
 * per (dataset, k, precision) group, a workspace of job slots, a stream,
 * three events and two pinned copies of the group's job states (read once
 * their copy has completed: the loop never waits for the device while it has
 * other work to issue); all of it is freed before the call returns.  The slots of all groups together hold at most
 * budget_bytes (stats->slot_bytes); every group needs at least one slot.
 * Returns BM_E_ARG for invalid jobs or a budget too small for one slot of
 * every group.  Synchronises the stream. */
BM_API int bm_serve(bm_ctx* ctx, const bm_dataset* datasets, int32_t nds, const bm_job* jobs,
                    int32_t njobs, const bm_serve_params* params, bm_job_result* results,
                    bm_serve_stats* stats);

/* Kernel timing of the Lloyd assignment (the dominant kernel), for
 * measurement.  With profiling on, every assignment launch of a Lloyd
 * iteration is bracketed by HIP events on the context's stream and the
 * device time is accumulated; enabling resets the counters.  Counters:
 *   assign_launches  assignment kernel launches
 *   assign_seconds   their summed device time
 *   assign_dists     point-centre distances those launches computed for
 *                    active jobs (sum over jobs of s * k per assignment)
 *   finalize_seconds summed device time of the update/convergence kernel
 * Profiling adds event records between launches; leave it off otherwise. */
typedef struct bm_stats {
  int64_t assign_launches;
  int64_t assign_dists;
  double assign_seconds;
  double finalize_seconds;
} bm_stats;

BM_API int bm_set_profiling(bm_ctx* ctx, int on);
BM_API int bm_get_stats(bm_ctx* ctx, bm_stats* out);

/* Tile-size tuning of the Lloyd launches that run one assignment step per
 * launch (bm_lloyd, bm_bigmeans_run with batched = 0 or 2 or wide points;
 * bm_serve always takes the heuristic's tile size, since a timing waits for
 * the device and would hold up every other job group).  On (the default),
 * the first batch of each (padded dimension, k, log2 of its points) times an
 * objective-mode assignment per candidate tile size (the heuristic's choice
 * and the sizes a quarter, half, twice and four times it, best of two timed
 * launches after one warm-up) and keeps the fastest for the context; results
 * never depend on the tile size.  Off: the heuristic alone.  Either call
 * clears the kept choices.  Returns BM_E_ARG for a null context. */
BM_API int bm_set_tuning(bm_ctx* ctx, int on);

/* Host-only: the sample size of `worker` in round t under params' policy,
 * given the BINS statistics so far (bin_acc/bin_passes: 5 counts each, may
 * be NULL for other policies) and the list L of earlier rounds (l_sum, l_count:
 * sum and number of its sizes; SHRINK).  Writes the size and its bin (0..4).
 * Needs no device. */
BM_API int bm_draw_size(const bm_params* params, uint32_t worker, int32_t t,
                        const int64_t* bin_acc, const int64_t* bin_passes, int64_t l_sum,
                        int64_t l_count, int64_t* s_out, int32_t* bin_out);

/* Host-only: Philox4x64-10 block B(ctr, key) -> out[4].  Needs no device. */
BM_API void bm_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

#ifdef __cplusplus
}
#endif

#endif /* BIGMEANS_H */
