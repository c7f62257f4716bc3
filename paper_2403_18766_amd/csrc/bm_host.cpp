// Host side of libbigmeans: context, workspace, the C ABI of
// include/bigmeans.h and the driver of Algorithm 1.
//
// Every device buffer is allocated in bm_create / bm_reserve (or by a call
// whose sizes exceed the reservation, before it enqueues any work); the
// per-iteration and per-pass paths only enqueue kernels and small copies.
// Small per-batch tables (sizes, tile maps, Feistel round keys) travel
// host->device through a ring of pinned staging slots guarded by events.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/bigmeans.h"
#include "bm_internal.h"
#include "bm_precision.h"
#include "bm_rng.h"

using bm::JobState;
using bm::KppState;

namespace {

constexpr int kNumStage = 16;
constexpr size_t kStageBytes = 256 * 1024;
constexpr int kNBins = 5;
constexpr int kMaxDim = 4096;            // largest point dimension
constexpr size_t kMaxLds = 160 * 1024;   // LDS of one compute unit
constexpr int kStagedKppDim = 32;        // rows this wide: K-means++ potentials staged through LDS

int round_up4(int n) { return (n + 3) & ~3; }

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct bm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  // reservation
  int64_t max_s = 0;
  int max_n = 0, max_k = 0, max_jobs = 0, cpmax = 0;
  int64_t max_chunks = 0;  // 256-point chunks per job
  int64_t obj_chunks = 0;  // chunks reserved for a full-data objective

  // device workspace
  DevBuf S, idx, labels, Cp, cn, Cinc, deg_work, deg_inc, fhat, acc, cnt, tf, tnear, js, sizes, tile_job, tile_idx, rkeys, seed_worker, absmax, scale, inv_scale,
      fjob, nearjob, D, Dt, ks, todo, picks, gs, rflags, wgmap, rargs, rres, bars, rwork, labels2;
  int xcd_cap = 0;                  // grid size the XCD layout below was measured for
  int xcd_wgs[bm::kMaxXcd] = {0};   // workgroups of that grid on each XCD
  bool round_ok = true;             // the persistent round kernel fits this device
  int64_t tile_cap = 0;  // entries of tile_job / tile_idx

  // pinned staging ring
  void* stage[kNumStage] = {};
  hipEvent_t stage_ev[kNumStage] = {};
  bool stage_used[kNumStage] = {};
  int stage_next = 0;
  // pinned readback area
  void* rb = nullptr;
  size_t rb_bytes = 0;

  void* scratch = nullptr;  // this device's static workspace (bm_objective_noalloc)

  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
  hipEvent_t tev0 = nullptr, tev1 = nullptr;  // tile tuning

  // profiling of the Lloyd kernels (bm_set_profiling)
  bool prof = false;
  std::vector<hipEvent_t> pev;  // 3 events per iteration: before assign, after assign, after finalize
  // tile sizes chosen by timing (key: padded dimension, k, log2 of the
  // batch's points); bm_set_tuning switches the timing off
  bool tune = true;
  std::map<uint64_t, int> tuned_tile;
  bm_stats stats{};

  int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }
  int hip_fail(hipError_t e, const char* what) {
    return fail(BM_E_HIP, "%s: %s", what, hipGetErrorString(e));
  }
};

#define HIP_TRY(ctx, expr)                                      \
  do {                                                          \
    hipError_t e_ = (expr);                                     \
    if (e_ != hipSuccess) return (ctx)->hip_fail(e_, #expr);    \
  } while (0)

#define BM_TRY(expr)              \
  do {                            \
    int r_ = (expr);              \
    if (r_ != BM_OK) return r_;   \
  } while (0)

namespace {

template <typename T>
T* P(const DevBuf& b) {
  return static_cast<T*>(b.p);
}

int dev_alloc(bm_ctx* c, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return BM_OK;
  if (b.p) {
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return c->fail(BM_E_NOMEM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
  }
  b.bytes = bytes;
  return BM_OK;
}

void dev_free(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

// Copy `bytes` from host memory to device memory through a pinned slot.
int upload(bm_ctx* c, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return BM_OK;
  if (bytes > kStageBytes) return c->fail(BM_E_ARG, "upload of %zu bytes exceeds staging", bytes);
  const int i = c->stage_next;
  c->stage_next = (i + 1) % kNumStage;
  if (c->stage_used[i]) HIP_TRY(c, hipEventSynchronize(c->stage_ev[i]));
  std::memcpy(c->stage[i], src, bytes);
  HIP_TRY(c, hipMemcpyAsync(dst, c->stage[i], bytes, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipEventRecord(c->stage_ev[i], c->stream));
  c->stage_used[i] = true;
  return BM_OK;
}

// Copy device memory to the pinned readback area and wait for it.
int readback(bm_ctx* c, const void* src, size_t bytes, void* dst) {
  if (bytes == 0) return BM_OK;
  if (bytes > c->rb_bytes) {
    if (c->rb) (void)hipHostFree(c->rb);
    c->rb = nullptr;
    HIP_TRY(c, hipHostMalloc(&c->rb, bytes, hipHostMallocDefault));
    c->rb_bytes = bytes;
  }
  HIP_TRY(c, hipMemcpyAsync(c->rb, src, bytes, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::memcpy(dst, c->rb, bytes);
  return BM_OK;
}

int reserve_impl(bm_ctx* c, int64_t max_s, int max_n, int max_k, int max_jobs) {
  max_s = std::max<int64_t>(max_s, c->max_s);
  max_n = std::max(max_n, c->max_n);
  max_k = std::max(max_k, c->max_k);
  max_jobs = std::max(max_jobs, c->max_jobs);
  if (max_s == c->max_s && max_n == c->max_n && max_k == c->max_k && max_jobs == c->max_jobs &&
      c->S.p)
    return BM_OK;
  // the stream may still use the old buffers
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int cp = round_up4(max_n);
  const int64_t mc = (max_s + bm::kWG - 1) / bm::kWG;
  const size_t J = (size_t)max_jobs;
  const size_t T = 256;  // initial tile-map capacity per job
  BM_TRY(dev_alloc(c, c->S, J * max_s * cp * sizeof(float)));
  BM_TRY(dev_alloc(c, c->idx, J * max_s * sizeof(int32_t)));
  BM_TRY(dev_alloc(c, c->labels, J * max_s * sizeof(int32_t)));
  BM_TRY(dev_alloc(c, c->Cp, J * max_k * cp * sizeof(float)));
  BM_TRY(dev_alloc(c, c->cn, J * max_k * sizeof(float)));
  BM_TRY(dev_alloc(c, c->Cinc, J * max_k * max_n * sizeof(float)));
  BM_TRY(dev_alloc(c, c->deg_work, J * max_k));
  BM_TRY(dev_alloc(c, c->deg_inc, J * max_k));
  BM_TRY(dev_alloc(c, c->fhat, J * sizeof(double)));
  BM_TRY(dev_alloc(c, c->acc, J * max_k * cp * sizeof(unsigned long long)));
  BM_TRY(dev_alloc(c, c->cnt, J * max_k * sizeof(int32_t)));
  const size_t tfn = std::max<size_t>(J * mc, (size_t)c->obj_chunks);
  BM_TRY(dev_alloc(c, c->tf, tfn * sizeof(double)));
  BM_TRY(dev_alloc(c, c->tnear, tfn * sizeof(int32_t)));
  BM_TRY(dev_alloc(c, c->js, J * sizeof(JobState)));
  BM_TRY(dev_alloc(c, c->sizes, J * sizeof(int64_t)));
  const int64_t tcap = std::max<int64_t>((int64_t)J * T, c->tile_cap);
  BM_TRY(dev_alloc(c, c->tile_job, tcap * sizeof(int32_t)));
  BM_TRY(dev_alloc(c, c->tile_idx, tcap * sizeof(int32_t)));
  c->tile_cap = tcap;
  BM_TRY(dev_alloc(c, c->rkeys, J * 4 * sizeof(uint64_t)));
  BM_TRY(dev_alloc(c, c->seed_worker, J * 2 * sizeof(uint64_t)));
  BM_TRY(dev_alloc(c, c->absmax, (size_t)std::max(max_n, 1) * sizeof(unsigned int)));
  BM_TRY(dev_alloc(c, c->scale, (size_t)cp * sizeof(double)));
  BM_TRY(dev_alloc(c, c->inv_scale, (size_t)cp * sizeof(double)));
  BM_TRY(dev_alloc(c, c->fjob, J * sizeof(double)));
  BM_TRY(dev_alloc(c, c->nearjob, J * sizeof(long long)));
  BM_TRY(dev_alloc(c, c->D, 4 * J * max_s * sizeof(float)));
  BM_TRY(dev_alloc(c, c->Dt, 4 * J * mc * sizeof(double)));
  BM_TRY(dev_alloc(c, c->ks, J * sizeof(KppState)));
  BM_TRY(dev_alloc(c, c->todo, J * max_k * sizeof(int32_t)));
  BM_TRY(dev_alloc(c, c->picks, J * max_k * 4 * sizeof(int32_t)));
  BM_TRY(dev_alloc(c, c->gs, J * sizeof(uint64_t)));
  BM_TRY(dev_alloc(c, c->rflags, J * sizeof(int32_t)));
  BM_TRY(dev_alloc(c, c->bars, J * sizeof(bm::GroupBar)));
  BM_TRY(dev_alloc(c, c->rargs, sizeof(bm::RoundArgs)));
  c->max_s = max_s;
  c->max_n = max_n;
  c->max_k = max_k;
  c->max_jobs = max_jobs;
  c->cpmax = cp;
  c->max_chunks = mc;
  return BM_OK;
}

int ensure(bm_ctx* c, int64_t s, int n, int k, int jobs) {
  if (s <= c->max_s && n <= c->max_n && k <= c->max_k && jobs <= c->max_jobs && c->S.p)
    return BM_OK;
  return reserve_impl(c, s, n, k, jobs);
}

int ensure_objective(bm_ctx* c, int64_t m) {
  const int64_t ch = (m + bm::kWG - 1) / bm::kWG;
  if (ch > (int64_t)(c->tf.bytes / sizeof(double))) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    BM_TRY(dev_alloc(c, c->tf, (size_t)ch * sizeof(double)));
    BM_TRY(dev_alloc(c, c->tnear, (size_t)ch * sizeof(int32_t)));
    c->obj_chunks = ch;
  }
  return BM_OK;
}

// Points per assignment workgroup: a multiple of 512 (two 256-point chunks,
// one per register-blocked point of a lane), large enough that the whole
// batch fits in about 2,048 workgroups, two residency rounds of the chip
// (256 compute units x 4 workgroups at the kernel's register use), so that
// the second round evens out the first one's uneven finishing times (serving
// measured 2 % faster than with one round, and 3 % slower with half a round).
int choose_tile_pts(const std::vector<int64_t>& sizes) {
  int64_t total = 0;
  for (int64_t s : sizes) total += s;
  const int64_t step = 2 * bm::kWG;
  const int64_t target = 2048;
  int64_t steps = (total + step * target - 1) / (step * target);
  steps = std::max<int64_t>(steps, 1);
  return (int)(steps * step);
}

struct TileMap {
  int tile_pts = bm::kWG;
  int total = 0;
  std::vector<int32_t> ntiles, job, idx;
};

TileMap make_tiles(const std::vector<int64_t>& sizes, int tile_pts) {
  TileMap t;
  t.tile_pts = tile_pts;
  for (size_t j = 0; j < sizes.size(); ++j) {
    const int nt = (int)((sizes[j] + tile_pts - 1) / tile_pts);
    t.ntiles.push_back(nt);
    for (int q = 0; q < nt; ++q) {
      t.job.push_back((int32_t)j);
      t.idx.push_back(q);
    }
  }
  t.total = (int)t.job.size();
  return t;
}

int upload_tiles(bm_ctx* c, const TileMap& t) {
  if ((int64_t)t.total > c->tile_cap) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    BM_TRY(dev_alloc(c, c->tile_job, (size_t)t.total * sizeof(int32_t)));
    BM_TRY(dev_alloc(c, c->tile_idx, (size_t)t.total * sizeof(int32_t)));
    c->tile_cap = t.total;
  }
  const size_t chunk = kStageBytes / sizeof(int32_t);
  for (size_t off = 0; off < (size_t)t.total; off += chunk) {
    const size_t cntv = std::min(chunk, (size_t)t.total - off);
    BM_TRY(upload(c, P<int32_t>(c->tile_job) + off, t.job.data() + off, cntv * sizeof(int32_t)));
    BM_TRY(upload(c, P<int32_t>(c->tile_idx) + off, t.idx.data() + off, cntv * sizeof(int32_t)));
  }
  return BM_OK;
}

// Fixed-point scales from the data (max |x_d| over rows x n at stride ld).
int compute_scales(bm_ctx* c, const float* X, int64_t rows, int n, int ld, int cp, int64_t max_s) {
  HIP_TRY(c, hipMemsetAsync(c->absmax.p, 0, (size_t)n * sizeof(unsigned int), c->stream));
  HIP_TRY(c, bm::launch_absmax(c->stream, X, rows, n, ld, P<unsigned int>(c->absmax)));
  HIP_TRY(c, bm::launch_scales(c->stream, P<unsigned int>(c->absmax), n, cp, max_s,
                               P<double>(c->scale), P<double>(c->inv_scale)));
  return BM_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// A batch of jobs with shared n and k.  Job j's sample, centroids and
// per-job state live at the job-j offsets of the workspace arrays, shifted
// by `first` (so one worker can run alone in the plain path).
struct BatchView {
  int first = 0;     // first workspace job slot
  int njobs = 0;
  int n = 0, cp = 0, k = 0;
  const float* S = nullptr;  // sample of slot `first`
  int64_t S_stride = 0;      // floats between jobs (0: shared sample)
  int ld = 0;
  std::vector<int64_t> sizes;
};

// Points per assignment workgroup for a batch: the first batch of each
// (padded dimension, k, log2 points) times one assignment launch per
// candidate — the heuristic's choice, half and twice it — in objective mode
// (no labels, sums or job state touched; only the chunk partials, which the
// next assignment rewrites) and keeps the fastest.  The batch's sizes, centroids
// and norms must be on the device.  Results do not depend on the choice (every
// reduction is per 256-point chunk, in a fixed order).
int tuned_tile_pts(bm_ctx* c, const BatchView& b, const std::vector<int64_t>& sizes, int* out) {
  const int base = choose_tile_pts(sizes);
  *out = base;
  int64_t total = 0;
  for (int64_t v : sizes) total += v;
  if (!c->tune || total < 4 * 1024) return BM_OK;
  int lg = 0;
  while ((int64_t)1 << (lg + 1) <= total) ++lg;
  const uint64_t key = ((uint64_t)b.cp << 40) | ((uint64_t)b.k << 16) | (uint64_t)lg;
  auto it = c->tuned_tile.find(key);
  if (it != c->tuned_tile.end()) {
    *out = it->second;
    return BM_OK;
  }
  // the heuristic size and two sizes either side of it (powers of two apart)
  std::vector<int> cands;
  for (int t : {base / 4, base / 2, base, base * 2, base * 4})
    if (t >= 2 * bm::kWG && t % (2 * bm::kWG) == 0) cands.push_back(t);
  if (!c->tev0) {
    HIP_TRY(c, hipEventCreate(&c->tev0));
    HIP_TRY(c, hipEventCreate(&c->tev1));
  }
  bm::AssignArgs a{};
  a.S = b.S;
  a.S_stride = b.S_stride;
  a.ld = b.ld;
  a.n = b.n;
  a.cp = b.cp;
  a.k = b.k;
  a.max_chunks = (int32_t)c->max_chunks;
  a.vec = (b.ld == b.cp && aligned16(b.S) && (b.S_stride % 4) == 0) ? 1 : 0;
  a.s = P<int64_t>(c->sizes) + b.first;
  a.Cp = P<float>(c->Cp) + (int64_t)b.first * b.k * b.cp;
  a.C_stride = (int64_t)b.k * b.cp;
  a.cn = P<float>(c->cn) + (int64_t)b.first * b.k;
  a.cn_stride = b.k;
  a.tf = P<double>(c->tf) + (int64_t)b.first * c->max_chunks;
  const bool wide = b.cp > bm::kMaxRegDim;
  float best_ms = 0.f;
  for (int t : cands) {
    TileMap tm = make_tiles(sizes, t);
    BM_TRY(upload_tiles(c, tm));
    a.tile_pts = t;
    a.tile_job = P<int32_t>(c->tile_job);
    a.tile_idx = P<int32_t>(c->tile_idx);
    float ms = 0.f;
    for (int rep = 0; rep < 3; ++rep) {  // the first launch warms the caches; best of two
      HIP_TRY(c, hipEventRecord(c->tev0, c->stream));
      if (wide)
        HIP_TRY(c, bm::launch_assign_wide(c->stream, a, tm.total, false));
      else
        HIP_TRY(c, bm::launch_assign(c->stream, a, tm.total, false));
      HIP_TRY(c, hipEventRecord(c->tev1, c->stream));
      HIP_TRY(c, hipEventSynchronize(c->tev1));
      float r = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&r, c->tev0, c->tev1));
      if (rep == 1 || (rep == 2 && r < ms)) ms = r;
    }
    if (t == cands.front() || ms < best_ms) {
      best_ms = ms;
      *out = t;
    }
  }
  c->tuned_tile[key] = *out;
  return BM_OK;
}

// Kernel arguments of Lloyd iterations over the jobs (slots) of a batch.
struct LloydSetup {
  bm::AssignArgs a{};
  bm::FinalizeArgs f{};
  bool wide = false;
  bool bf16 = false;  // wide points: dot products on the BF16 matrix cores (split operands)
  int32_t* lab[2] = {nullptr, nullptr};  // wide points: assignment q writes lab[q % 2]
  int64_t lab_stride = 0;
  JobState* js = nullptr;
  unsigned long long* acc = nullptr;
  int32_t* cnt = nullptr;
};

// Arguments for the slots first..first+J-1 (tile map set separately).  With
// `accept`, a stopping job replaces the slot's incumbent on strict improvement.
int lloyd_setup(bm_ctx* c, const BatchView& b, int max_iter, double tol, int32_t* labels,
                int64_t lab_stride, bool accept, LloydSetup* L, int prec = BM_FP32) {
  const int J = b.njobs, first = b.first, k = b.k, cp = b.cp;
  if (!labels) {
    labels = P<int32_t>(c->labels) + (int64_t)first * c->max_s;
    lab_stride = c->max_s;
  }
  L->js = P<JobState>(c->js) + first;
  L->acc = P<unsigned long long>(c->acc) + (int64_t)first * k * cp;
  L->cnt = P<int32_t>(c->cnt) + (int64_t)first * k;
  bm::AssignArgs& a = L->a;
  a = bm::AssignArgs{};
  a.S = b.S;
  a.S_stride = b.S_stride;
  a.ld = b.ld;
  a.n = b.n;
  a.cp = cp;
  a.k = k;
  a.tile_pts = bm::kWG;
  a.max_chunks = (int32_t)c->max_chunks;
  a.vec = (b.ld == cp && aligned16(b.S) && (b.S_stride % 4) == 0) ? 1 : 0;
  a.s = P<int64_t>(c->sizes) + first;
  a.tile_job = P<int32_t>(c->tile_job);
  a.tile_idx = P<int32_t>(c->tile_idx);
  a.Cp = P<float>(c->Cp) + (int64_t)first * k * cp;
  a.C_stride = (int64_t)k * cp;
  a.cn = P<float>(c->cn) + (int64_t)first * k;
  a.cn_stride = k;
  a.labels = labels;
  a.lab_stride = lab_stride;
  a.tf = P<double>(c->tf) + (int64_t)first * c->max_chunks;
  a.tnear = nullptr;
  a.acc = L->acc;
  a.cnt = L->cnt;
  a.scale = P<double>(c->scale);
  a.st = L->js;

  bm::FinalizeArgs& f = L->f;
  f = bm::FinalizeArgs{};
  f.n = b.n;
  f.cp = cp;
  f.k = k;
  f.max_chunks = (int32_t)c->max_chunks;
  f.max_iter = max_iter;
  f.tol = tol;
  f.acc = L->acc;
  f.cnt = L->cnt;
  f.tf = a.tf;
  f.inv_scale = P<double>(c->inv_scale);
  f.Cp = P<float>(c->Cp) + (int64_t)first * k * cp;
  f.cn = P<float>(c->cn) + (int64_t)first * k;
  f.st = L->js;
  f.deg = P<uint8_t>(c->deg_work) + (int64_t)first * k;
  if (accept) {
    f.Cinc = P<float>(c->Cinc) + (int64_t)first * k * b.n;
    f.deg_inc = P<uint8_t>(c->deg_inc) + (int64_t)first * k;
    f.fhat = P<double>(c->fhat) + first;
  }

  // Wide points: assignment q of a job (q = its iteration count) writes its
  // labels to lab[q % 2] (lab[0] = labels, lab[1] = a second buffer with the
  // same layout); a separate kernel adds the label changes to the sums.
  L->wide = cp > bm::kMaxRegDim;
  L->bf16 = L->wide && prec == BM_BF16;
  L->lab[0] = labels;
  L->lab[1] = nullptr;
  L->lab_stride = lab_stride;
  if (L->wide) {
    if (J > 1 && lab_stride != c->max_s) return c->fail(BM_E_STATE, "label layout");
    const size_t need = (size_t)c->max_jobs * c->max_s;
    if (c->labels2.bytes < need * sizeof(int32_t)) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      BM_TRY(dev_alloc(c, c->labels2, need * sizeof(int32_t)));
    }
    L->lab[1] = J == 1 ? P<int32_t>(c->labels2) : P<int32_t>(c->labels2) + (int64_t)first * c->max_s;
  }
  a.labels2 = L->lab[1];
  return BM_OK;
}

// One Lloyd iteration (assignment, update, finalize) of every active job of
// the batch over the tile map tm.
int lloyd_launch(bm_ctx* c, LloydSetup& L, const BatchView& b, const TileMap& tm, int64_t max_size,
                 int prof_slot) {
  const int J = b.njobs;
  L.a.tile_pts = tm.tile_pts;
  // the tile arrays may have been reallocated by upload_tiles since the setup
  L.a.tile_job = P<int32_t>(c->tile_job);
  L.a.tile_idx = P<int32_t>(c->tile_idx);
  if (tm.total > c->tile_cap) return c->fail(BM_E_STATE, "tile map not uploaded");
  if (prof_slot >= 0) HIP_TRY(c, hipEventRecord(c->pev[2 * prof_slot], c->stream));
  if (L.wide) {
    if (L.bf16)
      HIP_TRY(c, bm::launch_assign_wide_bf16(c->stream, L.a, tm.total, true));
    else
      HIP_TRY(c, bm::launch_assign_wide(c->stream, L.a, tm.total, true));
    HIP_TRY(c, bm::launch_update_wide(c->stream, b.S, b.S_stride, b.ld, b.n, b.cp, b.k, L.a.s, L.js,
                                      J, max_size, L.lab[0], L.lab[1], L.lab_stride, L.acc, L.cnt,
                                      L.a.scale));
  } else {
    HIP_TRY(c, bm::launch_assign(c->stream, L.a, tm.total, true));
  }
  if (prof_slot >= 0) HIP_TRY(c, hipEventRecord(c->pev[2 * prof_slot + 1], c->stream));
  if (L.wide)
    HIP_TRY(c, bm::launch_finalize_wide(c->stream, L.f, J));
  else
    HIP_TRY(c, bm::launch_finalize(c->stream, L.f, J));
  return BM_OK;
}

// Run Lloyd on every job of the batch from the centroids in Cp (slots
// first..first+njobs-1).  Leaves the final centroids in Cp, the job states in
// js, degenerate flags in deg_work and the final labels in `labels` (or in
// the workspace label buffer when labels is null).
int lloyd_batch(bm_ctx* c, const BatchView& b, int max_iter, double tol, int32_t* labels,
                int64_t lab_stride, bool accept = false, std::vector<JobState>* out = nullptr,
                int prec = BM_FP32) {
  const int J = b.njobs, first = b.first, k = b.k, cp = b.cp;
  LloydSetup L;
  BM_TRY(lloyd_setup(c, b, max_iter, tol, labels, lab_stride, accept, &L, prec));
  BM_TRY(upload(c, P<int64_t>(c->sizes) + first, b.sizes.data(), J * sizeof(int64_t)));
  HIP_TRY(c, bm::launch_job_init(c->stream, L.js, P<int64_t>(c->sizes) + first, J, k, cp, L.acc,
                                 L.cnt, P<float>(c->Cp) + (int64_t)first * k * cp,
                                 P<float>(c->cn) + (int64_t)first * k));
  int tp = 0;
  BM_TRY(tuned_tile_pts(c, b, b.sizes, &tp));  // after the norms: timing launches read them
  TileMap tm = make_tiles(b.sizes, tp);
  BM_TRY(upload_tiles(c, tm));
  int64_t max_size = 0;
  for (int64_t v : b.sizes) max_size = std::max(max_size, v);

  // Each job makes at most max_iter + 1 assignments.  Launch a few
  // iterations between checks of the job states; after each check the tile
  // map keeps only the jobs that still iterate.
  std::vector<JobState> hs(J);
  std::vector<int32_t> prev_iter(J, -1);  // updates seen at the previous check
  std::vector<int64_t> live(b.sizes);
  int launched = 0;
  int chunk = 4;
  while (true) {
    const int todo = std::min(chunk, max_iter + 1 - launched);
    if (c->prof && (int)c->pev.size() < 2 * todo) {
      for (int q = (int)c->pev.size(); q < 2 * todo; ++q) {
        hipEvent_t e;
        HIP_TRY(c, hipEventCreate(&e));
        c->pev.push_back(e);
      }
    }
    for (int q = 0; q < todo; ++q) BM_TRY(lloyd_launch(c, L, b, tm, max_size, c->prof ? q : -1));
    launched += todo;
    BM_TRY(readback(c, L.js, J * sizeof(JobState), hs.data()));
    if (c->prof) {
      for (int q = 0; q < todo; ++q) {
        float ms_a = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms_a, c->pev[2 * q], c->pev[2 * q + 1]));
        c->stats.assign_seconds += ms_a * 1e-3;
        c->stats.assign_launches += 1;
      }
      // distances of this chunk: job j made (assignments now - before)
      for (int j = 0; j < J; ++j) {
        const int before = prev_iter[j] < 0 ? 0 : prev_iter[j] + 1;
        const int now = hs[j].iter + 1;
        if (now > before) c->stats.assign_dists += (int64_t)(now - before) * b.sizes[j] * k;
        prev_iter[j] = hs[j].iter;
      }
    }
    bool any = false, shrink = false;
    for (int j = 0; j < J; ++j) {
      any = any || hs[j].active;
      if (!hs[j].active && live[j] != 0) {
        live[j] = 0;
        shrink = true;
      }
    }
    if (!any) {
      if (out) *out = hs;
      if (L.wide) {  // final labels of a job whose last assignment was odd are in lab[1]
        for (int j = 0; j < J; ++j)
          if (hs[j].iter & 1)
            HIP_TRY(c, hipMemcpyAsync(L.lab[0] + (int64_t)j * L.lab_stride,
                                      L.lab[1] + (int64_t)j * L.lab_stride,
                                      (size_t)b.sizes[j] * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                      c->stream));
      }
      break;
    }
    if (launched >= max_iter + 1) return c->fail(BM_E_STATE, "Lloyd did not stop after %d steps", launched);
    if (shrink) {
      // fewer points left: smaller tiles spread them over more compute units
      BM_TRY(tuned_tile_pts(c, b, live, &tp));
      tm = make_tiles(live, tp);
      BM_TRY(upload_tiles(c, tm));
    }
    chunk = std::min(chunk * 2, 16);
  }
  return BM_OK;
}

// Objective of each job of the batch (no centroid update): fjob[first + j].
int objective_batch(bm_ctx* c, const BatchView& b, int32_t* labels, int64_t lab_stride,
                    int64_t max_chunks, bool near, int prec = BM_FP32) {
  const int J = b.njobs, first = b.first, k = b.k, cp = b.cp;
  TileMap tm = make_tiles(b.sizes, choose_tile_pts(b.sizes));
  BM_TRY(upload_tiles(c, tm));
  BM_TRY(upload(c, P<int64_t>(c->sizes) + first, b.sizes.data(), J * sizeof(int64_t)));
  bm::AssignArgs a{};
  a.S = b.S;
  a.S_stride = b.S_stride;
  a.ld = b.ld;
  a.n = b.n;
  a.cp = cp;
  a.k = k;
  a.tile_pts = tm.tile_pts;
  a.max_chunks = (int32_t)max_chunks;
  a.vec = (b.ld == cp && aligned16(b.S) && (b.S_stride % 4) == 0) ? 1 : 0;
  a.s = P<int64_t>(c->sizes) + first;
  a.tile_job = P<int32_t>(c->tile_job);
  a.tile_idx = P<int32_t>(c->tile_idx);
  a.Cp = P<float>(c->Cp) + (int64_t)first * k * cp;
  a.C_stride = (int64_t)k * cp;
  a.cn = P<float>(c->cn) + (int64_t)first * k;
  a.cn_stride = k;
  a.labels = labels;
  a.lab_stride = lab_stride;
  a.tf = P<double>(c->tf);
  a.tnear = near ? P<int32_t>(c->tnear) : nullptr;
  a.acc = nullptr;
  a.cnt = nullptr;
  a.scale = nullptr;
  a.st = nullptr;
  if (cp > bm::kMaxRegDim && prec == BM_BF16)
    HIP_TRY(c, bm::launch_assign_wide_bf16(c->stream, a, tm.total, false));
  else if (cp > bm::kMaxRegDim)
    HIP_TRY(c, bm::launch_assign_wide(c->stream, a, tm.total, false));
  else
    HIP_TRY(c, bm::launch_assign(c->stream, a, tm.total, false));
  HIP_TRY(c, bm::launch_reduce_f(c->stream, P<double>(c->tf), a.tnear,
                                 P<int64_t>(c->sizes) + first, (int32_t)max_chunks, J,
                                 P<double>(c->fjob) + first,
                                 near ? P<long long>(c->nearjob) + first : nullptr));
  return BM_OK;
}

// K-means++ initial D of wide points on the matrix cores: jobs (slots
// base..base+J-1 of the workspace) with sizes `sizes` (0: no tiles), whose
// working centroids and flags are in place (launch_kpp_init_wide).
int kpp_init_wide(bm_ctx* c, hipStream_t st, const bm::KppArgs& ka, int base, int J,
                  const std::vector<int64_t>& sizes) {
  const int k = ka.k, cp = ka.cp;
  float* cn = P<float>(c->cn) + (int64_t)base * k;
  // norms of the working centroids (the same values the Lloyd kernels keep)
  HIP_TRY(c, bm::launch_centroid_norms(st, ka.Cp, cp, k, J, cn));
  TileMap tm = make_tiles(sizes, choose_tile_pts(sizes));
  if (tm.total == 0) return BM_OK;
  BM_TRY(upload_tiles(c, tm));
  bm::AssignArgs a{};
  a.S = ka.S;
  a.S_stride = ka.S_stride;
  a.ld = ka.ld;
  a.n = ka.n;
  a.cp = cp;
  a.k = k;
  a.tile_pts = tm.tile_pts;
  a.max_chunks = (int32_t)c->max_chunks;
  a.vec = (ka.ld == cp && aligned16(ka.S) && (ka.S_stride % 4) == 0) ? 1 : 0;
  a.s = ka.s;
  a.tile_job = P<int32_t>(c->tile_job);
  a.tile_idx = P<int32_t>(c->tile_idx);
  a.Cp = ka.Cp;
  a.C_stride = ka.C_stride;
  a.cn = cn;
  a.cn_stride = k;
  a.tf = P<double>(c->tf);
  bm::KppInitOut kp{};
  kp.ks = ka.ks;
  kp.deg = ka.deg;
  kp.D = ka.D;  // slot 0 of the D buffers
  kp.D_job_stride = ka.D_job_stride;
  kp.Dt = ka.Dt;
  kp.Dt_job_stride = ka.ndt_max;
  HIP_TRY(c, bm::launch_kpp_init_wide(st, a, tm.total, kp));
  return BM_OK;
}

struct KppBatch {
  const uint64_t* seed_worker_host;  // [J][2]
  uint64_t g;
  int n_cand;
  int steps;  // number of steps to run (max degenerate count over jobs)
  int32_t* picks;
};

// Greedy K-means++ for the degenerate centroids of every job (Cp, deg_work).
int kpp_batch(bm_ctx* c, const BatchView& b, const KppBatch& kb) {
  const int J = b.njobs, first = b.first, k = b.k, cp = b.cp;
  if (kb.steps <= 0) return BM_OK;
  BM_TRY(upload(c, P<int64_t>(c->sizes) + first, b.sizes.data(), J * sizeof(int64_t)));
  BM_TRY(upload(c, P<uint64_t>(c->seed_worker) + 2 * first, kb.seed_worker_host,
                J * 2 * sizeof(uint64_t)));
  int64_t smax = 0;
  for (int64_t s : b.sizes) smax = std::max(smax, s);
  bm::KppArgs a{};
  a.S = b.S;
  a.S_stride = b.S_stride;
  a.ld = b.ld;
  a.n = b.n;
  a.cp = cp;
  a.k = k;
  a.ndt_max = (int32_t)c->max_chunks;
  a.njobs = c->max_jobs;
  a.s = P<int64_t>(c->sizes) + first;
  a.Cp = P<float>(c->Cp) + (int64_t)first * k * cp;
  a.C_stride = (int64_t)k * cp;
  a.deg = P<uint8_t>(c->deg_work) + (int64_t)first * k;
  a.D = P<float>(c->D) + (int64_t)first * c->max_s;
  a.D_slot_stride = (int64_t)c->max_jobs * c->max_s;
  a.D_job_stride = c->max_s;
  a.Dt = P<double>(c->Dt) + (int64_t)first * c->max_chunks;
  a.ks = P<KppState>(c->ks) + first;
  a.todo = P<int32_t>(c->todo) + (int64_t)first * k;
  a.picks = kb.picks;
  a.seed_worker = P<uint64_t>(c->seed_worker) + 2 * first;
  a.g = kb.g;
  a.n_cand = kb.n_cand;
  HIP_TRY(c, bm::launch_kpp_setup(c->stream, a, J));
  if (cp > bm::kMaxRegDim)
    BM_TRY(kpp_init_wide(c, c->stream, a, first, J, b.sizes));
  else
    HIP_TRY(c, bm::launch_kpp_init(c->stream, a, J, smax));
  for (int step = 0; step < kb.steps; ++step) {
    HIP_TRY(c, bm::launch_kpp_step(c->stream, a, J));
    if (cp >= kStagedKppDim)
      HIP_TRY(c, bm::launch_kpp_pot_staged(c->stream, a, J, smax));
    else
      HIP_TRY(c, bm::launch_kpp_pot(c->stream, a, J, smax));
  }
  HIP_TRY(c, bm::launch_kpp_step(c->stream, a, J));  // commits the last step
  return BM_OK;
}

// One round of Algorithm 1 for all workers in a single cooperative launch of
// the persistent round kernel: workgroups are split among the workers in
// proportion to their sample sizes; each worker runs its re-evaluation (if
// its size changed) and its passes on its own group.  Fills, per worker, the
// re-evaluated f (recalc_f) and the per-pass results (out[w * p + q]).
struct RoundResult {
  std::vector<double> recalc_f;
  std::vector<bm::PassOut> out;
  double seconds = 0.0;
};

// Returned by round_persistent when the device's workgroup placement does not
// fit the worker layout; nothing ran and the round goes to the multi-launch path.
constexpr int kRoundNoFit = 1;

// Workgroups per XCD of a co-resident grid of `cap` workgroups (measured once).
int xcd_layout(bm_ctx* c, int cap) {
  if (c->xcd_cap == cap) return BM_OK;
  DevBuf tmp;
  BM_TRY(dev_alloc(c, tmp, (size_t)cap * sizeof(uint32_t)));
  hipError_t e = bm::launch_xcd_probe(c->stream, P<uint32_t>(tmp), cap);
  std::vector<uint32_t> ids(cap);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ids.data(), tmp.p, (size_t)cap * sizeof(uint32_t), hipMemcpyDeviceToHost,
                       c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_free(tmp);
  if (e != hipSuccess) return c->fail(BM_E_HIP, "XCD probe: %s", hipGetErrorString(e));
  for (int x = 0; x < bm::kMaxXcd; ++x) c->xcd_wgs[x] = 0;
  for (uint32_t v : ids) c->xcd_wgs[v % bm::kMaxXcd] += 1;
  c->xcd_cap = cap;
  return BM_OK;
}

// One round of Algorithm 1 for all workers in one cooperative launch.
//
// Placement: a worker's Lloyd iteration costs about F + L * u, u = assignment
// steps of its busiest workgroup (units of 512 points), and it runs about
// iters[w] iterations in the round.  Workers go to XCDs largest predicted work
// (iters x units) first, each to the XCD with the least work per workgroup.
// On each XCD every worker starts with one workgroup; the spare workgroups
// then go to the worker with the largest predicted time, each time as many as
// it needs for one assignment step fewer.
int round_persistent(bm_ctx* c, const float* X, const bm_params& p, int t,
                     const std::vector<int64_t>& sizes, const std::vector<int32_t>& recalc,
                     const std::vector<double>& iters, RoundResult* res) {
  const int W = p.workers, k = p.k, n = p.n, cp = round_up4(n);
  const size_t lds = bm::round_lds_bytes(cp, k);
  int cap = 0;
  HIP_TRY(c, bm::round_capacity(cp, k, lds, &cap));
  if (cap < W) return kRoundNoFit;
  BM_TRY(xcd_layout(c, cap));
  const int ppl = (cp <= 32 && k < bm::kMfmaMinK) ? 2 : 1;  // points per lane of k_round
  constexpr double kF = 20.0, kL = 16.0;  // relative costs (microseconds, measured)
  std::vector<int64_t> units(W);
  std::vector<double> work(W);
  for (int w = 0; w < W; ++w) {
    const int64_t nch = (sizes[w] + bm::kWG - 1) / bm::kWG;
    units[w] = std::max<int64_t>(1, (nch + ppl - 1) / ppl);
    work[w] = std::max(1.0, iters[w]) * (double)units[w];
  }
  std::vector<int> order(W);
  for (int w = 0; w < W; ++w) order[w] = w;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  std::vector<int32_t> xnw(bm::kMaxXcd, 0), xw((size_t)bm::kMaxXcd * W, 0),
      xg((size_t)bm::kMaxXcd * W, 0);
  std::vector<double> load(bm::kMaxXcd, 0.0);
  for (int w : order) {
    int best = -1;
    double best_v = 0.0;
    for (int x = 0; x < bm::kMaxXcd; ++x) {
      if (xnw[x] >= c->xcd_wgs[x]) continue;
      const double v = (load[x] + work[w]) / (double)c->xcd_wgs[x];
      if (best < 0 || v < best_v) {
        best = x;
        best_v = v;
      }
    }
    if (best < 0) return kRoundNoFit;
    xw[(size_t)best * W + xnw[best]] = w;
    xnw[best] += 1;
    load[best] += work[w];
  }
  auto steps = [&](int w, int64_t g) { return (units[w] + g - 1) / g; };
  auto t_of = [&](int w, int64_t g) {
    return std::max(1.0, iters[w]) * (kF + kL * (double)steps(w, g));
  };
  for (int x = 0; x < bm::kMaxXcd; ++x) {
    const int nw = xnw[x];
    if (nw == 0) continue;
    int32_t* g = &xg[(size_t)x * W];
    const int32_t* wl = &xw[(size_t)x * W];
    for (int i = 0; i < nw; ++i) g[i] = 1;
    for (int64_t spare = c->xcd_wgs[x] - nw; spare > 0;) {
      int bi = -1;
      double bt = 0.0;
      int64_t bneed = 0;
      for (int i = 0; i < nw; ++i) {
        const int w = wl[i];
        const int64_t st = steps(w, g[i]);
        if (st <= 1) continue;
        const int64_t gn = (units[w] + st - 2) / (st - 1);  // workgroups for one step fewer
        if (gn - g[i] > spare) continue;
        const double tw = t_of(w, g[i]);
        if (bi < 0 || tw > bt) {
          bi = i;
          bt = tw;
          bneed = gn - g[i];
        }
      }
      if (bi < 0) break;
      g[bi] += (int32_t)bneed;
      spare -= bneed;
    }
  }
  const int64_t mc = c->max_chunks;
  // work buffer: [reg kMaxXcd][grid barrier][W barriers][delta W*3*k*cp][dcnt W*3*k]
  //              [claim W*3] | [tf3 W*3*mc]; zero up to tf3
  const size_t off_gbar = 64, off_bar = 128;
  const size_t off_delta = off_bar + (size_t)W * sizeof(bm::GroupBar);
  const size_t off_dcnt = off_delta + (size_t)W * 3 * k * cp * sizeof(unsigned long long);
  const size_t off_claim = off_dcnt + (size_t)W * 3 * k * sizeof(int32_t);
  const size_t off_tf3 = (off_claim + (size_t)W * 3 * sizeof(unsigned int) + 255) / 256 * 256;
  const size_t work_bytes = off_tf3 + (size_t)W * 3 * mc * sizeof(double);
  const size_t map_bytes = (size_t)bm::kMaxXcd * (2 * W + 1) * sizeof(int32_t);
  const size_t rres_bytes = 16 + (size_t)W * sizeof(double) + (size_t)W * p.passes_p * sizeof(bm::PassOut);
  if (c->rwork.bytes < work_bytes || c->wgmap.bytes < map_bytes || c->rres.bytes < rres_bytes) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->rwork.bytes < work_bytes) BM_TRY(dev_alloc(c, c->rwork, work_bytes));
    if (c->wgmap.bytes < map_bytes) BM_TRY(dev_alloc(c, c->wgmap, map_bytes));
    if (c->rres.bytes < rres_bytes) BM_TRY(dev_alloc(c, c->rres, rres_bytes));
  }
  int32_t* d_map = P<int32_t>(c->wgmap);
  BM_TRY(upload(c, d_map, xnw.data(), bm::kMaxXcd * sizeof(int32_t)));
  BM_TRY(upload(c, d_map + bm::kMaxXcd, xw.data(), (size_t)bm::kMaxXcd * W * sizeof(int32_t)));
  BM_TRY(upload(c, d_map + bm::kMaxXcd * (1 + W), xg.data(), (size_t)bm::kMaxXcd * W * sizeof(int32_t)));
  BM_TRY(upload(c, P<int64_t>(c->sizes), sizes.data(), W * sizeof(int64_t)));
  BM_TRY(upload(c, P<int32_t>(c->rflags), recalc.data(), W * sizeof(int32_t)));
  unsigned char* rr = P<unsigned char>(c->rres);
  unsigned char* wk = P<unsigned char>(c->rwork);
  HIP_TRY(c, hipMemsetAsync(rr, 0, 16, c->stream));
  HIP_TRY(c, hipMemsetAsync(wk, 0, off_tf3, c->stream));

  const int64_t Sj = c->max_s * cp;
  bm::RoundArgs r{};
  r.X = X;
  r.m = p.m;
  r.n = n;
  r.cp = cp;
  r.k = k;
  r.W = W;
  r.passes_p = p.passes_p;
  r.max_iter = p.max_iter;
  r.n_cand = p.n_candidates;
  r.t = t;
  r.seed = p.seed;
  r.tol = p.tol;
  r.s = P<int64_t>(c->sizes);
  r.recalc = P<int32_t>(c->rflags);
  r.xcd_nw = d_map;
  r.xcd_workers = d_map + bm::kMaxXcd;
  r.xcd_g = d_map + bm::kMaxXcd * (1 + W);
  r.reg = reinterpret_cast<unsigned int*>(wk);
  r.gbar = reinterpret_cast<bm::GroupBar*>(wk + off_gbar);
  r.bar = reinterpret_cast<bm::GroupBar*>(wk + off_bar);
  r.delta = reinterpret_cast<unsigned long long*>(wk + off_delta);
  r.dcnt = reinterpret_cast<int32_t*>(wk + off_dcnt);
  r.claim = reinterpret_cast<unsigned int*>(wk + off_claim);
  r.tf3 = reinterpret_cast<double*>(wk + off_tf3);
  bm::AssignArgs& a = r.as;
  a.S = P<float>(c->S);
  a.S_stride = Sj;
  a.ld = cp;
  a.n = n;
  a.cp = cp;
  a.k = k;
  a.tile_pts = 0;
  a.max_chunks = (int32_t)mc;
  a.vec = 1;
  a.s = r.s;
  a.Cp = P<float>(c->Cp);
  a.C_stride = (int64_t)k * cp;
  a.cn = P<float>(c->cn);
  a.cn_stride = k;
  a.labels = P<int32_t>(c->labels);
  a.lab_stride = c->max_s;
  a.tf = P<double>(c->tf);
  a.tnear = nullptr;
  a.acc = P<unsigned long long>(c->acc);
  a.cnt = P<int32_t>(c->cnt);
  a.scale = P<double>(c->scale);
  a.st = nullptr;
  bm::KppArgs& ka = r.ka;
  ka.S = a.S;
  ka.S_stride = Sj;
  ka.ld = cp;
  ka.n = n;
  ka.cp = cp;
  ka.k = k;
  ka.ndt_max = (int32_t)mc;
  ka.njobs = c->max_jobs;
  ka.s = r.s;
  ka.Cp = P<float>(c->Cp);
  ka.C_stride = (int64_t)k * cp;
  ka.deg = P<uint8_t>(c->deg_work);
  ka.D = P<float>(c->D);
  ka.D_slot_stride = (int64_t)c->max_jobs * c->max_s;
  ka.D_job_stride = c->max_s;
  ka.Dt = P<double>(c->Dt);
  ka.ks = P<KppState>(c->ks);
  ka.todo = P<int32_t>(c->todo);
  ka.picks = nullptr;
  ka.seed_worker = P<uint64_t>(c->seed_worker);
  ka.g = 0;
  ka.gs = P<uint64_t>(c->gs);
  ka.n_cand = p.n_candidates;
  r.inv_scale = P<double>(c->inv_scale);
  r.Cinc = P<float>(c->Cinc);
  r.deg_inc = P<uint8_t>(c->deg_inc);
  r.fhat = P<double>(c->fhat);
  r.Cp = P<float>(c->Cp);
  r.deg_work = P<uint8_t>(c->deg_work);
  r.err = reinterpret_cast<int32_t*>(rr);
  r.recalc_f = reinterpret_cast<double*>(rr + 16);
  r.out = reinterpret_cast<bm::PassOut*>(rr + 16 + (size_t)W * sizeof(double));
  BM_TRY(upload(c, c->rargs.p, &r, sizeof r));

  HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
  HIP_TRY(c, bm::launch_round(c->stream, P<bm::RoundArgs>(c->rargs), cp, k, cap, lds));
  HIP_TRY(c, hipEventRecord(c->ev2, c->stream));
  std::vector<unsigned char> h(rres_bytes);
  BM_TRY(readback(c, rr, rres_bytes, h.data()));
  float ms = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&ms, c->ev1, c->ev2));
  res->seconds = ms * 1e-3;
  int32_t err;
  std::memcpy(&err, h.data(), sizeof err);
  if (err == 2) return kRoundNoFit;
  if (err) return c->fail(BM_E_STATE, "persistent round kernel: a group barrier timed out");
  res->recalc_f.assign(W, 0.0);
  std::memcpy(res->recalc_f.data(), h.data() + 16, W * sizeof(double));
  res->out.resize((size_t)W * p.passes_p);
  std::memcpy(res->out.data(), h.data() + 16 + W * sizeof(double),
              (size_t)W * p.passes_p * sizeof(bm::PassOut));
  return BM_OK;
}

int check_prec(bm_ctx* c, int prec) {
  if (prec != BM_FP32 && prec != BM_BF16)
    return c->fail(BM_E_ARG, "precision %d is not one of BM_FP32, BM_BF16", prec);
  return BM_OK;
}

int check_dim(bm_ctx* c, int n, int k) {
  if (n < 1) return c->fail(BM_E_ARG, "n must be >= 1");
  if (n > kMaxDim) return c->fail(BM_E_ARG, "n = %d exceeds the supported dimension %d", n, kMaxDim);
  if (k < 1) return c->fail(BM_E_ARG, "k must be >= 1");
  // LDS of the Lloyd-step kernels: centroids, norms and fixed-point sums
  // (k x cp floats and int64, narrow) or the update's label changes sorted by
  // cluster (wide), plus each kernel's static LDS
  const int cp = round_up4(n);
  size_t lds = 0, st = 0;
  HIP_TRY(c, hipSetDevice(c->device));
  if (cp > bm::kMaxRegDim) {
    HIP_TRY(c, bm::update_wide_static_lds(&st));
    lds = bm::update_wide_lds(k) + st;
  } else {
    HIP_TRY(c, bm::assign_static_lds(cp, &st));
    lds = (((size_t)k * cp + k) * 4 + 15) / 16 * 16 + (size_t)k * cp * 8 + (size_t)k * 4 + st;
  }
  if (lds > kMaxLds)
    return c->fail(BM_E_ARG, "k = %d is too large for n = %d (%zu bytes of LDS)", k, n, lds);
  return BM_OK;
}

uint64_t philox_word(uint64_t seed, uint32_t worker, uint32_t purpose, uint64_t c0, int word) {
  uint64_t k0, k1;
  bm::stream_key(seed, worker, purpose, &k0, &k1);
  return bm::philox_ctr(c0, 0, 0, 0, k0, k1).w[word];
}

void round_keys(uint64_t m, uint64_t seed, uint32_t worker, uint32_t purpose, uint64_t g,
                uint64_t out[4]) {
  const bm::FeistelKey fk = bm::feistel_key(m, seed, worker, purpose, g);
  for (int r = 0; r < 4; ++r) out[r] = fk.rk[r];
}

// Sample-size draw of Algorithm 1 under the configured policy.
int64_t draw_size(const bm_params& p, uint32_t worker, int t, const int64_t* bacc,
                  const int64_t* bpass, int64_t l_sum, int64_t l_count, int32_t* bin) {
  uint64_t k0, k1;
  bm::stream_key(p.seed, worker, BM_PURPOSE_SIZE, &k0, &k1);
  const bm::U64x4 w = bm::philox_ctr((uint64_t)t, 0, 0, 0, k0, k1);
  const int64_t a = p.s_min, b = p.s_max;
  *bin = 0;
  if (p.size_policy == BM_SIZE_UNIFORM) return a + (int64_t)bm::bounded(w.w[0], (uint64_t)(b - a + 1));
  if (p.size_policy == BM_SIZE_FIXED) return a;
  const double la = std::log((double)a);
  const double width = std::log((double)(b + 1)) - la;
  if (p.size_policy == BM_SIZE_SHRINK && t > 0 && l_count > 0) {
    // log-uniform in [mu / r_t, mu r_t] around the mean of L, ln r_t = width / 2 * 2^-t
    const int64_t mu = (l_sum + l_count / 2) / l_count;
    const double lm = std::log((double)mu);
    const double half = std::ldexp(width / 2.0, -t);
    const double lo = std::max(la, lm - half);
    const double hi = std::min(la + width, lm + half);
    const double v = lo + bm::u01(w.w[0]) * (hi - lo);
    const int64_t s = (int64_t)std::floor(std::exp(v));
    *bin = std::min(kNBins - 1, (int)((v - la) / width * kNBins));
    return std::min(std::max(s, a), b);
  }
  if (p.size_policy == BM_SIZE_LOGUNIFORM || p.size_policy == BM_SIZE_SHRINK || t == 0) {
    const double u = bm::u01(w.w[0]);
    int64_t s = (int64_t)std::floor(std::exp(la + u * width));
    *bin = std::min(kNBins - 1, (int)(u * kNBins));
    return std::min(std::max(s, a), b);
  }
  // BINS
  double weights[kNBins];
  double total = 0.0;
  for (int i = 0; i < kNBins; ++i) {
    weights[i] = ((double)bacc[i] + 1.0) / ((double)bpass[i] + 2.0);
  }
  for (int i = 0; i < kNBins; ++i) total += weights[i];  // in bin order
  const double x = bm::u01(w.w[1]) * total;
  double accw = 0.0;
  int ib = kNBins - 1;
  for (int i = 0; i < kNBins; ++i) {
    accw += weights[i];
    if (x < accw) {
      ib = i;
      break;
    }
  }
  *bin = ib;
  const double v = la + ((double)ib + bm::u01(w.w[2])) * (width / kNBins);
  const int64_t s = (int64_t)std::floor(std::exp(v));
  return std::min(std::max(s, a), b);
}

int validate_params(bm_ctx* c, const bm_params* p) {
  if (!p) return c->fail(BM_E_ARG, "params is NULL");
  if (p->m < 1 || p->m >= (1ll << 31)) return c->fail(BM_E_ARG, "m must be in [1, 2^31)");
  if (p->k < 1 || p->k > p->s_min || p->s_min > p->s_max || p->s_max > p->m)
    return c->fail(BM_E_ARG, "need 1 <= k <= s_min <= s_max <= m");
  if (p->workers < 1 || p->rounds_T < 0 || p->passes_p < 1)
    return c->fail(BM_E_ARG, "need workers >= 1, rounds_T >= 0, passes_p >= 1");
  if (p->max_iter < 0 || !(p->tol >= 0.0)) return c->fail(BM_E_ARG, "need max_iter >= 0, tol >= 0");
  if (p->n_candidates < 1 || p->n_candidates > 3) return c->fail(BM_E_ARG, "n_candidates in 1..3");
  if (p->size_policy < 0 || p->size_policy > BM_SIZE_SHRINK) return c->fail(BM_E_ARG, "unknown size policy");
  if (p->size_policy == BM_SIZE_FIXED && p->s_min != p->s_max)
    return c->fail(BM_E_ARG, "FIXED size policy needs s_min == s_max");
  BM_TRY(check_prec(c, p->prec));
  BM_TRY(check_dim(c, p->n, p->k));
  return BM_OK;
}

// ---------------------------------------------------------------------------
// Serving loop (bm_serve): single-pass jobs of competing workers, batched
// continuously.  Every (dataset, k) has its own context whose job slots hold
// the running jobs; every (dataset, k, worker) has an incumbent in a device
// store for the whole call.
// ---------------------------------------------------------------------------
struct ServeWorker {
  int d = 0, k = 0, w = 0;
  int store_group = -1;  // group whose stream last wrote this worker's incumbent
  uint32_t rng_worker = 0;
  int64_t off_c = 0, off_deg = 0;  // offsets in the incumbent store
  double fhat = std::numeric_limits<double>::infinity();
  int ndeg = 0;
  int64_t s_prev = -1;
  uint64_t passes = 0;
  bool busy = false;
  std::deque<int> queue;  // arrived jobs, arrival order
};

struct ServeGroup {
  int d = 0, k = 0, n = 0, cp = 0;
  int prec = BM_FP32;  // BM_BF16 only for wide points (the narrow kernels have one precision)
  bm_ctx* c = nullptr;
  int slots = 0;
  int64_t s_max = 0;
  int64_t jobs = 0;
  std::vector<int> slot_job;   // job of each slot, -1 when free
  std::vector<int64_t> sizes;  // its sample size, 0 when free
  LloydSetup L;
  int running = 0;
  hipStream_t stream = nullptr;   // the group's own stream (groups run concurrently)
  hipEvent_t store_ev = nullptr;  // recorded after the group's latest incumbent writes
  // job states copied after a Lloyd iteration (pinned, two buffers), read
  // once the copy has completed: the host never waits for the device, and a
  // group has at most two Lloyd iterations in flight
  JobState* snap[2] = {nullptr, nullptr};
  hipEvent_t snap_ev[2] = {nullptr, nullptr};
  std::vector<int> snap_job[2];  // slot_job when each copy was taken
  int snap_head = 0;             // oldest copy not yet read
  int snap_count = 0;            // copies in flight
};

// Device bytes one running job of sample size s uses (sample, indices, two
// label arrays, K-means++ D slots and tile sums, chunk partials, centroid
// state).
int64_t serve_job_bytes(int64_t s, int n, int k) {
  const int64_t cp = round_up4(n), ch = (s + bm::kWG - 1) / bm::kWG;
  return s * (cp * 4 + 4 + 8 + 16) + ch * (4 * 8 + 12) + (int64_t)k * (cp * 12 + n * 4 + 16) + 1024;
}

struct ServeState {
  std::vector<ServeGroup> groups;
  float* store_c = nullptr;
  uint8_t* store_deg = nullptr;
  hipEvent_t start_ev = nullptr;
  ~ServeState() {
    for (ServeGroup& g : groups) {
      if (g.c) bm_destroy(g.c);  // synchronises the group's stream
      if (g.store_ev) (void)hipEventDestroy(g.store_ev);
      for (int b = 0; b < 2; ++b) {
        if (g.snap_ev[b]) (void)hipEventDestroy(g.snap_ev[b]);
        if (g.snap[b]) (void)hipHostFree(g.snap[b]);
      }
      if (g.stream) (void)hipStreamDestroy(g.stream);
    }
    if (start_ev) (void)hipEventDestroy(start_ev);
    if (store_c) (void)hipFree(store_c);
    if (store_deg) (void)hipFree(store_deg);
  }
};

// Start the jobs `adm` (job, slot) of group G together: incumbents into their
// slots, re-evaluation of incumbents whose size changed, the passes' samples,
// K-means++ of every job's degenerate centroids in one batch over its slots,
// and the jobs' Lloyd states.
int serve_admit(bm_ctx* c, ServeState& st, std::vector<ServeWorker>& workers,
                const std::vector<int>& job_worker, ServeGroup& G, const std::vector<std::pair<int, int>>& adm,
                const bm_dataset& ds, const bm_job* jobs, const bm_serve_params& sp) {
  bm_ctx* gc = G.c;
  const int k = G.k, n = G.n, cp = G.cp, J = G.slots;
  const int64_t Sj = gc->max_s * cp;
  hipStream_t str = gc->stream;
  BatchView all;
  all.first = 0;
  all.njobs = J;
  all.n = n;
  all.cp = cp;
  all.k = k;
  all.S = P<float>(gc->S);
  all.S_stride = Sj;
  all.ld = cp;
  std::vector<uint64_t> rk(4 * (size_t)J, 0);
  std::vector<int64_t> sz(J, 0);
  int64_t smax = 0;
  for (const auto& jq : adm) {
    const ServeWorker& W = workers[job_worker[jq.first]];
    const int q = jq.second;
    if (W.store_group >= 0 && st.groups[W.store_group].stream != str)
      HIP_TRY(c, hipStreamWaitEvent(str, st.groups[W.store_group].store_ev, 0));
    HIP_TRY(c, hipMemcpyAsync(P<float>(gc->Cinc) + (int64_t)q * k * n, st.store_c + W.off_c,
                              (size_t)k * n * sizeof(float), hipMemcpyDeviceToDevice, str));
    HIP_TRY(c, hipMemcpyAsync(P<uint8_t>(gc->deg_inc) + (int64_t)q * k, st.store_deg + W.off_deg,
                              (size_t)k, hipMemcpyDeviceToDevice, str));
  }
  // re-evaluate incumbents whose sample size changed (Algorithm 1; Section 4.2)
  std::vector<int> re;
  for (size_t i = 0; i < adm.size(); ++i) {
    const ServeWorker& W = workers[job_worker[adm[i].first]];
    if (std::isfinite(W.fhat) && jobs[adm[i].first].s != W.s_prev) re.push_back((int)i);
  }
  if (!re.empty()) {
    for (int i : re) {
      const int j = adm[i].first, q = adm[i].second;
      const ServeWorker& W = workers[job_worker[j]];
      sz[q] = jobs[j].s;
      smax = std::max(smax, sz[q]);
      round_keys((uint64_t)ds.m, sp.seed, W.rng_worker, BM_PURPOSE_RECALC, W.passes, &rk[4 * q]);
      HIP_TRY(c, bm::launch_pad_centroids(str, P<float>(gc->Cinc) + (int64_t)q * k * n, (int64_t)k * n,
                                          n, cp, k, 1, P<float>(gc->Cp) + (int64_t)q * k * cp,
                                          (int64_t)k * cp, P<float>(gc->cn) + (int64_t)q * k, k));
    }
    BM_TRY(upload(gc, P<int64_t>(gc->sizes), sz.data(), J * sizeof(int64_t)));
    BM_TRY(upload(gc, P<uint64_t>(gc->rkeys), rk.data(), 4 * (size_t)J * sizeof(uint64_t)));
    HIP_TRY(c, bm::launch_sample(str, ds.X, ds.m, n, J, smax, P<int64_t>(gc->sizes),
                                 P<uint64_t>(gc->rkeys), P<int32_t>(gc->idx), gc->max_s,
                                 P<float>(gc->S), Sj, cp));
    all.sizes = sz;
    BM_TRY(objective_batch(gc, all, nullptr, 0, gc->max_chunks, false, G.prec));
    std::vector<double> fr(J);
    BM_TRY(readback(gc, P<double>(gc->fjob), J * sizeof(double), fr.data()));
    for (int i : re) workers[job_worker[adm[i].first]].fhat = fr[adm[i].second];
  }
  // the passes' samples; incumbents as working copies; f_hat of every slot
  std::fill(sz.begin(), sz.end(), 0);
  std::fill(rk.begin(), rk.end(), 0);
  smax = 0;
  std::vector<uint64_t> sw(2 * (size_t)J, 0), gs(J, 0);
  std::vector<int32_t> slots;
  int steps = 0;
  for (const auto& jq : adm) {
    const int j = jq.first, q = jq.second;
    const ServeWorker& W = workers[job_worker[j]];
    sz[q] = jobs[j].s;
    smax = std::max(smax, sz[q]);
    round_keys((uint64_t)ds.m, sp.seed, W.rng_worker, BM_PURPOSE_SAMPLE, W.passes, &rk[4 * q]);
    sw[2 * q] = sp.seed;
    sw[2 * q + 1] = W.rng_worker;
    gs[q] = W.passes;
    slots.push_back(q);
    steps = std::max(steps, W.ndeg);
    BM_TRY(upload(gc, P<double>(gc->fhat) + q, &W.fhat, sizeof(double)));
    HIP_TRY(c, bm::launch_copy_incumbent(str, P<float>(gc->Cinc) + (int64_t)q * k * n,
                                         P<uint8_t>(gc->deg_inc) + (int64_t)q * k, n, cp, k, 1,
                                         P<float>(gc->Cp) + (int64_t)q * k * cp,
                                         P<uint8_t>(gc->deg_work) + (int64_t)q * k));
  }
  BM_TRY(upload(gc, P<int64_t>(gc->sizes), sz.data(), J * sizeof(int64_t)));
  BM_TRY(upload(gc, P<uint64_t>(gc->rkeys), rk.data(), 4 * (size_t)J * sizeof(uint64_t)));
  HIP_TRY(c, bm::launch_sample(str, ds.X, ds.m, n, J, smax, P<int64_t>(gc->sizes),
                               P<uint64_t>(gc->rkeys), P<int32_t>(gc->idx), gc->max_s,
                               P<float>(gc->S), Sj, cp));
  // K-means++ of the degenerate centroids, all admitted slots in one batch
  if (steps > 0) {
    const int A = (int)slots.size();
    BM_TRY(upload(gc, P<int32_t>(gc->rflags), slots.data(), A * sizeof(int32_t)));
    BM_TRY(upload(gc, P<uint64_t>(gc->seed_worker), sw.data(), 2 * (size_t)J * sizeof(uint64_t)));
    BM_TRY(upload(gc, P<uint64_t>(gc->gs), gs.data(), J * sizeof(uint64_t)));
    bm::KppArgs a{};
    a.S = P<float>(gc->S);
    a.S_stride = Sj;
    a.ld = cp;
    a.n = n;
    a.cp = cp;
    a.k = k;
    a.ndt_max = (int32_t)gc->max_chunks;
    a.njobs = gc->max_jobs;
    a.s = P<int64_t>(gc->sizes);
    a.Cp = P<float>(gc->Cp);
    a.C_stride = (int64_t)k * cp;
    a.deg = P<uint8_t>(gc->deg_work);
    a.D = P<float>(gc->D);
    a.D_slot_stride = (int64_t)gc->max_jobs * gc->max_s;
    a.D_job_stride = gc->max_s;
    a.Dt = P<double>(gc->Dt);
    a.ks = P<KppState>(gc->ks);
    a.todo = P<int32_t>(gc->todo);
    a.picks = nullptr;
    a.seed_worker = P<uint64_t>(gc->seed_worker);
    a.g = 0;
    a.gs = P<uint64_t>(gc->gs);
    a.n_cand = sp.n_candidates;
    a.job_slot = P<int32_t>(gc->rflags);
    HIP_TRY(c, bm::launch_kpp_setup(str, a, A));
    if (cp > bm::kMaxRegDim)
      BM_TRY(kpp_init_wide(gc, str, a, 0, J, sz));
    else
      HIP_TRY(c, bm::launch_kpp_init(str, a, A, smax));
    for (int step = 0; step < steps; ++step) {
      HIP_TRY(c, bm::launch_kpp_step(str, a, A));
      if (a.cp >= kStagedKppDim)
        HIP_TRY(c, bm::launch_kpp_pot_staged(str, a, A, smax));
      else
        HIP_TRY(c, bm::launch_kpp_pot(str, a, A, smax));
    }
    HIP_TRY(c, bm::launch_kpp_step(str, a, A));  // commits the last step
  }
  // Lloyd state of every admitted slot
  for (int q : slots)
    HIP_TRY(c, bm::launch_job_init(str, G.L.js + q, P<int64_t>(gc->sizes) + q, 1, k, cp,
                                   G.L.acc + (int64_t)q * k * cp, G.L.cnt + (int64_t)q * k,
                                   P<float>(gc->Cp) + (int64_t)q * k * cp, P<float>(gc->cn) + (int64_t)q * k));
  return BM_OK;
}

int serve_impl(bm_ctx* c, const bm_dataset* ds, int nds, const bm_job* jobs, int njobs,
               const bm_serve_params& sp, bm_job_result* res, bm_serve_stats* stats) {
  using clock = std::chrono::steady_clock;
  ServeState st;
  std::vector<ServeWorker> workers;
  std::map<std::tuple<int, int, int>, int> wmap;
  std::map<std::tuple<int, int, int>, int> gmap;
  std::vector<int> job_worker(njobs), job_group(njobs);
  for (int j = 0; j < njobs; ++j) {
    const bm_job& jb = jobs[j];
    const auto key = std::make_tuple(jb.dataset, jb.k, jb.worker);
    auto it = wmap.find(key);
    if (it == wmap.end()) {
      ServeWorker W;
      W.d = jb.dataset;
      W.k = jb.k;
      W.w = jb.worker;
      W.rng_worker = ((uint32_t)jb.dataset << 20) | ((uint32_t)jb.k << 10) | (uint32_t)jb.worker;
      W.ndeg = jb.k;
      it = wmap.emplace(key, (int)workers.size()).first;
      workers.push_back(std::move(W));
    }
    job_worker[j] = it->second;
    // jobs of one (dataset, k) share launches; wide points also split by precision
    const int n = ds[jb.dataset].n;
    const int prec = round_up4(n) > bm::kMaxRegDim ? jb.prec : BM_FP32;
    const auto gk = std::make_tuple(jb.dataset, jb.k, prec);
    auto gi = gmap.find(gk);
    if (gi == gmap.end()) {
      ServeGroup G;
      G.d = jb.dataset;
      G.k = jb.k;
      G.n = n;
      G.cp = round_up4(n);
      G.prec = prec;
      gi = gmap.emplace(gk, (int)st.groups.size()).first;
      st.groups.push_back(std::move(G));
    }
    job_group[j] = gi->second;
    ServeGroup& G = st.groups[gi->second];
    G.s_max = std::max(G.s_max, jb.s);
    G.jobs += 1;
  }
  // slots per group within the budget, in proportion to the group's jobs
  int64_t total_slot_bytes = 0;
  for (ServeGroup& G : st.groups) {
    const int64_t per = serve_job_bytes(G.s_max, G.n, G.k);
    const double share = (double)sp.budget_bytes * (double)G.jobs / (double)njobs;
    if (per > sp.budget_bytes)
      return c->fail(BM_E_ARG, "budget too small for a job of dataset %d, k = %d", G.d, G.k);
    int64_t slots = (int64_t)(share / (double)per);
    slots = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(slots, sp.max_slots), G.jobs));
    G.slots = (int)slots;
    total_slot_bytes += slots * per;
  }
  // every group holds at least one slot; if the rounding up to one slot put
  // the total over the budget, take slots back from the groups holding the
  // most bytes in slots beyond their first
  while (total_slot_bytes > sp.budget_bytes) {
    ServeGroup* take = nullptr;
    int64_t most = 0;
    for (ServeGroup& G : st.groups) {
      const int64_t per = serve_job_bytes(G.s_max, G.n, G.k);
      if (G.slots > 1 && (G.slots - 1) * per > most) {
        most = (G.slots - 1) * per;
        take = &G;
      }
    }
    if (!take)
      return c->fail(BM_E_ARG, "budget of %lld bytes is too small for one job slot of each of "
                     "the %zu (dataset, k, precision) groups (%lld bytes)",
                     (long long)sp.budget_bytes, st.groups.size(), (long long)total_slot_bytes);
    take->slots -= 1;
    total_slot_bytes -= serve_job_bytes(take->s_max, take->n, take->k);
  }
  // incumbent store: all centroids degenerate, f = +inf
  int64_t nc = 0, ndg = 0;
  for (ServeWorker& W : workers) {
    W.off_c = nc;
    W.off_deg = ndg;
    nc += (int64_t)W.k * ds[W.d].n;
    ndg += W.k;
  }
  HIP_TRY(c, hipMalloc(&st.store_c, (size_t)nc * sizeof(float)));
  HIP_TRY(c, hipMalloc(&st.store_deg, (size_t)ndg));
  HIP_TRY(c, hipMemsetAsync(st.store_c, 0, (size_t)nc * sizeof(float), c->stream));
  HIP_TRY(c, hipMemsetAsync(st.store_deg, 1, (size_t)ndg, c->stream));
  // the groups' streams start after the caller's stream: the data sets it
  // produced and the store initialised above
  HIP_TRY(c, hipEventCreateWithFlags(&st.start_ev, hipEventDisableTiming));
  HIP_TRY(c, hipEventRecord(st.start_ev, c->stream));
  // one context per (dataset, k, precision): workspace for its slots, data
  // scales, idle job states
  for (ServeGroup& G : st.groups) {
    HIP_TRY(c, hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking));
    HIP_TRY(c, hipEventCreateWithFlags(&G.store_ev, hipEventDisableTiming));
    for (int b = 0; b < 2; ++b) {
      HIP_TRY(c, hipEventCreateWithFlags(&G.snap_ev[b], hipEventDisableTiming));
      HIP_TRY(c, hipHostMalloc((void**)&G.snap[b], (size_t)G.slots * sizeof(JobState),
                               hipHostMallocDefault));
    }
    HIP_TRY(c, hipStreamWaitEvent(G.stream, st.start_ev, 0));
    int rc = bm_create(c->device, G.stream, &G.c);
    if (rc != BM_OK) return c->fail(rc, "serving workspace: context creation failed");
    // no tile-size timing: it waits for the group's stream, which would stall
    // the host loop that feeds every group
    G.c->tune = false;
    rc = reserve_impl(G.c, G.s_max, G.n, G.k, G.slots);
    if (rc != BM_OK) return c->fail(rc, "serving workspace: %s", G.c->err.c_str());
    const bm_dataset& D = ds[G.d];
    rc = compute_scales(G.c, D.X, D.m, D.n, D.n, G.cp, G.s_max);
    if (rc != BM_OK) return c->fail(rc, "%s", G.c->err.c_str());
    HIP_TRY(c, hipMemsetAsync(G.c->js.p, 0, (size_t)G.slots * sizeof(JobState), G.stream));
    G.slot_job.assign(G.slots, -1);
    G.sizes.assign(G.slots, 0);
    BatchView b;
    b.first = 0;
    b.njobs = G.slots;
    b.n = G.n;
    b.cp = G.cp;
    b.k = G.k;
    b.S = P<float>(G.c->S);
    b.S_stride = G.c->max_s * G.cp;
    b.ld = G.cp;
    rc = lloyd_setup(G.c, b, sp.max_iter, sp.tol, nullptr, 0, true, &G.L, G.prec);
    if (rc != BM_OK) return c->fail(rc, "%s", G.c->err.c_str());
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));

  std::vector<int> order(njobs);
  for (int j = 0; j < njobs; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return jobs[a].arrival < jobs[b].arrival; });
  const auto t0 = clock::now();
  auto elapsed = [&]() { return std::chrono::duration<double>(clock::now() - t0).count(); };
  int next = 0, done = 0;
  int64_t inflight = 0, steps = 0, peak_running = 0, peak_bytes = 0, running = 0;
  while (done < njobs) {
    const double now = elapsed();
    while (next < njobs && (!sp.paced || jobs[order[next]].arrival <= now)) {
      const int j = order[next++];
      workers[job_worker[j]].queue.push_back(j);
    }
    // A group with two Lloyd iterations in flight neither admits nor steps
    // until the older one has finished on the device, so a group whose
    // stream holds a long K-means++ chain never holds up the host loop that
    // feeds the other groups.
    bool progress = false;
    // admissions, earliest arrival first
    std::vector<int> heads;
    for (ServeWorker& W : workers)
      if (!W.busy && !W.queue.empty()) heads.push_back(W.queue.front());
    std::stable_sort(heads.begin(), heads.end(), [&](int a, int b) {
      return jobs[a].arrival < jobs[b].arrival || (jobs[a].arrival == jobs[b].arrival && a < b);
    });
    int admitted = 0;
    std::vector<std::vector<std::pair<int, int>>> adm(st.groups.size());
    for (int j : heads) {
      ServeWorker& W = workers[job_worker[j]];
      ServeGroup& G = st.groups[job_group[j]];
      const int64_t bytes = serve_job_bytes(jobs[j].s, G.n, G.k);
      if (G.snap_count >= 2 || G.running >= G.slots || inflight + bytes > sp.budget_bytes) continue;
      int q = 0;
      while (G.slot_job[q] >= 0) ++q;
      adm[job_group[j]].push_back({j, q});
      W.queue.pop_front();
      W.busy = true;
      G.slot_job[q] = j;
      G.sizes[q] = jobs[j].s;
      G.running += 1;
      running += 1;
      inflight += bytes;
      ++admitted;
    }
    for (size_t gi = 0; gi < st.groups.size(); ++gi) {
      if (adm[gi].empty()) continue;
      ServeGroup& G = st.groups[gi];
      BM_TRY(serve_admit(c, st, workers, job_worker, G, adm[gi], ds[G.d], jobs, sp));
      const double t = elapsed();
      for (const auto& jq : adm[gi]) res[jq.first].admitted = t;
    }
    peak_running = std::max(peak_running, running);
    peak_bytes = std::max(peak_bytes, inflight);
    if (running == 0) {
      if (next < njobs && sp.paced) {  // idle until the next arrival
        const double wait = jobs[order[next]].arrival - elapsed();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 0.01)));
        continue;
      }
      if (admitted == 0) return c->fail(BM_E_STATE, "serving loop made no progress");
      continue;
    }
    // one Lloyd iteration of every running job
    std::vector<char> stepped(st.groups.size(), 0);
    for (size_t gi = 0; gi < st.groups.size(); ++gi) {
      ServeGroup& G = st.groups[gi];
      if (G.running == 0 || G.snap_count >= 2) continue;
      stepped[gi] = 1;
      progress = true;
      BatchView b;
      b.first = 0;
      b.njobs = G.slots;
      b.n = G.n;
      b.cp = G.cp;
      b.k = G.k;
      b.S = P<float>(G.c->S);
      b.S_stride = G.c->max_s * G.cp;
      b.ld = G.cp;
      b.sizes = G.sizes;
      BM_TRY(upload(G.c, P<int64_t>(G.c->sizes), G.sizes.data(), G.slots * sizeof(int64_t)));
      int tp = 0;
      BM_TRY(tuned_tile_pts(G.c, b, G.sizes, &tp));
      TileMap tm = make_tiles(G.sizes, tp);
      BM_TRY(upload_tiles(G.c, tm));
      BM_TRY(lloyd_launch(G.c, G.L, b, tm, G.s_max, -1));
    }
    ++steps;
    // finished jobs leave; an accepted result becomes the worker's incumbent.
    // The job states read here are copies taken after earlier iterations whose
    // copies have completed (the device meanwhile runs the later ones); a job
    // finished there is inactive in the later launches, which skip it.
    for (size_t gi = 0; gi < st.groups.size(); ++gi) {
      ServeGroup& G = st.groups[gi];
      while (G.snap_count > 0) {
        const int h = G.snap_head;
        const hipError_t e = hipEventQuery(G.snap_ev[h]);
        if (e == hipErrorNotReady) break;
        HIP_TRY(c, e);
        G.snap_head ^= 1;
        G.snap_count -= 1;
        progress = true;
        bool wrote = false;
        for (int q = 0; q < G.slots; ++q) {
          const int j = G.snap_job[h][q];
          if (j < 0 || G.slot_job[q] != j || G.snap[h][q].active) continue;
          const JobState& hq = G.snap[h][q];
          ServeWorker& W = workers[job_worker[j]];
          bm_job_result& r = res[j];
          r.f = hq.f;
          r.iters = hq.iter;
          r.accepted = hq.accepted;
          r.ndeg = hq.ndeg;
          if (hq.accepted) {
            HIP_TRY(c, hipMemcpyAsync(st.store_c + W.off_c, P<float>(G.c->Cinc) + (int64_t)q * G.k * G.n,
                                      (size_t)G.k * G.n * sizeof(float), hipMemcpyDeviceToDevice,
                                      G.stream));
            HIP_TRY(c, hipMemcpyAsync(st.store_deg + W.off_deg, P<uint8_t>(G.c->deg_inc) + (int64_t)q * G.k,
                                      (size_t)G.k, hipMemcpyDeviceToDevice, G.stream));
            W.store_group = (int)gi;
            wrote = true;
            W.fhat = hq.f;
            W.ndeg = hq.ndeg;
          }
          r.f_incumbent = W.fhat;
          r.finished = elapsed();
          W.s_prev = jobs[j].s;
          W.passes += 1;
          W.busy = false;
          G.slot_job[q] = -1;
          G.sizes[q] = 0;
          G.running -= 1;
          running -= 1;
          inflight -= serve_job_bytes(jobs[j].s, G.n, G.k);
          ++done;
        }
        if (wrote) HIP_TRY(c, hipEventRecord(G.store_ev, G.stream));
      }
      if (G.running > 0 && stepped[gi]) {
        const int t = (G.snap_head + G.snap_count) % 2;
        G.snap_job[t] = G.slot_job;
        HIP_TRY(c, hipMemcpyAsync(G.snap[t], G.L.js, (size_t)G.slots * sizeof(JobState),
                                  hipMemcpyDeviceToHost, G.stream));
        HIP_TRY(c, hipEventRecord(G.snap_ev[t], G.stream));
        G.snap_count += 1;
      }
    }
    // every group with running jobs is still busy on the device
    if (!progress && admitted == 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  for (ServeGroup& G : st.groups) HIP_TRY(c, hipStreamSynchronize(G.stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (stats) {
    stats->seconds = elapsed();
    stats->steps = steps;
    stats->peak_running = peak_running;
    stats->peak_bytes = peak_bytes;
    stats->slot_bytes = total_slot_bytes;
  }
  return BM_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

BM_API int bm_version(void) { return BM_VERSION; }

BM_API int bm_create(int device, void* hip_stream, bm_ctx** out) {
  if (!out) return BM_E_ARG;
  *out = nullptr;
  bm_ctx* c = new (std::nothrow) bm_ctx();
  if (!c) return BM_E_NOMEM;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    delete c;
    return BM_E_STATE;
  }
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return BM_E_STATE;
  }
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  // address of the no-allocation workspace on this device (device current)
  if (bm::noalloc_scratch(device, &c->scratch) != hipSuccess) {
    delete c;
    return BM_E_STATE;
  }
  bool ok = true;
  for (int i = 0; i < kNumStage && ok; ++i) {
    ok = hipHostMalloc(&c->stage[i], kStageBytes, hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&c->stage_ev[i], hipEventDisableTiming) == hipSuccess;
  }
  ok = ok && hipEventCreate(&c->ev0) == hipSuccess && hipEventCreate(&c->ev1) == hipSuccess &&
       hipEventCreate(&c->ev2) == hipSuccess;
  if (!ok) {
    bm_destroy(c);
    return BM_E_NOMEM;
  }
  *out = c;
  return BM_OK;
}

BM_API void bm_destroy(bm_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  DevBuf* bufs[] = {&c->S,        &c->idx,     &c->labels,   &c->Cp,        &c->cn,
                    &c->Cinc,     &c->deg_work, &c->deg_inc, &c->fhat,      &c->acc,
                    &c->cnt,      &c->tf,      &c->tnear,    &c->js,
                    &c->sizes,    &c->tile_job,  &c->tile_idx,
                    &c->rkeys,    &c->seed_worker, &c->absmax, &c->scale,   &c->inv_scale,
                    &c->fjob,     &c->nearjob, &c->D,         &c->Dt,
                    &c->ks,       &c->todo,    &c->picks,    &c->gs,        &c->rflags,
                    &c->wgmap,    &c->rargs,   &c->rres,     &c->bars, &c->rwork, &c->labels2};
  for (DevBuf* b : bufs) dev_free(*b);
  for (int i = 0; i < kNumStage; ++i) {
    if (c->stage[i]) (void)hipHostFree(c->stage[i]);
    if (c->stage_ev[i]) (void)hipEventDestroy(c->stage_ev[i]);
  }
  if (c->rb) (void)hipHostFree(c->rb);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->ev2) (void)hipEventDestroy(c->ev2);
  if (c->tev0) (void)hipEventDestroy(c->tev0);
  if (c->tev1) (void)hipEventDestroy(c->tev1);
  for (hipEvent_t e : c->pev) (void)hipEventDestroy(e);
  delete c;
}

BM_API const char* bm_strerror(const bm_ctx* c) { return c ? c->err.c_str() : "null context"; }

BM_API int bm_reserve(bm_ctx* c, int64_t max_s, int32_t max_n, int32_t max_k, int32_t max_jobs) {
  if (!c) return BM_E_ARG;
  if (max_s < 1 || max_n < 1 || max_k < 1 || max_jobs < 1)
    return c->fail(BM_E_ARG, "reserve sizes must be >= 1");
  HIP_TRY(c, hipSetDevice(c->device));
  return reserve_impl(c, max_s, max_n, max_k, max_jobs);
}

BM_API int bm_sample(bm_ctx* c, const float* X, int64_t m, int32_t n, int64_t s, uint64_t seed,
                     uint32_t worker, uint32_t purpose, uint64_t g, int32_t* idx_out,
                     float* S_out) {
  if (!c) return BM_E_ARG;
  if (!X || !idx_out) return c->fail(BM_E_ARG, "X and idx_out are required");
  if (n < 1 || s < 1 || s > m || m >= (1ll << 31)) return c->fail(BM_E_ARG, "need 1 <= s <= m < 2^31, n >= 1");
  HIP_TRY(c, hipSetDevice(c->device));
  BM_TRY(ensure(c, 1, 1, 1, 1));
  uint64_t rk[4];
  round_keys((uint64_t)m, seed, worker, purpose, g, rk);
  BM_TRY(upload(c, P<int64_t>(c->sizes), &s, sizeof(int64_t)));
  BM_TRY(upload(c, P<uint64_t>(c->rkeys), rk, sizeof rk));
  HIP_TRY(c, bm::launch_sample(c->stream, X, m, n, 1, s, P<int64_t>(c->sizes), P<uint64_t>(c->rkeys),
                               idx_out, 0, S_out, 0, n));
  return BM_OK;
}

BM_API int bm_seed(bm_ctx* c, const float* S, int64_t s, int32_t n, int32_t k, float* C,
                   uint8_t* degenerate, int32_t n_candidates, uint64_t seed, uint32_t worker,
                   uint64_t g, int32_t* picks_out) {
  if (!c) return BM_E_ARG;
  if (!S || !C || !degenerate) return c->fail(BM_E_ARG, "S, C and degenerate are required");
  if (k < 1 || s < k || n < 1) return c->fail(BM_E_ARG, "need 1 <= k <= s, n >= 1");
  if (n_candidates < 1 || n_candidates > 3) return c->fail(BM_E_ARG, "n_candidates must be 1..3");
  BM_TRY(check_dim(c, n, k));
  HIP_TRY(c, hipSetDevice(c->device));
  BM_TRY(ensure(c, s, n, k, 1));
  const int cp = round_up4(n);
  HIP_TRY(c, bm::launch_pad_centroids(c->stream, C, 0, n, cp, k, 1, P<float>(c->Cp), 0,
                                      P<float>(c->cn), 0));
  HIP_TRY(c, hipMemcpyAsync(c->deg_work.p, degenerate, (size_t)k, hipMemcpyDeviceToDevice, c->stream));
  BatchView b;
  b.first = 0;
  b.njobs = 1;
  b.n = n;
  b.cp = cp;
  b.k = k;
  b.S = S;
  b.S_stride = 0;
  b.ld = n;
  b.sizes = {s};
  const uint64_t sw[2] = {seed, worker};
  KppBatch kb{sw, g, n_candidates, k, picks_out};
  BM_TRY(kpp_batch(c, b, kb));
  HIP_TRY(c, bm::launch_unpad(c->stream, P<float>(c->Cp), cp, n, k, 1, C, 0));
  HIP_TRY(c, hipMemcpyAsync(degenerate, c->deg_work.p, (size_t)k, hipMemcpyDeviceToDevice, c->stream));
  return BM_OK;
}

BM_API int bm_lloyd(bm_ctx* c, const float* S, int64_t s, int32_t n, int32_t k, float* C,
                    int32_t max_iter, double tol, int32_t prec, double* f_out, int32_t* iters_out,
                    uint8_t* degenerate_out, int32_t* labels_out) {
  if (!c) return BM_E_ARG;
  if (!S || !C || !f_out) return c->fail(BM_E_ARG, "S, C and f_out are required");
  if (k < 1 || s < 1 || max_iter < 0 || !(tol >= 0.0)) return c->fail(BM_E_ARG, "need k >= 1, s >= 1, max_iter >= 0, tol >= 0");
  BM_TRY(check_prec(c, prec));
  BM_TRY(check_dim(c, n, k));
  HIP_TRY(c, hipSetDevice(c->device));
  BM_TRY(ensure(c, s, n, k, 1));
  const int cp = round_up4(n);
  BM_TRY(compute_scales(c, S, s, n, n, cp, s));
  HIP_TRY(c, bm::launch_pad_centroids(c->stream, C, 0, n, cp, k, 1, P<float>(c->Cp), 0,
                                      P<float>(c->cn), 0));
  BatchView b;
  b.first = 0;
  b.njobs = 1;
  b.n = n;
  b.cp = cp;
  b.k = k;
  b.S = S;
  b.S_stride = 0;
  b.ld = n;
  b.sizes = {s};
  BM_TRY(lloyd_batch(c, b, max_iter, tol, labels_out, 0, false, nullptr, prec));
  HIP_TRY(c, bm::launch_unpad(c->stream, P<float>(c->Cp), cp, n, k, 1, C, 0));
  if (degenerate_out)
    HIP_TRY(c, hipMemcpyAsync(degenerate_out, c->deg_work.p, (size_t)k, hipMemcpyDeviceToDevice, c->stream));
  JobState st;
  BM_TRY(readback(c, c->js.p, sizeof(JobState), &st));
  *f_out = st.f;
  if (iters_out) *iters_out = st.iter;
  if (!std::isfinite(st.f)) return c->fail(BM_E_NONFINITE, "objective is not finite");
  return BM_OK;
}

BM_API int bm_objective(bm_ctx* c, const float* X, int64_t m, int32_t n, const float* C, int32_t k,
                        int32_t prec, double* f_out, int32_t* labels_out, int64_t* near_ties_out) {
  if (!c) return BM_E_ARG;
  if (!X || !C || !f_out) return c->fail(BM_E_ARG, "X, C and f_out are required");
  if (k < 1 || m < 1) return c->fail(BM_E_ARG, "need k >= 1, m >= 1");
  BM_TRY(check_prec(c, prec));
  BM_TRY(check_dim(c, n, k));
  HIP_TRY(c, hipSetDevice(c->device));
  BM_TRY(ensure(c, 1, n, k, 1));
  BM_TRY(ensure_objective(c, m));
  const int cp = round_up4(n);
  HIP_TRY(c, bm::launch_pad_centroids(c->stream, C, 0, n, cp, k, 1, P<float>(c->Cp), 0,
                                      P<float>(c->cn), 0));
  BatchView b;
  b.first = 0;
  b.njobs = 1;
  b.n = n;
  b.cp = cp;
  b.k = k;
  b.S = X;
  b.S_stride = 0;
  b.ld = n;
  b.sizes = {m};
  BM_TRY(objective_batch(c, b, labels_out, 0, (m + bm::kWG - 1) / bm::kWG, near_ties_out != nullptr,
                         prec));
  double f;
  BM_TRY(readback(c, c->fjob.p, sizeof(double), &f));
  *f_out = f;
  if (near_ties_out) {
    long long nn;
    BM_TRY(readback(c, c->nearjob.p, sizeof(long long), &nn));
    *near_ties_out = nn;
  }
  if (!std::isfinite(f)) return c->fail(BM_E_NONFINITE, "objective is not finite");
  return BM_OK;
}

BM_API int bm_objective_noalloc(bm_ctx* c, const float* X, int64_t m, int32_t n, const float* C,
                                int32_t k, int32_t prec, double* f_out, int32_t* labels_out,
                                int64_t* near_ties_out) {
  if (!c) return BM_E_ARG;
  if (!X || !C || !f_out) return c->fail(BM_E_ARG, "X, C and f_out are required");
  if (k < 1 || m < 1) return c->fail(BM_E_ARG, "need k >= 1, m >= 1");
  BM_TRY(check_prec(c, prec));
  BM_TRY(check_dim(c, n, k));
  if (!c->scratch) return c->fail(BM_E_STATE, "no static workspace on device %d", c->device);
  // layout of the static workspace (256-byte aligned pieces)
  const int cp = round_up4(n);
  const int64_t chunks = (m + bm::kWG - 1) / bm::kWG;
  const int64_t step = 2 * bm::kWG;  // the tile size rule of the allocating path
  const int64_t tile_steps = std::max<int64_t>(1, (m + step * 1024 - 1) / (step * 1024));
  const int64_t tile_pts = tile_steps * step;
  const int64_t ntiles = (m + tile_pts - 1) / tile_pts;
  auto al = [](int64_t v) { return (v + 255) & ~(int64_t)255; };
  const int64_t o_tf = 0;
  const int64_t o_near = o_tf + al(chunks * 8);
  const int64_t o_tjob = o_near + al(chunks * 4);
  const int64_t o_tidx = o_tjob + al(ntiles * 4);
  const int64_t o_cp = o_tidx + al(ntiles * 4);
  const int64_t o_cn = o_cp + al((int64_t)k * cp * 4);
  const int64_t o_size = o_cn + al((int64_t)k * 4);
  const int64_t o_f = o_size + 256;
  const int64_t o_nn = o_f + 256;
  const int64_t total = o_nn + 256;
  if (total > (int64_t)bm::kNoallocScratchBytes)
    return c->fail(BM_E_ARG,
                   "m = %lld, n = %d, k = %d needs %lld bytes of workspace; the static workspace "
                   "holds %zu",
                   (long long)m, n, k, (long long)total, bm::kNoallocScratchBytes);
  HIP_TRY(c, hipSetDevice(c->device));
  unsigned char* base = static_cast<unsigned char*>(c->scratch);
  double* tf = reinterpret_cast<double*>(base + o_tf);
  int32_t* tnear = near_ties_out ? reinterpret_cast<int32_t*>(base + o_near) : nullptr;
  int32_t* tjob = reinterpret_cast<int32_t*>(base + o_tjob);
  int32_t* tidx = reinterpret_cast<int32_t*>(base + o_tidx);
  float* Cp = reinterpret_cast<float*>(base + o_cp);
  float* cn = reinterpret_cast<float*>(base + o_cn);
  int64_t* sizes = reinterpret_cast<int64_t*>(base + o_size);
  double* f_dev = reinterpret_cast<double*>(base + o_f);
  long long* near_dev = reinterpret_cast<long long*>(base + o_nn);
  hipStream_t st = c->stream;
  HIP_TRY(c, bm::launch_noalloc_tiles(st, tjob, tidx, (int32_t)ntiles, sizes, m));
  HIP_TRY(c, bm::launch_pad_centroids(st, C, 0, n, cp, k, 1, Cp, 0, cn, 0));
  bm::AssignArgs a{};
  a.S = X;
  a.S_stride = 0;
  a.ld = n;
  a.n = n;
  a.cp = cp;
  a.k = k;
  a.tile_pts = (int32_t)tile_pts;
  a.max_chunks = (int32_t)chunks;
  a.vec = (n == cp && aligned16(X)) ? 1 : 0;
  a.s = sizes;
  a.tile_job = tjob;
  a.tile_idx = tidx;
  a.Cp = Cp;
  a.C_stride = (int64_t)k * cp;
  a.cn = cn;
  a.cn_stride = k;
  a.labels = labels_out;
  a.lab_stride = 0;
  a.tf = tf;
  a.tnear = tnear;
  if (cp > bm::kMaxRegDim && prec == BM_BF16)
    HIP_TRY(c, bm::launch_assign_wide_bf16(st, a, (int32_t)ntiles, false));
  else if (cp > bm::kMaxRegDim)
    HIP_TRY(c, bm::launch_assign_wide(st, a, (int32_t)ntiles, false));
  else
    HIP_TRY(c, bm::launch_assign(st, a, (int32_t)ntiles, false));
  HIP_TRY(c, bm::launch_reduce_f(st, tf, tnear, sizes, (int32_t)chunks, 1, f_dev,
                                 near_ties_out ? near_dev : nullptr));
  double f = 0.0;
  long long nn = 0;
  HIP_TRY(c, hipMemcpyAsync(&f, f_dev, sizeof f, hipMemcpyDeviceToHost, st));
  if (near_ties_out) HIP_TRY(c, hipMemcpyAsync(&nn, near_dev, sizeof nn, hipMemcpyDeviceToHost, st));
  HIP_TRY(c, hipStreamSynchronize(st));
  *f_out = f;
  if (near_ties_out) *near_ties_out = nn;
  if (!std::isfinite(f)) return c->fail(BM_E_NONFINITE, "objective is not finite");
  return BM_OK;
}

BM_API int bm_draw_size(const bm_params* params, uint32_t worker, int32_t t, const int64_t* bin_acc,
                        const int64_t* bin_passes, int64_t l_sum, int64_t l_count, int64_t* s_out,
                        int32_t* bin_out) {
  if (!params || !s_out || t < 0) return BM_E_ARG;
  if (params->size_policy < 0 || params->size_policy > BM_SIZE_SHRINK) return BM_E_ARG;
  if (params->size_policy == BM_SIZE_BINS && t > 0 && (!bin_acc || !bin_passes)) return BM_E_ARG;
  if (params->s_min < 1 || params->s_min > params->s_max) return BM_E_ARG;
  if (l_count < 0 || l_sum < 0) return BM_E_ARG;
  int32_t bin = 0;
  *s_out = draw_size(*params, worker, t, bin_acc, bin_passes, l_sum, l_count, &bin);
  if (bin_out) *bin_out = bin;
  return BM_OK;
}

BM_API void bm_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  bm::U64x4 x;
  for (int i = 0; i < 4; ++i) x.w[i] = ctr[i];
  const bm::U64x4 y = bm::philox4x64_10(x, key[0], key[1]);
  for (int i = 0; i < 4; ++i) out[i] = y.w[i];
}

BM_API int bm_set_profiling(bm_ctx* c, int on) {
  if (!c) return BM_E_ARG;
  c->prof = on != 0;
  c->stats = bm_stats{};
  return BM_OK;
}

BM_API int bm_set_tuning(bm_ctx* c, int on) {
  if (!c) return BM_E_ARG;
  c->tune = on != 0;
  c->tuned_tile.clear();
  return BM_OK;
}

BM_API int bm_get_stats(bm_ctx* c, bm_stats* out) {
  if (!c || !out) return BM_E_ARG;
  *out = c->stats;
  return BM_OK;
}

// ---------------------------------------------------------------------------
// Algorithm 1
// ---------------------------------------------------------------------------
BM_API int bm_serve(bm_ctx* c, const bm_dataset* datasets, int32_t nds, const bm_job* jobs,
                    int32_t njobs, const bm_serve_params* params, bm_job_result* results,
                    bm_serve_stats* stats) {
  if (!c) return BM_E_ARG;
  if (!datasets || !jobs || !params || !results || nds < 1 || nds > 16 || njobs < 0)
    return c->fail(BM_E_ARG, "bm_serve: need datasets (1..16), jobs, params and results");
  const bm_serve_params& sp = *params;
  if (sp.max_slots < 1 || sp.max_iter < 0 || !(sp.tol >= 0.0) || sp.n_candidates < 1 ||
      sp.n_candidates > 3 || sp.budget_bytes < 1)
    return c->fail(BM_E_ARG, "bm_serve: need max_slots >= 1, max_iter >= 0, tol >= 0, "
                             "n_candidates in 1..3, budget > 0");
  for (int d = 0; d < nds; ++d) {
    const bm_dataset& D = datasets[d];
    if (!D.X || D.m < 1 || D.m >= (1ll << 31)) return c->fail(BM_E_ARG, "dataset %d: need X and 1 <= m < 2^31", d);
  }
  for (int j = 0; j < njobs; ++j) {
    const bm_job& jb = jobs[j];
    if (jb.dataset < 0 || jb.dataset >= nds) return c->fail(BM_E_ARG, "job %d: dataset out of range", j);
    const bm_dataset& D = datasets[jb.dataset];
    if (jb.k < 1 || jb.k >= 1024 || jb.worker < 0 || jb.worker >= 1024)
      return c->fail(BM_E_ARG, "job %d: need 1 <= k < 1024 and 0 <= worker < 1024", j);
    if (jb.s < jb.k || jb.s > D.m) return c->fail(BM_E_ARG, "job %d: need k <= s <= m", j);
    if (!(jb.arrival >= 0.0)) return c->fail(BM_E_ARG, "job %d: arrival must be >= 0", j);
    BM_TRY(check_prec(c, jb.prec));
    BM_TRY(check_dim(c, D.n, jb.k));
  }
  HIP_TRY(c, hipSetDevice(c->device));
  std::memset(results, 0, (size_t)njobs * sizeof(bm_job_result));
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (njobs == 0) return BM_OK;
  return serve_impl(c, datasets, nds, jobs, njobs, sp, results, stats);
}

BM_API int bm_bigmeans_run(bm_ctx* c, const float* X, const bm_params* params, float* C_best_out,
                           int32_t* Y_out, bm_result* out, bm_trace_cb cb, void* user) {
  if (!c) return BM_E_ARG;
  BM_TRY(validate_params(c, params));
  if (!X || !C_best_out || !out) return c->fail(BM_E_ARG, "X, C_best_out and out are required");
  const bm_params p = *params;
  const int W = p.workers, k = p.k, n = p.n, cp = round_up4(n);
  const int64_t m = p.m;
  HIP_TRY(c, hipSetDevice(c->device));
  BM_TRY(ensure(c, p.s_max, n, k, W));
  BM_TRY(ensure_objective(c, m));
  hipStream_t st = c->stream;

  HIP_TRY(c, hipEventRecord(c->ev0, st));
  BM_TRY(compute_scales(c, X, m, n, n, cp, p.s_max));

  // incumbents: all centroids degenerate, f_hat = +inf (Algorithm 1, initialisation)
  HIP_TRY(c, hipMemsetAsync(c->Cinc.p, 0, (size_t)W * k * n * sizeof(float), st));
  HIP_TRY(c, hipMemsetAsync(c->deg_inc.p, 1, (size_t)W * k, st));
  std::vector<double> fhat(W, std::numeric_limits<double>::infinity());
  BM_TRY(upload(c, c->fhat.p, fhat.data(), W * sizeof(double)));
  std::vector<int64_t> s_cur(W, -1), s_new(W, 0);
  std::vector<double> iters_prev(W, 1.0);  // Lloyd iterations of each worker's last round
  std::vector<int32_t> bin_cur(W, 0);
  std::vector<int32_t> ndeg(W, k);
  int64_t bacc[kNBins] = {0}, bpass[kNBins] = {0};
  int64_t Lsum = 0, Lcount = 0;
  int64_t lloyd_dists = 0, lloyd_iters = 0;
  double lloyd_ms = 0.0;
  std::vector<uint64_t> sw(2 * (size_t)W);
  for (int w = 0; w < W; ++w) {
    sw[2 * w] = p.seed;
    sw[2 * w + 1] = (uint64_t)w;
  }
  std::vector<uint64_t> rk(4 * (size_t)W);
  const int64_t Sj = c->max_s * cp;  // floats between job samples
  float* Sbase = P<float>(c->S);

  // The batch a pass runs on: all workers together, or one worker alone.
  std::vector<std::pair<int, int>> groups;
  if (p.batched != 0)
    groups.push_back({0, W});
  else
    for (int w = 0; w < W; ++w) groups.push_back({w, 1});

  if (p.batched == 1) BM_TRY(upload(c, c->seed_worker.p, sw.data(), 2 * W * sizeof(uint64_t)));

  for (int t = 0; t < p.rounds_T; ++t) {
    int64_t rpass[kNBins] = {0}, racc[kNBins] = {0};
    for (int w = 0; w < W; ++w)
      s_new[w] = draw_size(p, (uint32_t)w, t, bacc, bpass, Lsum, Lcount, &bin_cur[w]);

    // persistent round: re-evaluations and all passes of all workers in one
    // launch (the multi-launch path below runs when it does not fit the device)
    bool round_done = false;
    std::vector<int32_t> rflag(W, 0);
    // Lloyd iterations expected this round: a least-squares line in log2(s)
    // through the previous round's workers (smaller samples need more
    // iterations); before any round, more for smaller samples as well.
    std::vector<double> iters_pred(W, 1.0);
    {
      double sx = 0, sy = 0, sxx = 0, sxy = 0;
      for (int w = 0; w < W && t > 0; ++w) {
        const double lx = std::log2((double)std::max<int64_t>(1, s_cur[w]));
        sx += lx;
        sy += iters_prev[w];
        sxx += lx * lx;
        sxy += lx * iters_prev[w];
      }
      const double den = W * sxx - sx * sx;
      for (int w = 0; w < W; ++w) {
        const double lx = std::log2((double)std::max<int64_t>(1, s_new[w]));
        double v;
        if (t == 0 || !(den > 1e-9)) v = t == 0 ? 1.0 + std::max(0.0, 16.0 - lx) : sy / W;
        else v = (sy - (W * sxy - sx * sy) / den * sx) / W + (W * sxy - sx * sy) / den * lx;
        iters_pred[w] = std::max(1.0, v);
      }
    }
    RoundResult rres;
    if (p.batched == 1 && c->round_ok && cp <= bm::kMaxRegDim) {  // wide points: multi-launch
      for (int w = 0; w < W; ++w) rflag[w] = (std::isfinite(fhat[w]) && s_new[w] != s_cur[w]) ? 1 : 0;
      const int rc = round_persistent(c, X, p, t, s_new, rflag, iters_pred, &rres);
      if (rc == kRoundNoFit) c->round_ok = false;
      else BM_TRY(rc);
      round_done = rc == BM_OK;
    }
    if (round_done) {
      lloyd_ms += rres.seconds * 1e3;
      int64_t round_dists = 0;
      for (int w = 0; w < W; ++w) {
        s_cur[w] = s_new[w];
        if (rflag[w]) fhat[w] = rres.recalc_f[w];
        iters_prev[w] = 0.0;
        for (int q = 0; q < p.passes_p; ++q) iters_prev[w] += rres.out[(size_t)w * p.passes_p + q].iters + 1;
        for (int q = 0; q < p.passes_p; ++q) {
          const bm::PassOut& o = rres.out[(size_t)w * p.passes_p + q];
          lloyd_iters += o.iters + 1;
          round_dists += (int64_t)(o.iters + 1) * s_cur[w] * k;
          rpass[bin_cur[w]] += 1;
          if (o.accepted) {
            fhat[w] = o.f;
            ndeg[w] = o.ndeg;
            Lsum += s_cur[w];
            Lcount += 1;
            racc[bin_cur[w]] += 1;
          }
        }
      }
      lloyd_dists += round_dists;
      if (c->prof) {
        c->stats.assign_launches += 1;
        c->stats.assign_seconds += rres.seconds;
        c->stats.assign_dists += round_dists;
      }
    } else {  // multi-launch passes
    // Re-evaluate incumbents whose sample size changed (Algorithm 1; Section 4.2).
    std::vector<int> rec;
    for (int w = 0; w < W; ++w)
      if (std::isfinite(fhat[w]) && s_new[w] != s_cur[w]) rec.push_back(w);
    if (!rec.empty()) {
      // job slot = worker slot; run each recalc worker as its own group slot
      for (size_t r = 0; r < rec.size(); ++r) {
        const int w = rec[r];
        round_keys((uint64_t)m, p.seed, (uint32_t)w, BM_PURPOSE_RECALC, (uint64_t)t, &rk[4 * w]);
      }
      BM_TRY(upload(c, P<uint64_t>(c->rkeys), rk.data(), 4 * W * sizeof(uint64_t)));
      // one batch over all worker slots; slots not re-evaluated get size 0
      std::vector<int64_t> szs(W, 0);
      for (int w : rec) szs[w] = s_new[w];
      BM_TRY(upload(c, P<int64_t>(c->sizes), szs.data(), W * sizeof(int64_t)));
      HIP_TRY(c, bm::launch_sample(st, X, m, n, W, p.s_max, P<int64_t>(c->sizes),
                                   P<uint64_t>(c->rkeys), P<int32_t>(c->idx), c->max_s, Sbase, Sj,
                                   cp));
      HIP_TRY(c, bm::launch_pad_centroids(st, P<float>(c->Cinc), (int64_t)k * n, n, cp, k, W,
                                          P<float>(c->Cp), (int64_t)k * cp, P<float>(c->cn), k));
      BatchView b;
      b.first = 0;
      b.njobs = W;
      b.n = n;
      b.cp = cp;
      b.k = k;
      b.S = Sbase;
      b.S_stride = Sj;
      b.ld = cp;
      b.sizes = szs;  // zero-size jobs produce no tiles and f = 0
      BM_TRY(objective_batch(c, b, nullptr, 0, c->max_chunks, false, p.prec));
      std::vector<double> fr(W);
      BM_TRY(readback(c, c->fjob.p, W * sizeof(double), fr.data()));
      for (int w : rec) fhat[w] = fr[w];
      BM_TRY(upload(c, c->fhat.p, fhat.data(), W * sizeof(double)));
    }
    for (int w = 0; w < W; ++w) s_cur[w] = s_new[w];

    for (int q = 0; q < p.passes_p; ++q) {
      const uint64_t g = (uint64_t)t * p.passes_p + q;
      for (int w = 0; w < W; ++w)
        round_keys((uint64_t)m, p.seed, (uint32_t)w, BM_PURPOSE_SAMPLE, g, &rk[4 * w]);
      BM_TRY(upload(c, P<uint64_t>(c->rkeys), rk.data(), 4 * W * sizeof(uint64_t)));
      for (const auto& grp : groups) {
        const int first = grp.first, J = grp.second;
        std::vector<int64_t> szs(s_cur.begin() + first, s_cur.begin() + first + J);
        int64_t smax = 0;
        int steps = 0;
        for (int j = 0; j < J; ++j) {
          smax = std::max(smax, szs[j]);
          steps = std::max(steps, ndeg[first + j]);
        }
        BM_TRY(upload(c, P<int64_t>(c->sizes) + first, szs.data(), J * sizeof(int64_t)));
        // sample S_w (Algorithm 1)
        HIP_TRY(c, bm::launch_sample(st, X, m, n, J, smax, P<int64_t>(c->sizes) + first,
                                     P<uint64_t>(c->rkeys) + 4 * first,
                                     P<int32_t>(c->idx) + (int64_t)first * c->max_s, c->max_s,
                                     Sbase + (int64_t)first * Sj, Sj, cp));
        HIP_TRY(c, bm::launch_copy_incumbent(st, P<float>(c->Cinc) + (int64_t)first * k * n,
                                             P<uint8_t>(c->deg_inc) + (int64_t)first * k, n, cp, k,
                                             J, P<float>(c->Cp) + (int64_t)first * k * cp,
                                             P<uint8_t>(c->deg_work) + (int64_t)first * k));
        BatchView b;
        b.first = first;
        b.njobs = J;
        b.n = n;
        b.cp = cp;
        b.k = k;
        b.S = Sbase + (int64_t)first * Sj;
        b.S_stride = Sj;
        b.ld = cp;
        b.sizes = szs;
        // K-means++ for degenerate centroids
        KppBatch kb{sw.data() + 2 * first, g, p.n_candidates, steps, nullptr};
        BM_TRY(kpp_batch(c, b, kb));
        // Lloyd with acceptance (the finalize of each job's last iteration
        // replaces the incumbent on a strict improvement)
        HIP_TRY(c, hipEventRecord(c->ev1, st));
        std::vector<JobState> fin;
        BM_TRY(lloyd_batch(c, b, p.max_iter, p.tol, nullptr, 0, true, &fin, p.prec));
        HIP_TRY(c, hipEventRecord(c->ev2, st));
        HIP_TRY(c, hipEventSynchronize(c->ev2));
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev1, c->ev2));
        lloyd_ms += ms;
        for (int j = 0; j < J; ++j) {
          const int w = first + j;
          lloyd_iters += fin[j].iter + 1;
          lloyd_dists += (int64_t)(fin[j].iter + 1) * s_cur[w] * k;
          rpass[bin_cur[w]] += 1;
          if (fin[j].accepted) {
            fhat[w] = fin[j].f;
            ndeg[w] = fin[j].ndeg;
            Lsum += s_cur[w];
            Lcount += 1;
            racc[bin_cur[w]] += 1;
          }
        }
      }
    }
    }  // multi-launch passes
    for (int i = 0; i < kNBins; ++i) {
      bacc[i] += racc[i];
      bpass[i] += rpass[i];
    }
    if (cb) {
      HIP_TRY(c, hipEventRecord(c->ev1, st));
      HIP_TRY(c, hipEventSynchronize(c->ev1));
      float ms = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
      cb(user, t, P<float>(c->Cinc), fhat.data(), s_cur.data(), Lsum, Lcount, ms * 1e-3);
    }
  }

  // s_opt: round-half-up mean of L (Algorithm 1; Section 4.2 "simple mean")
  const int64_t s_opt = Lcount > 0 ? (Lsum + Lcount / 2) / Lcount : p.s_max;
  // one shared sample of size s_opt; every incumbent scored on it
  round_keys((uint64_t)m, p.seed, BM_FINAL_WORKER, BM_PURPOSE_FINAL, 0, rk.data());
  BM_TRY(upload(c, P<int64_t>(c->sizes), &s_opt, sizeof(int64_t)));
  BM_TRY(upload(c, P<uint64_t>(c->rkeys), rk.data(), 4 * sizeof(uint64_t)));
  HIP_TRY(c, bm::launch_sample(st, X, m, n, 1, s_opt, P<int64_t>(c->sizes), P<uint64_t>(c->rkeys),
                               P<int32_t>(c->idx), c->max_s, Sbase, Sj, cp));
  HIP_TRY(c, bm::launch_pad_centroids(st, P<float>(c->Cinc), (int64_t)k * n, n, cp, k, W,
                                      P<float>(c->Cp), (int64_t)k * cp, P<float>(c->cn), k));
  BatchView fb;
  fb.first = 0;
  fb.njobs = W;
  fb.n = n;
  fb.cp = cp;
  fb.k = k;
  fb.S = Sbase;
  fb.S_stride = 0;  // shared sample
  fb.ld = cp;
  fb.sizes.assign(W, s_opt);
  BM_TRY(objective_batch(c, fb, nullptr, 0, c->max_chunks, false, p.prec));
  std::vector<double> ffin(W);
  BM_TRY(readback(c, c->fjob.p, W * sizeof(double), ffin.data()));
  int best = -1;
  for (int w = 0; w < W; ++w) {
    if (!std::isfinite(fhat[w])) ffin[w] = std::numeric_limits<double>::infinity();
    // smallest value, NaN last, lowest worker on ties
    if (best < 0) {
      best = w;
      continue;
    }
    const bool nb = std::isnan(ffin[best]), nw = std::isnan(ffin[w]);
    if ((nb && !nw) || (!nw && !nb && ffin[w] < ffin[best])) best = w;
  }
  // full assignment of X with C_best (Algorithm 1, last step)
  HIP_TRY(c, hipMemcpyAsync(C_best_out, P<float>(c->Cinc) + (int64_t)best * k * n,
                            (size_t)k * n * sizeof(float), hipMemcpyDeviceToDevice, st));
  HIP_TRY(c, bm::launch_pad_centroids(st, C_best_out, 0, n, cp, k, 1, P<float>(c->Cp), 0,
                                      P<float>(c->cn), 0));
  BatchView xb;
  xb.first = 0;
  xb.njobs = 1;
  xb.n = n;
  xb.cp = cp;
  xb.k = k;
  xb.S = X;
  xb.S_stride = 0;
  xb.ld = n;
  xb.sizes = {m};
  BM_TRY(objective_batch(c, xb, Y_out, 0, (m + bm::kWG - 1) / bm::kWG, false, p.prec));
  double f_full;
  BM_TRY(readback(c, c->fjob.p, sizeof(double), &f_full));
  HIP_TRY(c, hipEventRecord(c->ev1, st));
  HIP_TRY(c, hipEventSynchronize(c->ev1));
  float total_ms = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&total_ms, c->ev0, c->ev1));

  out->f_full = f_full;
  out->f_best_sample = ffin[best];
  out->s_opt = s_opt;
  out->improvements = Lcount;
  out->lloyd_dists = lloyd_dists;
  out->lloyd_iters = lloyd_iters;
  out->best_worker = best;
  out->pad_ = 0;
  out->gpu_seconds = total_ms * 1e-3;
  out->lloyd_seconds = lloyd_ms * 1e-3;
  if (!std::isfinite(f_full)) return c->fail(BM_E_NONFINITE, "f(C_best, X) is not finite");
  return BM_OK;
}

}  // extern "C"
