"""Python binding of libbigmeans: torch tensors in, C ABI calls out.

Only argument marshalling lives here: every step of the clustering runs in
the library's HIP kernels.  Tensors must be on a ROCm ("cuda") device,
contiguous, float32 (points, centroids), int32 (labels, indices) or uint8
(degenerate flags).  Work is enqueued on torch's current stream of that
device; a context is created per (device, stream) and reused.
"""

import atexit
import ctypes as ct
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import (BM_BF16, BM_FP32, BM_PURPOSE_SAMPLE, BM_SIZE_UNIFORM, BM_E_NONFINITE, Params as _CParams,
                   Result as _CResult, STATUS_NAMES, TRACE_CB)


class BigmeansError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_contexts = {}


def _release_contexts():
    """At interpreter exit: finish each context's work and release its
    workspace, pinned staging and events while the HIP runtime is still up."""
    lib = _lib._lib
    if lib is None:
        return
    for c in list(_contexts.values()):
        lib.bm_destroy(c)
    _contexts.clear()


atexit.register(_release_contexts)


def _ctx(device):
    lib = _lib.load()
    stream = torch.cuda.current_stream(device)
    key = (device.index, stream.cuda_stream)
    c = _contexts.get(key)
    if c is None:
        out = ct.c_void_p()
        rc = lib.bm_create(device.index, ct.c_void_p(stream.cuda_stream), ct.byref(out))
        if rc != 0:
            raise BigmeansError(rc, f"bm_create(device={device.index}) failed")
        c = out.value
        _contexts[key] = c
    return lib, c


def _check(lib, ctx, rc, allow_nonfinite=False):
    if rc == 0 or (allow_nonfinite and rc == BM_E_NONFINITE):
        return rc
    raise BigmeansError(rc, lib.bm_strerror(ctx).decode())


def _dev(t, dtype, name, ndim=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")
    return t


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else ct.c_void_p(0)


def reserve(device, max_s, max_n, max_k, max_jobs=1):
    """Allocate the workspace up front (bm_reserve)."""
    device = torch.device(device)
    lib, c = _ctx(device)
    _check(lib, c, lib.bm_reserve(c, int(max_s), int(max_n), int(max_k), int(max_jobs)))


def sample(X, s, seed=0, worker=0, purpose=BM_PURPOSE_SAMPLE, g=0, gather=True):
    """bm_sample: indices (int32) of a sample of s distinct rows of X and, with
    gather, the rows themselves."""
    _dev(X, torch.float32, "X", 2)
    m, n = X.shape
    lib, c = _ctx(X.device)
    idx = torch.empty(int(s), dtype=torch.int32, device=X.device)
    S = torch.empty((int(s), n), dtype=torch.float32, device=X.device) if gather else None
    _check(lib, c, lib.bm_sample(c, _ptr(X), m, n, int(s), int(seed), int(worker), int(purpose),
                                 int(g), _ptr(idx), _ptr(S)))
    return idx, S


def seed(S, C, degenerate, n_candidates=3, seed=0, worker=0, g=0, return_picks=False):
    """bm_seed on copies of C and degenerate: greedy K-means++ for the
    degenerate centroids.  Returns (C, degenerate[, picks])."""
    _dev(S, torch.float32, "S", 2)
    s, n = S.shape
    C = _dev(C, torch.float32, "C", 2).clone()
    deg = _dev(degenerate, torch.uint8, "degenerate", 1).clone()
    k = C.shape[0]
    if C.shape[1] != n or deg.shape[0] != k:
        raise ValueError("shape mismatch between S, C and degenerate")
    picks = torch.empty((k, 4), dtype=torch.int32, device=S.device) if return_picks else None
    lib, c = _ctx(S.device)
    _check(lib, c, lib.bm_seed(c, _ptr(S), s, n, k, _ptr(C), _ptr(deg), int(n_candidates),
                               int(seed), int(worker), int(g), _ptr(picks)))
    return (C, deg, picks) if return_picks else (C, deg)


def lloyd(S, C0, max_iter=300, tol=1e-4, labels=True, prec=BM_FP32):
    """bm_lloyd from a copy of C0.  Returns a dict with C, f, iters, deg, labels."""
    _dev(S, torch.float32, "S", 2)
    s, n = S.shape
    C = _dev(C0, torch.float32, "C0", 2).clone()
    k = C.shape[0]
    if C.shape[1] != n:
        raise ValueError("C0 and S differ in dimension")
    deg = torch.empty(k, dtype=torch.uint8, device=S.device)
    lab = torch.empty(s, dtype=torch.int32, device=S.device) if labels else None
    f = ct.c_double()
    iters = ct.c_int32()
    lib, c = _ctx(S.device)
    rc = lib.bm_lloyd(c, _ptr(S), s, n, k, _ptr(C), int(max_iter), float(tol), int(prec),
                      ct.byref(f), ct.byref(iters), _ptr(deg), _ptr(lab))
    _check(lib, c, rc, allow_nonfinite=True)
    return {"C": C, "f": f.value, "iters": iters.value, "deg": deg, "labels": lab}


def objective(X, C, labels=True, near_ties=True, prec=BM_FP32):
    """bm_objective: (f, labels or None, near-tie count or None)."""
    _dev(X, torch.float32, "X", 2)
    _dev(C, torch.float32, "C", 2)
    m, n = X.shape
    k = C.shape[0]
    if C.shape[1] != n:
        raise ValueError("C and X differ in dimension")
    lab = torch.empty(m, dtype=torch.int32, device=X.device) if labels else None
    f = ct.c_double()
    near = ct.c_int64()
    lib, c = _ctx(X.device)
    rc = lib.bm_objective(c, _ptr(X), m, n, _ptr(C), k, int(prec), ct.byref(f), _ptr(lab),
                          ct.byref(near) if near_ties else None)
    _check(lib, c, rc, allow_nonfinite=True)
    return f.value, lab, (near.value if near_ties else None)


def objective_noalloc(X, C, labels_out=None, near_ties=True, prec=BM_FP32):
    """bm_objective_noalloc: bm_objective with the library's static workspace
    (no allocation in the call).  labels_out: an int32 device tensor of m
    entries, or None.  Returns (f, near-tie count or None)."""
    _dev(X, torch.float32, "X", 2)
    _dev(C, torch.float32, "C", 2)
    m, n = X.shape
    k = C.shape[0]
    if C.shape[1] != n:
        raise ValueError("C and X differ in dimension")
    if labels_out is not None:
        _dev(labels_out, torch.int32, "labels_out", 1)
        if labels_out.shape[0] != m:
            raise ValueError("labels_out must have one entry per row of X")
    f = ct.c_double()
    near = ct.c_int64()
    lib, c = _ctx(X.device)
    rc = lib.bm_objective_noalloc(c, _ptr(X), m, n, _ptr(C), k, int(prec), ct.byref(f),
                                  _ptr(labels_out), ct.byref(near) if near_ties else None)
    _check(lib, c, rc, allow_nonfinite=True)
    return f.value, (near.value if near_ties else None)


@dataclass
class RunParams:
    """Parameters of Algorithm 1 (defaults are those of Section 5)."""
    k: int
    workers: int
    rounds_T: int
    s_min: int
    s_max: int
    passes_p: int = 10
    max_iter: int = 300
    tol: float = 1e-4
    n_candidates: int = 3
    size_policy: int = BM_SIZE_UNIFORM
    seed: int = 0
    batched: int = 1   # 1 persistent rounds, 2 one launch per Lloyd step, 0 one worker per launch
    prec: int = BM_FP32  # BM_BF16: split-BF16 matrix-core distances for wide points

    def c_struct(self, m, n):
        return _CParams(m=int(m), s_min=int(self.s_min), s_max=int(self.s_max), n=int(n),
                        k=int(self.k), workers=int(self.workers), rounds_T=int(self.rounds_T),
                        passes_p=int(self.passes_p), max_iter=int(self.max_iter),
                        n_candidates=int(self.n_candidates), size_policy=int(self.size_policy),
                        prec=int(self.prec), batched=int(self.batched), tol=float(self.tol),
                        seed=int(self.seed))


def bigmeans_run(X, params, labels=True, trace=None):
    """bm_bigmeans_run (Algorithm 1).  `trace(round, C_all, fhat, sizes, t,
    l_sum, l_count)` is called after every round with a copy of the W
    incumbents (k x n each), the sum and count of the list L so far, and the
    device time since the start of the run."""
    _dev(X, torch.float32, "X", 2)
    m, n = X.shape
    k = params.k
    C = torch.empty((k, n), dtype=torch.float32, device=X.device)
    Y = torch.empty(m, dtype=torch.int32, device=X.device) if labels else None
    cp = params.c_struct(m, n)
    res = _CResult()
    lib, c = _ctx(X.device)
    W = params.workers
    cb = TRACE_CB(0)
    if trace is not None:
        def _cb(user, rnd, c_all, fhat, sizes, l_sum, l_count, tsec):
            # a device-to-device copy of the incumbents on the library's stream
            snap = torch.empty((W, k, n), dtype=torch.float32, device=X.device)
            torch.cuda.synchronize(X.device)       # snap's allocation is complete
            _copy_device(snap, c_all, W * k * n * 4)
            trace(rnd, snap, [fhat[i] for i in range(W)], [sizes[i] for i in range(W)], tsec,
                  l_sum, l_count)
        cb = TRACE_CB(_cb)
    rc = lib.bm_bigmeans_run(c, _ptr(X), ct.byref(cp), _ptr(C), _ptr(Y), ct.byref(res), cb, None)
    _check(lib, c, rc, allow_nonfinite=True)
    out = {f: getattr(res, f) for f, _ in _CResult._fields_ if f != "pad_"}
    out["C_best"] = C
    out["Y"] = Y
    return out


_hip = None


def _copy_device(dst, src_ptr, nbytes):
    """Copy nbytes of device memory at src_ptr into tensor dst (same device;
    the library has synchronised its stream before calling the trace)."""
    global _hip
    if _hip is None:
        _hip = ct.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = ct.c_int
        _hip.hipMemcpy.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_int]
    rc = _hip.hipMemcpy(ct.c_void_p(dst.data_ptr()), ct.c_void_p(src_ptr), nbytes,
                        3)  # hipMemcpyDeviceToDevice
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")


def set_profiling(device, on=True):
    """bm_set_profiling on the context of (device, current stream); resets counters."""
    device = torch.device(device)
    lib, c = _ctx(device)
    _check(lib, c, lib.bm_set_profiling(c, 1 if on else 0))


def set_tuning(device, on=True):
    """bm_set_tuning on the context of (device, current stream): tile-size timing
    of the one-step-per-launch Lloyd paths on or off (kept choices cleared;
    serving always takes the heuristic tile size)."""
    device = torch.device(device)
    lib, c = _ctx(device)
    _check(lib, c, lib.bm_set_tuning(c, 1 if on else 0))


def get_stats(device):
    """bm_get_stats: dict of the Lloyd kernel timing counters."""
    device = torch.device(device)
    lib, c = _ctx(device)
    st = _lib.Stats()
    _check(lib, c, lib.bm_get_stats(c, ct.byref(st)))
    return {f: getattr(st, f) for f, _ in _lib.Stats._fields_}


def draw_size(params, m, n, worker, t, bin_acc=None, bin_passes=None, l_sum=0, l_count=0):
    """bm_draw_size (host only): the sample size of `worker` in round t and its bin."""
    lib = _lib.load()
    cp = params.c_struct(m, n)
    arr = ct.c_int64 * 5
    ba = arr(*(bin_acc or [0] * 5))
    bp = arr(*(bin_passes or [0] * 5))
    s = ct.c_int64()
    b = ct.c_int32()
    rc = lib.bm_draw_size(ct.byref(cp), int(worker), int(t), ba, bp, int(l_sum), int(l_count),
                          ct.byref(s), ct.byref(b))
    if rc != 0:
        raise BigmeansError(rc, "bm_draw_size failed")
    return s.value, b.value


def philox4x64(ctr, key):
    """bm_philox4x64 (host only): one Philox4x64-10 block."""
    lib = _lib.load()
    c4 = (ct.c_uint64 * 4)(*[int(v) & ((1 << 64) - 1) for v in ctr])
    k2 = (ct.c_uint64 * 2)(*[int(v) & ((1 << 64) - 1) for v in key])
    o4 = (ct.c_uint64 * 4)()
    lib.bm_philox4x64(c4, k2, o4)
    return tuple(int(v) for v in o4)


def serve(datasets, jobs, seed=0, budget_bytes=200 << 30, max_slots=64, max_iter=300, tol=1e-4,
          n_candidates=3, paced=False):
    """bm_serve: run single-pass jobs of competing workers with continuous
    batching.  `datasets` are device tensors (m x n float32); `jobs` is a list
    of dicts with keys arrival (s), s, dataset, k, worker.  Returns (results,
    stats): one dict per job (f, f_incumbent, admitted, finished, iters,
    accepted, ndeg) and the call's statistics."""
    if not datasets:
        raise ValueError("need at least one dataset")
    dev = datasets[0].device
    lib, c = _ctx(dev)
    ds = (_lib.Dataset * len(datasets))()
    for i, X in enumerate(datasets):
        X = _dev(X, torch.float32, "X", 2)
        ds[i].X = X.data_ptr()
        ds[i].m = X.shape[0]
        ds[i].n = X.shape[1]
    nj = len(jobs)
    jb = (_lib.Job * max(1, nj))()
    for i, j in enumerate(jobs):
        jb[i].arrival = float(j.get("arrival", 0.0))
        jb[i].s = int(j["s"])
        jb[i].dataset = int(j["dataset"])
        jb[i].k = int(j["k"])
        jb[i].worker = int(j["worker"])
        jb[i].prec = int(j.get("prec", BM_FP32))
    sp = _lib.ServeParams(seed=seed, budget_bytes=int(budget_bytes), max_slots=max_slots,
                          max_iter=max_iter, n_candidates=n_candidates, paced=1 if paced else 0,
                          tol=tol)
    res = (_lib.JobResult * max(1, nj))()
    st = _lib.ServeStats()
    rc = lib.bm_serve(c, ds, len(datasets), jb, nj, ct.byref(sp), res, ct.byref(st))
    _check(lib, c, rc)
    out = [{"f": r.f, "f_incumbent": r.f_incumbent, "admitted": r.admitted,
            "finished": r.finished, "iters": r.iters, "accepted": bool(r.accepted),
            "ndeg": r.ndeg} for r in res[:nj]]
    stats = {"seconds": st.seconds, "steps": st.steps, "peak_running": st.peak_running,
             "peak_bytes": st.peak_bytes, "slot_bytes": st.slot_bytes}
    return out, stats
