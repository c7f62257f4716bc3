"""ctypes declarations of libbigmeans.so (the C ABI in include/bigmeans.h).

Loading fails loudly if the library has not been built: there is no other
implementation behind these names.
"""

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbigmeans.so")

BM_OK, BM_E_ARG, BM_E_NOMEM, BM_E_HIP, BM_E_NONFINITE, BM_E_STATE = 0, -1, -2, -3, -4, -5
BM_FP32, BM_BF16 = 0, 1
BM_SIZE_UNIFORM, BM_SIZE_FIXED, BM_SIZE_LOGUNIFORM, BM_SIZE_BINS, BM_SIZE_SHRINK = 0, 1, 2, 3, 4
BM_PURPOSE_SIZE, BM_PURPOSE_SAMPLE, BM_PURPOSE_KMPP, BM_PURPOSE_RECALC, BM_PURPOSE_FINAL = 1, 2, 3, 4, 5
BM_FINAL_WORKER = 0xFFFFFF

STATUS_NAMES = {BM_OK: "BM_OK", BM_E_ARG: "BM_E_ARG", BM_E_NOMEM: "BM_E_NOMEM",
                BM_E_HIP: "BM_E_HIP", BM_E_NONFINITE: "BM_E_NONFINITE", BM_E_STATE: "BM_E_STATE"}


class Params(ct.Structure):
    _fields_ = [("m", ct.c_int64), ("s_min", ct.c_int64), ("s_max", ct.c_int64),
                ("n", ct.c_int32), ("k", ct.c_int32), ("workers", ct.c_int32),
                ("rounds_T", ct.c_int32), ("passes_p", ct.c_int32), ("max_iter", ct.c_int32),
                ("n_candidates", ct.c_int32), ("size_policy", ct.c_int32), ("prec", ct.c_int32),
                ("batched", ct.c_int32), ("tol", ct.c_double), ("seed", ct.c_uint64)]


class Result(ct.Structure):
    _fields_ = [("f_full", ct.c_double), ("f_best_sample", ct.c_double),
                ("s_opt", ct.c_int64), ("improvements", ct.c_int64),
                ("lloyd_dists", ct.c_int64), ("lloyd_iters", ct.c_int64),
                ("best_worker", ct.c_int32), ("pad_", ct.c_int32),
                ("gpu_seconds", ct.c_double), ("lloyd_seconds", ct.c_double)]


class Stats(ct.Structure):
    _fields_ = [("assign_launches", ct.c_int64), ("assign_dists", ct.c_int64),
                ("assign_seconds", ct.c_double), ("finalize_seconds", ct.c_double)]


class Dataset(ct.Structure):
    _fields_ = [("X", ct.c_void_p), ("m", ct.c_int64), ("n", ct.c_int32), ("pad_", ct.c_int32)]


class Job(ct.Structure):
    _fields_ = [("arrival", ct.c_double), ("s", ct.c_int64), ("dataset", ct.c_int32),
                ("k", ct.c_int32), ("worker", ct.c_int32), ("prec", ct.c_int32)]


class JobResult(ct.Structure):
    _fields_ = [("f", ct.c_double), ("f_incumbent", ct.c_double), ("admitted", ct.c_double),
                ("finished", ct.c_double), ("iters", ct.c_int32), ("accepted", ct.c_int32),
                ("ndeg", ct.c_int32), ("pad_", ct.c_int32)]


class ServeParams(ct.Structure):
    _fields_ = [("seed", ct.c_uint64), ("budget_bytes", ct.c_int64), ("max_slots", ct.c_int32),
                ("max_iter", ct.c_int32), ("n_candidates", ct.c_int32), ("paced", ct.c_int32),
                ("tol", ct.c_double)]


class ServeStats(ct.Structure):
    _fields_ = [("seconds", ct.c_double), ("steps", ct.c_int64), ("peak_running", ct.c_int64),
                ("peak_bytes", ct.c_int64), ("slot_bytes", ct.c_int64)]


TRACE_CB = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_int32, ct.c_void_p,
                        ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64), ct.c_int64, ct.c_int64,
                        ct.c_double)

# (name, restype, argtypes) for every function the header declares.
SIGNATURES = [
    ("bm_version", ct.c_int, []),
    ("bm_create", ct.c_int, [ct.c_int, ct.c_void_p, ct.POINTER(ct.c_void_p)]),
    ("bm_destroy", None, [ct.c_void_p]),
    ("bm_strerror", ct.c_char_p, [ct.c_void_p]),
    ("bm_reserve", ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int32]),
    ("bm_sample", ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int64,
                             ct.c_uint64, ct.c_uint32, ct.c_uint32, ct.c_uint64, ct.c_void_p,
                             ct.c_void_p]),
    ("bm_seed", ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32,
                           ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_uint64, ct.c_uint32,
                           ct.c_uint64, ct.c_void_p]),
    ("bm_lloyd", ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32,
                            ct.c_void_p, ct.c_int32, ct.c_double, ct.c_int32,
                            ct.POINTER(ct.c_double), ct.POINTER(ct.c_int32), ct.c_void_p,
                            ct.c_void_p]),
    ("bm_objective", ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_void_p,
                                ct.c_int32, ct.c_int32, ct.POINTER(ct.c_double), ct.c_void_p,
                                ct.POINTER(ct.c_int64)]),
    ("bm_objective_noalloc", ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32,
                                        ct.c_void_p, ct.c_int32, ct.c_int32,
                                        ct.POINTER(ct.c_double), ct.c_void_p,
                                        ct.POINTER(ct.c_int64)]),
    ("bm_bigmeans_run", ct.c_int, [ct.c_void_p, ct.c_void_p, ct.POINTER(Params), ct.c_void_p,
                                   ct.c_void_p, ct.POINTER(Result), TRACE_CB, ct.c_void_p]),
    ("bm_draw_size", ct.c_int, [ct.POINTER(Params), ct.c_uint32, ct.c_int32,
                                ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64), ct.c_int64,
                                ct.c_int64, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32)]),
    ("bm_serve", ct.c_int, [ct.c_void_p, ct.POINTER(Dataset), ct.c_int32, ct.POINTER(Job),
                            ct.c_int32, ct.POINTER(ServeParams), ct.POINTER(JobResult),
                            ct.POINTER(ServeStats)]),
    ("bm_set_profiling", ct.c_int, [ct.c_void_p, ct.c_int]),
    ("bm_set_tuning", ct.c_int, [ct.c_void_p, ct.c_int]),
    ("bm_get_stats", ct.c_int, [ct.c_void_p, ct.POINTER(Stats)]),
    ("bm_philox4x64", None, [ct.POINTER(ct.c_uint64), ct.POINTER(ct.c_uint64),
                             ct.POINTER(ct.c_uint64)]),
]

_lib = None


def load():
    """Load libbigmeans.so (built by paper_2403_18766_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it first (python -m paper_2403_18766_amd.build); "
            "there is no fallback implementation")
    lib = ct.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
