"""MI355X (gfx950) implementation of the hot path of competitive
stochastic-sample-size Big-means (arXiv 2403.18766): sampling, greedy
K-means++, Lloyd iterations and the MSSC objective in hand-written HIP behind
the C ABI of include/bigmeans.h (libbigmeans.so), with Algorithm 1 driven by
the library's host code.

The binding (``api``) loads the library on first use and raises if it is
missing; ``datagen`` holds the seeded synthetic workloads.
"""

from ._lib import (BM_FP32, BM_PURPOSE_FINAL, BM_PURPOSE_KMPP, BM_PURPOSE_RECALC,  # noqa: F401
                   BM_PURPOSE_SAMPLE, BM_PURPOSE_SIZE, BM_SIZE_BINS, BM_SIZE_FIXED,
                   BM_SIZE_LOGUNIFORM, BM_SIZE_UNIFORM, LIB_PATH)


def __getattr__(name):
    if name in ("sample", "seed", "lloyd", "objective", "bigmeans_run", "RunParams",
                "draw_size", "philox4x64", "reserve", "BigmeansError"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
