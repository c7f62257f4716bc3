"""CPU oracle for competitive stochastic-sample-size Big-means.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, FP64 statement of
what the GPU path computes, written from the paper (Mussabayev & Mussabayev,
"Superior Parallel Big Data Clustering through Competitive Stochastic Sample
Size Optimization in Big-means", arXiv 2403.18766).  Only the tests, the
``smoke()`` check and the ``cpu_baseline`` leg of the benchmark may import it.
The product library never calls into it and shares no code with it.

Modules
-------
rng       Philox4x64-10 block function, the conversions used by the method's
          random draws, and the Feistel sampler (sampling without replacement).
kmeans    MSSC objective (Eq. 1), nearest-centre assignment, Lloyd iterations
          and greedy K-means++ seeding, in FP64.
bigmeans  Algorithm 1 (competitive sample-size Big-means) and its size draws.

Where the paper is silent (random-number contract, tie breaks, empty
clusters, rounding of the mean sample size, ...) each function states the
reading it takes.
"""

from . import rng, kmeans, bigmeans  # noqa: F401
