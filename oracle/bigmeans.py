"""Algorithm 1 (competitive stochastic-sample-size Big-means), oracle side.

Test infrastructure only.  Follows Section 4.2 (Algorithm 1 and the text
after it) and Section 4.3, with the parameters of Section 5.

Structure (rounds t < T, workers w, passes q < p, global pass g = t*p + q):
  * each worker starts with all k centroids degenerate and f_hat = +inf;
  * at the start of every round a worker draws its sample size s_w; if it
    already has an incumbent and the size changed, its f_hat is re-evaluated
    on a fresh sample of the new size (Section 4.2: any change of s_w
    requires recomputing the incumbent's objective);
  * each pass draws a new sample S_w, re-seeds the degenerate centroids with
    greedy K-means++ on S_w, runs K-means from the incumbent, and accepts the
    result only if its objective on S_w is strictly below f_hat (a NaN is
    never accepted); every acceptance appends s_w to the list L;
  * at the end s_opt = mean of L (Section 4.2: the simple mean, rounded half
    up to an integer), one shared sample of size s_opt re-scores every
    worker's incumbent, the worker with the smallest value wins (lowest
    worker on ties), and every point of X is assigned to its centroids.

Workers are independent apart from L; running them in lockstep rounds, as
here, is one valid interleaving.  The BINS size policy reads L's statistics
from earlier rounds only, which keeps it deterministic.

Size policies (the paper draws s_w uniformly in [s_min, s_max]):
  UNIFORM     s_min + mulhi(w0, s_max - s_min + 1)
  FIXED       s_min (s_min == s_max)
  LOGUNIFORM  floor(exp(ln a + u(w0) * (ln(b + 1) - ln a))) clamped to [a, b]
  BINS        round 0 as LOGUNIFORM; later rounds choose one of 5 equal-width
              bins of ln s with probability proportional to (a_i + 1)/(n_i + 2)
              (a_i acceptances and n_i passes seen in bin i so far), then draw
              log-uniformly inside the bin.
  SHRINK      (the exploration-then-exploitation the paper leaves to future
              work, Section 7) round 0, or while L is empty, as LOGUNIFORM;
              later rounds draw log-uniformly in [mu / r_t, mu r_t] clamped to
              [a, b + 1), where mu is the round-half-up mean of L over earlier
              rounds and ln r_t = (ln(b + 1) - ln a) / 2 * 2^-t.
with w = B((t, 0, 0, 0), key(seed, worker, SIZE)).
"""

import math
from dataclasses import dataclass

import numpy as np

from . import kmeans, rng

SIZE_UNIFORM, SIZE_FIXED, SIZE_LOGUNIFORM, SIZE_BINS, SIZE_SHRINK = 0, 1, 2, 3, 4
N_BINS = 5


@dataclass
class Params:
    k: int
    workers: int
    rounds_T: int
    passes_p: int = 10
    s_min: int = 0
    s_max: int = 0
    size_policy: int = SIZE_UNIFORM
    max_iter: int = 300
    tol: float = 1e-4
    n_candidates: int = 3
    seed: int = 0


def paper_size_range(s, m):
    """Section 5: s_min = 0.5 s (rounded up), s_max = min(2 s, m)."""
    return (int(s) + 1) // 2, min(2 * int(s), int(m))


def _log_edges(a, b):
    la = math.log(a)
    return la, (math.log(b + 1) - la)


def draw_size(params, worker, t, bin_stats, l_stats=None):
    """Sample size of `worker` for round t, and the bin (0..4) it falls in.
    bin_stats: BINS statistics of earlier rounds; l_stats: (sum, count) of
    the list L over earlier rounds (SHRINK)."""
    a, b = int(params.s_min), int(params.s_max)
    w = rng.philox_block_scalar((t, 0, 0, 0),
                                rng.stream_key(params.seed, worker, rng.PURPOSE_SIZE))
    pol = params.size_policy
    if pol == SIZE_UNIFORM:
        return a + rng.mulhi(w[0], b - a + 1), 0
    if pol == SIZE_FIXED:
        return a, 0
    la, width = _log_edges(a, b)
    if pol == SIZE_SHRINK and t > 0 and l_stats is not None and l_stats[1] > 0:
        l_sum, l_count = l_stats
        mu = (l_sum + l_count // 2) // l_count
        lm = math.log(mu)
        half = math.ldexp(width / 2.0, -t)
        lo = max(la, lm - half)
        hi = min(la + width, lm + half)
        v = lo + rng.u01(w[0]) * (hi - lo)
        s = int(math.floor(math.exp(v)))
        return min(max(s, a), b), min(N_BINS - 1, int((v - la) / width * N_BINS))
    if pol in (SIZE_LOGUNIFORM, SIZE_SHRINK) or (pol == SIZE_BINS and t == 0):
        u = rng.u01(w[0])
        s = int(math.floor(math.exp(la + u * width)))
        return min(max(s, a), b), min(N_BINS - 1, int(u * N_BINS))
    if pol == SIZE_BINS:
        weights = [(bin_stats["acc"][i] + 1.0) / (bin_stats["passes"][i] + 2.0)
                   for i in range(N_BINS)]
        total = 0.0
        for wt in weights:              # the weights' sum, added in bin order
            total += wt
        x = rng.u01(w[1]) * total
        acc, i_bin = 0.0, N_BINS - 1
        for i in range(N_BINS):
            acc += weights[i]
            if x < acc:
                i_bin = i
                break
        v = la + (i_bin + rng.u01(w[2])) * (width / N_BINS)
        s = int(math.floor(math.exp(v)))
        return min(max(s, a), b), i_bin
    raise ValueError("unknown size policy")


def _sample(X, s, seed, worker, purpose, g):
    idx = rng.sample_indices(X.shape[0], s, seed, worker, purpose, g)
    return X[idx]


def worker_pass(X, C, deg, fhat, s_prev, s, seed, worker, g, g_recalc, n_candidates=3,
                max_iter=300, tol=1e-4):
    """One pass of one worker of Algorithm 1 (the body of its inner loop).

    If the worker already has an incumbent (f_hat finite) and its sample size
    changed (s != s_prev), f_hat is first re-evaluated on a fresh sample of
    size s (purpose RECALC, counter g_recalc; Section 4.2).  Then a new sample
    S (purpose SAMPLE, counter g), greedy K-means++ for the degenerate
    centroids on S, K-means from the result, and acceptance only on a strict
    improvement of f_hat.  Returns a dict with the new incumbent (C, deg,
    fhat), the pass's Lloyd objective f and updates iters, and accepted."""
    if fhat < math.inf and s != s_prev:
        S_re = _sample(X, s, seed, worker, rng.PURPOSE_RECALC, g_recalc)
        fhat = kmeans.objective(S_re, C)
    S = _sample(X, s, seed, worker, rng.PURPOSE_SAMPLE, g)
    C0, _, _ = kmeans.kmeanspp(S, C, deg, n_candidates, seed, worker, g)
    res = kmeans.lloyd(S, C0, max_iter, tol)
    accepted = res["f"] < fhat
    if accepted:
        C, deg, fhat = res["C"], res["deg"], res["f"]
    return {"C": C, "deg": deg, "fhat": fhat, "f": res["f"], "iters": res["iters"],
            "accepted": accepted}


def worker_round(X, params, worker, t, state, bin_stats, l_stats):
    """Round t of one worker (Algorithm 1, the body of the loop over workers):
    its size draw, then p passes (the first one re-evaluates the incumbent if
    the size changed).  state = (C, deg, fhat, s_prev).  Returns the new state,
    the size, its bin and, per pass, (iters, accepted)."""
    P = params
    C, deg, fhat, s_prev = state
    s_new, b = draw_size(P, worker, t, bin_stats, l_stats)
    passes = []
    for q in range(P.passes_p):
        res = worker_pass(X, C, deg, fhat, s_prev, s_new, P.seed, worker, t * P.passes_p + q, t,
                          P.n_candidates, P.max_iter, P.tol)
        s_prev = s_new
        C, deg, fhat = res["C"], res["deg"], res["fhat"]
        passes.append((res["iters"], res["accepted"]))
    return (C, deg, fhat, s_new), s_new, b, passes


# Data of a process pool's workers (inherited through fork, never pickled).
_POOL_X = None


def _pool_init():
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)


def _pool_round(args):
    return worker_round(_POOL_X, *args)


def bigmeans_run(X, params, keep_trace=False, processes=1, rounds_done=None, final_stage=True):
    """Run Algorithm 1 on X (m x n).  Returns a dict with C_best, Y, s_opt,
    f_full, the winning worker, the list L and per-round statistics.

    Workers depend on each other only through the list L (and the BINS and
    SHRINK statistics of earlier rounds), so with processes > 1 each round's
    workers run in a pool of that many processes (one BLAS thread each, the
    paper's one worker per core); their results are merged in worker order,
    which gives exactly the sequential run.  rounds_done(t, state) is called
    after every round (optional).  With final_stage=False the run stops after
    the rounds (no s_opt, final sample or full assignment)."""
    global _POOL_X
    X = np.ascontiguousarray(X, dtype=np.float64)
    m, n = X.shape
    P = params
    W, k = P.workers, P.k
    if not (1 <= k <= P.s_min <= P.s_max <= m):
        raise ValueError("need 1 <= k <= s_min <= s_max <= m")
    state = [(np.zeros((k, n)), np.ones(k, dtype=bool), math.inf, None) for _ in range(W)]
    L = []                                  # (round, worker, pass, s, bin)
    bin_stats = {"acc": [0] * N_BINS, "passes": [0] * N_BINS}
    lloyd_dists = 0
    lloyd_iters = 0
    rounds = []
    pool = None
    if processes > 1:
        import multiprocessing as mp
        _POOL_X = X
        pool = mp.get_context("fork").Pool(processes, initializer=_pool_init)
    try:
        for t in range(P.rounds_T):
            round_acc = [0] * N_BINS
            round_passes = [0] * N_BINS
            l_stats = (sum(e[3] for e in L), len(L))   # L over earlier rounds
            stats_now = {"acc": list(bin_stats["acc"]), "passes": list(bin_stats["passes"])}
            tasks = [(P, w, t, state[w], stats_now, l_stats) for w in range(W)]
            if pool is None:
                outs = [worker_round(X, *a) for a in tasks]
            else:
                outs = pool.map(_pool_round, tasks, chunksize=1)
            for w, (st, s_new, b, passes) in enumerate(outs):
                state[w] = st
                for q, (iters, accepted) in enumerate(passes):
                    lloyd_iters += iters + 1
                    lloyd_dists += (iters + 1) * s_new * k
                    round_passes[b] += 1
                    if accepted:
                        L.append((t, w, q, s_new, b))
                        round_acc[b] += 1
            for i in range(N_BINS):
                bin_stats["acc"][i] += round_acc[i]
                bin_stats["passes"][i] += round_passes[i]
            if keep_trace:
                rounds.append({"C": [s_[0].copy() for s_ in state], "fhat": [s_[2] for s_ in state],
                               "s": [s_[3] for s_ in state]})
            if rounds_done is not None:
                rounds_done(t, state)
    finally:
        if pool is not None:
            pool.close()
            pool.join()
            _POOL_X = None
    C = [s_[0] for s_ in state]
    deg = [s_[1] for s_ in state]
    fhat = [s_[2] for s_ in state]
    if not final_stage:
        return {"L": L, "fhat": fhat, "C_all": C, "deg_all": deg, "lloyd_dists": lloyd_dists,
                "lloyd_iters": lloyd_iters, "rounds": rounds}
    if L:
        total = sum(e[3] for e in L)
        s_opt = (total + len(L) // 2) // len(L)
    else:
        s_opt = P.s_max
    S_fin = _sample(X, s_opt, P.seed, rng.FINAL_WORKER, rng.PURPOSE_FINAL, 0)
    f_fin = [kmeans.objective(S_fin, C[w]) if fhat[w] < math.inf else math.inf
             for w in range(W)]
    best = min(range(W), key=lambda w: (not (f_fin[w] == f_fin[w]), f_fin[w], w))
    Y, d1 = kmeans.assign(X, C[best])
    return {"C_best": C[best], "Y": Y, "s_opt": s_opt, "f_full": math.fsum(d1.tolist()),
            "best_worker": best, "f_final_sample": f_fin, "L": L, "fhat": fhat,
            "C_all": C, "deg_all": deg, "lloyd_dists": lloyd_dists,
            "lloyd_iters": lloyd_iters, "rounds": rounds}
