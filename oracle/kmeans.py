"""K-means building blocks of Big-means, in FP64 (test infrastructure only).

* ``assign`` / ``objective``: the MSSC criterion, Eq. (1): every point goes to
  its nearest centre in squared Euclidean distance, and f(C, X) is the sum of
  those squared distances.
* ``lloyd``: K-means (Lloyd) iterations as run on each sample in Algorithm 1,
  with the stopping rule of Section 5 (at most 300 iterations, relative
  tolerance 1e-4).
* ``kmeanspp``: K-means++ seeding (Section 3, Arthur & Vassilvitskii) in the
  greedy form with several candidates per centre (Section 5: three candidate
  points), used in Algorithm 1 to re-initialise only the centroids of
  degenerate clusters (Section 4.1).

Inputs stored in FP32 are widened to FP64 exactly; all arithmetic is FP64.

Readings taken where the paper is silent:
* ties in any argmin go to the lowest index;
* a cluster that loses all its points during Lloyd keeps its previous centre
  and is reported degenerate at the end (degenerate = empty under the final
  assignment of the K-means run that produced the centroids);
* "relative tolerance 1e-4" is on the objective: stop once
  f_prev - f <= 1e-4 * f; "300 iterations" caps the number of centroid
  updates, and the returned objective is that of the returned centroids;
* the first centre of a seeding with no existing centre is one uniform draw;
  later centres draw n_cand candidates with probability proportional to D^2
  and keep the one with the smallest potential; if every point coincides with
  a centre (total D^2 = 0), or the total is not finite, the pick is uniform.
"""

import math

import numpy as np

from . import rng

NEAR_TIE_REL = 1e-5
_CHUNK = 1 << 18


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def sqdist_direct(X, c):
    """||x_i - c||^2 for every row x_i of X, direct form sum_d (x_d - c_d)^2."""
    diff = _f64(X) - _f64(c)[None, :]
    return (diff * diff).sum(axis=1)


def assign(X, C, return_second=False):
    """Nearest centre of every row of X (the inner min of Eq. 1).

    Returns labels a (lowest index among equal distances) and d1 = ||x - c_a||^2
    in the direct form.  With return_second, also d2 (second-smallest squared
    distance, +inf when k == 1) and the near-tie mask (d2 - d1) < 1e-5 * d2.

    The expanded form ||x||^2 + ||c||^2 - 2 x.c is used only to shortlist,
    per row, the centres within a band far wider than its FP64 rounding error;
    the decision between shortlisted centres is taken in the direct form.
    """
    X, C = _f64(X), _f64(C)
    m, k = X.shape[0], C.shape[0]
    labels = np.empty(m, dtype=np.int64)
    d1 = np.empty(m)
    d2 = np.full(m, np.inf)
    cc = (C * C).sum(axis=1)
    for lo in range(0, m, _CHUNK):
        hi = min(m, lo + _CHUNK)
        Xc = X[lo:hi]
        xx = (Xc * Xc).sum(axis=1)
        G = (xx[:, None] + cc[None, :]) - 2.0 * (Xc @ C.T)
        gmin = G.min(axis=1)
        band = 1e-9 * (xx + cc.max()) + 1e-300
        short = G <= (gmin + band)[:, None]
        nshort = short.sum(axis=1)
        # Rows with a single shortlisted centre: that centre is the nearest.
        lab = np.argmax(short, axis=1)
        dd1 = ((Xc - C[lab]) ** 2).sum(axis=1)
        dd2 = np.full(hi - lo, np.inf)
        if k > 1:
            Gm = G.copy()
            Gm[np.arange(hi - lo), lab] = np.inf
            run = np.argmin(Gm, axis=1)
            dd2 = ((Xc - C[run]) ** 2).sum(axis=1)
        # Rows with several shortlisted centres: direct form over the shortlist.
        multi = np.nonzero(nshort > 1)[0]
        if multi.size:
            Dm = np.stack([((Xc[multi] - C[j]) ** 2).sum(axis=1) for j in range(k)], axis=1)
            Dm_short = np.where(short[multi], Dm, np.inf)
            lab_m = np.argmin(Dm_short, axis=1)          # first index of the minimum
            lab[multi] = lab_m
            dd1[multi] = Dm_short[np.arange(multi.size), lab_m]
            Dm_short[np.arange(multi.size), lab_m] = np.inf
            dd2[multi] = Dm_short.min(axis=1)
        labels[lo:hi] = lab
        d1[lo:hi] = dd1
        d2[lo:hi] = dd2
    if not return_second:
        return labels, d1
    near = (d2 - d1) < NEAR_TIE_REL * d2
    return labels, d1, d2, near


def objective(X, C):
    """f(C, X) of Eq. (1): sum over points of the squared distance to the nearest centre."""
    _, d1 = assign(X, C)
    return math.fsum(d1.tolist())


def cluster_means(S, labels, k, C_prev):
    """Centroid update: mean of each cluster (FP64); an empty cluster keeps C_prev[j].

    Returns (C_new, counts)."""
    S = _f64(S)
    labels = np.asarray(labels, dtype=np.int64)
    counts = np.bincount(labels, minlength=k)
    C_new = _f64(C_prev).copy()
    for d in range(S.shape[1]):
        sums = np.bincount(labels, weights=S[:, d], minlength=k)
        nz = counts > 0
        C_new[nz, d] = sums[nz] / counts[nz]
    return C_new, counts


def lloyd(S, C0, max_iter=300, tol=1e-4):
    """K-means (Lloyd) on sample S from initial centroids C0.

    Each iteration assigns every point to its nearest centre and evaluates
    f = f(C, S); it stops when f_prev - f <= tol * f, when f is not finite,
    or when max_iter centroid updates have been made, otherwise it moves each
    centroid to the mean of its cluster.  Returns a dict with the final centroids C, their objective f,
    the labels, the degenerate mask (empty clusters under the final
    assignment), the number of updates 'iters', and the objective trace.
    """
    S = _f64(S)
    C = _f64(C0).copy()
    k = C.shape[0]
    f_prev = None
    it = 0
    trace = []
    while True:
        labels, d1 = assign(S, C)
        f = math.fsum(d1.tolist())
        trace.append(f)
        counts = np.bincount(labels, minlength=k)
        if f_prev is not None and f_prev - f <= tol * f:
            break
        if not math.isfinite(f):      # NaN/inf points: the objective can never improve
            break
        if it >= max_iter:
            break
        C, _ = cluster_means(S, labels, k, C)
        f_prev = f
        it += 1
    return {"C": C, "f": f, "labels": labels, "deg": counts == 0,
            "counts": counts, "iters": it, "trace": trace}


def kmeanspp(S, C, deg, n_cand, seed, worker, g):
    """Greedy K-means++ re-seeding of the degenerate centroids of C on sample S.

    Existing (non-degenerate) centres E fix D_i = min_{j in E} ||S_i - C_j||^2.
    The degenerate centroids are filled in ascending index order; step number
    'step' draws one Philox block w = B((step, g, 0, 0), key(seed, worker, KMPP)):
      * no centre yet, or T = sum D not a finite positive number (all points
        covered, or NaN/inf data): i* = mulhi(w[3], s);
      * otherwise candidate c < n_cand is the first i whose FP64 prefix sum of D
        exceeds u(w[c]) * T (T = total of D), its potential is
        sum_i min(D_i, ||S_i - S_cand||^2), and i* is the candidate with the
        smallest potential (lowest c on ties).
    Then C_j = S_i* and D_i <- min(D_i, ||S_i - S_i*||^2).

    Returns (C, deg, log) where log lists, per step, the centroid index, the
    candidates, their potentials, T and the chosen sample index.
    """
    S = _f64(S)
    C = _f64(C).copy()
    deg = np.asarray(deg, dtype=bool).copy()
    s = S.shape[0]
    key = rng.stream_key(seed, worker, rng.PURPOSE_KMPP)
    existing = [j for j in range(C.shape[0]) if not deg[j]]
    todo = [j for j in range(C.shape[0]) if deg[j]]
    D = None
    for j in existing:
        dj = sqdist_direct(S, C[j])
        D = dj if D is None else np.minimum(D, dj)
    log = []
    for step, j in enumerate(todo):
        w = rng.philox_block_scalar((step, g, 0, 0), key)
        cands, pots, T = [], [], None
        if D is not None:
            prefix = np.cumsum(D)
            T = float(prefix[-1])
        if D is None or not (0.0 < T < math.inf):
            # no centre yet, every point covered (T = 0), or a NaN/inf total
            i_star = rng.mulhi(w[3], s)
        else:
            for c in range(n_cand):
                tau = rng.u01(w[c]) * T
                i_c = int(np.searchsorted(prefix, tau, side="right"))
                cands.append(i_c)
                pots.append(math.fsum(np.minimum(D, sqdist_direct(S, S[i_c])).tolist()))
            best = 0                      # smallest potential, lowest c on ties
            for c in range(1, n_cand):
                if pots[c] < pots[best]:
                    best = c
            i_star = cands[best]
        C[j] = S[i_star]
        dnew = sqdist_direct(S, S[i_star])
        D = dnew if D is None else np.minimum(D, dnew)   # NaN propagates into D and T
        deg[j] = False
        log.append({"centroid": j, "candidates": cands, "potentials": pots,
                    "total": T, "chosen": i_star})
    return C, deg, log
