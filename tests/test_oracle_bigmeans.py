"""Pins of the oracle's Algorithm 1 (competitive sample-size Big-means):
invariants of the incumbent and of the list L, the reduction to one plain
K-means++ + K-means run, determinism, the size policies, and NaN handling."""

import json
import math
import os

import numpy as np
import pytest

from oracle import bigmeans, kmeans, rng
from paper_2403_18766_amd import datagen


@pytest.fixture(scope="module")
def blobs():
    return datagen.make("blobs2d", m=4000).astype(np.float64)


def test_paper_parameters_are_the_defaults(golden_dir):
    with open(os.path.join(golden_dir, "paper_parameters.json")) as f:
        g = json.load(f)
    p = bigmeans.Params(k=5, workers=1, rounds_T=1)
    assert (p.max_iter, p.tol, p.n_candidates, p.passes_p) == \
        (g["max_iter"], g["tol"], g["n_candidates"], g["passes_p"])
    assert bigmeans.paper_size_range(2000, 20000) == (1000, 4000)
    assert bigmeans.paper_size_range(2000, 3000) == (1000, 3000)
    assert bigmeans.paper_size_range(7, 100) == (4, 14)


def test_invariants(blobs):
    P = bigmeans.Params(k=5, workers=3, rounds_T=3, passes_p=4, s_min=200, s_max=800,
                        size_policy=bigmeans.SIZE_UNIFORM, seed=1)
    out = bigmeans.bigmeans_run(blobs, P, keep_trace=True)
    L = out["L"]
    # every worker's first pass beats +inf
    assert len(L) >= P.workers
    assert {e[1] for e in L} == set(range(P.workers))
    sizes = [e[3] for e in L]
    assert min(sizes) <= out["s_opt"] <= max(sizes)
    assert out["s_opt"] == (sum(sizes) + len(sizes) // 2) // len(sizes)
    # the winner minimises the objective on the shared final sample
    ff = out["f_final_sample"]
    assert ff[out["best_worker"]] == min(ff)
    # the returned labels and f are those of C_best on all of X
    lab, d1 = kmeans.assign(blobs, out["C_best"])
    assert np.array_equal(lab, out["Y"])
    assert out["f_full"] == pytest.approx(d1.sum(), rel=1e-12)


def test_incumbent_never_worsens_at_fixed_size(blobs):
    P = bigmeans.Params(k=5, workers=2, rounds_T=4, passes_p=3, s_min=500, s_max=500,
                        size_policy=bigmeans.SIZE_FIXED, seed=2)
    out = bigmeans.bigmeans_run(blobs, P, keep_trace=True)
    for w in range(P.workers):
        fh = [r["fhat"][w] for r in out["rounds"]]
        for a, b in zip(fh, fh[1:]):
            assert b <= a


def test_reduces_to_one_kmeanspp_plus_lloyd(blobs):
    # W = 1, T = 1, p = 1, s = m, FIXED: one seeding + one K-means on the whole data
    X = blobs[:1500]
    m = X.shape[0]
    P = bigmeans.Params(k=5, workers=1, rounds_T=1, passes_p=1, s_min=m, s_max=m,
                        size_policy=bigmeans.SIZE_FIXED, seed=3)
    out = bigmeans.bigmeans_run(X, P)
    idx = rng.sample_indices(m, m, 3, 0, rng.PURPOSE_SAMPLE, 0)
    S = X[idx]
    C0, _, _ = kmeans.kmeanspp(S, np.zeros((5, 2)), np.ones(5, bool), 3, 3, 0, 0)
    res = kmeans.lloyd(S, C0)
    assert np.array_equal(out["C_best"], res["C"])
    # S is a permutation of X, so f on S equals f on X up to summation order
    assert out["f_full"] == pytest.approx(res["f"], rel=1e-12)


def test_deterministic(blobs):
    P = bigmeans.Params(k=5, workers=2, rounds_T=2, passes_p=2, s_min=300, s_max=600,
                        size_policy=bigmeans.SIZE_LOGUNIFORM, seed=4)
    a = bigmeans.bigmeans_run(blobs, P)
    b = bigmeans.bigmeans_run(blobs, P)
    assert np.array_equal(a["C_best"], b["C_best"]) and a["L"] == b["L"]
    assert a["f_full"] == b["f_full"]


def test_size_policies_ranges():
    for pol in (bigmeans.SIZE_UNIFORM, bigmeans.SIZE_LOGUNIFORM, bigmeans.SIZE_BINS):
        P = bigmeans.Params(k=2, workers=1, rounds_T=1, s_min=4096, s_max=131072,
                            size_policy=pol, seed=0)
        stats_ = {"acc": [0] * 5, "passes": [0] * 5}
        seen = []
        for t in range(400):
            for w in range(4):
                s, b = bigmeans.draw_size(P, w, t, stats_)
                assert 4096 <= s <= 131072 and 0 <= b < 5
                seen.append(s)
        seen = np.array(seen)
        if pol == bigmeans.SIZE_UNIFORM:
            assert abs(seen.mean() - (4096 + 131072) / 2) < 0.05 * 131072
        else:   # log-uniform: ln s roughly uniform on [ln a, ln(b+1))
            ls = np.log(seen)
            mid = 0.5 * (math.log(4096) + math.log(131073))
            assert abs(ls.mean() - mid) < 0.1


def test_bins_follow_improvement_statistics():
    P = bigmeans.Params(k=2, workers=1, rounds_T=1, s_min=4096, s_max=131072,
                        size_policy=bigmeans.SIZE_BINS, seed=0)
    # bin 3 improved on every pass, the others never
    st = {"acc": [0, 0, 0, 50, 0], "passes": [50, 50, 50, 50, 50]}
    bins = [bigmeans.draw_size(P, w, t, st)[1] for t in range(1, 200) for w in range(3)]
    frac3 = np.mean(np.array(bins) == 3)
    # weights (1/52, 1/52, 1/52, 51/52, 1/52): bin 3 has probability 51/55
    assert abs(frac3 - 51 / 55) < 0.05
    edges = [4096 * 2 ** i for i in range(6)]
    for t in range(1, 50):
        s, b = bigmeans.draw_size(P, 0, t, st)
        assert edges[b] <= s <= edges[b + 1]


def test_shrink_policy_narrows_around_mean_of_L():
    # Section 7 leaves the choice of sizes beyond uniform draws open; SHRINK draws
    # log-uniformly around the mean of L with a log-width halving every round
    a, b = 4096, 131072
    P = bigmeans.Params(k=2, workers=1, rounds_T=1, s_min=a, s_max=b,
                        size_policy=bigmeans.SIZE_SHRINK, seed=3)
    PL = bigmeans.Params(k=2, workers=1, rounds_T=1, s_min=a, s_max=b,
                         size_policy=bigmeans.SIZE_LOGUNIFORM, seed=3)
    # round 0 and an empty L: the log-uniform draw itself
    for w in range(5):
        assert bigmeans.draw_size(P, w, 0, None, (5000, 1)) == bigmeans.draw_size(PL, w, 0, None)
        assert bigmeans.draw_size(P, w, 4, None, (0, 0)) == bigmeans.draw_size(PL, w, 4, None)
    width = math.log(b + 1) - math.log(a)
    for mu in (4096, 20000, 131072):
        for t in range(1, 12):
            r = math.exp(width / 2 * 2.0 ** -t)
            lo, hi = max(a, mu / r), min(b + 1, mu * r)
            sizes = [bigmeans.draw_size(P, w, t, None, (3 * mu, 3))[0] for w in range(200)]
            assert all(math.floor(lo) <= s <= min(b, math.ceil(hi)) for s in sizes), (mu, t)
            if t >= 8:   # late rounds: within 1% of the mean (clamped to the range)
                assert all(abs(s - min(max(mu, a), b)) <= 0.01 * mu + 1 for s in sizes)
    # with a vanishing range the draw is the mean of L up to the floor of exp(ln mu)
    s1 = bigmeans.draw_size(P, 0, 30, None, (4097 + 4098, 2))[0]
    assert 4097 <= s1 <= 4098


def test_uniform_size_matches_contract():
    P = bigmeans.Params(k=2, workers=1, rounds_T=1, s_min=1000, s_max=4000, seed=9)
    w = rng.philox_block_scalar((3, 0, 0, 0), rng.stream_key(9, 2, rng.PURPOSE_SIZE))
    assert bigmeans.draw_size(P, 2, 3, None)[0] == 1000 + rng.mulhi(w[0], 3001)


def test_nan_sample_never_accepted(blobs):
    X = blobs[:2000].copy()
    X[::7] = np.nan                       # every sample of 300 rows contains NaN rows
    P = bigmeans.Params(k=3, workers=2, rounds_T=1, passes_p=2, s_min=300, s_max=300,
                        size_policy=bigmeans.SIZE_FIXED, seed=5)
    out = bigmeans.bigmeans_run(X, P)
    assert out["L"] == []
    assert all(f == math.inf for f in out["fhat"])


def test_recalc_on_size_change(blobs):
    # With UNIFORM sizes the incumbent is re-scored whenever s changes; the final
    # f_hat values stay finite and each is a sample objective of that worker's C.
    P = bigmeans.Params(k=5, workers=2, rounds_T=3, passes_p=2, s_min=200, s_max=1000,
                        size_policy=bigmeans.SIZE_UNIFORM, seed=6)
    out = bigmeans.bigmeans_run(blobs, P, keep_trace=True)
    for r in out["rounds"]:
        for w in range(2):
            assert math.isfinite(r["fhat"][w])


def test_process_pool_equals_sequential(blobs):
    # workers in a process pool, merged in worker order: exactly the sequential run
    P = bigmeans.Params(k=4, workers=5, rounds_T=3, passes_p=2, s_min=300, s_max=1200,
                        size_policy=bigmeans.SIZE_BINS, seed=8)
    a = bigmeans.bigmeans_run(blobs, P, keep_trace=True)
    b = bigmeans.bigmeans_run(blobs, P, keep_trace=True, processes=3)
    assert a["L"] == b["L"] and a["f_full"] == b["f_full"] and a["s_opt"] == b["s_opt"]
    assert np.array_equal(a["C_best"], b["C_best"])
    assert a["lloyd_dists"] == b["lloyd_dists"]
    for ra, rb in zip(a["rounds"], b["rounds"]):
        assert ra["fhat"] == rb["fhat"] and ra["s"] == rb["s"]
