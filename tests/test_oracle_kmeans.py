"""Pins of the oracle's K-means pieces against things other than itself:
brute-force enumeration on tiny inputs, closed forms, invariants, scikit-learn's
Lloyd, and the statistics and cited expected-cost bound of K-means++."""

import itertools
import math

import numpy as np
import pytest
from scipy import stats

from oracle import kmeans, rng


def _brute_assign(X, C):
    X = np.asarray(X, float)
    C = np.asarray(C, float)
    labels, d1 = [], []
    for x in X:
        ds = [math.fsum(((x - c) ** 2).tolist()) for c in C]
        j = min(range(len(C)), key=lambda t: (ds[t], t))
        labels.append(j)
        d1.append(ds[j])
    return np.array(labels), np.array(d1)


def test_objective_equals_min_over_all_labelings():
    # Eq. (1): f(C, X) = sum_i min_j ||x_i - c_j||^2 = min over all k^m labelings.
    r = np.random.default_rng(0)
    for trial in range(30):
        m = int(r.integers(1, 9))
        k = int(r.integers(1, 4))
        n = int(r.integers(1, 4))
        X = r.integers(-5, 6, size=(m, n)).astype(float)
        C = r.integers(-5, 6, size=(k, n)).astype(float)
        best = min(math.fsum(((X[i] - C[a[i]]) ** 2).sum() for i in range(m))
                   for a in itertools.product(range(k), repeat=m))
        assert kmeans.objective(X, C) == best          # small integers: exact


def test_assign_matches_direct_form_with_ties():
    r = np.random.default_rng(1)
    X = r.integers(-3, 4, size=(400, 3)).astype(float)
    C = r.integers(-3, 4, size=(7, 3)).astype(float)
    C[5] = C[2]                                       # duplicate centre: ties everywhere it wins
    lab, d1 = kmeans.assign(X, C)
    blab, bd1 = _brute_assign(X, C)
    assert np.array_equal(lab, blab)
    assert np.array_equal(d1, bd1)
    assert not np.any(lab == 5)                       # lowest index wins ties


def test_assign_large_offset_data_direct_decision():
    # Data far from the origin: expanded-form cancellation must not decide.
    r = np.random.default_rng(2)
    X = 1e4 + r.standard_normal((2000, 5))
    C = 1e4 + r.standard_normal((6, 5))
    lab, d1, d2, near = kmeans.assign(X, C, return_second=True)
    blab, bd1 = _brute_assign(X, C)
    ok = ~near
    assert np.array_equal(lab[ok], blab[ok])
    assert np.allclose(d1, bd1, rtol=1e-12, atol=0)
    assert np.all(d2 >= d1)


def _mssc_optimum(X, k):
    m = X.shape[0]
    best, best_lab = math.inf, None
    for lab in itertools.product(range(k), repeat=m):
        lab = np.array(lab)
        tot = 0.0
        for j in range(k):
            P = X[lab == j]
            if len(P):
                tot += ((P - P.mean(axis=0)) ** 2).sum()
        if tot < best:
            best, best_lab = tot, lab
    return best, best_lab


def test_lloyd_never_below_brute_force_optimum_and_optimum_is_fixed_point():
    r = np.random.default_rng(3)
    for trial in range(6):
        m, k = 8, 3
        X = r.standard_normal((m, 2)) * 3
        fstar, lab = _mssc_optimum(X, k)
        for s in range(5):
            C0 = X[r.choice(m, k, replace=False)]
            res = kmeans.lloyd(X, C0, max_iter=300, tol=0.0)
            assert res["f"] >= fstar * (1 - 1e-12)
        Copt, _ = kmeans.cluster_means(X, lab, k, np.zeros((k, 2)))
        res = kmeans.lloyd(X, Copt, max_iter=300, tol=1e-4)
        assert abs(res["f"] - fstar) <= 1e-12 * max(1.0, fstar)
        assert np.allclose(res["C"], Copt, rtol=0, atol=1e-12)


def test_lloyd_monotone_and_exit_state():
    r = np.random.default_rng(4)
    X = np.concatenate([r.standard_normal((300, 4)) + 6 * r.standard_normal(4) for _ in range(6)])
    C0 = X[r.choice(len(X), 6, replace=False)]
    res = kmeans.lloyd(X, C0, max_iter=300, tol=0.0)
    tr = res["trace"]
    for a, b in zip(tr, tr[1:]):
        assert b <= a * (1 + 1e-12)
    # with tol = 0 the run stops when f stops decreasing: the labels are stable, so
    # every non-empty centroid is the mean of its cluster.
    Cm, counts = kmeans.cluster_means(X, res["labels"], 6, res["C"])
    assert np.allclose(res["C"], Cm, rtol=0, atol=1e-10)
    assert res["f"] == pytest.approx(kmeans.objective(X, res["C"]), rel=1e-15)


def test_lloyd_k1_closed_form():
    r = np.random.default_rng(5)
    X = r.standard_normal((500, 3)) * 2 + 1
    res = kmeans.lloyd(X, X[:1], max_iter=300, tol=1e-4)
    mu = X.mean(axis=0)
    assert np.allclose(res["C"][0], mu, atol=1e-12)
    assert res["f"] == pytest.approx(((X - mu) ** 2).sum(), rel=1e-12)


def test_lloyd_empty_cluster_keeps_centre_and_is_degenerate():
    X = np.array([[0.0], [1.0], [10.0], [11.0]])
    C0 = np.array([[0.5], [10.5], [100.0]])
    res = kmeans.lloyd(X, C0)
    assert res["C"][2, 0] == 100.0
    assert list(res["deg"]) == [False, False, True]


def test_lloyd_iteration_cap():
    r = np.random.default_rng(6)
    X = r.standard_normal((400, 2))
    C0 = X[:20]
    res = kmeans.lloyd(X, C0, max_iter=2, tol=0.0)
    assert res["iters"] == 2 and len(res["trace"]) == 3
    res0 = kmeans.lloyd(X, C0, max_iter=0, tol=0.0)
    assert res0["iters"] == 0 and np.array_equal(res0["C"], C0)


def test_lloyd_matches_sklearn():
    from sklearn.cluster import KMeans
    r = np.random.default_rng(7)
    X = np.concatenate([r.standard_normal((200, 3)) + 5 * r.standard_normal(3) for _ in range(5)])
    C0 = X[r.choice(len(X), 5, replace=False)].copy()
    for iters in (1, 2, 5, 50):
        ours = kmeans.lloyd(X, C0, max_iter=iters, tol=0.0)
        km = KMeans(n_clusters=5, init=C0, n_init=1, algorithm="lloyd", tol=0.0,
                    max_iter=iters).fit(X)
        assert np.allclose(ours["C"], km.cluster_centers_, rtol=0, atol=1e-10)
        assert np.array_equal(ours["labels"], km.labels_)
        assert ours["f"] == pytest.approx(km.inertia_, rel=1e-10)


def test_kmeanspp_picks_sample_points_and_minimal_potential():
    r = np.random.default_rng(8)
    S = np.concatenate([r.standard_normal((100, 2)) + 8 * r.standard_normal(2) for _ in range(4)])
    C = np.zeros((4, 2))
    deg = np.ones(4, bool)
    C1, deg1, log = kmeans.kmeanspp(S, C, deg, 3, seed=3, worker=1, g=2)
    assert not deg1.any()
    D = None
    for step, e in enumerate(log):
        assert any(np.array_equal(C1[e["centroid"]], p) for p in S[[e["chosen"]]])
        if step == 0:
            assert e["candidates"] == []
        else:
            for c, p in zip(e["candidates"], e["potentials"]):
                assert D[c] > 0                        # D^2 sampling never picks a covered point
                assert p == pytest.approx(np.minimum(D, kmeans.sqdist_direct(S, S[c])).sum(), rel=1e-12)
            assert e["chosen"] == e["candidates"][int(np.argmin(e["potentials"]))]
        dn = kmeans.sqdist_direct(S, S[e["chosen"]])
        D = dn if D is None else np.minimum(D, dn)


def test_kmeanspp_only_degenerate_reseeded():
    r = np.random.default_rng(9)
    S = r.standard_normal((300, 3))
    C = r.standard_normal((5, 3))
    deg = np.array([False, True, False, True, False])
    C1, deg1, log = kmeans.kmeanspp(S, C, deg, 3, seed=0, worker=0, g=0)
    assert [e["centroid"] for e in log] == [1, 3]
    assert np.array_equal(C1[[0, 2, 4]], C[[0, 2, 4]])
    assert log[0]["candidates"] != []                  # existing centres give D, so D^2 sampling


def test_kmeanspp_zero_potential_uniform_and_exact_cover():
    S = np.array([[0.0, 0.0], [1.0, 1.0], [0.0, 0.0], [1.0, 1.0]])
    C, deg, log = kmeans.kmeanspp(S, np.zeros((3, 2)), np.ones(3, bool), 3, 0, 0, 0)
    # two distinct points, three centres: after both are covered T = 0 -> uniform pick
    assert kmeans.objective(S, C) == 0.0
    assert log[2]["candidates"] == [] and log[2]["total"] == 0.0


def test_kmeanspp_first_candidate_distribution_chi2():
    # P(candidate = i) = D_i / T under D^2 sampling.
    S = np.array([[0.0], [1.0], [2.0], [4.0], [7.0], [11.0]])
    C = np.array([[0.0], [0.0]])
    deg = np.array([False, True])
    D = S[:, 0] ** 2
    counts = np.zeros(len(S))
    trials = 20000
    for g in range(trials):
        _, _, log = kmeans.kmeanspp(S, C, deg, 1, seed=1, worker=0, g=g)
        counts[log[0]["candidates"][0]] += 1
    p = D / D.sum()
    nz = p > 0
    assert counts[~nz].sum() == 0
    chi = (((counts - trials * p) ** 2)[nz] / (trials * p[nz])).sum()
    assert stats.chi2.sf(chi, nz.sum() - 1) > 1e-4


def test_kmeanspp_expected_cost_bound():
    # Arthur & Vassilvitskii (cited in Section 3): plain K-means++ (one candidate)
    # has E[f] <= 8 (ln k + 2) f*.
    r = np.random.default_rng(10)
    X = np.concatenate([r.standard_normal((3, 2)) * 0.3 + c for c in ([0, 0], [5, 0], [0, 5])])
    k = 3
    fstar, _ = _mssc_optimum(X, k)
    fs = []
    for g in range(1000):
        C, _, _ = kmeans.kmeanspp(X, np.zeros((k, 2)), np.ones(k, bool), 1, 2, 0, g)
        fs.append(kmeans.objective(X, C))
    assert np.mean(fs) <= 8 * (math.log(k) + 2) * fstar
    # greedy with three candidates is no worse on average on this instance
    fs3 = [kmeans.objective(X, kmeans.kmeanspp(X, np.zeros((k, 2)), np.ones(k, bool), 3, 2, 0, g)[0])
           for g in range(300)]
    assert np.mean(fs3) <= np.mean(fs) * 1.05


def test_kmeanspp_draws_follow_contract():
    S = np.arange(10.0)[:, None]
    _, _, log = kmeans.kmeanspp(S, np.zeros((1, 1)), np.ones(1, bool), 3, seed=4, worker=2, g=6)
    w = rng.philox_block_scalar((0, 6, 0, 0), rng.stream_key(4, 2, rng.PURPOSE_KMPP))
    assert log[0]["chosen"] == rng.mulhi(w[3], 10)
