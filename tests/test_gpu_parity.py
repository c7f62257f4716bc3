"""GPU parity of every hot-path step against the FP64 oracle, through the C ABI.

Bars (FP32 path):
  * sample indices and gathered rows: bit-identical;
  * labels: identical except points the oracle calls near ties
    ((d2 - d1) < 1e-5 d2);
  * objectives f: within 1e-6 relative;
  * centroid update: within 1 ulp of fp32(FP64 cluster mean of the GPU's own
    labels) (teacher-forced);
  * K-means++: every candidate a valid D^2 draw for the oracle's D (within
    1e-5 T of the drawn threshold), every choice the oracle's minimum
    potential unless two potentials are within 1e-5.
"""

import math

import numpy as np
import pytest

from oracle import bigmeans as obm
from oracle import kmeans as okm
from oracle import rng as orng
from paper_2403_18766_amd import datagen
from tests.gpu_common import require_gpu, say, to_dev, ulp_diff_f32

pytestmark = pytest.mark.gpu

F_TOL = 1e-6


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def api():
    from paper_2403_18766_amd import api as a
    return a


def _data(name, m, seed=0):
    return datagen.make(name, seed=seed, m=m)


# ---------------------------------------------------------------------------
# a1: sample + gather
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,s,seed,worker,g", [
    (20_000, 2, 2_000, 0, 0, 0),
    (1_000, 3, 1_000, 5, 1, 7),          # s = m: a full permutation, odd n (scalar gather)
    (100_003, 28, 257, 1, 3, 11),        # ragged tail
    (1_000_000, 28, 65_536, 2, 31, 49),
    (777, 5, 1, 9, 2, 3),
    (1 << 20, 4, 262_144, 3, 0, 0),      # largest sample size of the workloads
])
def test_sample_bit_identical(dev, api, m, n, s, seed, worker, g):
    say("sample", m, n, s, seed, worker, g)
    rs = np.random.default_rng(m + n)
    X = rs.standard_normal((m, n)).astype(np.float32)
    Xd = to_dev(X, dev)
    idx, S = api.sample(Xd, s, seed=seed, worker=worker, purpose=2, g=g)
    idx = idx.cpu().numpy().astype(np.int64)
    want = orng.sample_indices(m, s, seed, worker, orng.PURPOSE_SAMPLE, g)
    assert np.array_equal(idx, want)
    assert np.array_equal(S.cpu().numpy(), X[want])


# ---------------------------------------------------------------------------
# a6: objective + labels
# ---------------------------------------------------------------------------
def _check_objective(api, dev, X, C, label):
    say("objective", label, X.shape, C.shape)
    f, lab, near = api.objective(to_dev(X, dev), to_dev(C, dev))
    lab = lab.cpu().numpy()
    olab, od1, od2, onear = okm.assign(X, C, return_second=True)
    fo = math.fsum(od1.tolist())
    assert abs(f - fo) <= F_TOL * abs(fo) + 1e-300, (f, fo)
    ok = ~onear
    mism = np.nonzero(lab[ok] != olab[ok])[0]
    assert mism.size == 0, f"{mism.size} label mismatches outside near ties"
    # near-tie counts agree up to points whose gap sits at the 1e-5 boundary
    assert abs(int(near) - int(onear.sum())) <= max(2, int(0.01 * onear.sum()))
    return f, lab


@pytest.mark.parametrize("name,m,k,seed", [("blobs2d", 20_000, 5, 0), ("aniso28", 60_000, 25, 1),
                                           ("noisy28", 100_000, 50, 2)])
def test_objective_workloads(dev, api, name, m, k, seed):
    X = _data(name, m, seed)
    r = np.random.default_rng(seed)
    C = (X[r.choice(len(X), k, replace=False)] + 0.1 * r.standard_normal((k, X.shape[1]))).astype(np.float32)
    _check_objective(api, dev, X, C, name)


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (255, 3, 7), (257, 5, 1), (4_097, 64, 13),
                                   (10_000, 16, 200), (3_000, 61, 9), (70_001, 12, 33)])
def test_objective_shapes(dev, api, m, n, k):
    r = np.random.default_rng(m * 7 + n)
    X = r.standard_normal((m, n)).astype(np.float32) * 3
    C = r.standard_normal((k, n)).astype(np.float32) * 3
    _check_objective(api, dev, X, C, f"shape m={m} n={n} k={k}")


@pytest.mark.parametrize("n,k", [(64, 63), (64, 64), (64, 200), (28, 100), (8, 300)])
def test_objective_narrow_many_redecisions(dev, api, n, k):
    # noisy mixture with centres near data points: many points have several
    # centres of their own cluster at nearly the same distance; from k = 64 on
    # the wave re-decides its flagged points together (lanes over centres)
    X = datagen.serving_dataset(n, m=8_000, seed=4)
    r = np.random.default_rng(k)
    C = (X[r.choice(len(X), k, replace=False)] + 0.05 * r.standard_normal((k, n))).astype(np.float32)
    _check_objective(api, dev, X, C, f"narrow re-decisions n={n} k={k}")


def test_objective_far_from_origin_needs_recheck(dev, api):
    # cancellation in ||c||^2 - 2 x.c is large here: the certified recheck decides
    r = np.random.default_rng(3)
    X = (1e4 + r.standard_normal((50_000, 8))).astype(np.float32)
    C = (1e4 + r.standard_normal((20, 8))).astype(np.float32)
    _check_objective(api, dev, X, C, "offset 1e4")


def test_objective_ties_go_to_lowest_index(dev, api):
    r = np.random.default_rng(4)
    X = r.integers(-4, 5, size=(5_000, 4)).astype(np.float32)
    C = r.integers(-4, 5, size=(9, 4)).astype(np.float32)
    C[6] = C[1]
    C[8] = C[1]
    f, lab = _check_objective(api, dev, X, C, "duplicate centres")
    assert not np.any(lab == 6) and not np.any(lab == 8)
    # integer data: exact ties are exact in FP32 as well
    olab, _ = okm.assign(X, C)
    assert np.array_equal(lab, olab)


def test_objective_full_size_sampled(dev, api):
    # the aniso28 workload at its full size (1,000,000 x 28, k = 25): f against
    # the oracle, labels on 20,000 sampled rows
    X = _data("aniso28", None, 0)
    r = np.random.default_rng(5)
    C = X[r.choice(len(X), 25, replace=False)].copy()
    say("objective full aniso28", X.shape)
    f, lab, near = api.objective(to_dev(X, dev), to_dev(C, dev))
    lab = lab.cpu().numpy()
    fo = okm.objective(X, C)
    assert abs(f - fo) <= F_TOL * fo
    rows = r.choice(len(X), 20_000, replace=False)
    olab, _, _, onear = okm.assign(X[rows], C, return_second=True)
    assert np.array_equal(lab[rows][~onear], olab[~onear])


def test_objective_nan_is_reported(dev, api):
    from paper_2403_18766_amd._lib import BM_E_NONFINITE  # noqa: F401
    X = np.ones((600, 4), np.float32)
    X[17, 2] = np.nan
    f, lab, near = api.objective(to_dev(X, dev), to_dev(X[:3].copy(), dev))
    assert math.isnan(f)


# ---------------------------------------------------------------------------
# a3-a5: Lloyd
# ---------------------------------------------------------------------------
def _lloyd_case(name, m, k, seed):
    X = datagen.serving_dataset(64, m=m, seed=seed) if name == "mix64" else _data(name, m, seed)
    r = np.random.default_rng(seed + 100)
    C0 = X[r.choice(len(X), k, replace=False)].copy()
    return X, C0


@pytest.mark.parametrize("name,m,k,seed", [("blobs2d", 2_000, 5, 0), ("aniso28", 22_161, 25, 1),
                                           ("noisy28", 40_000, 50, 2),
                                           ("mix64", 30_000, 150, 3)])   # matrix-core ranking
def test_lloyd_one_update_teacher_forced(dev, api, name, m, k, seed):
    S, C0 = _lloyd_case(name, m, k, seed)
    say("lloyd one update", name, S.shape, k)
    res = api.lloyd(to_dev(S, dev), to_dev(C0, dev), max_iter=1, tol=0.0)
    C1 = res["C"].cpu().numpy()
    assert res["iters"] == 1
    lab0, _, _, near0 = okm.assign(S, C0, return_second=True)
    want, counts = okm.cluster_means(S, lab0, k, C0)
    want32 = want.astype(np.float32)
    # clusters touched by a near-tie point may legitimately differ
    touched = np.zeros(k, bool)
    touched[np.unique(lab0[near0])] = True
    u = ulp_diff_f32(C1[~touched], want32[~touched])
    assert u.max() <= 1, u.max()
    # the returned f, labels and flags are those of C1
    lab1 = res["labels"].cpu().numpy()
    olab1, od1, _, onear1 = okm.assign(S, C1, return_second=True)
    assert np.array_equal(lab1[~onear1], olab1[~onear1])
    fo = math.fsum(od1.tolist())
    assert abs(res["f"] - fo) <= F_TOL * fo
    cnt1 = np.bincount(olab1, minlength=k)
    assert np.array_equal(res["deg"].cpu().numpy().astype(bool), cnt1 == 0)


def test_lloyd_update_dimension_set_by_an_outlier(dev, api):
    # The centroid sums are exact fixed-point integers with 2^-shift_d
    # resolution, shift_d = 62 - e_d - ceil(log2 s) where |x_d| < 2^e_d over the
    # data: a mean whose magnitude is far below the dimension's largest value
    # (here one point at 1e7 among values near 1e-2) is only good to 2^-shift_d
    # absolute, many FP32 ulps.  Check that documented bound everywhere, and
    # 1 ulp where |mean| >= 2^-21 max|x_d|.
    r = np.random.default_rng(11)
    m, n, k = 4096, 4, 6
    centres = r.uniform(-1e-2, 1e-2, size=(k - 1, n))
    S = centres[r.integers(k - 1, size=m)] + 1e-3 * r.standard_normal((m, n))
    S[17, 2] = 1.0e7
    S = S.astype(np.float32)
    C0 = np.ascontiguousarray(S[[0, 1, 2, 3, 4, 17]])
    res = api.lloyd(to_dev(S, dev), to_dev(C0, dev), max_iter=1, tol=0.0)
    assert res["iters"] == 1
    C1 = res["C"].cpu().numpy().astype(np.float64)
    lab0, _, _, near0 = okm.assign(S, C0, return_second=True)
    want, _ = okm.cluster_means(S, lab0, k, C0)
    touched = np.zeros(k, bool)
    touched[np.unique(lab0[near0])] = True
    L = int(math.ceil(math.log2(m)))
    e = np.array([math.frexp(float(v))[1] for v in np.abs(S.astype(np.float64)).max(axis=0)])
    shift = 62 - e - L
    w32 = want.astype(np.float32)
    half_ulp = 0.5 * np.abs(np.spacing(w32)).astype(np.float64)
    bound = np.ldexp(1.0, -shift)[None, :] + half_ulp
    err = np.abs(C1 - want)
    assert np.all(err[~touched] <= bound[~touched]), (err / bound)[~touched].max()
    big = np.abs(want) >= np.ldexp(np.abs(S.astype(np.float64)).max(axis=0), -21)[None, :]
    u = ulp_diff_f32(C1.astype(np.float32), w32)
    assert np.all(u[~touched][big[~touched]] <= 1)
    # the outlier's own cluster is exact, and dimension 2 is the limited one
    assert C1[5, 2] == 1.0e7
    assert not big[:5, 2].any()
    say("outlier dimension: max ulp error where the bound is relaxed", int(u[~touched][~big[~touched]].max()))


@pytest.mark.parametrize("name,m,k,seed", [("blobs2d", 2_000, 5, 3), ("aniso28", 22_161, 25, 4),
                                           ("noisy28", 40_000, 50, 5)])
def test_lloyd_full_run_matches_oracle(dev, api, name, m, k, seed):
    S, C0 = _lloyd_case(name, m, k, seed)
    say("lloyd full", name, S.shape, k)
    res = api.lloyd(to_dev(S, dev), to_dev(C0, dev), max_iter=300, tol=1e-4)
    o = okm.lloyd(S, C0, 300, 1e-4)
    assert abs(res["iters"] - o["iters"]) <= 1
    if res["iters"] == o["iters"]:
        scale = np.abs(S).max()
        assert np.abs(res["C"].cpu().numpy() - o["C"]).max() <= 1e-5 * scale
        assert abs(res["f"] - o["f"]) <= 1e-5 * o["f"]
    # the GPU's own result is self-consistent: f = f(C_gpu, S)
    fo = okm.objective(S, res["C"].cpu().numpy())
    assert abs(res["f"] - fo) <= F_TOL * fo


def test_lloyd_empty_cluster_is_degenerate_and_kept(dev, api):
    r = np.random.default_rng(6)
    S = r.standard_normal((3_000, 6)).astype(np.float32)
    C0 = S[:4].copy()
    C0[2] = 1e3
    res = api.lloyd(to_dev(S, dev), to_dev(C0, dev))
    deg = res["deg"].cpu().numpy()
    assert deg[2] == 1 and deg.sum() == 1
    assert np.array_equal(res["C"].cpu().numpy()[2], C0[2])


@pytest.mark.parametrize("s,n,k", [(1, 1, 1), (7, 3, 7), (300, 2, 1), (513, 64, 40), (5_000, 16, 200)])
def test_lloyd_edge_shapes(dev, api, s, n, k):
    r = np.random.default_rng(s + k)
    S = r.standard_normal((s, n)).astype(np.float32)
    C0 = S[r.choice(s, k, replace=False)].copy()
    say("lloyd edge", s, n, k)
    res = api.lloyd(to_dev(S, dev), to_dev(C0, dev))
    fo = okm.objective(S, res["C"].cpu().numpy())
    assert abs(res["f"] - fo) <= F_TOL * fo + 1e-30
    o = okm.lloyd(S, C0)
    assert abs(res["f"] - o["f"]) <= 1e-4 * o["f"] + 1e-30


def test_lloyd_max_iter_zero(dev, api):
    r = np.random.default_rng(7)
    S = r.standard_normal((1000, 4)).astype(np.float32)
    C0 = S[:10].copy()
    res = api.lloyd(to_dev(S, dev), to_dev(C0, dev), max_iter=0)
    assert res["iters"] == 0
    assert np.array_equal(res["C"].cpu().numpy(), C0)


def test_lloyd_deterministic(dev, api):
    S, C0 = _lloyd_case("noisy28", 30_000, 50, 8)
    a = api.lloyd(to_dev(S, dev), to_dev(C0, dev))
    b = api.lloyd(to_dev(S, dev), to_dev(C0, dev))
    assert a["f"] == b["f"] and a["iters"] == b["iters"]
    assert np.array_equal(a["C"].cpu().numpy(), b["C"].cpu().numpy())


# ---------------------------------------------------------------------------
# a2: greedy K-means++
# ---------------------------------------------------------------------------
def _replay_kmeanspp(S, C_init, deg_init, picks, n_cand, seed, worker, g):
    """Check every GPU step against the oracle's D built from the GPU's own
    earlier choices.  Returns the number of steps whose choice equals the
    oracle's own draw."""
    S = S.astype(np.float64)
    k = C_init.shape[0]
    key = orng.stream_key(seed, worker, orng.PURPOSE_KMPP)
    D = None
    for j in range(k):
        if not deg_init[j]:
            dj = okm.sqdist_direct(S, C_init[j])
            D = dj if D is None else np.minimum(D, dj)
    exact = 0
    step = 0
    for j in range(k):
        if not deg_init[j]:
            assert (picks[j] == -1).all()
            continue
        chosen, cands = int(picks[j, 0]), [int(v) for v in picks[j, 1:] if v >= 0]
        w = orng.philox_block_scalar((step, g, 0, 0), key)
        s = S.shape[0]
        T = None if D is None else float(np.cumsum(D)[-1])
        if D is None or not (0.0 < T < math.inf):
            assert cands == [] and chosen == orng.mulhi(w[3], s)
            exact += 1
        else:
            assert len(cands) == n_cand
            prefix = np.cumsum(D)
            pots = []
            for c, ic in enumerate(cands):
                tau = orng.u01(w[c]) * T
                before = prefix[ic - 1] if ic > 0 else 0.0
                assert D[ic] > 0
                assert before <= tau + 1e-5 * T and prefix[ic] >= tau - 1e-5 * T
                pots.append(math.fsum(np.minimum(D, okm.sqdist_direct(S, S[ic])).tolist()))
            best = int(np.argmin(pots))
            pc = pots[cands.index(chosen)]
            assert pc <= pots[best] * (1 + 1e-5)
            oc = [int(np.searchsorted(prefix, orng.u01(w[c]) * T, side="right")) for c in range(n_cand)]
            exact += int(oc == cands)
        dn = okm.sqdist_direct(S, S[chosen])
        D = dn if D is None else np.minimum(D, dn)
        step += 1
    return exact, step


@pytest.mark.parametrize("name,m,k,n_cand,seed", [("blobs2d", 2_000, 5, 3, 0),
                                                  ("aniso28", 22_161, 25, 3, 1),
                                                  ("noisy28", 30_001, 50, 3, 2),
                                                  ("aniso28", 5_000, 25, 1, 3)])
def test_kmeanspp_all_degenerate(dev, api, name, m, k, n_cand, seed):
    S = _data(name, m, seed)
    n = S.shape[1]
    C = np.zeros((k, n), np.float32)
    deg = np.ones(k, np.uint8)
    say("kmeans++", name, S.shape, k, n_cand)
    Cg, dg, picks = api.seed(to_dev(S, dev), to_dev(C, dev), to_dev(deg, dev), n_cand,
                             seed=seed, worker=2, g=5, return_picks=True)
    picks = picks.cpu().numpy()
    Cg = Cg.cpu().numpy()
    assert dg.cpu().numpy().sum() == 0
    assert np.array_equal(Cg, S[picks[:, 0]])
    exact, steps = _replay_kmeanspp(S, C, deg.astype(bool), picks, n_cand, seed, 2, 5)
    assert exact >= steps - 1
    # and against the oracle's own run from the same draws
    Co, _, log = okm.kmeanspp(S, C, deg.astype(bool), n_cand, seed, 2, 5)
    same = sum(int(e["chosen"] == p) for e, p in zip(log, picks[:, 0]))
    assert same >= k - 1


def test_kmeanspp_partial_reseed(dev, api):
    S = _data("noisy28", 20_000, 4)
    r = np.random.default_rng(9)
    k = 50
    C = S[r.choice(len(S), k, replace=False)].copy()
    deg = (r.random(k) < 0.2).astype(np.uint8)
    deg[0] = 1
    Cg, dg, picks = api.seed(to_dev(S, dev), to_dev(C, dev), to_dev(deg, dev), 3, seed=4,
                             worker=9, g=123, return_picks=True)
    Cg = Cg.cpu().numpy()
    picks = picks.cpu().numpy()
    keep = deg == 0
    assert np.array_equal(Cg[keep], C[keep])
    exact, steps = _replay_kmeanspp(S, C, deg.astype(bool), picks, 3, 4, 9, 123)
    assert steps == deg.sum() and exact >= steps - 1


def test_kmeanspp_duplicate_points_zero_total(dev, api):
    # two distinct points, four centres: once both are covered T = 0 -> uniform picks
    S = np.array([[0, 0], [1, 1]] * 50, np.float32)
    C = np.zeros((4, 2), np.float32)
    deg = np.ones(4, np.uint8)
    Cg, dg, picks = api.seed(to_dev(S, dev), to_dev(C, dev), to_dev(deg, dev), 3, 1, 0, 0,
                             return_picks=True)
    exact, steps = _replay_kmeanspp(S, C, deg.astype(bool), picks.cpu().numpy(), 3, 1, 0, 0)
    assert steps == 4
    assert okm.objective(S, Cg.cpu().numpy()) == 0.0


# ---------------------------------------------------------------------------
# a7 + everything: Algorithm 1 end to end
# ---------------------------------------------------------------------------
def test_bigmeans_blobs2d_end_to_end(dev, api):
    # 20,000 points in 2-D from 5 Gaussians; k = 5; s = 2,000; 4 workers; 20 rounds of 10 passes
    X = _data("blobs2d", None, 0)
    P = dict(k=5, workers=4, rounds_T=20, passes_p=10, s_min=2000, s_max=2000, seed=0)
    say("bigmeans blobs2d", X.shape, P)
    g = api.bigmeans_run(to_dev(X, dev), api.RunParams(size_policy=1, **P))
    o = obm.bigmeans_run(X, obm.Params(size_policy=obm.SIZE_FIXED, **P))
    assert abs(g["f_full"] - o["f_full"]) <= 0.01 * o["f_full"]
    assert g["s_opt"] == 2000
    # f_full is f(C_best, X) of the returned centroids
    fo = okm.objective(X, g["C_best"].cpu().numpy())
    assert abs(g["f_full"] - fo) <= F_TOL * fo
    lab, _, _, near = okm.assign(X, g["C_best"].cpu().numpy(), return_second=True)
    assert np.array_equal(g["Y"].cpu().numpy()[~near], lab[~near])


def test_bigmeans_uniform_sizes_matches_oracle(dev, api):
    X = _data("aniso28", 100_000, 1)
    P = dict(k=25, workers=6, rounds_T=3, passes_p=4, s_min=2000, s_max=8000, seed=3)
    say("bigmeans aniso28 uniform", X.shape, P)
    g = api.bigmeans_run(to_dev(X, dev), api.RunParams(size_policy=0, **P))
    o = obm.bigmeans_run(X, obm.Params(size_policy=obm.SIZE_UNIFORM, **P))
    assert abs(g["f_full"] - o["f_full"]) <= 0.01 * o["f_full"]
    assert g["improvements"] >= P["workers"]


@pytest.mark.parametrize("policy,seed", [(2, 11), (0, 12), (3, 13), (4, 14)])
def test_bigmeans_execution_modes_identical(dev, api, policy, seed):
    # persistent rounds (1), one launch per Lloyd step (2) and one worker per
    # launch (0) compute the same arithmetic: results are bitwise identical
    X = _data("noisy28", 50_000, 2)
    P = dict(k=20, workers=5, rounds_T=3, passes_p=3, s_min=1000, s_max=6000, seed=seed,
             size_policy=policy)
    say("bigmeans modes", X.shape, P)
    runs = [api.bigmeans_run(to_dev(X, dev), api.RunParams(batched=b, **P)) for b in (1, 2, 0)]
    a = runs[0]
    for b in runs[1:]:
        assert a["f_full"] == b["f_full"] and a["s_opt"] == b["s_opt"]
        assert a["best_worker"] == b["best_worker"] and a["lloyd_dists"] == b["lloyd_dists"]
        assert a["improvements"] == b["improvements"]
        assert np.array_equal(a["C_best"].cpu().numpy(), b["C_best"].cpu().numpy())
        assert np.array_equal(a["Y"].cpu().numpy(), b["Y"].cpu().numpy())


@pytest.mark.parametrize("k", [10, 20])
def test_bigmeans_modes_identical_shared_units(dev, api, k):
    # 64 workers with samples of 4,096 to 262,144 points: each XCD holds about
    # eight of them, so in the persistent rounds the workgroups of a worker
    # have several assignment units each and share them dynamically (claimed
    # from a counter), while workers left with one workgroup keep their own
    # range; the result is bitwise the one of one launch per Lloyd step
    # (k = 10: ranking on the FP32 FMAs, two points per lane; k = 20: on the
    # matrix cores, one point per lane)
    X = _data("noisy28", 400_000, 4)
    P = dict(k=k, workers=64, rounds_T=2, passes_p=2, s_min=4096, s_max=262_144, seed=40 + k,
             size_policy=2)
    say("bigmeans modes, shared units", X.shape, P)
    a, b = [api.bigmeans_run(to_dev(X, dev), api.RunParams(batched=m, **P)) for m in (1, 2)]
    assert a["f_full"] == b["f_full"] and a["s_opt"] == b["s_opt"]
    assert a["best_worker"] == b["best_worker"] and a["lloyd_dists"] == b["lloyd_dists"]
    assert a["lloyd_iters"] == b["lloyd_iters"] and a["improvements"] == b["improvements"]
    assert np.array_equal(a["C_best"].cpu().numpy(), b["C_best"].cpu().numpy())
    assert np.array_equal(a["Y"].cpu().numpy(), b["Y"].cpu().numpy())


@pytest.mark.parametrize("k", [100, 150])
def test_bigmeans_execution_modes_identical_cooperative_redecision(dev, api, k):
    # k = 100 and 150 in 64-D: the round kernel re-decides a flagged point in
    # one lane, the per-step kernels with the whole wave -- the same values and
    # choices; at k = 150 the per-step kernels rank on the matrix cores too
    X = datagen.serving_dataset(64, m=40_000, seed=5)
    P = dict(k=k, workers=3, rounds_T=2, passes_p=2, s_min=3000, s_max=6000, seed=21,
             size_policy=2)
    say("bigmeans modes, cooperative re-decision", X.shape, P)
    runs = [api.bigmeans_run(to_dev(X, dev), api.RunParams(batched=b, **P)) for b in (1, 2, 0)]
    a = runs[0]
    for b in runs[1:]:
        assert a["f_full"] == b["f_full"] and a["s_opt"] == b["s_opt"]
        assert a["best_worker"] == b["best_worker"] and a["lloyd_dists"] == b["lloyd_dists"]
        assert np.array_equal(a["C_best"].cpu().numpy(), b["C_best"].cpu().numpy())
        assert np.array_equal(a["Y"].cpu().numpy(), b["Y"].cpu().numpy())
    o = obm.bigmeans_run(X, obm.Params(**P))
    assert abs(a["f_full"] - o["f_full"]) <= 0.01 * o["f_full"]


def test_bigmeans_shrink_policy_matches_oracle(dev, api):
    # sizes narrowing around the mean of L (Section 7's open question)
    X = _data("aniso28", 100_000, 3)
    P = dict(k=25, workers=6, rounds_T=4, passes_p=4, s_min=2000, s_max=16000, seed=6,
             size_policy=4)
    say("bigmeans shrink", X.shape, P)
    g = api.bigmeans_run(to_dev(X, dev), api.RunParams(**P))
    o = obm.bigmeans_run(X, obm.Params(**P))
    assert abs(g["f_full"] - o["f_full"]) <= 0.01 * o["f_full"]
    assert 2000 <= g["s_opt"] <= 16000


def test_bigmeans_bins_policy_runs(dev, api):
    X = _data("noisy28", 60_000, 3)
    P = dict(k=10, workers=8, rounds_T=4, passes_p=2, s_min=1 << 10, s_max=1 << 14, seed=5,
             size_policy=3)
    g = api.bigmeans_run(to_dev(X, dev), api.RunParams(**P))
    o = obm.bigmeans_run(X, obm.Params(**P))
    assert abs(g["f_full"] - o["f_full"]) <= 0.01 * o["f_full"]


def test_bigmeans_trace_and_nan_rows(dev, api):
    X = _data("blobs2d", 4_000, 4).copy()
    X[::9] = np.nan                      # every sample of 500 rows contains NaN rows
    P = api.RunParams(k=3, workers=2, rounds_T=2, passes_p=2, s_min=500, s_max=500,
                      size_policy=1, seed=5)
    seen = []
    g = api.bigmeans_run(to_dev(X, dev), P, trace=lambda r, C, fh, s, t, *L: seen.append((r, list(fh), L)))
    assert g["improvements"] == 0
    assert [r for r, _, _ in seen] == [0, 1]
    assert all(math.isinf(f) for _, fh, _ in seen for f in fh)
    assert all(L == (0, 0) for _, _, L in seen)     # nothing accepted: L stays empty


@pytest.mark.parametrize("n", [36, 64])
def test_bigmeans_modes_identical_wider_rows(dev, api, n):
    # rows of 32 floats or more: outside the round kernel the K-means++
    # potentials stage the rows through LDS; every mode still gives the same bits
    X = datagen.noisy_mixture(30_000, n, 10, seed=n)
    P = dict(k=12, workers=4, rounds_T=2, passes_p=3, s_min=1500, s_max=5000, seed=3,
             size_policy=2)
    say("bigmeans modes, n =", n)
    runs = [api.bigmeans_run(to_dev(X, dev), api.RunParams(batched=b, **P)) for b in (1, 2, 0)]
    a = runs[0]
    for b in runs[1:]:
        assert a["f_full"] == b["f_full"] and a["lloyd_dists"] == b["lloyd_dists"]
        assert np.array_equal(a["C_best"].cpu().numpy(), b["C_best"].cpu().numpy())


def test_tile_tuning_changes_no_result(dev, api):
    # the tile size of the one-step-per-launch Lloyd paths is chosen by timing;
    # every choice gives the same bits (narrow and wide points, Algorithm 1)
    r = np.random.default_rng(21)
    out = {}
    for on in (False, True):
        api.set_tuning(dev, on)
        res = []
        for n, k in ((20, 17), (96, 40)):
            S = (r.standard_normal((60_000, n)) + 3 * r.integers(0, 8, (60_000, 1))).astype(np.float32) \
                if on is False else out["S", n]
            out["S", n] = S
            C0 = S[:k].copy()
            g = api.lloyd(to_dev(S, dev), to_dev(C0, dev))
            res.append((g["f"], g["iters"], g["C"].cpu().numpy().tobytes(), g["labels"].cpu().numpy().tobytes()))
        X = _data("aniso28", 80_000, 4)
        b = api.bigmeans_run(to_dev(X, dev), api.RunParams(k=25, workers=6, rounds_T=2, passes_p=2,
                                                           s_min=4096, s_max=30_000, size_policy=2,
                                                           seed=2, batched=2))
        res.append((b["f_full"], b["C_best"].cpu().numpy().tobytes()))
        out[on] = res
    api.set_tuning(dev, True)
    assert out[False] == out[True]
