"""GPU parity of the BF16 matrix-core path (BM_BF16: split BF16 operands, FP32
accumulation) against the FP64 oracle and against the FP32 path, through the
C ABI.

The rigorous error bound of the split arithmetic sends every point whose two
best centres it cannot separate to the FP32 direct-form re-decision, and the
winner's distance is always the FP32 direct form, so the bars are those of
the FP32 path (tighter than the 1e-3 objective tolerance allowed for BF16):

  * labels identical to the oracle's except its near ties ((d2 - d1) < 1e-5 d2);
  * objectives within 1e-6 relative of the oracle;
  * labels and objective the same as the FP32 path's (except oracle near ties);
  * Lloyd runs: iterations within 1 of the oracle, the same f when equal;
  * Algorithm 1 end to end within 1% of the oracle's f(C, X), bitwise
    identical between the execution modes, and within 1% of the FP32 run.
"""

import math

import numpy as np
import pytest

from oracle import bigmeans as obm
from oracle import kmeans as okm
from paper_2403_18766_amd import datagen
from tests.gpu_common import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu

F_TOL = 1e-6
BF16 = 1


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def api():
    from paper_2403_18766_amd import api as a
    return a


@pytest.fixture(scope="module")
def vmf():
    return datagen.make("vmf768", m=20_000, seed=5)


def _check_objective(api, dev, X, C, label):
    say("objective bf16", label, X.shape, C.shape)
    Xd, Cd = to_dev(X, dev), to_dev(C, dev)
    f, lab, near = api.objective(Xd, Cd, prec=BF16)
    lab = lab.cpu().numpy()
    olab, od1, od2, onear = okm.assign(X, C, return_second=True)
    fo = math.fsum(od1.tolist())
    assert abs(f - fo) <= F_TOL * abs(fo) + 1e-300, (f, fo)
    ok = ~onear
    mism = np.nonzero(lab[ok] != olab[ok])[0]
    assert mism.size == 0, f"{mism.size} label mismatches outside near ties"
    assert abs(int(near) - int(onear.sum())) <= max(2, int(0.01 * onear.sum()))
    # the FP32 path on the same input
    f32, lab32, _ = api.objective(Xd, Cd)
    lab32 = lab32.cpu().numpy()
    assert np.array_equal(lab[ok], lab32[ok])
    assert abs(f - f32) <= F_TOL * abs(f32) + 1e-300
    return f, lab


def test_objective_bf16_vmf768(dev, api, vmf):
    r = np.random.default_rng(0)
    C = vmf[r.choice(len(vmf), 100, replace=False)].copy()
    _check_objective(api, dev, vmf, C, "vmf768 k=100")


def test_objective_bf16_vmf768_cluster_means(dev, api, vmf):
    # centroids at cluster means (the Lloyd regime: close top-2 gaps)
    r = np.random.default_rng(1)
    C = vmf[r.choice(len(vmf), 100, replace=False)].astype(np.float64)
    for _ in range(5):
        lab, _, _, _ = okm.assign(vmf, C, return_second=True)
        C, _ = okm.cluster_means(vmf, lab, 100, C)
    _check_objective(api, dev, vmf, C.astype(np.float32), "vmf768 cluster means")


@pytest.mark.parametrize("m,n,k", [(1, 65, 1), (300, 65, 7), (4_099, 101, 33), (2_049, 256, 200),
                                   (1_000, 768, 129), (513, 1_000, 5)])
def test_objective_bf16_shapes(dev, api, m, n, k):
    r = np.random.default_rng(m + n + k + 1)
    X = r.standard_normal((m, n)).astype(np.float32)
    C = r.standard_normal((k, n)).astype(np.float32)
    _check_objective(api, dev, X, C, f"m={m} n={n} k={k}")


@pytest.mark.parametrize("k", [129, 200, 256, 257])
def test_objective_bf16_two_groups_many_redecisions(dev, api, k):
    # noisy 256-D mixture, centres near data points: most points have several
    # centres of their own cluster at nearly the same distance, so a large
    # share goes through the re-decision (and the FP32 path) -- among the candidates of
    # both centre groups up to k = 256, among all centres above
    X = datagen.serving_dataset(256, m=6_000, seed=3)
    r = np.random.default_rng(k)
    C = (X[r.choice(len(X), k, replace=False)] + 0.05 * r.standard_normal((k, 256))).astype(np.float32)
    _check_objective(api, dev, X, C, f"two groups k={k}")


def test_objective_bf16_far_from_origin(dev, api):
    # large ||x|| and ||c||: the bound sends most points to the FP32 direct form
    r = np.random.default_rng(3)
    X = (300.0 + r.standard_normal((3_000, 96))).astype(np.float32)
    C = (300.0 + r.standard_normal((12, 96))).astype(np.float32)
    _check_objective(api, dev, X, C, "offset 300")


def test_objective_bf16_ties_and_small_values(dev, api):
    r = np.random.default_rng(4)
    X = r.integers(-3, 4, size=(2_000, 72)).astype(np.float32)
    C = r.integers(-3, 4, size=(9, 72)).astype(np.float32)
    C[7] = C[2]
    f, lab = _check_objective(api, dev, X, C, "duplicate centres")
    assert not np.any(lab == 7)
    # values that are not exact in BF16 (residual parts matter), tiny scale
    X = (r.standard_normal((1_500, 80)) * 1e-3 + 1e-3 / 3).astype(np.float32)
    C = X[r.choice(1_500, 17, replace=False)].copy()
    _check_objective(api, dev, X, C, "scale 1e-3")


@pytest.mark.parametrize("s,n,k,seed", [(5_000, 768, 20, 4), (3_001, 130, 150, 5), (700, 66, 3, 6)])
def test_lloyd_bf16_full_run(dev, api, s, n, k, seed):
    r = np.random.default_rng(seed)
    centres = r.standard_normal((k, n)) * 4
    S = (centres[r.integers(0, k, s)] + r.standard_normal((s, n))).astype(np.float32)
    C0 = S[r.choice(s, k, replace=False)].copy()
    say("lloyd bf16 full", S.shape, k)
    res = api.lloyd(to_dev(S, dev), to_dev(C0, dev), max_iter=300, tol=1e-4, prec=BF16)
    o = okm.lloyd(S, C0, 300, 1e-4)
    assert abs(res["iters"] - o["iters"]) <= 1
    if res["iters"] == o["iters"]:
        assert np.abs(res["C"].cpu().numpy() - o["C"]).max() <= 1e-5 * np.abs(S).max()
        assert abs(res["f"] - o["f"]) <= 1e-5 * o["f"]
    fo = okm.objective(S, res["C"].cpu().numpy())
    assert abs(res["f"] - fo) <= F_TOL * fo
    lab = res["labels"].cpu().numpy()
    olab, _, _, onear = okm.assign(S, res["C"].cpu().numpy(), return_second=True)
    assert np.array_equal(lab[~onear], olab[~onear])
    deg = res["deg"].cpu().numpy().astype(bool)
    assert np.array_equal(deg, np.bincount(olab, minlength=k) == 0)


def test_lloyd_bf16_matches_fp32_path(dev, api, vmf):
    # same start: the same updates as the FP32 path unless a near tie flips
    S = vmf[:12_000]
    C0 = vmf[-100:].copy()
    Sd, Cd = to_dev(S, dev), to_dev(C0, dev)
    a = api.lloyd(Sd, Cd, prec=BF16)
    b = api.lloyd(Sd, Cd)
    say("lloyd bf16 vs fp32: iters", a["iters"], b["iters"], "f", a["f"], b["f"])
    assert abs(a["iters"] - b["iters"]) <= 1
    assert abs(a["f"] - b["f"]) <= 1e-5 * b["f"]
    if a["iters"] == b["iters"]:
        assert np.abs(a["C"].cpu().numpy() - b["C"].cpu().numpy()).max() <= 1e-5
    # and deterministic
    c = api.lloyd(Sd, Cd, prec=BF16)
    assert c["f"] == a["f"] and np.array_equal(c["labels"].cpu().numpy(), a["labels"].cpu().numpy())


def test_bigmeans_bf16_end_to_end_and_modes(dev, api):
    X = datagen.make("vmf768", m=20_000, seed=4)
    P = dict(k=10, workers=4, rounds_T=2, passes_p=3, s_min=2000, s_max=2000, seed=7,
             size_policy=1)
    say("bigmeans bf16", X.shape, P)
    Xd = to_dev(X, dev)
    runs = [api.bigmeans_run(Xd, api.RunParams(batched=b, prec=BF16, **P)) for b in (1, 2, 0)]
    o = obm.bigmeans_run(X, obm.Params(**P))
    g = runs[0]
    assert abs(g["f_full"] - o["f_full"]) <= 0.01 * o["f_full"]
    fo = okm.objective(X, g["C_best"].cpu().numpy())
    assert abs(g["f_full"] - fo) <= F_TOL * fo
    for b in runs[1:]:
        assert g["f_full"] == b["f_full"] and g["best_worker"] == b["best_worker"]
        assert np.array_equal(g["C_best"].cpu().numpy(), b["C_best"].cpu().numpy())
        assert np.array_equal(g["Y"].cpu().numpy(), b["Y"].cpu().numpy())
    f32 = api.bigmeans_run(Xd, api.RunParams(**P))
    assert abs(g["f_full"] - f32["f_full"]) <= 0.01 * f32["f_full"]


def test_serve_bf16_alone_equals_mix(dev, api):
    # one wide data set, jobs of both precisions (one launch group per precision)
    Xs = [datagen.noisy_mixture(20_000, 96, 12, seed=11), datagen.noisy_mixture(20_000, 16, 12, seed=12)]
    Xd = [to_dev(X, dev) for X in Xs]
    r = np.random.default_rng(5)
    jobs = [dict(s=int(r.integers(500, 4_000)), dataset=int(r.integers(2)), k=int(r.choice([5, 12])),
                 worker=int(r.integers(3)), prec=int(r.integers(2))) for _ in range(40)]
    say("serve bf16 mix", len(jobs), "jobs")
    mix, st = api.serve(Xd, jobs, seed=2, max_slots=16)
    alone, _ = api.serve(Xd, jobs, seed=2, max_slots=1)
    key = lambda res: [(q["f"], q["f_incumbent"], q["iters"], q["accepted"], q["ndeg"]) for q in res]
    assert st["peak_running"] > 1
    assert key(mix) == key(alone)


@pytest.mark.parametrize("prec", [0, BF16])
def test_nonfinite_inputs_wide(dev, api, prec):
    # NaN or infinity in a point: the objective is reported non-finite and a
    # Lloyd run stops at once (its f cannot decrease)
    r = np.random.default_rng(9)
    X = r.standard_normal((600, 96)).astype(np.float32)
    C = X[:5].copy()
    for bad in (np.nan, np.inf):
        Y = X.copy()
        Y[311, 40] = bad
        say("non-finite wide", prec, bad)
        f, _, _ = api.objective(to_dev(Y, dev), to_dev(C, dev), prec=prec)
        assert not math.isfinite(f)
        res = api.lloyd(to_dev(Y, dev), to_dev(C, dev), prec=prec)
        assert not math.isfinite(res["f"]) and res["iters"] == 0
    # finite data far beyond BF16's exact range still gives the FP32 path's result
    Z = (X * 3e4).astype(np.float32)
    fz, lz, _ = api.objective(to_dev(Z, dev), to_dev(Z[:5].copy(), dev), prec=prec)
    f32, l32, _ = api.objective(to_dev(Z, dev), to_dev(Z[:5].copy(), dev))
    assert abs(fz - f32) <= F_TOL * f32


def test_precision_argument_is_checked(dev, api):
    from paper_2403_18766_amd.api import BigmeansError
    X = to_dev(np.ones((100, 70), np.float32), dev)
    with pytest.raises(BigmeansError):
        api.objective(X, X[:3].clone(), prec=2)
    with pytest.raises(BigmeansError):
        api.lloyd(X, X[:3].clone(), prec=-1)
    # a narrow data set accepts BF16 and runs the FP32 vector path (same bits)
    Y = to_dev(np.random.default_rng(0).standard_normal((500, 12)).astype(np.float32), dev)
    a = api.objective(Y, Y[:4].clone(), prec=BF16)
    b = api.objective(Y, Y[:4].clone())
    assert a[0] == b[0] and np.array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())
