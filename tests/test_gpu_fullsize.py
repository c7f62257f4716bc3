"""GPU parity at the full sizes of the measured workloads, in the launch
configurations bench.py times (fewer rounds, same per-launch shapes), checked
on outputs the FP64 oracle can compute: f(C_best, X) over every point, and
the labels of sampled points.

  * vmf768: 2,000,000 unit vectors in 768-D, k = 100, 16 workers with samples
    of 131,072 (one launch per Lloyd step), FP32 and BF16 matrix cores;
  * noisy28: 10,000,000 points in 28-D, k = 50, 64 workers with BINS sizes in
    [2^12, 2^17] (one persistent launch per round);
  * serving: the three resident 4,000,000-point data sets (n = 16, 64, 256)
    with a slice of the job stream; each result is the same served alone, and
    each worker's chain matches the oracle's chain of single passes;
  * Algorithm 1 against the oracle's own Algorithm-1 result on the same data
    (tests/golden/<workload>_reference.json, written by make_reference.py):
    noisy28 with all 100 rounds, vmf768 in both precisions, f(C_best, X)
    within 1 %.
"""

import json
import math
import os

import numpy as np
import pytest

from oracle import kmeans as okm
from paper_2403_18766_amd import datagen
from tests.gpu_common import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu

F_TOL = 1e-6


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def api():
    from paper_2403_18766_amd import api as a
    return a


def _check_run(X_host, g, label, rng):
    C = g["C_best"].cpu().numpy()
    Y = g["Y"].cpu().numpy()
    rows = np.sort(rng.choice(X_host.shape[0], 20_000, replace=False))
    olab, _, _, onear = okm.assign(X_host[rows], C, return_second=True)
    mism = np.count_nonzero(Y[rows][~onear] != olab[~onear])
    assert mism == 0, f"{label}: {mism} sampled labels differ outside near ties"
    say(label, "oracle f over all", X_host.shape[0], "points")
    fo = okm.objective(X_host, C)
    assert abs(g["f_full"] - fo) <= F_TOL * fo, (label, g["f_full"], fo)
    return fo


def test_vmf768_full_size_both_precisions(dev, api):
    say("vmf768 full size: generating 2,000,000 x 768 on the device")
    X = datagen.vmf_mixture_device(20_000, 768, 100, dev, seed=0)
    P = dict(k=100, workers=16, rounds_T=1, passes_p=2, s_min=131_072, s_max=131_072,
             size_policy=1, seed=0, batched=2)
    runs = {}
    for prec in (0, 1):
        say("vmf768 full size: run, prec", prec)
        runs[prec] = api.bigmeans_run(X, api.RunParams(prec=prec, **P))
    Xh = X.cpu().numpy()
    del X
    rng = np.random.default_rng(0)
    fo = _check_run(Xh, runs[0], "vmf768 fp32", rng)
    if np.array_equal(runs[1]["C_best"].cpu().numpy(), runs[0]["C_best"].cpu().numpy()):
        assert runs[1]["f_full"] == runs[0]["f_full"]
    else:
        _check_run(Xh, runs[1], "vmf768 bf16", rng)
    assert abs(runs[1]["f_full"] - fo) <= 0.01 * fo


@pytest.fixture(scope="module")
def noisy28_host():
    say("noisy28 full size: generating 10,000,000 x 28 on the host")
    return datagen.make("noisy28")


def test_noisy28_full_size_persistent_rounds(dev, api, noisy28_host):
    from paper_2403_18766_amd import _lib
    Xh = noisy28_host
    X = to_dev(Xh, dev)
    P = api.RunParams(k=50, workers=64, rounds_T=3, passes_p=10, s_min=1 << 12, s_max=1 << 17,
                      size_policy=_lib.BM_SIZE_BINS, seed=0, batched=1)
    say("noisy28 full size: run")
    g = api.bigmeans_run(X, P)
    assert 1 << 12 <= g["s_opt"] <= 1 << 17
    _check_run(Xh, g, "noisy28", np.random.default_rng(1))
    # the same run in one launch per Lloyd step gives the same bits
    say("noisy28 full size: run, one launch per Lloyd step")
    P.batched = 2
    g2 = api.bigmeans_run(X, P)
    assert g2["f_full"] == g["f_full"]
    assert np.array_equal(g2["C_best"].cpu().numpy(), g["C_best"].cpu().numpy())


@pytest.fixture(scope="module")
def serving_host():
    say("serving full size: generating three 4,000,000-point data sets on the host")
    return [datagen.serving_dataset(n, m=4_000_000) for n in (16, 64, 256)]


def test_serving_full_size_datasets_alone_equals_mix(dev, api, serving_host):
    Xs = [to_dev(X, dev) for X in serving_host]
    r = np.random.default_rng(0)
    jobs = []
    for _ in range(60):
        s = int(math.floor(math.exp(r.uniform(math.log(1024), math.log(262_145)))))
        jobs.append(dict(s=min(s, 262_144), dataset=int(r.integers(3)), k=int(r.choice([10, 50, 200])),
                         worker=int(r.integers(4)), prec=int(r.integers(2))))
    say("serving full size: mix")
    mix, st = api.serve(Xs, jobs, seed=0, max_slots=64)
    say("serving full size: alone")
    alone, _ = api.serve(Xs, jobs, seed=0, max_slots=1)
    key = lambda res: [(q["f"], q["f_incumbent"], q["iters"], q["accepted"], q["ndeg"]) for q in res]
    assert st["peak_running"] > 1
    assert key(mix) == key(alone)
    for q in mix:
        assert math.isfinite(q["f"])
        if q["accepted"]:
            assert q["f_incumbent"] == q["f"]


def test_serving_full_size_matches_oracle_chains(dev, api, serving_host):
    """100 sampled jobs of the serving stream on the three 4,000,000-point data
    sets (FP32 and BF16 jobs, k in {10, 50}, three workers per group, samples
    of 1,024 to 4,096 points so that the FP64 replay stays short): every
    worker's chain of jobs is replayed with the oracle's single passes of
    Algorithm 1 on the same data."""
    from oracle import bigmeans as obm
    Xd = [to_dev(X, dev) for X in serving_host]
    r = np.random.default_rng(7)
    jobs = []
    for _ in range(100):
        s = int(math.floor(math.exp(r.uniform(math.log(1024), math.log(4097)))))
        jobs.append(dict(s=min(s, 4096), dataset=int(r.integers(3)), k=int(r.choice([10, 50])),
                         worker=int(r.integers(3)), prec=int(r.integers(2))))
    say("serving full size vs oracle:", len(jobs), "jobs")
    res, _ = api.serve(Xd, jobs, seed=11, max_slots=16)
    state = {}
    same_iters = 0
    for j, jb in enumerate(jobs):  # equal arrival times: list order
        key = (jb["dataset"], jb["k"], jb["worker"])
        X = serving_host[jb["dataset"]]
        if key not in state:
            state[key] = dict(C=np.zeros((jb["k"], X.shape[1])), deg=np.ones(jb["k"], bool),
                              fhat=math.inf, s_prev=None, g=0)
        S = state[key]
        wid = (jb["dataset"] << 20) | (jb["k"] << 10) | jb["worker"]
        say("oracle replay job", j, "n", X.shape[1], "k", jb["k"], "s", jb["s"])
        o = obm.worker_pass(X, S["C"], S["deg"], S["fhat"], S["s_prev"], jb["s"], 11, wid,
                            S["g"], S["g"], 3, 300, 1e-4)
        S.update(C=o["C"], deg=o["deg"], fhat=o["fhat"], s_prev=jb["s"], g=S["g"] + 1)
        g = res[j]
        if g["iters"] == o["iters"]:
            same_iters += 1
            assert abs(g["f"] - o["f"]) <= 1e-5 * abs(o["f"]), (j, g["f"], o["f"])
        assert g["accepted"] == o["accepted"] or abs(g["f"] - g["f_incumbent"]) <= 1e-5 * g["f"]
        assert abs(g["f_incumbent"] - o["fhat"]) <= 0.01 * o["fhat"], (j, g, o["fhat"])
    assert same_iters >= 0.8 * len(jobs)


def _reference(name):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        f"{name}_reference.json")
    if not os.path.exists(path):
        pytest.skip(f"no oracle reference for {name}")
    with open(path) as f:
        return json.load(f)


def _params_of(api, ref, **kw):
    c = ref["params"]
    return api.RunParams(k=c["k"], workers=c["workers"], rounds_T=c["rounds_T"],
                         passes_p=c["passes_p"], s_min=c["s_min"], s_max=c["s_max"],
                         size_policy=c["size_policy"], max_iter=c.get("max_iter", 300),
                         tol=c.get("tol", 1e-4), n_candidates=c.get("n_candidates", 3),
                         seed=c["seed"], **kw)


def test_noisy28_algorithm1_within_1pct_of_oracle(dev, api, noisy28_host):
    """The whole competitive run (64 workers, BINS sizes, 100 rounds, the final
    stage's selection) against the oracle's Algorithm-1 run on the same data."""
    ref = _reference("noisy28")
    assert datagen.sha256_chunked(noisy28_host) == ref["x_sha256_chunked"]
    X = to_dev(noisy28_host, dev)
    say("noisy28 Algorithm 1,", ref["params"]["rounds_T"], "rounds, persistent rounds")
    g = api.bigmeans_run(X, _params_of(api, ref, batched=1), labels=False)
    gap = (g["f_full"] - ref["f_full"]) / ref["f_full"]
    say("noisy28 f", g["f_full"], "oracle", ref["f_full"], "gap", gap)
    assert abs(gap) <= 0.01
    assert ref["params"]["s_min"] <= g["s_opt"] <= ref["params"]["s_max"]


def test_vmf768_algorithm1_within_1pct_of_oracle_both_precisions(dev, api):
    ref = _reference("vmf768")
    say("vmf768: generating 2,000,000 x 768 on the host")
    Xh = datagen.make("vmf768")
    assert datagen.sha256_chunked(Xh) == ref["x_sha256_chunked"]
    X = to_dev(Xh, dev)
    del Xh
    runs = {}
    for prec in (0, 1):
        say("vmf768 Algorithm 1, prec", prec)
        g = api.bigmeans_run(X, _params_of(api, ref, batched=2, prec=prec), labels=False)
        runs[prec] = g
        gap = (g["f_full"] - ref["f_full"]) / ref["f_full"]
        say("vmf768 prec", prec, "f", g["f_full"], "oracle", ref["f_full"], "gap", gap)
        assert abs(gap) <= 0.01
    # equal centroids (the certified labels coincide) give equal objectives
    if np.array_equal(runs[0]["C_best"].cpu().numpy(), runs[1]["C_best"].cpu().numpy()):
        assert runs[0]["f_full"] == runs[1]["f_full"]
