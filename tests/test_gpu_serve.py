"""GPU tests of the serving loop (bm_serve) through the C ABI.

* Each job's result is the same alone (one running job at a time) and in the
  mix (many running jobs of several data sets, dimensions and k): bitwise.
* Each worker's chain of jobs matches the oracle's chain of single passes of
  Algorithm 1 (oracle.bigmeans.worker_pass): the Lloyd objective of every job
  within 1e-5 relative when both take the same number of updates, the
  acceptance decisions identical, and the final incumbent objective within 1%.
* Paced arrivals: no job starts before it arrives; latencies are reported.
"""

import math

import numpy as np
import pytest

from oracle import bigmeans as obm
from paper_2403_18766_amd import datagen
from tests.gpu_common import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def api():
    from paper_2403_18766_amd import api as a
    return a


def _datasets():
    # the noisy Gaussian-mixture recipe in three dimensions (narrow, narrow, wide)
    return [datagen.noisy_mixture(20_000, n, 12, seed=n) for n in (16, 28, 96)]


def _jobs(nds, njobs, seed, ks=(5, 12), workers=4, s_lo=500, s_hi=4_000, rate=None):
    r = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for _ in range(njobs):
        if rate:
            t += float(r.exponential(1.0 / rate))
        s = int(math.floor(math.exp(r.uniform(math.log(s_lo), math.log(s_hi + 1)))))
        jobs.append(dict(arrival=t, s=min(s, s_hi), dataset=int(r.integers(nds)),
                         k=int(ks[r.integers(len(ks))]), worker=int(r.integers(workers))))
    return jobs


def _fields(res):
    return [(r["f"], r["f_incumbent"], r["iters"], r["accepted"], r["ndeg"]) for r in res]


def test_serve_alone_equals_mix(dev, api):
    Xs = _datasets()
    Xd = [to_dev(X, dev) for X in Xs]
    jobs = _jobs(len(Xs), 48, 1)
    say("serve mix", len(jobs), "jobs")
    mix, st_mix = api.serve(Xd, jobs, seed=3, max_slots=16)
    alone, st_alone = api.serve(Xd, jobs, seed=3, max_slots=1)
    assert st_mix["peak_running"] > 1 and st_alone["peak_running"] <= len(Xs) * 2
    assert _fields(mix) == _fields(alone)
    # a smaller budget (but room for one slot of every group) admits fewer
    # jobs at once and still gives the same results
    budget = max(st_mix["peak_bytes"] // 2, st_alone["slot_bytes"])
    small, st_small = api.serve(Xd, jobs, seed=3, max_slots=16, budget_bytes=budget)
    assert st_small["peak_bytes"] <= budget and st_small["slot_bytes"] <= budget
    assert st_small["peak_running"] <= st_mix["peak_running"]
    assert st_mix["slot_bytes"] <= 200 << 30
    assert _fields(small) == _fields(mix)


def test_serve_matches_oracle_chains(dev, api):
    Xs = _datasets()
    Xd = [to_dev(X, dev) for X in Xs]
    jobs = _jobs(len(Xs), 30, 2, ks=(4, 9), workers=3)
    say("serve vs oracle", len(jobs), "jobs")
    res, _ = api.serve(Xd, jobs, seed=5, max_slots=8)
    # replay every worker's chain in arrival order with the oracle
    state = {}
    same_iters = 0
    for j, jb in sorted(enumerate(jobs), key=lambda e: (e[1]["arrival"], e[0])):
        key = (jb["dataset"], jb["k"], jb["worker"])
        X = Xs[jb["dataset"]]
        if key not in state:
            state[key] = dict(C=np.zeros((jb["k"], X.shape[1])), deg=np.ones(jb["k"], bool),
                              fhat=math.inf, s_prev=None, g=0)
        S = state[key]
        wid = (jb["dataset"] << 20) | (jb["k"] << 10) | jb["worker"]
        o = obm.worker_pass(X, S["C"], S["deg"], S["fhat"], S["s_prev"], jb["s"], 5, wid, S["g"],
                            S["g"], 3, 300, 1e-4)
        S.update(C=o["C"], deg=o["deg"], fhat=o["fhat"], s_prev=jb["s"], g=S["g"] + 1)
        g = res[j]
        if g["iters"] == o["iters"]:
            same_iters += 1
            assert abs(g["f"] - o["f"]) <= 1e-5 * abs(o["f"]), (j, g["f"], o["f"])
        assert g["accepted"] == o["accepted"] or abs(g["f"] - g["f_incumbent"]) <= 1e-5 * g["f"]
        assert abs(g["f_incumbent"] - o["fhat"]) <= 0.01 * o["fhat"], (j, g, o["fhat"])
    assert same_iters >= 0.8 * len(jobs)


def test_serve_paced_latency(dev, api):
    Xs = _datasets()
    Xd = [to_dev(X, dev) for X in Xs]
    jobs = _jobs(len(Xs), 40, 3, rate=400.0)
    res, st = api.serve(Xd, jobs, seed=1, max_slots=16, paced=True)
    for r, jb in zip(res, jobs):
        assert r["admitted"] >= jb["arrival"] - 1e-6
        assert r["finished"] >= r["admitted"]
    lat = np.array([r["finished"] - jb["arrival"] for r, jb in zip(res, jobs)])
    say("serve paced: p50", np.percentile(lat, 50), "p99", np.percentile(lat, 99), "s")
    assert np.all(lat > 0)
    # unpaced, the same jobs give the same results
    unpaced, _ = api.serve(Xd, jobs, seed=1, max_slots=16)
    assert _fields(unpaced) == _fields(res)


def test_serve_rejects_invalid(dev, api):
    from paper_2403_18766_amd.api import BigmeansError
    X = to_dev(datagen.noisy_mixture(1_000, 8, 3, seed=0), dev)
    with pytest.raises(BigmeansError):
        api.serve([X], [dict(s=5, dataset=0, k=10, worker=0)])       # k > s
    with pytest.raises(BigmeansError):
        api.serve([X], [dict(s=50, dataset=1, k=2, worker=0)])       # no such data set
    with pytest.raises(BigmeansError):
        api.serve([X], [dict(s=50, dataset=0, k=2, worker=0)], budget_bytes=1)


def test_serve_budget_bounds_reserved_slots(dev, api):
    # many (dataset, k) groups and a budget just above one slot each: the
    # reserved slots stay within the budget, results unchanged; below one
    # slot per group the call is refused
    from paper_2403_18766_amd.api import BigmeansError
    Xs = _datasets()
    Xd = [to_dev(X, dev) for X in Xs]
    jobs = _jobs(len(Xs), 36, 4, ks=(3, 5, 8), workers=2)
    ref, st_ref = api.serve(Xd, jobs, seed=2, max_slots=16)
    one_each = st_ref["slot_bytes"] // max(1, st_ref["peak_running"])
    # the bytes of one slot of every group, from a run with one slot each
    _, st_one = api.serve(Xd, jobs, seed=2, max_slots=1)
    budget = st_one["slot_bytes"] + st_one["slot_bytes"] // 4
    res, st = api.serve(Xd, jobs, seed=2, max_slots=16, budget_bytes=budget)
    say("serve budget", budget, "slots", st["slot_bytes"], "one each", st_one["slot_bytes"], one_each)
    assert st["slot_bytes"] <= budget and st["peak_bytes"] <= budget
    assert _fields(res) == _fields(ref)
    with pytest.raises(BigmeansError):
        api.serve(Xd, jobs, seed=2, max_slots=16, budget_bytes=st_one["slot_bytes"] - 1)
