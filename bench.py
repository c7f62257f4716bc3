#!/usr/bin/env python3
"""Benchmark of the Big-means hot path on one MI355X.

Headline step = one run of Algorithm 1 (bm_bigmeans_run) on the noisy28
workload, competitive Big-means at scale: 10,000,000 points in 28-D from 50
Gaussians with 5 % uniform background noise, k = 50, 64 competing workers
whose sample sizes are re-drawn every round from the best-performing of five
log-width bins over [2^12, 2^17], 100 rounds of 10 passes (sampling,
K-means++, Lloyd, acceptance), then the final selection and the full
assignment of X with f(C, X) in FP64 accumulation.  X is resident in HBM
before the timed region.

Printed (one JSON line):
  value           Lloyd point-centre distances per second over the whole job
                  (sum over Lloyd runs of s * k * assignment steps / wall time)
  roofline        the persistent round kernel k_round<28> (one launch per
                  round): algorithmic FLOPs (2 n per distance) over its device
                  time, HIP events on the library's stream inside the timed
                  region, against the FP32 vector peak (the binding roofline
                  at n = 28, k = 50); beside it the algorithmic HBM bytes
                  (4 n / k per distance) against 8 TB/s and the counted traffic
  cpu_baseline    the FP64 oracle on a process pool of this host's cores, on a
                  bounded slice of the same workload
  time_to_target  device seconds until Algorithm 1's final stage, applied after
                  round R, returns C with f(C, X) within 1 % of the oracle's
                  final f; assignment agreement of the final labels
  seeds           the headline run with algorithm seeds 0-4: wall time and
                  f(C_best, X), median / min / max
Secondary legs: aniso28 (1,000,000 x 28, k = 25, 32 workers; HBM-bound;
speed-up of the persistent rounds over one launch per Lloyd step and over one
worker's sample per launch), vmf768 (2,000,000 x 768, k = 100; FP32 and BF16
matrix cores against the oracle's f), serving (three resident 4,000,000-point
data sets, Poisson arrivals at 2,000/s for 1 s of warm-up and 10 s measured:
sustained jobs/s, p50/p99 latency).
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Lloyd point·centre dists/s & time to f(C,X) within 1% of oracle; p99 latency"
PEAK_FP32_VECTOR_TFLOPS = 157.3      # published, counts packed FP32 (two FMAs per lane)
PEAK_FP32_NONPACKED_TFLOPS = 78.6    # plain FP32 VALU code: 16 FMA lanes per SIMD per clock
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0}  # dense matrix-core peaks of the MI355X
PEAK_HBM_GBS = 8000.0

HEAD = dict(name="noisy28", k=50, workers=64, rounds_T=100, passes_p=10, s_min=1 << 12,
            s_max=1 << 17, policy="BINS")
C2 = dict(name="aniso28", k=25, workers=32, rounds_T=5, passes_p=10, s_min=4096, s_max=65536,
          policy="LOGUNIFORM")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha256():
    """Hash of the kernel sources; HBM traffic counted for other sources is stale."""
    h = hashlib.sha256()
    for name in ("bm_kernels.hip", "bm_device.h", "bm_internal.h", "bm_rng.h"):
        with open(os.path.join(ROOT, "paper_2403_18766_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counted_traffic(key):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None
    when the summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    entry = rec.get(key)
    if not entry or entry.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return entry["fetch_bytes_per_launch"] + entry["write_bytes_per_launch"]


def calibrate_copy(torch, dev, mib=512):
    """A plain device copy of known size, for scaling the memory counters."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 x {mib} MiB read + {mib} MiB written")


def reference(name, X=None, digest=None):
    """The oracle's final f on a workload (tests/golden), if its data digest matches."""
    from paper_2403_18766_amd import datagen
    path = os.path.join(ROOT, "tests", "golden", f"{name}_reference.json")
    if not os.path.exists(path):
        log(f"no oracle reference for {name}")
        return None
    with open(path) as f:
        ref = json.load(f)
    if "x_sha256_chunked" in ref:
        ok = ref["x_sha256_chunked"] == (digest or datagen.sha256_chunked(X))
    else:
        ok = ref.get("x_sha256") == datagen.sha256(X)
    if not ok:
        log(f"{name}: reference data digest differs; no oracle comparison")
        return None
    return ref


def run_params(api, _lib, w, mode):
    pol = {"BINS": _lib.BM_SIZE_BINS, "LOGUNIFORM": _lib.BM_SIZE_LOGUNIFORM}[w["policy"]]
    return api.RunParams(k=w["k"], workers=w["workers"], rounds_T=w["rounds_T"],
                         passes_p=w["passes_p"], s_min=w["s_min"], s_max=w["s_max"],
                         size_policy=pol, seed=0, batched=mode)


def timed_runs(torch, api, dev, Xd, P, steps, warmup):
    """W warm-up runs, then K timed runs between synchronisations, with the
    round kernel timed by HIP events on the library's stream."""
    for w in range(warmup):
        log("warmup", w)
        api.bigmeans_run(Xd, P, labels=True)
    torch.cuda.synchronize()
    api.set_profiling(dev, True)
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        results.append(api.bigmeans_run(Xd, P, labels=True))
        log("step", s, "f_full", results[-1]["f_full"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = api.get_stats(dev)
    api.set_profiling(dev, False)
    return results, wall, st


def kernel_roofline(st, n, k, mode, traffic_key):
    """The dominant kernel's algorithmic rates per launch: 2 n FLOPs and
    4 n / k bytes per distance over the kernel's average device time."""
    launches = max(1, st["assign_launches"])
    sec = st["assign_seconds"]
    dpl = st["assign_dists"] / launches
    avg = sec / launches
    tflops = dpl * 2.0 * n / avg / 1e12 if avg > 0 else 0.0
    gbs = dpl * 4.0 * n / k / avg / 1e9 if avg > 0 else 0.0
    kernel = f"k_round<{(n + 3) // 4 * 4}>" if mode == 1 else f"k_assign_small<{(n + 3) // 4 * 4}>"
    traffic = counted_traffic(traffic_key)
    return {"kernel": kernel, "avg_launch_us": 1e6 * avg, "launches": st["assign_launches"],
            "dists_per_launch": dpl, "alu_tflops": tflops,
            "alu_frac": tflops / PEAK_FP32_VECTOR_TFLOPS, "algorithmic_gbs": gbs,
            "hbm_frac": gbs / PEAK_HBM_GBS, "traffic": traffic,
            "traffic_over_algorithmic": (traffic / (dpl * 4.0 * n / k)) if traffic else None}


def final_stage_pick(api, Xd, C_all, fhat, l_sum, l_count, s_max, seed=0):
    """What Algorithm 1's final stage would return from these incumbents: the
    shared sample of size s_opt (round-half-up mean of L) from the FINAL
    stream, each incumbent's objective on it, the smallest (lowest worker on
    ties, workers without an incumbent never), and that worker's f(C, X)."""
    from paper_2403_18766_amd import _lib
    s_opt = (l_sum + l_count // 2) // l_count if l_count > 0 else s_max
    _, S = api.sample(Xd, s_opt, seed=seed, worker=_lib.BM_FINAL_WORKER,
                      purpose=_lib.BM_PURPOSE_FINAL, g=0)
    best, fb = -1, math.inf
    for w in range(C_all.shape[0]):
        if not math.isfinite(fhat[w]):
            continue
        f = api.objective(S, C_all[w].contiguous(), labels=False, near_ties=False)[0]
        if best < 0 or f < fb:
            best, fb = w, f
    if best < 0:
        return None, None
    f_full = api.objective(Xd, C_all[best].contiguous(), labels=False, near_ties=False)[0]
    return best, f_full


def time_to_target(torch, api, Xd, P, f_ref):
    """Device time until the final stage applied after round R gives
    f(C, X) <= 1.01 f_oracle, plus one final stage (off the clock, from the
    per-round snapshots of an identical run)."""
    snaps = []
    r = api.bigmeans_run(Xd, P, labels=False,
                         trace=lambda rnd, C, fh, sz, t, ls, lc: snaps.append((rnd, C, fh, ls, lc, t)))
    final_stage = r["gpu_seconds"] - snaps[-1][5] if snaps else 0.0
    curve = []
    hit = None
    for rnd, C, fh, ls, lc, t in snaps:
        best, f = final_stage_pick(api, Xd, C, fh, ls, lc, P.s_max)
        curve.append(f)
        if hit is None and f is not None and f <= 1.01 * f_ref:
            hit = {"seconds": t + final_stage, "round": rnd, "f": f, "worker": best,
                   "f_oracle": f_ref, "final_stage_seconds": final_stage}
    del snaps
    torch.cuda.empty_cache()
    step = max(1, len(curve) // 20)
    return hit, {"rounds": len(curve), "f_after_round": {i: curve[i] for i in range(0, len(curve), step)},
                 "f_last_round": curve[-1] if curve else None}


def assignment_agreement(Xh, Y, C, f_gpu):
    """Labels of the final run against the oracle's nearest centres for the
    same C over every point: disagreements outside near ties (top-two gap
    below 1e-5 relative, decided by the oracle) and the near-tie count."""
    import numpy as np

    from oracle import kmeans as okm
    lab, d1, _, near = okm.assign(Xh, C, return_second=True)
    diff = Y != lab
    fo = math.fsum(d1.tolist())
    return {"points": int(Xh.shape[0]), "near_ties": int(near.sum()),
            "disagree_outside_near_ties": int(np.count_nonzero(diff & ~near)),
            "disagree_at_near_ties": int(np.count_nonzero(diff & near)),
            "f_oracle_same_C": fo, "f_rel_diff": abs(f_gpu - fo) / fo}


def cpu_baseline(Xh, w):
    """The oracle as it is, on a process pool of this host's cores (one BLAS
    thread each, one worker per core as in the paper's setup): the first pass
    of round 0 of every worker (K-means++ of every centroid, then Lloyd)."""
    from oracle import bigmeans as obm
    cores = len(os.sched_getaffinity(0))
    pol = {"BINS": obm.SIZE_BINS, "LOGUNIFORM": obm.SIZE_LOGUNIFORM}[w["policy"]]
    P = obm.Params(k=w["k"], workers=w["workers"], rounds_T=1, passes_p=1, s_min=w["s_min"],
                   s_max=w["s_max"], size_policy=pol, seed=0)
    t0 = time.perf_counter()
    out = obm.bigmeans_run(Xh, P, processes=cores, final_stage=False)
    dt = time.perf_counter() - t0
    return {"value": out["lloyd_dists"] / dt, "unit": "dists/s", "cores": cores, "kind": "oracle",
            "sample": (f"Algorithm 1 on the same {Xh.shape[0]:,} x {Xh.shape[1]} data: the first "
                       f"pass of round 0 of all {w['workers']} workers (same size law and seed; "
                       f"K-means++ of all {w['k']} centroids, then Lloyd), FP64 NumPy oracle on a "
                       f"pool of {cores} processes with one BLAS thread each; "
                       f"{out['lloyd_dists']:.3e} distances in {dt:.1f} s")}


def c2_leg(torch, api, _lib, dev, steps, with_modes):
    """aniso28: k_round at n = 28, k = 25 (HBM-bound) and the speed-up of the
    persistent rounds over the multi-launch and plain per-sample paths at
    identical results."""
    import dataclasses

    from paper_2403_18766_amd import datagen
    log("generating aniso28")
    Xh = datagen.make("aniso28")
    Xd = torch.from_numpy(Xh).to(dev)
    P = run_params(api, _lib, C2, 1)
    api.reserve(dev, C2["s_max"], 28, C2["k"], C2["workers"])
    res, wall, st = timed_runs(torch, api, dev, Xd, P, steps, 1)
    ms = 1e3 * wall / steps
    roof = kernel_roofline(st, 28, C2["k"], 1, "k_round<28>@aniso28")
    ref = reference("aniso28", Xh)
    f = res[-1]["f_full"]
    out = {"workload": ("aniso28: 1,000,000 x 28 anisotropic Gaussian mixture (25 components), "
                        "k=25, 32 workers, sizes log-uniform [4096, 65536], T=5 x p=10"),
           "ms_per_run": ms, "dists_per_s": sum(r["lloyd_dists"] for r in res) / wall,
           "roofline": dict(roof, bound="hbm"), "f_full": f,
           "f_oracle": ref["f_full"] if ref else None,
           "f_gap_vs_oracle": (f - ref["f_full"]) / ref["f_full"] if ref else None}
    if with_modes:
        modes = {}
        for name, mode in (("one_launch_per_lloyd_step", 2), ("one_worker_per_launch", 0)):
            Pm = dataclasses.replace(P, batched=mode)
            api.bigmeans_run(Xd, Pm, labels=False)  # warm-up (tile-size tuning)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = api.bigmeans_run(Xd, Pm, labels=False)
            torch.cuda.synchronize()
            mms = 1e3 * (time.perf_counter() - t0)
            modes[name] = {"ms_per_run": mms, "f_full": r["f_full"], "same_f_bits": r["f_full"] == f,
                           "speedup_of_persistent_rounds": mms / ms}
            log("mode", mode, "ms", mms, "f_full", r["f_full"])
        out["modes"] = modes
    del Xd
    torch.cuda.empty_cache()
    return out


def seed_spread(torch, api, Xd, P, seeds=(0, 1, 2, 3, 4)):
    """The headline run once per algorithm seed (same data): wall time and
    f(C_best, X) per seed, with their median, min and max."""
    import dataclasses
    import statistics
    ms, fs = [], []
    for sd in seeds:
        log("headline run, seed", sd)
        q = dataclasses.replace(P, seed=sd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = api.bigmeans_run(Xd, q, labels=False)
        torch.cuda.synchronize()
        ms.append(1e3 * (time.perf_counter() - t0))
        fs.append(r["f_full"])
    return {"seeds": list(seeds), "ms": ms, "f_full": fs,
            "ms_median": statistics.median(ms), "ms_min": min(ms), "ms_max": max(ms),
            "f_median": statistics.median(fs), "f_min": min(fs), "f_max": max(fs)}


SERVE = dict(m=4_000_000, dims=(16, 64, 256), ks=(10, 50, 200), s_min=1024, s_max=262144,
             workers=32, rate=2000.0, budget_gb=200, warmup_s=1.0)


def serve_run(torch, dev, seconds):
    """The serving workload: Poisson arrivals of single-pass jobs against three
    resident data sets for warmup_s + `seconds` seconds.  Jobs that arrive in
    the warm-up are served but not counted; for the others: latency
    percentiles (completion - arrival) and the sustained rate (their number
    over the time from the first one's arrival to the last one's completion)."""
    import numpy as np

    from paper_2403_18766_amd import api, datagen
    log("generating serving data sets")
    Xs = [torch.from_numpy(datagen.serving_dataset(n, m=SERVE["m"])).to(dev) for n in SERVE["dims"]]
    r = np.random.default_rng(0)
    t = 0.0
    jobs = []
    ls, lb = math.log(SERVE["s_min"]), math.log(SERVE["s_max"] + 1)
    horizon = SERVE["warmup_s"] + seconds
    while True:
        t += float(r.exponential(1.0 / SERVE["rate"]))
        if t >= horizon:
            break
        s = min(SERVE["s_max"], int(math.floor(math.exp(r.uniform(ls, lb)))))
        jobs.append(dict(arrival=t, s=s, dataset=int(r.integers(len(Xs))),
                         k=int(SERVE["ks"][r.integers(len(SERVE["ks"]))]),
                         worker=int(r.integers(SERVE["workers"])), prec=int(r.integers(2))))
    log("serving", len(jobs), "jobs over", horizon, "s of arrivals")
    res, st = api.serve(Xs, jobs, seed=0, budget_bytes=SERVE["budget_gb"] << 30, max_slots=64,
                        paced=True)
    arr = np.array([j["arrival"] for j in jobs])
    fin = np.array([x["finished"] for x in res])
    m = arr >= SERVE["warmup_s"]
    lat = (fin[m] - arr[m]) * 1e3
    del Xs
    torch.cuda.empty_cache()
    return {"workload": (f"3 resident data sets of {SERVE['m']:,} points (noisy Gaussian mixtures, "
                         f"n = 16, 64, 256); Poisson arrivals at {SERVE['rate']:.0f}/s for "
                         f"{SERVE['warmup_s']:g} s of warm-up + {seconds:g} s measured "
                         f"({len(jobs)} jobs, {int(m.sum())} measured); k in (10, 50, 200); "
                         f"s log-uniform in [{SERVE['s_min']}, {SERVE['s_max']}]; FP32 or BF16 with "
                         f"equal odds (matrix-core distances at n = 256); 32 workers per "
                         f"(data set, k); {SERVE['budget_gb']} GiB budget"),
            "offered_per_s": SERVE["rate"],
            "jobs_per_s": float(m.sum() / (fin[m].max() - arr[m].min())),
            "p50_latency_ms": float(np.percentile(lat, 50)),
            "p99_latency_ms": float(np.percentile(lat, 99)),
            "jobs": len(jobs), "measured_jobs": int(m.sum()), "wall_s": st["seconds"],
            "lloyd_steps": st["steps"], "peak_running": st["peak_running"],
            "peak_bytes": st["peak_bytes"], "slot_bytes": st["slot_bytes"]}


PREC = dict(m=2_000_000, n=768, k=100, workers=16, s=131_072, rounds_T=2, passes_p=1)


def precision_run(torch, dev):
    """Algorithm 1 on 2,000,000 unit vectors in 768-D (100 vMF clusters),
    k = 100, 16 workers with fixed samples of 131,072: once with FP32 and once
    with BF16 matrix-core distances, each against the oracle's final f on the
    same data.  Per precision: wall time, Lloyd distances/s, and the assignment
    + update kernels timed with HIP events (algorithmic FLOP/s against the
    precision's matrix-core peak, and algorithmic bytes/s: each sample row read
    once per Lloyd step)."""
    from paper_2403_18766_amd import _lib, api, datagen
    log("generating the vmf768 workload on the host")
    Xh = datagen.make("vmf768")
    ref = reference("vmf768", digest=datagen.sha256_chunked(Xh))
    X = torch.from_numpy(Xh).to(dev)
    del Xh
    torch.cuda.synchronize()
    n, k, s = PREC["n"], PREC["k"], PREC["s"]
    api.reserve(dev, s, n, k, PREC["workers"])
    f_ref = ref["f_full"] if ref else None
    out = {"workload": (f"{PREC['m']:,} unit vectors in {n}-D from 100 von Mises-Fisher clusters "
                        f"(kappa U[50,200]), k={k}, {PREC['workers']} workers, fixed s={s:,}, "
                        f"T={PREC['rounds_T']} rounds x p={PREC['passes_p']} passes, "
                        "one launch per Lloyd step"), "f_oracle": f_ref}
    for name, prec in (("f32", _lib.BM_FP32), ("bf16", _lib.BM_BF16)):
        common = dict(k=k, workers=PREC["workers"], s_min=s, s_max=s,
                      size_policy=_lib.BM_SIZE_FIXED, seed=0, batched=2, prec=prec)
        api.bigmeans_run(X, api.RunParams(rounds_T=1, passes_p=1, **common), labels=False)
        torch.cuda.synchronize()
        api.set_profiling(dev, True)
        t0 = time.perf_counter()
        r = api.bigmeans_run(X, api.RunParams(rounds_T=PREC["rounds_T"], passes_p=PREC["passes_p"],
                                              **common), labels=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = api.get_stats(dev)
        api.set_profiling(dev, False)
        ksec = st["assign_seconds"]
        tflops = st["assign_dists"] * 2.0 * n / ksec / 1e12 if ksec > 0 else 0.0
        gbs = st["assign_dists"] * 4.0 * n / k / ksec / 1e9 if ksec > 0 else 0.0
        out[name] = {"seconds": wall, "lloyd_dists": r["lloyd_dists"],
                     "dists_per_s": r["lloyd_dists"] / wall,
                     "lloyd_phase_dists_per_s": r["lloyd_dists"] / r["lloyd_seconds"],
                     "f_full": r["f_full"],
                     "f_gap_vs_oracle": (r["f_full"] - f_ref) / f_ref if f_ref else None,
                     "kernels": f"k_assign_wide<true,{'true' if name == 'bf16' else 'false'}> "
                                "+ k_update_wide",
                     "kernel_launches": st["assign_launches"],
                     "kernel_avg_us": 1e6 * ksec / max(1, st["assign_launches"]),
                     "kernel_dists_per_s": st["assign_dists"] / ksec if ksec > 0 else None,
                     "achieved_tflops": tflops, "peak_tflops": PEAK_TFLOPS[name],
                     "mfma_frac": tflops / PEAK_TFLOPS[name],
                     "algorithmic_gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS}
        log("precision", name, "wall", wall, "f_full", r["f_full"], "oracle", f_ref)
    out["bf16_speedup"] = out["f32"]["seconds"] / out["bf16"]["seconds"]
    out["bf16_f_gap"] = (out["bf16"]["f_full"] - out["f32"]["f_full"]) / out["f32"]["f_full"]
    del X
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-ttt", action="store_true",
                    help="skip the time-to-target run and the assignment agreement")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="measured seconds of serving arrivals after 1 s of warm-up (0 skips it)")
    ap.add_argument("--serve-jobs", type=int, default=None,
                    help="0 skips the serving measurement (as --serve-seconds 0)")
    ap.add_argument("--no-seeds", action="store_true",
                    help="skip the headline runs with algorithm seeds 0-4")
    ap.add_argument("--no-c2", action="store_true", help="skip the aniso28 leg")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the comparison with the multi-launch and plain per-sample modes")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP32 / BF16 matrix-core measurement")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed steps, copy 512 MiB three times (counter scaling)")
    ap.add_argument("--mode", type=int, default=1,
                    help="1 persistent rounds (default), 2 one launch per Lloyd step, "
                         "0 one worker's sample per launch")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of the workers is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2403_18766_amd import _lib, api, datagen
    if not os.path.exists(_lib.LIB_PATH):
        raise SystemExit(f"{_lib.LIB_PATH} is missing: build it first (python __graft_entry__.py build)")
    dev = torch.device("cuda:0")
    log("generating workload", HEAD["name"])
    Xh = datagen.make(HEAD["name"])
    m, n = Xh.shape
    k = HEAD["k"]
    Xd = torch.from_numpy(Xh).to(dev)
    P = run_params(api, _lib, HEAD, args.mode)
    api.reserve(dev, HEAD["s_max"], n, k, HEAD["workers"])
    results, wall, st = timed_runs(torch, api, dev, Xd, P, args.steps, args.warmup)
    if args.calibrate_copy:
        calibrate_copy(torch, dev)
    dists = sum(r["lloyd_dists"] for r in results)
    value = dists / wall
    lloyd_sec = sum(r["lloyd_seconds"] for r in results)
    kr = kernel_roofline(st, n, k, args.mode, f"k_round<28>@{HEAD['name']}")
    roof = {"bound": "alu", "kernel": kr["kernel"] + (" (persistent round: re-evaluation, sampling, "
                                                      "K-means++, Lloyd, acceptance)"
                                                      if args.mode == 1 else " (Lloyd step)"),
            "achieved": kr["alu_tflops"], "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
            "frac": kr["alu_frac"], "traffic": kr["traffic"],
            "nonpacked_peak": PEAK_FP32_NONPACKED_TFLOPS,
            "nonpacked_frac": kr["alu_tflops"] / PEAK_FP32_NONPACKED_TFLOPS,
            "flops_per_dist": 2 * n, "avg_launch_us": kr["avg_launch_us"],
            "launches": kr["launches"], "dists_per_launch": kr["dists_per_launch"],
            "hbm": {"algorithmic_gbs": kr["algorithmic_gbs"], "frac": kr["hbm_frac"],
                    "bytes_per_dist": 4.0 * n / k,
                    "traffic_over_algorithmic": kr["traffic_over_algorithmic"]}}
    f_full = results[-1]["f_full"]
    ref = reference(HEAD["name"], Xh)
    f_ref = ref["f_full"] if ref else None

    ttt = curve = agree = None
    if not args.no_ttt:
        if f_ref is not None:
            log("time to target")
            ttt, curve = time_to_target(torch, api, Xd, P, f_ref)
        log("assignment agreement")
        r = results[-1]
        agree = assignment_agreement(Xh, r["Y"].cpu().numpy(), r["C_best"].cpu().numpy().astype("float64"),
                                     f_full)
        agree["gpu_near_ties"] = api.objective(Xd, r["C_best"], labels=False, near_ties=True)[2]
    seeds = None if args.no_seeds else seed_spread(torch, api, Xd, P)
    del results
    del Xd
    torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu:
        log("oracle baseline")
        cpu = cpu_baseline(Xh, HEAD)
    del Xh
    c2 = None if args.no_c2 else c2_leg(torch, api, _lib, dev, 3, not args.no_modes)
    want_serving = args.serve_seconds > 0 and args.serve_jobs != 0
    serving = serve_run(torch, dev, args.serve_seconds) if want_serving else None
    precision = None if args.no_precision else precision_run(torch, dev)
    out = {
        "metric": METRIC, "value": value, "unit": "dists/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": ("noisy28: 10,000,000 x 28 Gaussian mixture (50 components, sigma "
                                "U[0.5,3]) with 5% uniform background noise, k=50, 64 competing "
                                "workers, sizes from the best-performing of 5 log-width bins over "
                                "[4096, 131072], T=100 rounds x p=10 passes, Lloyd <=300 iters "
                                "tol 1e-4, 3 K-means++ candidates, full-data f in FP64"),
                   "m": m, "n": n, "k": k, "workers": HEAD["workers"],
                   "rounds": HEAD["rounds_T"], "passes": HEAD["passes_p"],
                   "mode": {1: "persistent rounds", 2: "one launch per Lloyd step",
                            0: "one worker per launch"}[args.mode]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "lloyd_phase_dists_per_s": dists / lloyd_sec if lloyd_sec > 0 else None,
        "f_full": f_full,
        "f_oracle": f_ref,
        "f_gap_vs_oracle": (f_full - f_ref) / f_ref if f_ref else None,
        "time_to_target": ttt,
        "f_curve": curve,
        "assignment": agree,
        "seeds": seeds,
        "p99_latency_ms": serving["p99_latency_ms"] if serving else None,
        "aniso28": c2,
        "serving": serving,
        "precision": precision,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
