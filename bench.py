#!/usr/bin/env python3
"""Benchmark of the Big-means hot path on one MI355X.

One step = one run of Algorithm 1 (bm_bigmeans_run) on the aniso28 workload:
1,000,000 points in 28-D from 25 anisotropic Gaussians, k = 25, 32 competing
workers with sample sizes log-uniform in [4,096, 65,536], 5 rounds of 10
passes (sampling, K-means++, Lloyd, acceptance, final selection and the full
assignment of X).  X is resident in HBM before the timed region.

Printed (one JSON line):
  value          Lloyd point-centre distances per second over the whole job
                 (sum over Lloyd runs of s * k * assignment steps / wall time)
  roofline       the Lloyd assignment kernel: algorithmic FLOPs (2 n per
                 distance) over its device time, measured with HIP events on
                 the library's stream inside the timed region
  cpu_baseline   the FP64 oracle timed on this host on a bounded slice of the
                 same workload
  time_to_target seconds until f(C, X) is within 1% of the oracle's final f
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
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0}  # dense matrix-core peaks of the MI355X
PEAK_HBM_GBS = 8000.0

WORKLOAD = dict(name="aniso28", k=25, workers=32, rounds_T=5, passes_p=10, s_min=4096,
                s_max=65536)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(X, workers, passes):
    """The oracle as it is, on a bounded slice of the same workload."""
    from threadpoolctl import threadpool_limits

    from oracle import bigmeans as obm
    P = obm.Params(k=WORKLOAD["k"], workers=workers, rounds_T=1, passes_p=passes,
                   s_min=WORKLOAD["s_min"], s_max=WORKLOAD["s_max"],
                   size_policy=obm.SIZE_LOGUNIFORM, seed=0)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        out = obm.bigmeans_run(X, P)
        dt = time.perf_counter() - t0
    return {"value": out["lloyd_dists"] / dt, "unit": "dists/s", "cores": 1, "kind": "oracle",
            "sample": (f"Algorithm 1 on the same 1,000,000 x 28 data: {workers} workers x 1 "
                       f"round x {passes} passes (same size law and seed), FP64 NumPy, "
                       f"one BLAS thread; {out['lloyd_dists']:.3e} distances in {dt:.1f} s")}


def kernel_sources_sha256():
    """Hash of the kernel sources; HBM traffic counted for other sources is stale."""
    h = hashlib.sha256()
    for name in ("bm_kernels.hip", "bm_device.h", "bm_internal.h", "bm_rng.h"):
        with open(os.path.join(ROOT, "paper_2403_18766_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counted_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size),
    or None when the summary is missing or was taken on other sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    entry = rec.get(kernel)
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


SERVE = dict(m=4_000_000, dims=(16, 64, 256), ks=(10, 50, 200), s_min=1024, s_max=262144,
             workers=32, rate=2000.0, budget_gb=200)


def serve_run(torch, dev, njobs):
    """The serving workload: Poisson arrivals of single-pass jobs against three
    resident data sets; returns the latency summary."""
    import numpy as np

    from paper_2403_18766_amd import api, datagen
    log("generating serving data sets")
    Xs = [torch.from_numpy(datagen.serving_dataset(n, m=SERVE["m"])).to(dev) for n in SERVE["dims"]]
    r = np.random.default_rng(0)
    t = 0.0
    jobs = []
    ls, lb = math.log(SERVE["s_min"]), math.log(SERVE["s_max"] + 1)
    for _ in range(njobs):
        t += float(r.exponential(1.0 / SERVE["rate"]))
        s = min(SERVE["s_max"], int(math.floor(math.exp(r.uniform(ls, lb)))))
        jobs.append(dict(arrival=t, s=s, dataset=int(r.integers(len(Xs))),
                         k=int(SERVE["ks"][r.integers(len(SERVE["ks"]))]),
                         worker=int(r.integers(SERVE["workers"])), prec=int(r.integers(2))))
    log("serving", njobs, "jobs")
    res, st = api.serve(Xs, jobs, seed=0, budget_bytes=SERVE["budget_gb"] << 30, max_slots=64,
                        paced=True)
    lat = np.array([x["finished"] - j["arrival"] for x, j in zip(res, jobs)]) * 1e3
    del Xs
    torch.cuda.empty_cache()
    return {"workload": (f"3 resident data sets of {SERVE['m']:,} points (noisy Gaussian mixtures, "
                         f"n = 16, 64, 256); {njobs} jobs, Poisson arrivals at "
                         f"{SERVE['rate']:.0f}/s; k in (10, 50, 200); s log-uniform in "
                         f"[{SERVE['s_min']}, {SERVE['s_max']}]; FP32 or BF16 with equal odds (matrix-core "
                         f"distances at n = 256); 32 workers per (data set, k); "
                         f"{SERVE['budget_gb']} GiB budget"),
            "jobs_per_s": njobs / st["seconds"], "p50_latency_ms": float(np.percentile(lat, 50)),
            "p99_latency_ms": float(np.percentile(lat, 99)), "wall_s": st["seconds"],
            "lloyd_steps": st["steps"], "peak_running": st["peak_running"],
            "peak_bytes": st["peak_bytes"]}


PREC = dict(m=2_000_000, n=768, k=100, workers=16, s=131_072, rounds_T=2, passes_p=10)


def precision_run(torch, dev):
    """Algorithm 1 on 2,000,000 unit vectors in 768-D (100 vMF clusters),
    k = 100, 16 workers with fixed samples of 131,072: once with FP32 and once
    with BF16 matrix-core distances.  Per precision: wall time, Lloyd
    distances/s, and the assignment + update kernels timed with HIP events
    (algorithmic FLOP/s against the precision's matrix-core peak, and
    algorithmic bytes/s: each sample row read once per Lloyd step)."""
    from paper_2403_18766_amd import _lib, api, datagen
    log("generating the vmf768 workload on the device")
    X = datagen.vmf_mixture_device(PREC["m"] // 100, PREC["n"], 100, dev, seed=0)
    torch.cuda.synchronize()
    n, k, s = PREC["n"], PREC["k"], PREC["s"]
    api.reserve(dev, s, n, k, PREC["workers"])
    out = {"workload": (f"{PREC['m']:,} unit vectors in {n}-D from 100 von Mises-Fisher clusters "
                        f"(kappa U[50,200]), k={k}, {PREC['workers']} workers, fixed s={s:,}, "
                        f"T={PREC['rounds_T']} rounds x p={PREC['passes_p']} passes, "
                        "one launch per Lloyd step")}
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
                     "kernels": f"k_assign_wide<true,{'true' if name == 'bf16' else 'false'}> "
                                "+ k_update_wide",
                     "kernel_launches": st["assign_launches"],
                     "kernel_avg_us": 1e6 * ksec / max(1, st["assign_launches"]),
                     "kernel_dists_per_s": st["assign_dists"] / ksec if ksec > 0 else None,
                     "achieved_tflops": tflops, "peak_tflops": PEAK_TFLOPS[name],
                     "mfma_frac": tflops / PEAK_TFLOPS[name],
                     "algorithmic_gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS}
        log("precision", name, "wall", wall, "f_full", r["f_full"])
    out["bf16_speedup"] = out["f32"]["seconds"] / out["bf16"]["seconds"]
    out["bf16_f_gap"] = (out["bf16"]["f_full"] - out["f32"]["f_full"]) / out["f32"]["f_full"]
    del X
    torch.cuda.empty_cache()
    return out


def mode_comparison(torch, api, Xd, P, ms_mode1, f_mode1):
    """The same Algorithm-1 step with one launch per Lloyd step (mode 2) and one
    worker's sample per launch (mode 0, the plain per-sample GPU path): the
    batched mode's speed-up at equal results (the modes give the same bits)."""
    import dataclasses
    out = {}
    for name, mode in (("one_launch_per_lloyd_step", 2), ("one_worker_per_launch", 0)):
        Pm = dataclasses.replace(P, batched=mode)
        api.bigmeans_run(Xd, Pm, labels=False)  # warm-up (tile-size tuning)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = api.bigmeans_run(Xd, Pm, labels=False)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        out[name] = {"ms_per_step": ms, "f_full": r["f_full"], "same_f_bits": r["f_full"] == f_mode1,
                     "speedup_of_persistent_rounds": ms / ms_mode1}
        log("mode", mode, "ms", ms, "f_full", r["f_full"])
    return out


def reference_f(X):
    from paper_2403_18766_amd import datagen
    path = os.path.join(ROOT, "tests", "golden", f"{WORKLOAD['name']}_reference.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        ref = json.load(f)
    if ref.get("x_sha256") != datagen.sha256(X):
        log("reference data hash differs; time-to-target not reported")
        return None
    return ref["f_full"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--cpu-workers", type=int, default=32)
    ap.add_argument("--cpu-passes", type=int, default=10)
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-target run")
    ap.add_argument("--serve-jobs", type=int, default=2000,
                    help="jobs of the serving measurement (0 skips it)")
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

    import numpy as np
    import torch

    from paper_2403_18766_amd import _lib, api, datagen
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2403_18766_amd import build
        build.build()
    dev = torch.device("cuda:0")
    log("generating workload", WORKLOAD["name"])
    X = datagen.make(WORKLOAD["name"])
    m, n = X.shape
    Xd = torch.from_numpy(X).to(dev)
    P = api.RunParams(k=WORKLOAD["k"], workers=WORKLOAD["workers"], rounds_T=WORKLOAD["rounds_T"],
                      passes_p=WORKLOAD["passes_p"], s_min=WORKLOAD["s_min"],
                      s_max=WORKLOAD["s_max"], size_policy=_lib.BM_SIZE_LOGUNIFORM, seed=0,
                      batched=args.mode)
    api.reserve(dev, WORKLOAD["s_max"], n, WORKLOAD["k"], WORKLOAD["workers"])
    for w in range(args.warmup):
        log("warmup", w)
        api.bigmeans_run(Xd, P, labels=True)
    torch.cuda.synchronize()

    api.set_profiling(dev, True)
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        results.append(api.bigmeans_run(Xd, P, labels=True))
        log("step", s, "f_full", results[-1]["f_full"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = api.get_stats(dev)
    api.set_profiling(dev, False)
    wall = t1 - t0
    if args.calibrate_copy:
        calibrate_copy(torch, dev)

    dists = sum(r["lloyd_dists"] for r in results)
    value = dists / wall
    lloyd_sec = sum(r["lloyd_seconds"] for r in results)
    flops = st["assign_dists"] * 2.0 * n
    achieved = flops / st["assign_seconds"] / 1e12 if st["assign_seconds"] > 0 else 0.0
    kernel = "k_round<28>" if args.mode == 1 else "k_assign_small<28,2,true>"
    kname = (kernel + (" (persistent round: sampling, K-means++, Lloyd, acceptance)"
                       if args.mode == 1 else " (Lloyd assignment + update)"))
    traffic = counted_traffic(kernel)
    roof = {"bound": "alu", "kernel": kname,
            "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic,
            "avg_launch_us": 1e6 * st["assign_seconds"] / max(1, st["assign_launches"]),
            "launches": st["assign_launches"],
            "dists_per_launch": st["assign_dists"] / max(1, st["assign_launches"])}

    ttt = None
    f_ref = reference_f(X)
    if not args.no_ttt and f_ref is not None:
        snaps = []
        r = api.bigmeans_run(Xd, P, labels=False,
                             trace=lambda rnd, C, fh, sz, t: snaps.append((rnd, C.clone(), t)))
        final_stage = r["gpu_seconds"] - snaps[-1][2] if snaps else 0.0
        for rnd, C, t in snaps:
            best = min(api.objective(Xd, C[w].contiguous(), labels=False, near_ties=False)[0]
                       for w in range(C.shape[0]))
            if best <= 1.01 * f_ref:
                ttt = {"seconds": t + final_stage, "round": rnd, "f": best, "f_oracle": f_ref}
                break

    modes = None
    if not args.no_modes and args.mode == 1:
        modes = mode_comparison(torch, api, Xd, P, 1e3 * wall / args.steps, results[-1]["f_full"])
    cpu = None if args.no_cpu else cpu_baseline(X, args.cpu_workers, args.cpu_passes)
    del Xd
    serving = serve_run(torch, dev, args.serve_jobs) if args.serve_jobs > 0 else None
    precision = None if args.no_precision else precision_run(torch, dev)
    f_full = results[-1]["f_full"]
    out = {
        "metric": METRIC, "value": value, "unit": "dists/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "aniso28: 1,000,000 x 28 anisotropic Gaussian mixture (25 "
                               "components), k=25, 32 workers, sizes log-uniform [4096, 65536], "
                               "T=5 rounds x p=10 passes, Lloyd <=300 iters tol 1e-4, "
                               "3 K-means++ candidates",
                   "m": m, "n": n, "k": WORKLOAD["k"], "workers": WORKLOAD["workers"],
                   "mode": {1: "persistent rounds", 2: "one launch per Lloyd step",
                            0: "one worker per launch"}[args.mode]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "lloyd_phase_dists_per_s": dists / lloyd_sec if lloyd_sec > 0 else None,
        "f_full": f_full,
        "f_oracle": f_ref,
        "f_gap_vs_oracle": (f_full - f_ref) / f_ref if f_ref else None,
        "time_to_target": ttt,
        "p99_latency_ms": serving["p99_latency_ms"] if serving else None,
        "serving": serving,
        "precision": precision,
        "modes": modes,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
