"""Write the oracle's Algorithm-1 result on a named workload (expected values
for the time-to-target and oracle-gap measurements).  Calls only the oracle;
the input is the seeded generator's data set, identified by its sha256.
Workers run in a process pool of the host's cores (one BLAS thread each);
the result is the same as the sequential run.

    python tests/golden/make_reference.py noisy28 [processes]
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import bigmeans as obm  # noqa: E402
from paper_2403_18766_amd import datagen  # noqa: E402

# Algorithm-1 settings of each measured workload (k, workers, rounds, passes,
# size range and policy; Section 5 parameters otherwise).
CONFIGS = {
    "blobs2d": dict(k=5, workers=4, rounds_T=20, passes_p=10, s_min=2000, s_max=2000,
                    size_policy=obm.SIZE_FIXED, seed=0),
    "aniso28": dict(k=25, workers=32, rounds_T=5, passes_p=10, s_min=4096, s_max=65536,
                    size_policy=obm.SIZE_LOGUNIFORM, seed=0),
    "noisy28": dict(k=50, workers=64, rounds_T=100, passes_p=10, s_min=1 << 12, s_max=1 << 17,
                    size_policy=obm.SIZE_BINS, seed=0),
    "vmf768": dict(k=100, workers=16, rounds_T=2, passes_p=1, s_min=131_072, s_max=131_072,
                   size_policy=obm.SIZE_FIXED, seed=0),
}
# large inputs are identified by the chunked digest
CHUNKED = ("noisy28", "vmf768")


def main(name, processes):
    X = datagen.make(name)
    digest = datagen.sha256_chunked(X) if name in CHUNKED else datagen.sha256(X)
    cfg = CONFIGS[name]
    t0 = time.time()

    def progress(t, state):
        print(f"[{name}] round {t} done at {time.time() - t0:.0f} s", file=sys.stderr, flush=True)

    out = obm.bigmeans_run(X, obm.Params(**cfg), processes=processes, rounds_done=progress)
    wall = time.time() - t0
    rec = {"workload": name, "params": cfg,
           ("x_sha256_chunked" if name in CHUNKED else "x_sha256"): digest,
           "f_full": out["f_full"], "s_opt": out["s_opt"], "best_worker": out["best_worker"],
           "improvements": len(out["L"]), "lloyd_dists": out["lloyd_dists"],
           "lloyd_iters": out["lloyd_iters"], "oracle_wall_seconds": wall,
           "processes": processes}
    path = os.path.join(HERE, f"{name}_reference.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    nm = sys.argv[1] if len(sys.argv) > 1 else "aniso28"
    procs = int(sys.argv[2]) if len(sys.argv) > 2 else len(os.sched_getaffinity(0))
    main(nm, procs)
