"""Oracle study of the 10-d Rosenbrock workload (Eq. (6) chained over d = 10,
prior [-5,5]^10, N = 500): log Z of complete FP64 oracle runs against the
transfer-matrix quadrature value, per batch size m, slice iterations n*d and
cluster-tree depth.  It separates the error of batching (Sec. 3) from the
mixing of the slice sampler (Sec. 2.2) and from the cluster-dependent
whitening of its directions (Sec. 2.1-2.2).

Calls only the oracle and the seeded workload constructor.  Writes
``c2_oracle_ensemble.json`` beside this file: per setting the seeds, every
run's log Z, sigma = sqrt(H/N) and H, their mean, run-to-run standard
deviation and standard error of the mean.  The GPU tests and the benchmark
compare the GPU sampler against these ensembles.

Usage: python tests/golden/c2_oracle_study.py [--procs 8]
"""
import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N_LIVE = 500
# (m, n, depth, seeds): the production setting (m = 50, n = 5, depth 2) and
# m = 1, 10 with more seeds, since the GPU ensembles are compared with them
SETTINGS = [(1, 5, 2, 48), (10, 5, 2, 48), (50, 5, 2, 48),
            (1, 10, 2, 32), (10, 10, 2, 32), (50, 10, 2, 32),
            (1, 25, 2, 32),
            (1, 5, 0, 32), (50, 5, 0, 32), (1, 10, 0, 32), (1, 25, 0, 32)]


def quadrature_logZ(d=10, lo=-5.0, hi=5.0, n=4001):
    """log Z of the chained Rosenbrock likelihood on [lo, hi]^d by the
    transfer matrix K[a, b] = exp(-100 (b - a^2)^2 - (1 - a)^2) on a trapezoid
    grid, rescaled at every product."""
    import numpy as np
    x = np.linspace(lo, hi, n)
    w = np.full(n, (hi - lo) / (n - 1))
    w[0] *= 0.5
    w[-1] *= 0.5
    K = np.exp(-100.0 * (x[None, :] - x[:, None] ** 2) ** 2 - (1.0 - x[:, None]) ** 2)
    f = np.ones(n)
    logscale = 0.0
    for _ in range(d - 1):
        f = (w * f) @ K
        s = f.max()
        f /= s
        logscale += math.log(s)
    return math.log((w * f).sum()) + logscale - d * math.log(hi - lo)


def _one(args):
    m, n, depth, seed = args
    import oracle
    from paper_2608_28514_amd import workloads
    oracle.set_threads(1)
    o = oracle.Oracle(workloads.likelihood(2), N_LIVE, seed=seed, tree_depth=depth, slice_steps_per_dim=n)
    t0 = time.perf_counter()
    o.run(m)
    dt = time.perf_counter() - t0
    lz, sig, H = o.logZ()
    return m, n, depth, seed, lz, sig, H, o.n_dead(), dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    truth = quadrature_logZ()
    jobs = [(m, n, dep, s) for (m, n, dep, S) in SETTINGS for s in range(S)]
    # longest first: m = 1 with many slice iterations
    jobs.sort(key=lambda j: -(j[1] * (60 if j[0] == 1 else 1)))
    t0 = time.time()
    res = {}
    with ProcessPoolExecutor(max_workers=args.procs) as ex:
        for r in ex.map(_one, jobs):
            res.setdefault(r[:3], []).append(r[3:])
    rows = []
    for (m, n, dep, S) in SETTINGS:
        rr = sorted(res[(m, n, dep)])
        lz = [x[1] for x in rr]
        mean = sum(lz) / len(lz)
        std = math.sqrt(sum((z - mean) ** 2 for z in lz) / (len(lz) - 1))
        sem = std / math.sqrt(len(lz))
        sig = sum(x[2] for x in rr) / len(rr)
        rows.append({"m": m, "n": n, "depth": dep, "seeds": [x[0] for x in rr], "logZ": lz,
                     "sigma": [x[2] for x in rr], "H": [x[3] for x in rr], "dead": [x[4] for x in rr],
                     "mean": mean, "std": std, "sem": sem, "sigma_mean": sig,
                     "diff_vs_quadrature": mean - truth, "diff_in_sem": (mean - truth) / sem,
                     "cpu_s": sum(x[5] for x in rr)})
        print(f"m={m:3d} n={n:2d} depth={dep}: mean {mean:.4f}  diff {mean - truth:+.4f}  "
              f"({(mean - truth) / sem:+.1f} SEM)  std {std:.3f}  sigma {sig:.3f}  seeds {len(lz)}", flush=True)
    try:
        commit = subprocess.run(["git", "-C", ROOT, "rev-parse", "--short=12", "HEAD"], capture_output=True,
                                text=True).stdout.strip()
    except OSError:
        commit = ""
    out = {"workload": "rosenbrock10d prior[-5,5]^10 N_live=500, FP64 oracle, history correction K=1",
           "quadrature_logZ": truth, "n_live": N_LIVE, "settings": rows,
           "generated_by": "tests/golden/c2_oracle_study.py", "commit": commit, "host": platform.node(),
           "cpu": platform.processor() or platform.machine(), "procs": args.procs,
           "wall_s": time.time() - t0}
    with open(os.path.join(HERE, "c2_oracle_ensemble.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
