"""Reference evidence of the 27-d emulator workloads (the random-MLP
27-512-512-512-1024 emulator, diagonal chi^2 likelihood, prior [0,1]^27;
workloads 4 and 5 share the seed-0 likelihood).

Calls only the oracle (oracle.evidence_is: posterior mode by Gauss-Newton,
Hessian by differences of the analytic gradient, importance sampling from a
Student-t around the mode with the oracle's FP64 likelihood) and the seeded
workload constructor.  Two independent proposals are used and must agree.
Writes ``emulator27d_reference.json`` beside this file.

Usage: python tests/golden/make_emulator_reference.py [--threads 8]
"""
import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    import numpy as np
    import oracle
    from oracle import evidence_is as E
    from paper_2608_28514_amd import workloads

    oracle.set_threads(args.threads)
    out = {"workload": "emulator27d MLP 27-512-512-512-1024 tanh, linear output, diagonal chi^2, "
                       "prior [0,1]^27, network and data of seed 0 (workloads 4 and 5)",
           "method": "importance sampling from a multivariate Student-t at the posterior mode, scale from "
                     "the Hessian of -log L (FP64 oracle likelihood)",
           "generated_by": "tests/golden/make_emulator_reference.py"}
    t0 = time.time()
    spec = workloads.likelihood(4, seed=0)
    main_est = E.emulator_evidence(spec, n=200_000, seed=0, nu=10.0, scale=1.2)
    alt = E.importance_logZ(spec, main_est["mode"], main_est["cov"], 100_000, 1, nu=30.0, scale=1.0)
    comb = math.sqrt(main_est["se"] ** 2 + alt["se"] ** 2)
    if abs(main_est["logZ"] - alt["logZ"]) > 4.0 * comb:
        raise SystemExit(f"proposals disagree: {main_est['logZ']} vs {alt['logZ']} (se {comb})")
    H = main_est["H"]
    out.update({
        "seed": 0,
        "logZ": main_est["logZ"], "logZ_se": main_est["se"], "H": H,
        "ess": main_est["ess"], "n_samples": main_est["n"], "nu": main_est["nu"], "scale": main_est["scale"],
        "check_logZ": alt["logZ"], "check_se": alt["se"], "check_nu": alt["nu"], "check_scale": alt["scale"],
        "laplace_logZ": main_est["laplace_logZ"], "laplace_gauss_newton_logZ": main_est["laplace_gn_logZ"],
        "logL_mode": main_est["logL_mode"],
        "mode": main_est["mode"].tolist(), "cov": main_est["cov"].tolist(),
        "posterior_sd": main_est["posterior_sd"].tolist(),
        "mode_to_box_edge_in_sd": main_est["mode_to_box_edge_in_sd"],
        "sigma_sqrt_H_over_N": {"2000": math.sqrt(H / 2000.0), "4000": math.sqrt(H / 4000.0)},
    })
    try:
        commit = subprocess.run(["git", "-C", ROOT, "rev-parse", "--short=12", "HEAD"], capture_output=True,
                                text=True).stdout.strip()
    except OSError:
        commit = ""
    out.update({"commit": commit, "host": platform.node(), "threads": args.threads,
                "wall_s": time.time() - t0})
    with open(os.path.join(HERE, "emulator27d_reference.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"log Z = {out['logZ']:.5f} +- {out['logZ_se']:.5f} (check {alt['logZ']:.5f} +- {alt['se']:.5f}; "
          f"Laplace {out['laplace_logZ']:.5f}); H = {H:.3f}; ESS {out['ess']:.0f}; {out['wall_s']:.1f} s")
    del np


if __name__ == "__main__":
    main()
