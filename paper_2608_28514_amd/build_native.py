"""Build libns.so (the HIP library behind include/ns.h) for gfx950, in-tree.

Every source is compiled by hipcc with contraction off (the FP64 paths keep
the operation order of the algorithm statement) and packed FP32 disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["k_select.hip", "k_slice.hip", "k_slice_rounds.hip", "k_gemm.hip", "k_surrogate.hip",
           "k_cluster.hip", "k_correct.hip", "ns_api.hip"]
LIB = os.path.join(HERE, "libns.so")
FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-shared", "-std=c++17", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall"]


def build(verbose=False):
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ["hipcc"] + FLAGS + ["-o", tmp] + srcs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libns.so")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
