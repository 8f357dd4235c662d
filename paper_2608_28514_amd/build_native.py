"""Build libns.so (the HIP library behind include/ns.h) for gfx950, in-tree.

Every source is compiled by hipcc with contraction off (the FP64 paths keep
the operation order of the algorithm statement) and packed FP32 disabled.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["k_select.hip", "k_select_large.hip", "k_slice.hip", "k_slice_rounds.hip", "k_emu_chains.hip",
           "k_gemm.hip", "k_surrogate.hip",
           "k_cluster.hip", "k_cluster_large.hip", "k_correct.hip", "ns_api.hip"]
LIB = os.path.join(HERE, "libns.so")
FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall"]
OBJDIR = os.path.join(HERE, "_build")


def _run(cmd):
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose=False, jobs=None):
    """Compile every source to an object (in parallel), then link libns.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    jobs = jobs or min(len(srcs), os.cpu_count() or 1, 8)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        res = list(ex.map(_run, [["hipcc"] + FLAGS + ["-c", s, "-o", o] for s, o in zip(srcs, objs)]))
    tmp = LIB + ".tmp"
    res.append(_run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs))
    for r in res:
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed building libns.so")
        if verbose:
            sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
