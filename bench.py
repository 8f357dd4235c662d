"""Benchmark of the batched nested sampler on one MI355X.

A "step" here is one complete nested-sampling run of the benchmark workload
(init -> batched updates until the stopping rule -> final evidence), which
passes through every stage of the hot path: selection, clustering, slice
sampling with the vectorised likelihood, batch correction and evidence.

Default workload: 10-d Rosenbrock chain, prior [-5,5]^10, N_live = 500,
batch m = 50, FP64 likelihood, FP32 sampler state, cluster tree depth 2,
5 d slice iterations, stop at remaining-evidence fraction 1e-3.

value = live-point updates per second over the timed runs (dead rows / wall
time of ns_run, inputs and live set already on the device); evaluations per
second are reported beside it.  Every run's log Z is checked against the
oracle's mean on the same workload (|dlogZ| < 2 combined sigma) and against
the transfer-matrix quadrature value.

Other modes (one JSON line each): --workload 4 / 5 (27-d emulator runs, with
--prec f32|bf16x3 and --no-screen), --lik-sweep (the batched emulator
likelihood at 200 ... 25,600 rows per call), --select-sweep (worst-1000
selection at N = 2^16 ... 2^24), --cluster-sweep (one cluster-tree node at
N = 2^16 ... 2^24) and --train-sweep (a dense network's training step at
batch 1,024 ... 65,536).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

ROSEN_QUADRATURE_LOGZ = -43.10836   # transfer-matrix quadrature of the 10-d chain on [-5,5]^10
FP64_PEAK = 78.6e12                 # MI355X FP64 vector FLOP/s


EMU_FLOPS = 2 * (27 * 512 + 512 * 512 * 2 + 512 * 1024)   # one emulator evaluation
# MFMA work actually issued per row by the split-bfloat16 path: nine products of
# 32 (padded) inputs in the first layer, three activation terms afterwards
EMU_MFMA_ISSUED = 2 * (9 * 32 * 512 + 3 * (512 * 512 * 2 + 512 * 1024))
BF16_PEAK = 2.5e15                                          # MI355X dense BF16 MFMA FLOP/s

# HBM bytes per launch of the fused slice kernel on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled
# by what the counter reads for a 256 MiB device copy (FETCH_SIZE reads half the
# bytes moved: x2.0; WRITE_SIZE: x1.0).  Valid only for the kernel sources they
# were taken with: reported as null once those sources change.
SLICE_TRAFFIC = {
    "sources": ["paper_2608_28514_amd/csrc/k_slice.hip", "paper_2608_28514_amd/csrc/ns_device.hpp",
                "paper_2608_28514_amd/csrc/ns_internal.hpp"],
    "sha256": "f25b04853910a423c7b68b7fcf73d8aed303ab83ed738ecb825572fcbc8c59cb",
    "fetch_kib": 325.30, "fetch_scale": 2.0, "write_kib": 18.31, "write_scale": 1.0,
}


def slice_traffic_bytes():
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in SLICE_TRAFFIC["sources"]:
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != SLICE_TRAFFIC["sha256"]:
        return None
    t = SLICE_TRAFFIC
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])
FP32_PEAK = 157.3e12                                        # MI355X FP32 vector FLOP/s


def rosen_flops_per_eval(d):
    # theta = lo + span*u (2d) + 9 terms of 8 flops + proposal x + t v (2d)
    return 2 * d + 8 * (d - 1) + 2 * d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--workload", type=int, default=2,
                    help="2: 10-d Rosenbrock (default); 4: 27-d emulator; 5: emulator + learned screen")
    ap.add_argument("--prec", default=None, help="emulator layers: bf16x3 (default) or f32")
    ap.add_argument("--max-steps", type=int, default=0,
                    help="emulator workloads: stop each run after this many batched steps (timing probe)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stepout-spec", type=int, default=None,
                    help="batched rounds: stepping-out offsets per side evaluated per round")
    ap.add_argument("--shrink-spec", type=int, default=None,
                    help="batched rounds: shrink proposals evaluated per round")
    ap.add_argument("--screen", default="",
                    help="workload 5: surrogate settings as k=v pairs, e.g. margin=3,train_every=4")
    ap.add_argument("--no-screen", action="store_true",
                    help="workload 5 without the learned pre-screen (the plain sampler)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--select-sweep", action="store_true",
                    help="worst-1000 selection alone at N = 2^16 ... 2^24 (HBM streaming passes)")
    ap.add_argument("--cluster-sweep", action="store_true",
                    help="one cluster-tree node (mean, covariance, 2-means) at N = 2^16 ... 2^24, d = 10")
    ap.add_argument("--lik-sweep", action="store_true",
                    help="batched emulator likelihood alone at M = 200 ... 25600 rows per call")
    ap.add_argument("--train-sweep", action="store_true",
                    help="network training step alone (forward + backward) at batch 1024 ... 65536")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; run with --gpus 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2608_28514_amd import native, workloads

    torch.cuda.set_device(0)
    if args.lik_sweep:
        return bench_lik_sweep(args, np, torch, native, workloads)
    if args.select_sweep:
        return bench_select_sweep(args, np, torch, native)
    if args.cluster_sweep:
        return bench_cluster_sweep(args, np, torch, native)
    if args.train_sweep:
        return bench_train_sweep(args, np, torch, native)
    if args.workload in (4, 5):
        return bench_emulator(args, np, torch, native, workloads)
    spec = workloads.likelihood(2)
    N, m, d, depth = 500, args.m or 50, 10, 2
    kw = dict(prec="f64", state="f32", tree_depth=depth)

    for k in range(args.warmup):
        s = native.Sampler(spec, N, seed=999 + k, **kw)
        s.run(m)
        s.logZ()
        s.close()

    torch.cuda.synchronize()
    runs = []
    t_total = 0.0
    kern = {c: [0.0, 0] for c in native.TIMING_CLASSES}
    for k in range(args.steps):
        s = native.Sampler(spec, N, seed=k, **kw)
        # events around the slice kernel only: it is the roofline kernel, and
        # the other launches run without extra stream records
        native.ns_set_timing(s.ctx, 1 << native.TIMING_CLASSES.index("slice"))
        native.ns_sync(s.ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run(m)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        t_total += t1 - t0
        tm = native.ns_get_timing(s.ctx)
        for c, (ms, n) in tm.items():
            kern[c][0] += ms
            kern[c][1] += n
        st = s.stats()
        lz, sig, H = s.logZ()
        runs.append({"seed": k, "time_s": t1 - t0, "dead": st["dead"], "steps": st["steps"],
                     "evals": st["evals"] - N, "logZ": lz, "sigma": sig, "H": H})
        s.close()

    dead = sum(r["dead"] for r in runs)
    evals = sum(r["evals"] for r in runs)
    steps_sum = sum(r["steps"] for r in runs)
    value = dead / t_total
    # dominant kernel class and its roofline (ALU bound: FP64 likelihood arithmetic)
    dom = "slice"
    slice_ms, slice_n = kern["slice"]
    # useful work of the slice kernel: the counted likelihood calls (the
    # directions are formed by the separate draw kernel)
    flops = evals * rosen_flops_per_eval(d)
    achieved = flops / (slice_ms * 1e-3) if slice_ms > 0 else 0.0
    roof = {"kernel": "k_slice<float,double,10>", "bound": "alu", "achieved": achieved / 1e12,
            "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK,
            "traffic": slice_traffic_bytes(), "traffic_unit": "bytes per launch",
            "avg_launch_us": 1e3 * slice_ms / max(slice_n, 1),
            "flops_per_launch": flops / max(slice_n, 1), "dominant_class": dom}

    out = {
        "metric": "live-point updates/s at |dlogZ|<2sigma vs oracle, 1 GPU",
        "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_total / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"rosenbrock10d prior[-5,5]^10 N_live={N} m={m} depth={depth} "
                               f"slice=5d f64-likelihood f32-state stop=1e-3",
                   "n_live": N, "m": m, "d": d},
        "evals_per_s": evals / t_total,
        "kernel_ms": {"slice": round(kern["slice"][0], 3)},
        "kernel_launches": {"slice": kern["slice"][1]},
        "roofline": roof,
        "runs": [{k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()} for r in runs],
        "quadrature_logZ": ROSEN_QUADRATURE_LOGZ,
    }

    if not args.no_cpu_baseline:
        import oracle
        threads = min(os.cpu_count() or 1, 16)
        oracle.set_threads(threads)
        o_dead, o_time, o_lz = 0, 0.0, []
        seed = 0
        while o_time < args.cpu_seconds and seed < 16:
            o = oracle.Oracle(spec, N, seed=seed, tree_depth=depth)
            t0 = time.perf_counter()
            o.run(m)
            o_time += time.perf_counter() - t0
            o_dead += o.n_dead()
            o_lz.append(o.logZ())
            seed += 1
        o_vals = np.array([x[0] for x in o_lz])
        o_mean = float(o_vals.mean())
        o_sig = float(np.mean([x[1] for x in o_lz]))
        # per-run scatter: the larger of sqrt(H/N) and the oracle's own spread
        o_spread = float(o_vals.std(ddof=1)) if len(o_vals) > 1 else o_sig
        out["cpu_baseline"] = {"value": o_dead / o_time, "unit": "updates/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{len(o_lz)} complete FP64 oracle runs of the same workload "
                                         f"(seeds 0..{len(o_lz) - 1}), OpenMP over the m chains"}
        out["oracle_logZ_mean"] = o_mean
        out["oracle_logZ_run_std"] = o_spread
        out["gpu_logZ_mean"] = float(np.mean([r["logZ"] for r in runs]))
        gate = [abs(r["logZ"] - o_mean) < 2 * math.sqrt(max(r["sigma"], o_spread) ** 2 + o_spread ** 2 / len(o_lz))
                for r in runs]
        out["pass_2sigma_vs_oracle"] = f"{sum(gate)}/{len(gate)}"
        gate_s = [abs(r["logZ"] - o_mean) < 2 * math.sqrt(r["sigma"] ** 2 + o_spread ** 2 / len(o_lz))
                  for r in runs]
        out["pass_2sigma_vs_oracle_sqrtHN"] = f"{sum(gate_s)}/{len(gate_s)}"
        g_vals = np.array([r["logZ"] for r in runs])
        sem = math.sqrt((g_vals.var(ddof=1) if len(g_vals) > 1 else o_spread ** 2) / len(g_vals)
                        + o_spread ** 2 / len(o_lz))
        out["mean_logZ_diff_vs_oracle_in_sem"] = float((g_vals.mean() - o_mean) / sem)
    out["pass_2sigma_vs_quadrature"] = \
        f"{sum(abs(r['logZ'] - ROSEN_QUADRATURE_LOGZ) < 2 * r['sigma'] for r in runs)}/{len(runs)}"
    print(json.dumps(out))


HBM_PEAK = 8.0e12                   # MI355X HBM3E bytes/s


def bench_select_sweep(args, np, torch, native):
    """ns_select_worst (the m = 1000 worst of N FP64 likelihoods, drawn from
    N(-100, 30^2)) at N = 2^16 ... 2^24, timed with torch events on the stream
    it runs on.  Each pass streams N doubles from HBM; the achieved rate counts
    8 N bytes per pass over the whole call (initialisation, the early-exiting
    launches and the final sort of at most 8192 candidates included)."""
    m = 1000
    work = torch.empty(native.ns_select_worst_work_bytes(), dtype=torch.uint8, device="cuda:0")
    gen = torch.Generator().manual_seed(0)
    res = []
    for lg in (16, 18, 20, 22, 24):
        N = 1 << lg
        x = (torch.randn(N, generator=gen, dtype=torch.float64) * 30.0 - 100.0).to("cuda:0")
        slots = torch.empty(m, dtype=torch.int32, device="cuda:0")
        passes = torch.zeros(1, dtype=torch.int32, device="cuda:0")
        native.ns_select_worst(x, m, slots, work, passes)
        torch.cuda.synchronize()
        reps = max(10, min(200, (1 << 28) // N))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            native.ns_select_worst(x, m, slots, work, passes)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3 / reps
        npass = int(passes.item())
        ok = bool(torch.equal(slots.cpu().long(), torch.argsort(x, stable=True)[:m].cpu()))
        bw = npass * 8.0 * N / t
        res.append({"N": N, "m": m, "us_per_call": 1e6 * t, "passes": npass, "hbm_gbs": bw / 1e9,
                    "hbm_frac": bw / HBM_PEAK, "matches_stable_sort": ok})
        print(f"[bench] select N=2^{lg}: {1e6 * t:.1f} us, {npass} passes, {bw / 1e9:.0f} GB/s",
              file=sys.stderr, flush=True)
    print(json.dumps({"metric": "worst-m selection, N sweep", "dtype": "f64", "data": "synthetic",
                      "peak_gbs": HBM_PEAK / 1e9, "config": {"workload": "select worst 1000 of N(-100,30^2)"},
                      "sweep": res}))


def bench_cluster_sweep(args, np, torch, native):
    """ns_cluster_split (mean, covariance, k-means split of one node) on N
    points in d = 10 (two Gaussian blobs, sd 0.05, clipped to the unit cube;
    FP32) at N = 2^16 ... 2^24, timed with torch events on its stream.  Each
    pass streams the N x d FP32 points (the Lloyd passes also read and write
    one side byte per point); the achieved rate counts 4 N d bytes per pass."""
    d, iters = 10, 20
    work = torch.empty(native.ns_cluster_split_work_bytes(), dtype=torch.uint8, device="cuda:0")
    gen = torch.Generator().manual_seed(0)
    res = []
    for lg in (16, 18, 20, 22, 24):
        N = 1 << lg
        c = torch.rand((2, d), generator=gen, dtype=torch.float64) * 0.6 + 0.2
        lab = torch.randint(0, 2, (N,), generator=gen)
        u = (c[lab] + 0.05 * torch.randn((N, d), generator=gen, dtype=torch.float64)).clamp(0, 1)
        u = u.to(torch.float32).to("cuda:0")
        mean = torch.zeros(d, dtype=torch.float64, device="cuda:0")
        cov = torch.zeros((d, d), dtype=torch.float64, device="cuda:0")
        cen = torch.zeros((2, 32), dtype=torch.float64, device="cuda:0")
        side = torch.zeros(N, dtype=torch.uint8, device="cuda:0")
        passes = torch.zeros(1, dtype=torch.int32, device="cuda:0")
        native.ns_cluster_split(u, iters, mean, cov, cen, side, work, passes)
        torch.cuda.synchronize()
        reps = max(5, min(100, (1 << 26) // N))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            native.ns_cluster_split(u, iters, mean, cov, cen, side, work, passes)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3 / reps
        npass = int(passes.item())
        bw = npass * 4.0 * N * d / t
        res.append({"N": N, "d": d, "us_per_call": 1e6 * t, "passes": npass, "hbm_gbs": bw / 1e9,
                    "hbm_frac": bw / HBM_PEAK})
        print(f"[bench] cluster N=2^{lg}: {1e6 * t:.1f} us, {npass} passes, {bw / 1e9:.0f} GB/s",
              file=sys.stderr, flush=True)
    print(json.dumps({"metric": "cluster-tree node (mean, covariance, 2-means), N sweep", "dtype": "f64",
                      "data": "synthetic", "peak_gbs": HBM_PEAK / 1e9,
                      "config": {"workload": "two blobs in [0,1]^10, FP32 points"}, "sweep": res}))


def bench_train_sweep(args, np, torch, native):
    """One training step of a dense network on the library's kernels
    (ns_mlp_forward keeping the pre-activations and hidden outputs, then
    ns_mlp_backward for dW, db; no input gradient), for the learned pre-screen
    (27-256-256-1, SiLU) and the 27-d emulator shape (27-512-512-512-1024,
    tanh), at batch B, in bfloat16 MFMA and FP32 FMA.  Timed with torch events
    on the stream the calls run on.  Work per sample: 2 sum_l w_l w_{l+1}
    forward, the same for dW and again for the input gradients of every layer
    but the first."""
    nets = [("screen 27-256-256-1 silu", (27, 256, 256, 1), "silu", (1024, 4096, 16384, 65536)),
            ("emulator 27-512-512-512-1024 tanh", (27, 512, 512, 512, 1024), "tanh", (1024, 4096, 16384))]
    gen = torch.Generator().manual_seed(0)
    res = []
    for name, widths, act, batches in nets:
        Ws = [((torch.rand((widths[l], widths[l + 1]), generator=gen) * 2 - 1) *
               math.sqrt(6.0 / (widths[l] + widths[l + 1]))).to("cuda:0") for l in range(len(widths) - 1)]
        bs = [torch.zeros(widths[l + 1], device="cuda:0") for l in range(len(widths) - 1)]
        desc = native.mlp_desc(Ws, bs, act)
        prods = [widths[l] * widths[l + 1] for l in range(len(widths) - 1)]
        flops = 2 * sum(prods) + 2 * sum(prods) + 2 * sum(prods[1:])
        for prec in ("bf16", "f32"):
            peak = BF16_PEAK if prec == "bf16" else FP32_PEAK
            for B in batches:
                X = torch.rand((B, widths[0]), generator=gen).to("cuda:0")
                tot = B * sum(widths[1:])
                Z = torch.empty(tot, device="cuda:0")
                H = torch.empty(tot, device="cuda:0")
                Y = torch.empty((B, widths[-1]), device="cuda:0")
                dY = torch.randn((B, widths[-1]), generator=gen).to("cuda:0")
                dWs = [torch.empty_like(w) for w in Ws]
                dbs = [torch.empty_like(b) for b in bs]
                work = torch.empty(2 * B * max(widths), device="cuda:0")

                def step():
                    native.ns_mlp_forward(desc, prec, X, Y, Z, H)
                    native.ns_mlp_backward(desc, prec, X, Z, H, dY, dWs, dbs, None, work)

                step()
                torch.cuda.synchronize()
                reps = max(5, min(200, (1 << 22) // B))
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    step()
                e1.record()
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1) * 1e-3 / reps
                tf = B * flops / t
                res.append({"net": name, "prec": prec, "batch": B, "us_per_step": 1e6 * t,
                            "tflops": tf / 1e12, "frac": tf / peak})
                print(f"[bench] train {name} {prec} B={B}: {1e6 * t:.1f} us, {tf / 1e12:.1f} TFLOP/s "
                      f"({100 * tf / peak:.1f} % of peak)", file=sys.stderr, flush=True)
                del X, Z, H, Y, dY, work
    print(json.dumps({"metric": "dense network training step (forward + backward), batch sweep",
                      "dtype": "bf16 / f32", "data": "synthetic",
                      "peaks_tflops": {"bf16": BF16_PEAK / 1e12, "f32": FP32_PEAK / 1e12}, "sweep": res}))


def bench_lik_sweep(args, np, torch, native, workloads):
    """The 27-d emulator likelihood of M prior-uniform rows per call (the
    batched-likelihood path of the rounds: row compaction, four dense layers,
    chi^2 and the scatter back), timed with HIP events on the sampler's stream,
    for M in {200, 400, 1600, 6400, 25600} (calls of more than 8192 rows run in
    chunks of 8192)."""
    prec = args.prec or "bf16x3"
    spec = workloads.likelihood(4, seed=0)
    s = native.Sampler(spec, 2000, seed=0, prec=prec, state="f32", tree_depth=1)
    gen = torch.Generator().manual_seed(0)
    peak = BF16_PEAK if prec.startswith("bf16") else FP32_PEAK
    res = []
    for M in (200, 400, 1600, 6400, 25600):
        u = torch.rand((M, 27), generator=gen, dtype=torch.float64).to("cuda:0")
        out = torch.empty(M, dtype=torch.float64, device="cuda:0")
        native.ns_loglike_batch(s.ctx, u, out)
        native.ns_sync(s.ctx)
        reps = max(20, (400 * 1600) // M)
        native.ns_set_timing(s.ctx, 1 << native.TIMING_CLASSES.index("lik"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            native.ns_loglike_batch(s.ctx, u, out)
        native.ns_sync(s.ctx)
        t1 = time.perf_counter()
        ms, n = native.ns_get_timing(s.ctx)["lik"]
        per_call = 1e-3 * ms / reps
        useful = M * EMU_FLOPS / per_call
        r = {"rows": M, "calls": reps, "us_per_call": 1e6 * per_call, "wall_us_per_call": 1e6 * (t1 - t0) / reps,
             "rows_per_s": M / per_call, "useful_tflops": useful / 1e12, "useful_frac": useful / peak}
        if prec == "bf16x3":
            issued = M * EMU_MFMA_ISSUED / per_call
            r["mfma_issued_tflops"] = issued / 1e12
            r["mfma_issued_frac"] = issued / peak
        res.append(r)
        print(f"[bench] lik sweep M={M}: {1e6 * per_call:.1f} us per call", file=sys.stderr, flush=True)
    s.close()
    print(json.dumps({"metric": "batched emulator likelihood, rows per call sweep", "dtype": prec,
                      "data": "synthetic", "peak_tflops": peak / 1e12,
                      "config": {"workload": "emulator27d MLP 27-512-512-512-1024, prior-uniform rows"},
                      "sweep": res}))


def bench_emulator(args, np, torch, native, workloads):
    """27-d random-MLP emulator (workload 4) or the same with the learned screen
    and N=4000, m=400 (workload 5).  One step = one complete run; the dominant
    kernels are the dense layers (MFMA for bf16x3)."""
    wl = args.workload
    prec = args.prec or "bf16x3"
    N, m = (2000, 200) if wl == 4 else (4000, 400)
    m = args.m or m
    spec = workloads.likelihood(wl, seed=0)
    kw = dict(prec=prec, state="f32", tree_depth=1)
    if args.stepout_spec:
        kw["stepout_spec"] = args.stepout_spec
    if args.shrink_spec:
        kw["shrink_spec"] = args.shrink_spec
    screen_kw = {"prec": "bf16"}
    for item in filter(None, args.screen.split(",")):
        k, v = item.split("=")
        screen_kw[k] = float(v) if "." in v or "e" in v else int(v)
    runs, t_total = [], 0.0
    kern = {c: [0.0, 0] for c in native.TIMING_CLASSES}
    for k in range(args.warmup + args.steps):
        s = native.Sampler(spec, N, seed=(999 + k) if k < args.warmup else k - args.warmup, **kw)
        if wl == 5 and not args.no_screen:
            s.enable_surrogate(**screen_kw)
        timed = k >= args.warmup
        if timed:
            native.ns_set_timing(s.ctx, True)
        native.ns_sync(s.ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # chunks of 100 steps with a progress line each (a full run takes minutes)
        left = args.max_steps if args.max_steps else None
        while True:
            chunk = 100 if left is None else min(100, left)
            rc, _ = s.run(m, max_steps=chunk)
            done = rc == native.NS_DONE
            if left is not None:
                left -= chunk
            st_p = s.stats()
            print(f"[bench] workload {wl} run {k}: {st_p['steps']} steps, {st_p['dead']} dead, "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
            if done or (left is not None and left <= 0):
                break
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        print(f"[bench] workload {wl} run {k} ({'timed' if timed else 'warm-up'}): {t1 - t0:.1f} s",
              file=sys.stderr, flush=True)
        if not timed:
            s.close()
            continue
        t_total += t1 - t0
        for c, (ms, n) in native.ns_get_timing(s.ctx).items():
            kern[c][0] += ms
            kern[c][1] += n
        st = s.stats()
        lz, sig, H = s.logZ()
        r = {"seed": k - args.warmup, "time_s": t1 - t0, "dead": st["dead"], "steps": st["steps"],
             "evals": st["evals"] - N, "net_rows": st["net_rows"], "screened": st["screened"],
             "logZ": lz, "sigma": sig, "H": H}
        if wl == 5 and not args.no_screen:
            r["surrogate"] = s.surrogate_stats()
        runs.append(r)
        s.close()
    dead = sum(r["dead"] for r in runs)
    evals = sum(r["evals"] for r in runs)
    rows = sum(r["net_rows"] for r in runs)
    lik_ms = kern["lik"][0]
    flops = rows * EMU_FLOPS
    peak = BF16_PEAK if prec.startswith("bf16") else FP32_PEAK
    achieved = flops / (lik_ms * 1e-3) if lik_ms > 0 else 0.0
    out = {
        "metric": "live-point updates/s at |dlogZ|<2sigma vs oracle, 1 GPU",
        "value": dead / t_total, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_total / max(args.steps, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if prec.startswith("bf16") else "f32", "data": "synthetic",
        "config": {"workload": f"emulator27d MLP 27-512-512-512-1024 N_live={N} m={m} depth=1 "
                               f"spec={kw.get('stepout_spec', 4)}/{kw.get('shrink_spec', 8)} "
                               f"layers={prec}{' +learned-screen' if wl == 5 and not args.no_screen else ''}"
                               f"{f' PARTIAL first {args.max_steps} steps' if args.max_steps else ''}",
                   "n_live": N, "m": m, "d": 27},
        "evals_per_s": evals / t_total, "net_rows_per_s": rows / t_total,
        "kernel_ms": {c: round(v[0], 3) for c, v in kern.items()},
        "kernel_launches": {c: v[1] for c, v in kern.items()},
        "roofline": {"kernel": ("k_dense_frag (emulator layers, chi^2 partials fused; the row sums run in "
                                "the next round's advance kernel)"
                                if prec.startswith("bf16") else "k_gemm<F32> + k_chi2"),
                     "bound": "mfma" if prec.startswith("bf16") else "alu", "achieved": achieved / 1e12,
                     "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "note": "network rows x 2,124,800 FLOP over the batched-likelihood time (HIP events); "
                             "the split activations issue 3x this MFMA work (9x in the first layer)"},
        "runs": runs,
    }
    print(json.dumps(out, default=float))


if __name__ == "__main__":
    main()
