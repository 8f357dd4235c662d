"""Benchmark of the batched nested sampler on one MI355X.

Default workload (the largest of the five): the 27-d emulator likelihood, a
random-weight 27-512-512-512-1024 tanh network with a diagonal chi^2 against
seeded data (stand-in for the cosmological emulator of Sec. 5), prior
[0,1]^27, N_live = 4000, batch m = 400, FP32 sampler state, cluster tree depth
1, 5 d slice iterations, network layers on bfloat16 MFMA with the activations
split in three bfloat16 terms and FP32 accumulation, chi^2 in FP64.

A "step" is one ns_step_batch(m): select the m worst, m slice-sampling chains
with the batched network likelihood, cluster tree, batch correction, live and
dead update, evidence.  One complete run (seed 0) is made: `warmup` steps,
then exactly `steps` timed steps (HIP-event timing of the dense layers on the
context's stream), then the rest of the run untimed.  value = live-point
updates per second over the timed steps (inputs and live set resident on the
device).  The run's log Z is checked against the stored FP64 reference of this
likelihood (importance-sampling integral computed by the oracle) within 2
combined sigma, sigma = sqrt(H/N); the line says whether the gate passed.
The same run with the learned pre-screen is reported beside it.

cpu_baseline: the FP64 oracle (plain C, OpenMP over chains) on the same
likelihood and live-set size: one batched step from the prior live set, on
all host threads (up to 16) and on one thread.

Other modes (one JSON line each): --workload 2 (10-d Rosenbrock, N = 500,
m = 50; complete runs), --workload 4 (27-d emulator, N = 2000, m = 200),
--no-screen-run, --lik-sweep, --select-sweep, --cluster-sweep, --train-sweep.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
GOLDEN = os.path.join(ROOT, "tests", "golden")

FP64_PEAK = 78.6e12                 # MI355X FP64 vector FLOP/s
FP32_PEAK = 157.3e12                # MI355X FP32 vector FLOP/s
BF16_PEAK = 2.5e15                  # MI355X dense BF16 MFMA FLOP/s
EMU_FLOPS = 2 * (27 * 512 + 512 * 512 * 2 + 512 * 1024)   # one emulator evaluation: 2,124,800
# MFMA work issued per row by the split-bfloat16 path: three activation terms
# against the bfloat16 weights in every layer (the first layer's 32 padded
# inputs; its weights are bfloat16 values, so their zero split planes are
# skipped)
EMU_MFMA_ISSUED = 2 * (3 * 32 * 512 + 3 * (512 * 512 * 2 + 512 * 1024))
METRIC = "live-point updates/s at |dlogZ|<2sigma vs oracle, 1 GPU"
# Counters of the persistent chain kernel at N = 4000, m = 400, BF16x3 (the
# default workload), per launch over its first 12 steps, from
#   rocprofv3 --pmc FETCH_SIZE  / WRITE_SIZE / TCP_TCC_READ_REQ_sum TCC_HIT_sum ... -- python3 bench.py --steps 10 --warmup 2 --timed-only --no-cpu-baseline
# FETCH_SIZE is scaled by 2.0 and WRITE_SIZE by 1.0 (the factors a plain
# 256 MiB device copy reads for the same counters); L1-to-L2 read requests
# are 128-byte lines.  Valid only for the kernel source they were taken on.
EMU_CHAINS_COUNTERS = {"source_sha256": "32cb8e0fea3d760e32d4b95f1c88baf6b6e100929c85599d2b62ac8cdd27fbd9",
                       "fetch_kib": 10784.9, "write_kib": 19877.4, "tcp_tcc_read_req": 9.1290e8,
                       "tcc_hit": 9.1744e8, "tcc_miss": 3.1675e5}
L2_CU_PEAK = 64 * 256 * 2.4e9       # MI355X L2-to-CU fill bandwidth: 64 B per clock per CU, 256 CUs


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--workload", type=int, default=5,
                    help="5: 27-d emulator N=4000 m=400 (default); 4: N=2000 m=200; 2: 10-d Rosenbrock")
    ap.add_argument("--prec", default=None, help="emulator layers: bf16x3 (default) or f32")
    ap.add_argument("--timed-only", action="store_true",
                    help="emulator: stop after the timed steps (no complete run, no gate; for profiling)")
    ap.add_argument("--no-screen-run", action="store_true", help="emulator: skip the learned-screen run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--screen", default="",
                    help="learned-screen settings as k=v pairs, e.g. margin=3,train_every=4")
    ap.add_argument("--rounds-driver", action="store_true",
                    help="emulator: the batched-rounds driver (layer kernels per round) instead of the persistent chain kernel")
    ap.add_argument("--stepout-spec", type=int, default=None)
    ap.add_argument("--shrink-spec", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--select-sweep", action="store_true")
    ap.add_argument("--cluster-sweep", action="store_true")
    ap.add_argument("--lik-sweep", action="store_true")
    ap.add_argument("--train-sweep", action="store_true")
    ap.add_argument("--runs", default="",
                    help="independent runs at once, e.g. 1,2,4,8,16: aggregate throughput of R concurrent runs "
                         "(one stream and host thread each) of --workload 2 or 4/5")
    ap.add_argument("--corr-sweep", action="store_true",
                    help="Sec. 3.2 study: batch corrections vs m/N on the 2-d Gaussian of Eq. (5)")
    ap.add_argument("--cluster-study", action="store_true",
                    help="Sec. 2.3 study: Tests 1-3 with and without clustering, and the Test 2 depth sweep")
    ap.add_argument("--suite", action="store_true",
                    help="Sec. 4 workloads: Gaussians d = 2..32, 2-d Rosenbrock and the 49-mode array vs N_live")
    ap.add_argument("--seeds", type=int, default=0, help="study modes: runs per setting (0: the paper's count)")
    ap.add_argument("--seed-study", type=int, default=0,
                    help="emulator (--workload 4/5): this many complete runs, seeds 0 .., one after another; "
                         "log Z of each against the reference and the spread over seeds")
    ap.add_argument("--concurrent", type=int, default=16, help="study modes: runs at once (ns_run_many)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the build targets a single "
                                   "MI355X); run with --gpus 1", "n_gpus": args.gpus}))
        sys.exit(2)
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

    if args.runs or args.corr_sweep or args.cluster_study or args.suite:
        # one hardware queue per concurrent run's stream (read when the HIP runtime starts)
        need = max(int(r) for r in args.runs.split(",")) if args.runs else args.concurrent
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, max(4, need)))
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
    if args.runs:
        return bench_runs(args, np, torch, native, workloads)
    if args.corr_sweep:
        return study_corrections(args, np, torch, native, workloads)
    if args.cluster_study:
        return study_clustering(args, np, torch, native, workloads)
    if args.suite:
        return study_suite(args, np, torch, native, workloads)
    if args.workload in (4, 5) and args.seed_study:
        return study_emulator_seeds(args, np, torch, native, workloads)
    if args.workload in (4, 5):
        return bench_emulator(args, np, torch, native, workloads)
    if args.workload == 2:
        return bench_rosenbrock(args, np, torch, native, workloads)
    raise SystemExit(f"unknown workload {args.workload}")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------- 27-d emulator (default)
def _emu_sampler(native, spec, N, prec, seed, args, screen):
    kw = dict(prec=prec, state="f32", tree_depth=1, seed=seed)
    if args.rounds_driver:
        kw["fused_chains"] = 0
    if args.stepout_spec:
        kw["stepout_spec"] = args.stepout_spec
    if args.shrink_spec:
        kw["shrink_spec"] = args.shrink_spec
    s = native.Sampler(spec, N, **kw)
    if screen:
        skw = {"prec": "bf16"}
        for item in filter(None, args.screen.split(",")):
            k, v = item.split("=")
            skw[k] = float(v) if "." in v or "e" in v else int(v)
        s.enable_surrogate(**skw)
    return s


def _finish_run(native, s, m, t_start, label):
    """Run s to the stopping rule, printing progress; returns wall seconds from t_start."""
    while True:
        rc, _ = s.run(m, max_steps=200)
        st = s.stats()
        log(f"{label}: {st['steps']} steps, {st['dead']} dead, {time.perf_counter() - t_start:.1f} s")
        if rc == native.NS_DONE:
            break
    return time.perf_counter() - t_start


def bench_emulator(args, np, torch, native, workloads):
    wl = args.workload
    prec = args.prec or "bf16x3"
    N, m = (2000, 200) if wl == 4 else (4000, 400)
    m = args.m or m
    spec = workloads.likelihood(wl, seed=0)
    ref = json.load(open(os.path.join(GOLDEN, "emulator27d_reference.json")))
    # events around the dominant kernels: the persistent chain kernel (class
    # "slice", one launch per step) or, on the rounds driver, the batched
    # likelihood of each round (class "lik")
    tm_bits = (1 << native.TIMING_CLASSES.index("lik")) | (1 << native.TIMING_CLASSES.index("slice"))

    # ---- the timed steps, inside a complete run of the plain sampler (seed 0)
    s = _emu_sampler(native, spec, N, prec, 0, args, screen=False)
    native.ns_sync(s.ctx)
    t_run0 = time.perf_counter()
    s.run(m, max_steps=args.warmup)
    st0 = s.stats()
    native.ns_set_timing(s.ctx, tm_bits)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, nsteps = s.run(m, max_steps=args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = s.stats()
    tmg = s.timing()
    fused = tmg["lik"][1] == 0
    k_ms, k_launches = tmg["slice"] if fused else tmg["lik"]
    native.ns_set_timing(s.ctx, False)
    if nsteps != args.steps:
        raise SystemExit(f"the run stopped after {nsteps} of {args.steps} timed steps")
    t_steps = t1 - t0
    dead = st1["dead"] - st0["dead"]
    rows = st1["net_rows"] - st0["net_rows"]
    evals = st1["evals"] - st0["evals"]
    log(f"timed {args.steps} steps: {t_steps:.3f} s, {dead / t_steps:.0f} updates/s, "
        f"{rows} network rows, dominant kernel {k_ms:.1f} ms over {k_launches} launches")
    useful = rows * EMU_FLOPS / (k_ms * 1e-3)
    # split-bfloat16 layers issue three MFMA per product; FP32 layers one
    issued = rows * (EMU_MFMA_ISSUED if prec == "bf16x3" else EMU_FLOPS) / (k_ms * 1e-3)
    peak = BF16_PEAK if prec.startswith("bf16") else FP32_PEAK
    if fused and prec != "f32":
        kname = ("k_emu_chains: a step's chains in one persistent launch, each workgroup evaluating its "
                 "chains' rows through the four layers (27-512, 512-512, 512-512, 512-1024 + chi^2)")
        note = ("one launch per step, timed by HIP events on the context's stream; useful work 2,124,800 "
                "FLOP per network row (the split activations issue 3x that on MFMA); "
                "the chain logic runs inside the same launch")
    elif fused:
        kname = ("k_emu_chains<FP32>: a step's chains in one persistent launch, the four layers on the FP32 "
                 "MFMA (16x16x4) with FP32 activations in LDS")
        note = ("one launch per step, timed by HIP events on the context's stream; useful work 2,124,800 "
                "FLOP per network row against the FP32 matrix peak")
    else:
        kname = ("k_dense_frag: the four dense layers of one round" if prec.startswith("bf16") else
                 "k_gemm<F32> layers + k_chi2")
        note = ("one launch = the layer kernels of one batched round, timed by HIP events on the "
                "context's stream; useful work 2,124,800 FLOP per network row")
    traffic, l2 = None, None
    if fused and prec == "bf16x3" and (N, m) == (4000, 400):
        import hashlib
        src = os.path.join(ROOT, "paper_2608_28514_amd", "csrc", "k_emu_chains.hip")
        cnt = EMU_CHAINS_COUNTERS
        if hashlib.sha256(open(src, "rb").read()).hexdigest() == cnt["source_sha256"]:
            traffic = 1024.0 * (2.0 * cnt["fetch_kib"] + cnt["write_kib"])
            l2b = 128.0 * cnt["tcp_tcc_read_req"]
            t_launch = k_ms * 1e-3 / max(k_launches, 1)
            l2 = {"bytes_per_launch": l2b, "achieved_TBps": l2b / t_launch / 1e12,
                  "peak_TBps": L2_CU_PEAK / 1e12, "frac": l2b / t_launch / L2_CU_PEAK,
                  "l2_hit_rate": cnt["tcc_hit"] / (cnt["tcc_hit"] + cnt["tcc_miss"]),
                  "note": "L1-to-L2 read requests x 128 B: the weights every workgroup streams each round; "
                          "200 of the 256 CUs hold a workgroup"}
    roof = {"kernel": kname, "bound": "mfma" if prec.startswith("bf16") or fused else "alu",
            "achieved": useful / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s", "frac": useful / peak,
            "traffic": traffic, "l2_to_cu": l2,
            "flops_per_launch": rows * EMU_FLOPS / max(k_launches, 1),
            "avg_launch_us": 1e3 * k_ms / max(k_launches, 1), "launches": k_launches,
            "rows_per_launch": rows / max(k_launches, 1),
            "mfma_issued_tflops": issued / 1e12, "mfma_issued_frac": issued / peak, "note": note}
    out = {"metric": METRIC, "value": dead / t_steps, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * t_steps / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16" if prec.startswith("bf16") else "f32",
           "data": "synthetic",
           "config": {"workload": f"emulator27d random-MLP 27-512-512-512-1024 tanh + diagonal chi^2, "
                                  f"prior [0,1]^27, N_live={N}, m={m}, depth 1, 5d slice iterations, "
                                  f"layers {prec}, FP32 state, seed 0",
                      "n_live": N, "m": m, "d": 27},
           "evals_per_s": evals / t_steps, "net_rows_per_s": rows / t_steps, "roofline": roof}
    if args.timed_only:
        s.close()
        print(json.dumps(out, default=float))
        return
    wall = _finish_run(native, s, m, t_run0, "plain run")
    st = s.stats()
    lz, sig, H = s.logZ()
    s.close()
    lim = 2.0 * math.sqrt(sig ** 2 + ref["logZ_se"] ** 2)
    out["run"] = {"seed": 0, "wall_s": wall, "dead": st["dead"], "steps": st["steps"],
                  "updates_per_s_whole_run": st["dead"] / wall, "evals": st["evals"] - N,
                  "net_rows": st["net_rows"], "logZ": lz, "sigma": sig, "H": H}
    out["logZ_gate"] = {"reference_logZ": ref["logZ"], "reference_se": ref["logZ_se"],
                        "reference": "tests/golden/emulator27d_reference.json (oracle, importance sampling, FP64)",
                        "diff": lz - ref["logZ"], "limit_2sigma": lim, "pass": abs(lz - ref["logZ"]) < lim}
    out["meets_gate"] = bool(out["logZ_gate"]["pass"])
    log(f"plain run: log Z {lz:.4f} +- {sig:.4f} (reference {ref['logZ']:.4f}); {wall:.1f} s")

    # ---- the same run with the learned pre-screen
    if wl == 5 and not args.no_screen_run:
        t = _emu_sampler(native, spec, N, prec, 0, args, screen=True)
        native.ns_sync(t.ctx)
        ts0 = time.perf_counter()
        wall_s = _finish_run(native, t, m, ts0, "screened run")
        st_s = t.stats()
        lz_s, sig_s, H_s = t.logZ()
        ss = t.surrogate_stats()
        t.close()
        lim_s = 2.0 * math.sqrt(sig_s ** 2 + ref["logZ_se"] ** 2)
        out["screened_run"] = {"seed": 0, "wall_s": wall_s, "dead": st_s["dead"], "steps": st_s["steps"],
                               "updates_per_s_whole_run": st_s["dead"] / wall_s, "net_rows": st_s["net_rows"],
                               "screened": st_s["screened"], "logZ": lz_s, "sigma": sig_s,
                               "gate_pass": abs(lz_s - ref["logZ"]) < lim_s,
                               "speedup_vs_plain": wall / wall_s, "surrogate": ss}
        log(f"screened run: log Z {lz_s:.4f} +- {sig_s:.4f}; {wall_s:.1f} s")

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_emulator(np, spec, N)
    print(json.dumps(out, default=float))


def study_emulator_seeds(args, np, torch, native, workloads):
    """Complete runs of the emulator workload over seeds 0 .. K-1: each run's
    log Z against the oracle's reference, the mean's offset in standard errors
    of the mean, and the run-to-run spread against the single-run sqrt(H/N)."""
    wl = args.workload
    prec = args.prec or "bf16x3"
    N, m = (2000, 200) if wl == 4 else (4000, 400)
    m = args.m or m
    spec = workloads.likelihood(wl, seed=0)
    ref = json.load(open(os.path.join(GOLDEN, "emulator27d_reference.json")))
    runs = []
    for sd in range(args.seed_study):
        s = _emu_sampler(native, spec, N, prec, sd, args, screen=False)
        native.ns_sync(s.ctx)
        t0 = time.perf_counter()
        _finish_run(native, s, m, t0, f"seed {sd}")
        lz, sig, H = s.logZ()
        s.close()
        runs.append({"seed": sd, "logZ": lz, "sigma": sig, "H": H, "wall_s": time.perf_counter() - t0})
        log(f"seed {sd}: log Z {lz:.4f} +- {sig:.4f} ({(lz - ref['logZ']) / sig:+.2f} sigma)")
    z = np.array([r["logZ"] for r in runs])
    sg = np.array([r["sigma"] for r in runs])
    d = z - ref["logZ"]
    sd_runs = float(z.std(ddof=1)) if z.size > 1 else float("nan")
    sem = sd_runs / math.sqrt(z.size) if z.size > 1 else float("nan")
    print(json.dumps({"study": "emulator evidence over seeds", "workload": wl, "n_live": N, "m": m, "prec": prec,
                      "reference_logZ": ref["logZ"], "runs": runs, "mean_minus_reference": float(d.mean()),
                      "sem": sem, "mean_over_sem": float(d.mean()) / sem if z.size > 1 else None,
                      "run_std": sd_runs, "mean_sqrt_H_over_N": float(sg.mean()),
                      "within_2sigma": int(np.sum(np.abs(d) < 2 * sg))}, default=float))


def cpu_baseline_emulator(np, spec, N):
    """The FP64 oracle on the same likelihood and live-set size: one batched
    step from the prior live set (m chains), on all host threads and on one."""
    import oracle
    res = {}
    for threads, m in ((host_threads(), 4 * host_threads()), (1, 4)):
        oracle.set_threads(threads)
        o = oracle.Oracle(spec, N, seed=0, tree_depth=1)
        t0 = time.perf_counter()
        o.step(m)
        dt = time.perf_counter() - t0
        res[threads] = (m / dt, m, dt)
        log(f"oracle {threads} thread(s): one step of {m} chains in {dt:.2f} s")
    oracle.set_threads(1)
    nt = host_threads()
    return {"value": res[nt][0], "unit": "updates/s", "cores": nt, "kind": "oracle",
            "value_1core": res[1][0], "cpu": cpu_model(),
            "sample": f"one FP64 oracle step of the same workload from the prior live set (N={N}): "
                      f"{res[nt][1]} chains on {nt} threads ({res[nt][2]:.1f} s), {res[1][1]} chains on "
                      f"1 thread ({res[1][2]:.1f} s); OpenMP over the chains"}


# ---------------------------------------------------------------- R runs at once
def bench_runs(args, np, torch, native, workloads):
    """R independent complete runs at once (ns_run_many: a stream and a host
    thread per run), seeds 0..R-1, for each R in --runs: aggregate live-point
    updates/s, evaluations/s and the per-run log Z.  Workload 2: 10-d
    Rosenbrock (N = 500, m = 50, FP64 likelihood, FP32 state, depth 2), with
    the useful FP64 rate of the counted Rosenbrock calls; workload 4/5: the
    27-d emulator at N = 500, m = 100 (bf16x3)."""
    Rs = [int(r) for r in args.runs.split(",")]
    if args.workload == 2:
        spec, N, m = workloads.likelihood(2), 500, args.m or 50
        kw = dict(prec="f64", state="f32", tree_depth=2)
        flops_per_eval = 2 * 10 + 8 * 9 + 2 * 10      # box map, 9 chain terms, proposal x + t v
        desc = f"rosenbrock10d prior[-5,5]^10 N_live={N} m={m} depth 2 f64-likelihood f32-state"
    else:
        spec, N, m = workloads.likelihood(4, seed=0), 500, args.m or 100
        kw = dict(prec=args.prec or "bf16x3", state="f32", tree_depth=1)
        flops_per_eval = EMU_FLOPS
        desc = f"emulator27d N_live={N} m={m} depth 1 layers {kw['prec']}"
    streams = [torch.cuda.Stream() for _ in range(max(Rs))]
    # warm-up: one run per stream
    warm = [native.Sampler(spec, N, seed=900 + r, stream=streams[r], **kw) for r in range(min(2, max(Rs)))]
    native.run_many(warm, m)
    for w in warm:
        w.close()
    res = []
    for R in Rs:
        ss = [native.Sampler(spec, N, seed=r, stream=streams[r], **kw) for r in range(R)]
        for x in ss:
            native.ns_sync(x.ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        native.run_many(ss, m)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stats = [x.stats() for x in ss]
        lz = [x.logZ() for x in ss]
        for x in ss:
            x.close()
        dead = sum(st["dead"] for st in stats)
        evals = sum(st["evals"] - N for st in stats)
        r = {"R": R, "wall_s": dt, "updates_per_s": dead / dt, "evals_per_s": evals / dt,
             "useful_tflops": evals * flops_per_eval / dt / 1e12,
             "logZ_mean": float(np.mean([x[0] for x in lz])), "sigma_mean": float(np.mean([x[1] for x in lz]))}
        if R > 1:
            r["logZ_std"] = float(np.std([x[0] for x in lz], ddof=1))
        res.append(r)
        log(f"R={R}: {dt:.2f} s, {dead / dt:.0f} updates/s")
    peak = FP64_PEAK if args.workload == 2 else BF16_PEAK
    best = max(res, key=lambda x: x["updates_per_s"])
    print(json.dumps({"metric": "aggregate live-point updates/s of R independent runs at once, 1 GPU",
                      "unit": "updates/s", "data": "synthetic", "config": {"workload": desc},
                      "peak_tflops": peak / 1e12, "best_R": best["R"],
                      "best_frac_of_peak": best["useful_tflops"] * 1e12 / peak,
                      "speedup_best_vs_R1": best["updates_per_s"] / res[0]["updates_per_s"] if res[0]["R"] == 1
                      else None, "sweep": res}, default=float))


# ---------------------------------------------------------------- paper studies
def _ensemble(native, torch, spec, N, m, seeds, streams, **kw):
    """Complete runs of spec for the given seeds, len(streams) at a time
    (ns_run_many, one stream and host thread per run).  Returns the per-run
    results and the summed wall time of the batches."""
    out, wall = [], 0.0
    R = len(streams)
    for i in range(0, len(seeds), R):
        batch = seeds[i:i + R]
        ss = [native.Sampler(spec, N, seed=int(sd), stream=streams[k], **kw) for k, sd in enumerate(batch)]
        for x in ss:
            native.ns_sync(x.ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        native.run_many(ss, m)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        for sd, x in zip(batch, ss):
            st = x.stats()
            lz, sig, H = x.logZ()
            out.append({"seed": int(sd), "logZ": lz, "sigma": sig, "H": H, "dead": st["dead"],
                        "evals": st["evals"] - N, "steps": st["steps"]})
            x.close()
    return out, wall


def _summ(np, runs, truth, wall=None):
    z = np.array([r["logZ"] for r in runs])
    d = {"runs": len(runs), "mean_err": float(z.mean() - truth), "std": float(z.std(ddof=1)) if z.size > 1 else 0.0,
         "sem": float(z.std(ddof=1) / math.sqrt(z.size)) if z.size > 1 else 0.0,
         "sigma_mean": float(np.mean([r["sigma"] for r in runs])),
         "evals_mean": float(np.mean([r["evals"] for r in runs])), "dead_mean": float(np.mean([r["dead"] for r in runs]))}
    if wall is not None:
        d["wall_s"] = wall
        d["updates_per_s"] = sum(r["dead"] for r in runs) / wall
    return d


def _oracle_runs(spec, N, m, seeds, **kw):
    import oracle
    oracle.set_threads(host_threads())
    res = []
    for sd in seeds:
        o = oracle.Oracle(spec, N, seed=int(sd), **kw)
        o.run(m)
        lz, sig, H = o.logZ()
        res.append({"seed": int(sd), "logZ": lz, "sigma": sig, "H": H, "dead": o.n_dead(),
                    "evals": o.counters()["evals"] - N})
    oracle.set_threads(1)
    return res


def study_corrections(args, np, torch, native, workloads):
    """Sec. 3.2: log Z of the 2-d Gaussian of Eq. (5) on [-7,7]^2 (closed form
    d/2 log 2 pi - d log 14, up to the box truncation), N = 1000, against the
    batch fraction m/N in {0.001 ... 0.5} for (i) no correction, best-of-worst
    thresholds, (ii) batch sorting, (iii)-(v) history correction with K = 1,
    2, 10 iterations; 50 runs each (m = 1 is sequential nested sampling: one
    set of runs stands for every variant).  FP64.  Oracle runs of the same
    seeds check a subset."""
    from scipy.special import erf
    spec = workloads.paper_problem("eq5_gauss2d")
    truth = 2.0 * math.log(0.5 * (erf(7 / math.sqrt(2)) - erf(-7 / math.sqrt(2))) * math.sqrt(2 * math.pi) / 14)
    N = 1000
    S = args.seeds or 50
    seeds = list(range(S))
    streams = [torch.cuda.Stream() for _ in range(args.concurrent)]
    variants = [("none", 1), ("best_of_worst", 1), ("sort", 1), ("history", 1), ("history", 2), ("history", 10)]
    ms = [1, 2, 5, 10, 20, 50, 100, 200, 500]
    table = []
    for m in ms:
        for corr, K in (variants if m > 1 else [("history", 1)]):
            runs, wall = _ensemble(native, torch, spec, N, m, seeds, streams, correction=corr, history_iters=K)
            row = {"m": m, "m_over_N": m / N, "correction": corr if m > 1 else "all (m = 1)", "K": K}
            row.update(_summ(np, runs, truth, wall))
            table.append(row)
            log(f"m={m:4d} {row['correction']:>14s} K={K:2d}: err {row['mean_err']:+.4f} +- {row['sem']:.4f} "
                f"(std {row['std']:.3f}, sigma {row['sigma_mean']:.3f}), {wall:.1f} s")
    checks = []
    if not args.no_cpu_baseline:
        for corr, m in (("history", 100), ("none", 100), ("sort", 500)):
            o = _oracle_runs(spec, N, m, seeds[:16], correction=corr)
            g = next(r for r in table if r["m"] == m and r["correction"] == corr and r["K"] == 1)
            oz = _summ(np, o, truth)
            checks.append({"m": m, "correction": corr, "oracle_mean_err": oz["mean_err"], "oracle_sem": oz["sem"],
                           "gpu_mean_err": g["mean_err"], "gpu_sem": g["sem"],
                           "diff_in_sem": (g["mean_err"] - oz["mean_err"]) / math.sqrt(g["sem"] ** 2 + oz["sem"] ** 2)})
            log(f"oracle check {corr} m={m}: oracle {oz['mean_err']:+.4f} +- {oz['sem']:.4f}, "
                f"GPU {g['mean_err']:+.4f} +- {g['sem']:.4f}")
    print(json.dumps({"metric": "log Z error vs batch fraction m/N per correction (Sec. 3.2)", "truth": truth,
                      "data": "synthetic", "config": {"workload": "eq5 gauss2d prior[-7,7]^2 N_live=1000 FP64, "
                                                                  "depth 0, 5d slice iterations"},
                      "seeds": S, "table": table, "oracle_checks": checks}, default=float))


def _two_gauss_truth(d):
    import numpy as np
    var1 = np.array([0.1 if (i % 2 == 0) else 1.0 for i in range(d)])
    var2 = np.array([1.0 if (i % 2 == 0) else 0.1 for i in range(d)])
    a = math.log(0.1) + 0.5 * float(np.sum(np.log(2 * math.pi * var1)))
    b = 0.5 * float(np.sum(np.log(2 * math.pi * var2)))
    return float(np.logaddexp(a, b)) - d * math.log(40.0)


def _shell_truth():
    from scipy import integrate
    f = lambda r: r * math.exp(-0.5 * (r - 5.0) ** 2)
    disk = 2 * math.pi * integrate.quad(f, 0.0, 10.0, epsabs=1e-13)[0]
    # the square's four corners beyond r = 10: at radius r they span the angle
    # 2 pi - 8 acos(10 / r)
    corner = integrate.quad(lambda r: f(r) * (2 * math.pi - 8 * math.acos(10.0 / r)), 10.0, 10.0 * math.sqrt(2.0),
                            epsabs=1e-15)[0]
    return math.log((disk + corner) / 400.0)


def study_clustering(args, np, torch, native, workloads):
    """Sec. 2.3, Table 1: Test 1 (Eq. (2), 49 Gaussians, [-20,20]^2, depth 6),
    Test 2 (Eq. (3), two 10-d Gaussians, [-20,20]^10, depth 1), Test 3
    (Eq. (4), shell, [-10,10]^2, depth 4), each with and without clustering
    (depth 0), N = 1000, sequential (m = 1), recluster every 100 deaths, 50
    runs (Test 2: 20); and the Test 2 depth sweep over d in {2, 4, 6, 8, 10},
    10 runs.  FP64.  Evaluations and the paper's CPU numbers are reported
    beside the GPU's."""
    paper = {"test1": {"on": (-1.6470, 0.0207, 1.027, 102881), "off": (-1.6492, 0.0212, 0.113, 124568)},
             "test2": {"on": (-33.408, 0.198, 3.49, 10508225), "off": (-33.272, 0.221, 4.03, 14144037)},
             "test3": {"on": (-1.6261, 0.0274, 0.273, 96925), "off": (-1.6322, 0.0314, 0.048, 134944)}}
    tests = [("test1", workloads.paper_problem("test1_array49"), 6, math.log(49 * 2 * math.pi / 1600.0)),
             ("test2", workloads.paper_problem("test2_two_gauss_10d"), 1, _two_gauss_truth(10)),
             ("test3", workloads.paper_problem("test3_shell"), 4, _shell_truth())]
    streams = [torch.cuda.Stream() for _ in range(args.concurrent)]
    table = []
    for name, spec, depth, truth in tests:
        S = args.seeds or (20 if name == "test2" else 50)
        for on in (True, False):
            runs, wall = _ensemble(native, torch, spec, 1000, 1, list(range(S)), streams,
                                   tree_depth=depth if on else 0, recluster_every=100)
            row = {"test": name, "clustering": on, "depth": depth if on else 0, "truth": truth}
            row.update(_summ(np, runs, truth, wall))
            row["logZ_mean"] = truth + row["mean_err"]
            row["paper_cpu"] = dict(zip(("logZ", "std", "wall_s", "evals"), paper[name]["on" if on else "off"]))
            table.append(row)
            log(f"{name} clustering={on}: log Z {row['logZ_mean']:.4f} (truth {truth:.4f}) std {row['std']:.4f}, "
                f"evals {row['evals_mean']:.0f}, {wall:.1f} s for {S} runs")
    sweep = []
    for d in (2, 4, 6, 8, 10):
        spec = workloads.paper_problem(f"test2_two_gauss_{d}d")
        truth = _two_gauss_truth(d)
        for depth in (0, 1, 3, 6):
            runs, wall = _ensemble(native, torch, spec, 1000, 1, list(range(args.seeds or 10)), streams,
                                   tree_depth=depth, recluster_every=100)
            row = {"d": d, "depth": depth, "truth": truth}
            row.update(_summ(np, runs, truth, wall))
            sweep.append(row)
            log(f"test2 d={d} depth={depth}: err {row['mean_err']:+.4f} std {row['std']:.3f} "
                f"evals {row['evals_mean']:.0f}")
    for row in sweep:
        base = next(r for r in sweep if r["d"] == row["d"] and r["depth"] == 0)
        row["evals_ratio_vs_depth0"] = row["evals_mean"] / base["evals_mean"]
    print(json.dumps({"metric": "clustering study (Sec. 2.3, Table 1, Fig. 1)", "data": "synthetic",
                      "config": {"workload": "Tests 1-3, N_live=1000, m=1, recluster every 100 deaths, FP64"},
                      "table": table, "depth_sweep": sweep}, default=float))


def study_suite(args, np, torch, native, workloads):
    """Sec. 4 workloads (the comparison samplers themselves are not run):
    Gaussian of Eq. (5) on [-7,7]^d for d in {2, 4, 8, 16, 32} (N = 1000, 50
    runs; d = 32: 10), 2-d Rosenbrock of Eq. (6) on [-10,10]^2 and the
    49-Gaussian array of Eq. (2) for N in {100, 200, 500, 1000} (100 runs);
    sequential (m = 1), FP32 state and likelihood as the paper's Sec. 4 runs;
    log Z against the closed form or quadrature."""
    from scipy.special import erf
    streams = [torch.cuda.Stream() for _ in range(args.concurrent)]
    kw = dict(prec="f32", state="f32")
    gauss, ros, arr = [], [], []
    for d in (2, 4, 8, 16, 32):
        spec = workloads.paper_problem(f"eq5_gauss{d}d")
        truth = d * math.log(0.5 * (erf(7 / math.sqrt(2)) - erf(-7 / math.sqrt(2))) * math.sqrt(2 * math.pi) / 14)
        S = args.seeds or (10 if d == 32 else 50)
        runs, wall = _ensemble(native, torch, spec, 1000, 1, list(range(S)), streams, **kw)
        row = {"d": d, "N": 1000, "truth": truth}
        row.update(_summ(np, runs, truth, wall))
        gauss.append(row)
        log(f"gauss d={d}: err {row['mean_err']:+.4f} std {row['std']:.3f}, {wall:.1f} s / {S} runs")
    x = np.linspace(-10, 10, 400001)
    inner = math.sqrt(math.pi / 100) * 0.5 * (erf(10 * (10 - x ** 2)) - erf(10 * (-10 - x ** 2)))
    ros_truth = math.log(np.trapezoid(np.exp(-(1 - x) ** 2) * inner, x) / 400.0)
    arr_truth = math.log(49 * 2 * math.pi / 1600.0)
    for N in (100, 200, 500, 1000):
        S = args.seeds or 100
        for name, spec, truth, depth, out in (("rosenbrock2d", workloads.paper_problem("eq6_rosenbrock2d"), ros_truth, 0, ros),
                                              ("array49", workloads.paper_problem("test1_array49"), arr_truth, 6, arr)):
            runs, wall = _ensemble(native, torch, spec, N, 1, list(range(S)), streams, tree_depth=depth, **kw)
            row = {"N": N, "truth": truth, "depth": depth}
            row.update(_summ(np, runs, truth, wall))
            out.append(row)
            log(f"{name} N={N}: err {row['mean_err']:+.4f} std {row['std']:.3f}, {wall:.1f} s / {S} runs")
    print(json.dumps({"metric": "Sec. 4 workloads: log Z error and throughput", "data": "synthetic",
                      "config": {"workload": "sequential m=1, FP32 state and likelihood, 5d slice iterations"},
                      "gaussian": gauss, "rosenbrock2d": ros, "array49": arr}, default=float))


# ---------------------------------------------------------------- 10-d Rosenbrock
def bench_rosenbrock(args, np, torch, native, workloads):
    """10-d Rosenbrock, N = 500, m = 50 (or --m), FP64 likelihood, FP32 state,
    depth 2: one step = one complete run (seeds 0 .., after warm-up runs);
    log Z against the stored oracle ensemble of the same setting."""
    spec = workloads.likelihood(2)
    N, m, d, depth = 500, args.m or 50, 10, 2
    kw = dict(prec="f64", state="f32", tree_depth=depth)
    ens = json.load(open(os.path.join(GOLDEN, "c2_oracle_ensemble.json")))
    row = next((r for r in ens["settings"] if (r["m"], r["n"], r["depth"]) == (m, 5, depth)), None)
    for k in range(args.warmup):
        s = native.Sampler(spec, N, seed=999 + k, **kw)
        s.run(m)
        s.close()
    torch.cuda.synchronize()
    runs, t_total = [], 0.0
    slice_ms = slice_n = 0.0
    slice_bit = 1 << native.TIMING_CLASSES.index("slice")
    for k in range(args.steps):
        s = native.Sampler(spec, N, seed=k, **kw)
        native.ns_set_timing(s.ctx, slice_bit)
        native.ns_sync(s.ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run(m)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        t_total += t1 - t0
        ms, n = s.timing()["slice"]
        slice_ms += ms
        slice_n += n
        st = s.stats()
        lz, sig, H = s.logZ()
        runs.append({"seed": k, "time_s": t1 - t0, "dead": st["dead"], "evals": st["evals"] - N,
                     "logZ": lz, "sigma": sig, "H": H})
        s.close()
    dead = sum(r["dead"] for r in runs)
    evals = sum(r["evals"] for r in runs)
    out = {"metric": METRIC, "value": dead / t_total, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * t_total / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"rosenbrock10d prior[-5,5]^10 N_live={N} m={m} depth={depth} slice=5d "
                                  f"f64-likelihood f32-state; one step = one complete run", "n_live": N,
                      "m": m, "d": d},
           "evals_per_s": evals / t_total,
           "slice_kernel": {"avg_launch_us": 1e3 * slice_ms / max(slice_n, 1), "launches": int(slice_n),
                            "bound": "latency",
                            "note": "one wave per chain; m waves on 1,024 SIMDs"}}
    if row is not None:
        g = np.array([r["logZ"] for r in runs])
        o = np.array(row["logZ"])
        sem = math.sqrt((g.var(ddof=1) if g.size > 1 else 0.0) / g.size + o.var(ddof=1) / o.size)
        out["oracle_ensemble"] = {"mean": row["mean"], "runs": len(row["logZ"]), "std": row["std"]}
        out["gpu_logZ_mean"] = float(g.mean())
        out["mean_diff_in_sem"] = float((g.mean() - row["mean"]) / sem) if sem > 0 else None
        out["runs_within_2sigma"] = int(sum(abs(r["logZ"] - row["mean"]) < 2 * math.sqrt(r["sigma"] ** 2 +
                                                                                     row["sem"] ** 2)
                                            for r in runs))
        out["meets_gate"] = bool(abs(g.mean() - row["mean"]) < 3 * sem)
    out["runs"] = runs
    if not args.no_cpu_baseline:
        import oracle
        nt = host_threads()
        oracle.set_threads(nt)
        o_dead, o_time, seed = 0, 0.0, 0
        while o_time < args.cpu_seconds and seed < 16:
            o = oracle.Oracle(spec, N, seed=seed, tree_depth=depth)
            t0 = time.perf_counter()
            o.run(m)
            o_time += time.perf_counter() - t0
            o_dead += o.n_dead()
            seed += 1
        oracle.set_threads(1)
        out["cpu_baseline"] = {"value": o_dead / o_time, "unit": "updates/s", "cores": nt, "kind": "oracle",
                               "cpu": cpu_model(),
                               "sample": f"{seed} complete FP64 oracle runs of the same workload, OpenMP over "
                                         f"the m chains"}
    print(json.dumps(out, default=float))


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




if __name__ == "__main__":
    main()
