"""GPU parity at the shapes the benchmark runs, against the FP64 oracle.

* 10-d Rosenbrock (Eq. (6) chained), N = 500, m = 50, tree depth 2, FP32
  sampler state, FP64 likelihood: the cluster tree of the FP32 live set equals
  the oracle's tree of the same points (counts, labels, accepted set exact);
  over several steps fed the same live set, seeds and thresholds are bit-exact
  (Algorithm 1), every new point and recorded history point re-evaluated by the
  oracle matches the GPU's likelihood within 1e-12 relative, and every chain's
  final point clears its own threshold while no earlier recorded proposal
  does (Sec. 2.2).
* The same workload with FP64 state runs the same fused kernel template at
  d = 10: whole runs equal the oracle's within 1e-10 with equal call counts.
* The cap branches of the fused first round (stepping-out and shrink caps
  below the first round's width) against the oracle, FP64.
* Batched rounds and the fused kernel give identical runs at d = 10, FP32.
* A depth-6 tree (127 nodes, Test 1 of Sec. 2.3) and a whole run with it.
* Evidence ensembles: the mean log Z of >= 32 GPU runs against the mean of the
  oracle ensemble of the same setting, within 3 combined standard errors of the
  mean, for the 10-d Rosenbrock at m = 50 and 10 (m = 1 with 16 GPU runs), and
  the 5-d mixture with the FP64 likelihood.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2608_28514_amd import native, workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _close(got, ref, rtol):
    got, ref = np.asarray(got), np.asarray(ref)
    if not np.array_equal(np.isinf(got), np.isinf(ref)) or np.any(got[np.isinf(ref)] != ref[np.isinf(ref)]):
        return False
    f = np.isfinite(ref)
    return bool(np.all(np.abs(got[f] - ref[f]) <= rtol * np.maximum(1.0, np.abs(ref[f]))))


def _c2_sampler(seed, state="f32", **kw):
    return native.Sampler(W.likelihood(2), 500, prec="f64", state=state, seed=seed, tree_depth=2, **kw)


# ---------------------------------------------------------------- C2 shape, FP32 state
def test_c2_fp32_tree_equals_oracle_tree_of_the_same_points():
    for seed in (0, 3):
        s = _c2_sampler(seed)
        lv = s.live()
        # the FP32 state holds float values: the oracle clusters exactly these points
        assert np.array_equal(lv["u"], lv["u"].astype(np.float32).astype(np.float64))
        t_ref, lab_ref = oracle.cluster(lv["u"], 2, nmin=22)
        t = s.tree()
        assert np.array_equal(t["count"], t_ref["count"])
        assert np.array_equal(t["accepted"], t_ref["accepted"])
        assert np.array_equal(t["split_ok"], t_ref["split_ok"])
        assert np.array_equal(lv["label"], lab_ref)
        ok = t["count"] >= 2
        assert np.allclose(t["centre"][ok], t_ref["centre"][ok], rtol=1e-12, atol=1e-14)
        assert np.allclose(t["chol"][ok], t_ref["chol"][ok], rtol=1e-9, atol=1e-12)


def test_c2_fp32_tree_after_a_run_equals_oracle_tree():
    """Trees of live sets concentrated in the curved valley: a step that
    reclusters first builds the tree of the live set read just before it."""
    spec = W.likelihood(2)
    s = _c2_sampler(1)
    s.run(50, max_steps=150)          # past log X = -15; the valley splits into clusters later on
    compared = splits = 0
    for _ in range(300):
        if splits >= 2:
            break
        lv = s.live()
        n_cl = s.stats()["clusterings"]
        s.step(50)
        if s.stats()["clusterings"] == n_cl:
            continue
        t_ref, lab_ref = oracle.cluster(lv["u"], 2, nmin=22)
        t = s.tree()
        assert np.array_equal(t["count"], t_ref["count"])
        assert np.array_equal(t["accepted"], t_ref["accepted"])
        assert np.array_equal(t["split_ok"], t_ref["split_ok"])
        ok = t["count"] >= 2
        assert np.allclose(t["centre"][ok], t_ref["centre"][ok], rtol=1e-12, atol=1e-14)
        assert np.allclose(t["chol"][ok], t_ref["chol"][ok], rtol=1e-9, atol=1e-12)
        # slots the step left alone carry the tree's labels; replaced ones the
        # nearest accepted centre
        after = s.live()
        same = np.all(after["u"] == lv["u"], axis=1)
        assert np.array_equal(after["label"][same], lab_ref[same])
        acc = np.nonzero(t["accepted"])[0]
        d2 = ((after["u"][~same][:, None, :] - t["centre"][acc][None, :, :]) ** 2).sum(-1)
        assert np.array_equal(after["label"][~same], acc[np.argmin(d2, axis=1)])
        compared += 1
        splits += int(t["accepted"].sum() > 1)
    print(f"C2 trees compared: {compared}, with more than one cluster: {splits}")
    assert splits >= 2
    assert spec["d"] == 10


@pytest.mark.parametrize("seed", [0, 11])
def test_c2_fp32_steps_at_full_shape(seed):
    m, T = 50, 32
    s = _c2_sampler(seed)
    o = oracle.Oracle(W.likelihood(2), 500, seed=seed, tree_depth=2)
    spec = W.likelihood(2)
    for step in range(6):
        lv = s.live()
        o.set_live(u=lv["u"], logL=lv["logL"], label=lv["label"])
        s.step(m)
        o.step(m)
        g, r = s.last_batch(), o.last_batch(m)
        # selection and seeds: Algorithm 1 on identical keys, same Philox draws
        assert np.array_equal(g["seeds"], r["seeds"]), step
        assert np.array_equal(g["tau"], r["tau"]), step
        # every new point and recorded proposal, re-evaluated in FP64
        assert _close(g["new_logL"], oracle.loglike(spec, g["new_u"]), 1e-12)
        for j in range(m):
            n = int(g["hist_n"][j])
            assert 1 <= n <= T - 1
            h = g["hist_logL"][:n, j]
            assert _close(h, oracle.loglike(spec, g["hist_u"][j, :n]), 1e-12)
            assert g["hist_logL"][T - 1, j] == g["new_logL"][j]
            assert np.array_equal(g["hist_u"][j, T - 1], g["new_u"][j])
            # only the final shrink proposal of the last iteration clears tau_j
            # (unless that iteration hit the shrink cap)
            above = np.nonzero(h > g["tau"][j])[0]
            assert above.size == 0 or (above.size == 1 and above[0] == n - 1)
        # each chain's point clears its own threshold (shrink caps aside)
        st = s.stats()
        if st["shrink_caps"] == 0:
            assert np.all(g["new_logL"] > g["tau"])
        # points are FP32 values inside the box
        assert np.array_equal(g["new_u"], g["new_u"].astype(np.float32).astype(np.float64))
        assert np.all((g["new_u"] >= 0) & (g["new_u"] <= 1))


# ---------------------------------------------------------------- C2 shape, FP64 state
def test_c2_fp64_state_whole_run_matches_oracle():
    seed = 2
    s = _c2_sampler(seed, state="f64")
    o = oracle.Oracle(W.likelihood(2), 500, seed=seed, tree_depth=2)
    oracle.set_threads(8)
    try:
        for _ in range(3):
            s.step(50)
            o.step(50)
            g, r = s.last_batch(), o.last_batch(50)
            assert np.array_equal(g["seeds"], r["seeds"])
            assert np.array_equal(g["chain_evals"], r["chain_evals"])
            assert np.array_equal(g["hist_n"], r["hist_n"])
            assert np.allclose(g["new_u"], r["new_u"], rtol=0, atol=1e-10)
            for j in range(50):
                n = int(r["hist_n"][j])
                assert _close(g["hist_logL"][:n, j], r["hist_logL"][:n, j], 1e-10)
                assert _close(g["hist_logL"][-1:, j], r["hist_logL"][-1:, j], 1e-10)
        s.run(50)
        o.run(50)
    finally:
        oracle.set_threads(1)
    gd, rd = s.dead(), o.dead()
    assert gd["logL"].size == rd["logL"].size
    assert _close(gd["logL"], rd["logL"], 1e-10)
    assert np.allclose(gd["u"], rd["u"], rtol=0, atol=1e-10)
    lg, lr = s.logZ(), o.logZ()
    assert abs(lg[0] - lr[0]) <= 1e-10 * abs(lr[0])
    st, oc = s.stats(), o.counters()
    assert st["evals"] == oc["evals"] and st["oob"] == oc["oob"] and st["steps"] == oc["steps"]


@pytest.mark.parametrize("max_stepout,max_shrink", [(1, 64), (5, 64), (64, 1), (64, 2), (1, 1), (2, 3)])
def test_cap_branches_match_oracle(max_stepout, max_shrink):
    spec = W.paper_problem("eq5_gauss2d")
    kw = dict(seed=6, tree_depth=1, max_stepout=max_stepout, max_shrink=max_shrink)
    s = native.Sampler(spec, 200, **kw)
    o = oracle.Oracle(spec, 200, **kw)
    s.run(10, max_steps=60)
    o.run(10, 60)
    g, r = s.dead(), o.dead()
    assert g["logL"].size == r["logL"].size
    assert _close(g["logL"], r["logL"], 1e-10)
    assert np.allclose(g["u"], r["u"], rtol=0, atol=1e-10)
    st, oc = s.stats(), o.counters()
    for k in ("evals", "oob", "stepout_caps", "shrink_caps"):
        assert st[k] == oc[k], k


def test_cap_branches_at_d10_fp64_match_oracle():
    kw = dict(seed=8, tree_depth=2, max_stepout=2, max_shrink=3)
    s = _c2_sampler(8, state="f64", max_stepout=2, max_shrink=3)
    o = oracle.Oracle(W.likelihood(2), 500, **kw)
    s.run(50, max_steps=20)
    o.run(50, 20)
    g, r = s.dead(), o.dead()
    assert _close(g["logL"], r["logL"], 1e-10)
    st, oc = s.stats(), o.counters()
    for k in ("evals", "oob", "stepout_caps", "shrink_caps"):
        assert st[k] == oc[k], k
    assert st["shrink_caps"] > 0 and st["stepout_caps"] > 0


@pytest.mark.parametrize("so,sh", [(4, 8), (1, 1), (32, 64)])
def test_rounds_identical_to_fused_kernel_d10_fp32(so, sh):
    a = _c2_sampler(4)
    b = _c2_sampler(4, batch_rounds=1, stepout_spec=so, shrink_spec=sh)
    a.run(50, max_steps=40)
    b.run(50, max_steps=40)
    da, db = a.dead(), b.dead()
    assert np.array_equal(da["logL"], db["logL"])
    assert np.array_equal(da["u"], db["u"])
    sa, sb = a.stats(), b.stats()
    for k in ("evals", "oob", "stepout_caps", "shrink_caps", "steps", "dead"):
        assert sa[k] == sb[k], k


# ---------------------------------------------------------------- depth 6
def test_depth6_tree_matches_oracle():
    """127-node tree (Test 1, the 49-Gaussian array of Eq. (2)): after 250
    identical FP64 steps (the live points sit on the separate modes) the GPU
    tree equals the oracle's."""
    spec = W.paper_problem("test1_array49")
    s = native.Sampler(spec, 1000, seed=2, tree_depth=6)
    o = oracle.Oracle(spec, 1000, seed=2, tree_depth=6)
    s.run(10, max_steps=250)
    o.run(10, 250)
    g, r = s.tree(), o.tree()
    assert g["n_nodes"] == 127
    assert np.array_equal(g["count"], r["count"])
    assert np.array_equal(g["accepted"], r["accepted"])
    assert np.array_equal(g["split_ok"], r["split_ok"])
    assert np.array_equal(s.live()["label"], o.live()["label"])
    ok = g["count"] >= 2
    assert np.allclose(g["centre"][ok], r["centre"][ok], rtol=1e-12, atol=1e-14)
    assert np.allclose(g["chol"][ok], r["chol"][ok], rtol=1e-9, atol=1e-12)
    assert g["accepted"].sum() >= 32


def test_depth6_whole_run_matches_oracle():
    spec = W.paper_problem("test1_array49")
    s = native.Sampler(spec, 1000, seed=5, tree_depth=6)
    o = oracle.Oracle(spec, 1000, seed=5, tree_depth=6)
    s.run(10)
    o.run(10)
    g, r = s.dead(), o.dead()
    assert g["logL"].size == r["logL"].size
    assert _close(g["logL"], r["logL"], 1e-10)
    assert np.allclose(g["u"], r["u"], rtol=0, atol=1e-10)
    lg, lr = s.logZ(), o.logZ()
    assert abs(lg[0] - lr[0]) <= 1e-10 * max(1.0, abs(lr[0]))
    st, oc = s.stats(), o.counters()
    assert st["evals"] == oc["evals"] and st["clusterings"] == oc["clusterings"]


# ---------------------------------------------------------------- evidence ensembles
def _gate(g, r, k=3.0):
    g, r = np.asarray(g), np.asarray(r)
    sem = math.sqrt(g.var(ddof=1) / g.size + r.var(ddof=1) / r.size)
    return abs(g.mean() - r.mean()), k * sem


@pytest.mark.parametrize("m,n_gpu", [(50, 48), (10, 32), (1, 16)])
def test_c2_ensemble_matches_oracle_ensemble(m, n_gpu):
    ref = json.load(open(os.path.join(GOLDEN, "c2_oracle_ensemble.json")))
    row = next(r for r in ref["settings"] if (r["m"], r["n"], r["depth"]) == (m, 5, 2))
    g, sig = [], []
    for seed in range(n_gpu):
        s = _c2_sampler(seed)
        s.run(m)
        lz, sg, H = s.logZ()
        g.append(lz)
        sig.append(sg)
        assert 30 < H < 45
        s.close()
    diff, lim = _gate(g, row["logZ"])
    n2 = sum(abs(z - row["mean"]) < 2 * math.sqrt(sg ** 2 + row["sem"] ** 2) for z, sg in zip(g, sig))
    print(f"C2 m={m}: GPU mean {np.mean(g):.4f} ({n_gpu} runs), oracle {row['mean']:.4f} "
          f"({len(row['logZ'])} runs); |diff| {diff:.4f} < {lim:.4f}; runs within 2 sigma: {n2}/{n_gpu}")
    assert diff < lim


def _c3_truth(spec):
    from scipy.special import erf
    Phi = lambda x: 0.5 * (1 + erf(x / math.sqrt(2)))
    return math.log(0.25 * sum(np.prod(Phi((1 - mu) / 0.05) - Phi(-mu / 0.05)) for mu in spec["mu"]))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_c3_ensemble_matches_oracle_ensemble(prec):
    S = 32
    g, r, t = [], [], []
    oracle.set_threads(16)
    try:
        for seed in range(S):
            spec = W.likelihood(3, seed=seed)
            s = native.Sampler(spec, 1000, prec=prec, state="f32", seed=seed, tree_depth=3)
            s.run(100)
            g.append(s.logZ()[0])
            s.close()
            o = oracle.Oracle(spec, 1000, seed=seed, tree_depth=3)
            o.run(100)
            r.append(o.logZ()[0])
            t.append(_c3_truth(spec))
    finally:
        oracle.set_threads(1)
    g, r, t = np.array(g), np.array(r), np.array(t)
    # compare the errors against each seed's closed form (the centres differ per seed)
    diff, lim = _gate(g - t, r - t)
    print(f"C3 {prec}: GPU mean error {np.mean(g - t):+.4f}, oracle {np.mean(r - t):+.4f}; "
          f"|diff| {diff:.4f} < {lim:.4f}")
    assert diff < lim
