"""GPU parity of the batched-round slice sampler and of the dense-network
kernels (emulator likelihood, surrogate forward/backward) against the FP64
oracle.

* Rounds driver, FP64 state, analytic likelihood: the whole run equals the
  oracle's within 1e-10 (same draws, same decisions).
* Rounds driver, FP32 state: bit-identical to the single-kernel path.
* Dense layers: each GEMM output within the FP32-accumulation bound
  gamma_K * sum |a||w| (gamma_K = K 2^-24) of the FP64 product; single-bfloat16
  operands within the bfloat16 rounding bound.
* Network backward: against the oracle's FP64 backward within FP32 bounds.
* Emulator likelihood: quantiles of |dlogL| against the FP64 oracle, and every
  row within a forward error bound derived from the FP32 / split-bfloat16
  arithmetic of each layer (both the fragment-major path and the generic one).
"""
import math
import numpy as np
import pytest
import torch

import oracle
from paper_2608_28514_amd import native, workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _close(got, ref, rtol):
    got, ref = np.asarray(got), np.asarray(ref)
    if not np.array_equal(np.isinf(got), np.isinf(ref)):
        return False
    f = np.isfinite(ref)
    return bool(np.all(np.abs(got[f] - ref[f]) <= rtol * np.maximum(1.0, np.abs(ref[f]))))


@pytest.mark.parametrize("spec_name,N,m,depth,corr", [
    ("c1", 100, 1, 0, "history"),
    ("eq5", 200, 10, 1, "history"),
    ("array", 300, 30, 3, "sort"),
])
def test_rounds_fp64_matches_oracle(spec_name, N, m, depth, corr):
    spec = {"c1": W.likelihood(1), "eq5": W.paper_problem("eq5_gauss2d"),
            "array": W.paper_problem("test1_array49")}[spec_name]
    s = native.Sampler(spec, N, seed=4, tree_depth=depth, correction=corr, batch_rounds=1)
    o = oracle.Oracle(spec, N, seed=4, tree_depth=depth, correction=corr)
    s.run(m)
    o.run(m)
    g, r = s.dead(), o.dead()
    assert g["logL"].size == r["logL"].size
    assert _close(g["logL"], r["logL"], 1e-10)
    assert np.allclose(g["u"], r["u"], rtol=0, atol=1e-10)
    st, oc = s.stats(), o.counters()
    assert st["evals"] == oc["evals"] and st["oob"] == oc["oob"] and st["steps"] == oc["steps"]


@pytest.mark.parametrize("so,sh", [(4, 8), (1, 1), (32, 64), (3, 5)])
def test_rounds_fp32_identical_to_fused_kernel(so, sh):
    spec = W.likelihood(3, seed=2)
    kw = dict(prec="f32", state="f32", seed=2, tree_depth=3)
    a = native.Sampler(spec, 1000, **kw)
    b = native.Sampler(spec, 1000, batch_rounds=1, stepout_spec=so, shrink_spec=sh, **kw)
    a.run(100, max_steps=20)
    b.run(100, max_steps=20)
    da, db = a.dead(), b.dead()
    assert np.array_equal(da["logL"], db["logL"])
    assert np.array_equal(da["u"], db["u"])
    sa, sb = a.stats(), b.stats()
    for k in ("evals", "oob", "stepout_caps", "shrink_caps", "steps", "dead"):
        assert sa[k] == sb[k], k


def _gemm_ref(X, Wm):
    return X.astype(np.float64) @ Wm.astype(np.float64)


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "bf16"])
@pytest.mark.parametrize("M,K,N", [(1, 27, 512), (200, 512, 512), (77, 33, 130), (1600, 512, 1024)])
def test_dense_layer_bounds(prec, M, K, N):
    rng = np.random.default_rng(M + K + N)
    X = rng.normal(size=(M, K)).astype(np.float32)
    Wm = W._round_bf16(rng.normal(size=(K, N)) * 0.1).astype(np.float32)
    b = np.zeros(N, dtype=np.float32)
    Xd = torch.tensor(X, device=DEV)
    Yd = torch.zeros((M, N), dtype=torch.float32, device=DEV)
    Wt = [torch.tensor(Wm, device=DEV)]
    bt = [torch.tensor(b, device=DEV)]
    d = native.mlp_desc(Wt, bt, "tanh")
    native.ns_mlp_forward(d, prec, Xd, Yd)
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy().astype(np.float64)
    ref = _gemm_ref(X, Wm)
    mag = np.abs(X).astype(np.float64) @ np.abs(Wm).astype(np.float64)
    if prec == "bf16":
        bound = (2.0 * 2.0 ** -8 + K * 2.0 ** -24) * mag
    else:
        bound = 2.0 * (K + 3) * 2.0 ** -24 * mag
    assert np.all(np.abs(Y - ref) <= bound + 1e-30)


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "bf16"])
def test_network_backward_against_oracle(prec):
    rng = np.random.default_rng(7)
    widths = [27, 64, 48, 1]
    Ws = [W._round_bf16(rng.normal(size=(widths[l], widths[l + 1])) * 0.3) for l in range(3)]
    bs = [rng.normal(size=widths[l + 1]) * 0.1 for l in range(3)]
    B = 300
    X = rng.uniform(size=(B, 27)).astype(np.float32).astype(np.float64)
    dY = rng.normal(size=(B, 1)).astype(np.float32).astype(np.float64)
    Yr, acts = oracle.mlp_forward(widths, Ws, bs, 1, X)
    dWr, dbr, dXr = oracle.mlp_backward(widths, Ws, bs, 1, X, acts, dY)
    f32 = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device=DEV)
    Wd, bd = [f32(w) for w in Ws], [f32(b) for b in bs]
    desc = native.mlp_desc(Wd, bd, "silu")
    Xd = f32(X)
    Yd = torch.zeros((B, 1), dtype=torch.float32, device=DEV)
    tot = B * sum(widths[1:])
    Zd = torch.zeros(tot, dtype=torch.float32, device=DEV)
    Hd = torch.zeros(tot, dtype=torch.float32, device=DEV)
    native.ns_mlp_forward(desc, prec, Xd, Yd, Zd, Hd)
    dWd = [torch.zeros_like(w) for w in Wd]
    dbd = [torch.zeros_like(b) for b in bd]
    dXd = torch.zeros_like(Xd)
    work = torch.zeros(2 * B * max(widths), dtype=torch.float32, device=DEV)
    native.ns_mlp_backward(desc, prec, Xd, Zd, Hd, f32(dY), dWd, dbd, dXd, work)
    torch.cuda.synchronize()
    # FP32: accumulation-order bound; bfloat16 operands (the gradients in the
    # backward products are rounded once even in the split mode): 2^-7 relative
    tol = 1e-4 if prec == "f32" else 2.0 ** -7
    ytol = 1e-4 if prec != "bf16" else 2.0 ** -7
    assert np.max(np.abs(Yd.cpu().numpy() - Yr)) <= ytol * max(1.0, np.max(np.abs(Yr)))
    for l in range(3):
        g, r = dWd[l].cpu().numpy(), dWr[l]
        assert np.max(np.abs(g - r)) <= tol * max(1.0, np.max(np.abs(r))), l
        g, r = dbd[l].cpu().numpy(), dbr[l]
        assert np.max(np.abs(g - r)) <= tol * max(1.0, np.max(np.abs(r))), l
    assert np.max(np.abs(dXd.cpu().numpy() - dXr)) <= tol * max(1.0, np.max(np.abs(dXr)))


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_emulator_loglike_quantiles(prec):
    spec = W.emulator(seed=0)
    rng = np.random.default_rng(1)
    th0 = spec["theta0"]
    near = np.clip(th0 + rng.normal(0, 3e-4, size=(300, 27)), 0, 1)
    prior = rng.uniform(size=(200, 27))
    u = np.concatenate([near, prior]).astype(np.float32).astype(np.float64)
    s = native.Sampler(spec, 64, prec=prec, state="f32", seed=0, tree_depth=1)
    d_u = torch.tensor(u, device=DEV)
    d_o = torch.zeros(len(u), dtype=torch.float64, device=DEV)
    native.ns_loglike_batch(s.ctx, d_u, d_o)
    native.ns_sync(s.ctx)
    got = d_o.cpu().numpy()
    ref = oracle.loglike(spec, u)
    dn = np.abs(got[:300] - ref[:300])
    rel = np.abs(got[300:] - ref[300:]) / np.abs(ref[300:])
    print(f"{prec}: near-posterior |dlogL| p50={np.median(dn):.3g} p99={np.quantile(dn, 0.99):.3g} "
          f"(logL median {np.median(ref[:300]):.1f}); prior-typical rel p50={np.median(rel):.3g} "
          f"p99={np.quantile(rel, 0.99):.3g}")
    assert np.median(dn) < 1.0 and np.quantile(dn, 0.99) < 10.0
    assert np.quantile(rel, 0.99) < 1e-4


def test_small_emulator_run_agrees_with_oracle():
    """Evidence of a small emulator (5-32-32-32-16) from 32 GPU runs per
    precision against 32 FP64 oracle runs: means within 3 combined standard
    errors."""
    spec = W.emulator(seed=3, widths=(5, 32, 32, 32, 16), noise_frac=0.05)
    S = 32
    res = {}
    for prec in ("f32", "bf16x3"):
        z = []
        for seed in range(S):
            s = native.Sampler(spec, 200, prec=prec, state="f32", seed=seed, tree_depth=1)
            s.run(20)
            z.append(s.logZ()[0])
            s.close()
        res[prec] = np.array(z)
    oracle.set_threads(16)
    try:
        zo = []
        for seed in range(S):
            o = oracle.Oracle(spec, 200, seed=seed, tree_depth=1)
            o.run(20)
            zo.append(o.logZ()[0])
    finally:
        oracle.set_threads(1)
    zo = np.array(zo)
    for prec, z in res.items():
        sem = math.sqrt(z.var(ddof=1) / S + zo.var(ddof=1) / S)
        print(f"small emulator {prec}: GPU {z.mean():.4f}, oracle {zo.mean():.4f}, 3 SEM {3 * sem:.4f}")
        assert abs(z.mean() - zo.mean()) < 3.0 * sem


U32 = 2.0 ** -24


def _gamma(n):
    return n * U32 / (1.0 - n * U32)


def _emulator_logL_bound(spec, X):
    """Per-row bound on |logL_gpu - logL_exact| for the emulator likelihood
    evaluated on split-bfloat16 MFMA layers with FP32 accumulation, tanh hidden
    activations and an FP64 chi^2.  Products per (row, k): the first layer
    multiplies the three bfloat16 terms of the input by the three of the FP32
    weight (P = 9; the generic path instead runs an FP32 fused multiply-add
    chain, covered by the same bound), later layers the three terms of the
    activation by the bfloat16 weight (P = 3).  Layer by layer, with h exact:
      |dz| <= gamma(P K + 2) 1.02 (sum |h||w| + |b|) + sum |dh||w|
      tanh (1-Lipschitz, <= 2 ulp) and the three-term split: |dh| <= |dz| + 9 u |h|
      output y = z; chi^2: |dlogL| <= sum |r| d / sigma + (d / sigma)^2 / 2,
    r = (y - D) / sigma, plus 1e-12 |logL| for the FP64 sum."""
    Ws, bs = spec["weights"], spec["biases"]
    L = len(Ws)
    h = np.asarray(X, dtype=np.float64)
    dh = np.zeros_like(h)
    for l in range(L):
        Wl, bl = np.asarray(Ws[l], dtype=np.float64), np.asarray(bs[l], dtype=np.float64)
        K = Wl.shape[0]
        mag = np.abs(h) @ np.abs(Wl) + np.abs(bl)
        z = h @ Wl + bl
        P = 9 if l == 0 else 3
        dz = _gamma(P * K + 2) * 1.02 * mag + dh @ np.abs(Wl)
        if l + 1 < L:
            h = np.tanh(z)
            dh = dz + 9.0 * U32 * np.abs(h)
        else:
            h, dh = z, dz
    sig = np.asarray(spec["sigma"], dtype=np.float64)
    r = (h - np.asarray(spec["data"], dtype=np.float64)) / sig
    q = dh / sig
    logL = -0.5 * np.sum(r * r, axis=1)
    return np.sum(np.abs(r) * q, axis=1) + 0.5 * np.sum(q * q, axis=1) + 1e-12 * np.abs(logL)


def _bf16(x):
    """Round FP32 values to bfloat16 (nearest, ties to even), returned as FP32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _split3(x):
    x = np.asarray(x, dtype=np.float32)
    hi = _bf16(x)
    r1 = (x - hi).astype(np.float32)
    mid = _bf16(r1)
    return hi, mid, _bf16((r1 - mid).astype(np.float32))


def _emulator_logL_fp32_model(spec, X):
    """The intended arithmetic in numpy: per layer the activations (the input
    too) split into hi + mid + lo bfloat16 terms, the first layer's FP32
    weights likewise, later weights bfloat16; FP32 products summed in FP32,
    FP32 bias and tanh; chi^2 in FP64."""
    h = np.asarray(X, dtype=np.float32)
    L = len(spec["weights"])
    for l in range(L):
        Wl = np.asarray(spec["weights"][l], dtype=np.float32)
        bl = np.asarray(spec["biases"][l], dtype=np.float32)
        a = _split3(h)
        w = _split3(Wl) if l == 0 else (Wl,)
        z = np.zeros((h.shape[0], Wl.shape[1]), dtype=np.float32)
        for pa in (2, 1, 0):
            for pb in range(len(w)):
                z = (z + a[pa] @ w[pb]).astype(np.float32)
        z = (z + bl).astype(np.float32)
        h = np.tanh(z).astype(np.float32) if l + 1 < L else z
    r = (h.astype(np.float64) - spec["data"]) / spec["sigma"]
    return -0.5 * np.sum(r * r, axis=1)


@pytest.mark.parametrize("widths,n", [
    ((27, 64, 96, 64), 333),            # fragment-major path, ragged rows, several tiles
    ((27, 512, 512, 512, 1024), 300),   # the 27-d emulator on the fragment-major path
    ((5, 32, 32, 32, 16), 333),         # output width 16: the generic split path
])
def test_emulator_rows_within_error_bound(widths, n):
    """Every row within the worst-case forward bound, and the error
    distribution no wider than that of the numpy model of the same arithmetic
    (a lost bfloat16 term or a misplaced bias widens it by orders of magnitude)."""
    spec = W.emulator(seed=5, widths=widths, noise_frac=0.05)
    rng = np.random.default_rng(11)
    # FP32-representable non-zero biases; data regenerated around theta0
    spec["biases"] = [rng.normal(0, 0.1, size=w).astype(np.float32).astype(np.float64) for w in widths[1:]]
    y0 = W._forward_f64(spec["weights"], spec["biases"], spec["theta0"])
    spec["sigma"] = 0.05 * np.abs(y0)
    spec["data"] = y0 + rng.normal(size=y0.shape) * spec["sigma"]
    d = widths[0]
    near = np.clip(spec["theta0"] + rng.normal(0, 1e-3, size=(n - n // 4, d)), 0, 1)
    prior = rng.uniform(size=(n // 4, d))
    u = np.concatenate([near, prior]).astype(np.float32).astype(np.float64)
    s = native.Sampler(spec, 64, prec="bf16x3", state="f32", seed=0, tree_depth=1)
    d_u = torch.tensor(u, device=DEV)
    d_o = torch.zeros(len(u), dtype=torch.float64, device=DEV)
    native.ns_loglike_batch(s.ctx, d_u, d_o)
    native.ns_sync(s.ctx)
    got = d_o.cpu().numpy()
    s.close()
    ref = oracle.loglike(spec, u)
    bound = _emulator_logL_bound(spec, u)
    err = np.abs(got - ref)
    model = np.abs(_emulator_logL_fp32_model(spec, u) - ref)
    k = len(near)
    print(f"widths {widths}: max |dlogL|/bound = {np.max(err / bound):.3g}; near theta0 median |dlogL| "
          f"{np.median(err[:k]):.3g} (model {np.median(model[:k]):.3g}), p90 {np.quantile(err[:k], 0.9):.3g} "
          f"(model {np.quantile(model[:k], 0.9):.3g})")
    assert np.all(np.isfinite(got))
    assert np.all(err <= bound)
    for q in (0.5, 0.9):
        assert np.quantile(err[:k], q) <= 4.0 * np.quantile(model[:k], q) + 1e-9
        assert np.quantile(err[k:] / np.abs(ref[k:]), q) <= 4.0 * np.quantile(model[k:] / np.abs(ref[k:]), q) + 1e-15


def test_direct_rounds_equal_compacted_rounds():
    """Plain emulator rounds evaluate the advance kernel's compacted planes
    directly; with a surrogate attached (never trained here) every round goes
    through the row-compaction pass instead.  Placement aside the arithmetic
    per row is the same, so the two runs must agree bit for bit."""
    spec = W.emulator(seed=3, widths=(27, 64, 96, 64), noise_frac=0.05)
    out = []
    for attach in (False, True):
        s = native.Sampler(spec, 200, prec="bf16x3", state="f32", seed=4, tree_depth=1)
        if attach:
            s.enable_surrogate(min_pairs=2 ** 30, margin=1e30)   # never screens
        s.run(20, max_steps=40)
        out.append((s.dead(), s.stats()))
        s.close()
    (da, sa), (db, sb) = out
    assert len(da["logL"]) == len(db["logL"]) > 0
    assert np.array_equal(da["logL"], db["logL"])
    assert np.array_equal(da["u"], db["u"])
    for k in ("evals", "oob", "stepout_caps", "shrink_caps", "steps", "dead"):
        assert sa[k] == sb[k], k


@pytest.mark.parametrize("M,widths", [(4096, (27, 128, 64, 128)), (6001, (27, 64, 128, 64))])
def test_wide_blocks_equal_narrow_blocks(M, widths):
    """Calls of 4096 rows or more run the hidden and output layers on 32 x 64
    blocks per wave; each output tile sums its products in the same order, so
    the likelihoods equal those of the same rows in calls below 4096 rows,
    bit for bit (ragged row counts: a last wave with one row block)."""
    spec = W.emulator(seed=7, widths=widths, noise_frac=0.05)
    rng = np.random.default_rng(M)
    u = rng.uniform(size=(M, widths[0]))
    s = native.Sampler(spec, 64, prec="bf16x3", state="f32", seed=0, tree_depth=1)
    d_u = torch.tensor(u, device=DEV)
    wide = torch.zeros(M, dtype=torch.float64, device=DEV)
    native.ns_loglike_batch(s.ctx, d_u, wide)
    cut = 2039
    narrow = torch.zeros(M, dtype=torch.float64, device=DEV)
    for a in range(0, M, cut):
        native.ns_loglike_batch(s.ctx, d_u[a:a + cut].contiguous(), narrow[a:a + cut])
    native.ns_sync(s.ctx)
    s.close()
    got, ref = wide.cpu().numpy(), narrow.cpu().numpy()
    assert np.all(np.isfinite(got))
    assert np.array_equal(got, ref)


def test_tiled_layers_equal_narrow_blocks():
    """Layers with at least 256 tiles of 128 x 128 (here the 27-512-512-512-1024
    emulator at 8,155 rows: a ragged last tile) run on workgroup tiles with
    the operands staged in LDS; the likelihoods equal those of calls below
    4096 rows, bit for bit."""
    M, widths = 8155, (27, 512, 512, 512, 1024)
    spec = W.emulator(seed=9, widths=widths, noise_frac=0.05)
    rng = np.random.default_rng(M)
    u = rng.uniform(size=(M, widths[0]))
    s = native.Sampler(spec, 64, prec="bf16x3", state="f32", seed=0, tree_depth=1)
    d_u = torch.tensor(u, device=DEV)
    tiled = torch.zeros(M, dtype=torch.float64, device=DEV)
    native.ns_loglike_batch(s.ctx, d_u, tiled)
    cut = 3001
    narrow = torch.zeros(M, dtype=torch.float64, device=DEV)
    for a in range(0, M, cut):
        native.ns_loglike_batch(s.ctx, d_u[a:a + cut].contiguous(), narrow[a:a + cut])
    native.ns_sync(s.ctx)
    s.close()
    got, ref = tiled.cpu().numpy(), narrow.cpu().numpy()
    assert np.all(np.isfinite(got))
    assert np.array_equal(got, ref)
