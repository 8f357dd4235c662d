"""The persistent chain kernel with FP32 layers (FP32 MFMA, 16 x 16 x 4).

Its sums run in another order than the FP32 layer kernels of the rounds
driver, so the two agree to FP32 rounding rather than bit for bit.  Checked
here: every likelihood the kernel produced in a run (the step's new points and
the last-iteration histories) against the oracle's FP64 likelihood within the
worst-case FP32 forward bound, and with an error distribution no wider than
that of numpy's FP32 arithmetic on the same points, input widths 6, 12 and
27 (the first layer's input padded to 32); runs are deterministic; and a
complete run gives the rounds driver's evidence within the runs' combined
sigma (the 27-d emulator's complete runs are gated against the oracle's
reference in test_gpu_emulator_reference.py).
"""
import numpy as np
import pytest

import oracle
from paper_2608_28514_amd import native, workloads as W

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


def _gamma(n):
    return n * U32 / (1.0 - n * U32)


def _fp32_logL_bound(spec, X):
    """Per-row bound on |logL_gpu - logL_exact| for FP32 layers with FP32
    accumulation (at most K + 2 roundings per output), FP32 bias and tanh
    (1-Lipschitz, a few ulp), FP64 chi^2:
      |dz| <= gamma(K + 2) 1.02 (sum |h||w| + |b|) + sum |dh||w|,  |dh| <= |dz| + 4 u |h|."""
    h = np.asarray(X, dtype=np.float64)
    dh = np.zeros_like(h)
    L = len(spec["weights"])
    for l in range(L):
        Wl = np.asarray(spec["weights"][l], dtype=np.float64)
        bl = np.asarray(spec["biases"][l], dtype=np.float64)
        K = Wl.shape[0]
        mag = np.abs(h) @ np.abs(Wl) + np.abs(bl)
        z = h @ Wl + bl
        dz = _gamma(K + 2) * 1.02 * mag + dh @ np.abs(Wl)
        if l + 1 < L:
            h = np.tanh(z)
            dh = dz + 4.0 * U32 * np.abs(h)
        else:
            h, dh = z, dz
    sig = np.asarray(spec["sigma"], dtype=np.float64)
    r = (h - np.asarray(spec["data"], dtype=np.float64)) / sig
    q = dh / sig
    logL = -0.5 * np.sum(r * r, axis=1)
    return np.sum(np.abs(r) * q, axis=1) + 0.5 * np.sum(q * q, axis=1) + 1e-12 * np.abs(logL)


def _numpy_fp32_logL(spec, X):
    h = np.asarray(X, dtype=np.float32)
    L = len(spec["weights"])
    for l in range(L):
        z = (h @ np.asarray(spec["weights"][l], dtype=np.float32)
             + np.asarray(spec["biases"][l], dtype=np.float32)).astype(np.float32)
        h = np.tanh(z).astype(np.float32) if l + 1 < L else z
    r = (h.astype(np.float64) - spec["data"]) / spec["sigma"]
    return -0.5 * np.sum(r * r, axis=1)


def _kernel_rows(s):
    """(points, logL) the chain kernel evaluated in the last step."""
    lb = s.last_batch()
    pts, ll = [lb["new_u"]], [lb["new_logL"]]
    for j in range(lb["hist_n"].size):
        n = int(lb["hist_n"][j])
        pts.append(lb["hist_u"][j, :n])
        ll.append(lb["hist_logL"][:n, j])
    u, l = np.concatenate(pts), np.concatenate(ll)
    fin = np.isfinite(l)
    return u[fin], l[fin]


@pytest.mark.parametrize("spec_name,N,m,steps", [("emulator27d", 300, 30, 12), ("emulator12d_256", 300, 40, 25),
                                                  ("emulator6d_256", 200, 20, 30)])
def test_fp32_chain_kernel_rows_within_error_bound(spec_name, N, m, steps):
    if spec_name == "emulator27d":
        spec = W.likelihood(4, seed=0)
    elif spec_name == "emulator12d_256":
        spec = W.emulator(seed=5, widths=(12, 256, 256, 512), noise_frac=0.02)
    else:
        spec = W.emulator(seed=3, widths=(6, 256, 256, 512), noise_frac=0.05)
    print(f"fp32 chains: {spec_name} N={N} m={m} steps={steps}", flush=True)
    s = native.Sampler(spec, N, prec="f32", state="f32", tree_depth=1, seed=3)
    native.ns_set_timing(s.ctx, (1 << native.TIMING_CLASSES.index("lik")) | (1 << native.TIMING_CLASSES.index("slice")))
    s.run(m, max_steps=steps)
    tmg = s.timing()
    assert s.stats()["steps"] == steps
    # the chain kernel ran (one slice launch per step, no separate likelihood launches)
    assert tmg["lik"][1] == 0 and tmg["slice"][1] == steps
    u, got = _kernel_rows(s)
    s.close()
    assert u.shape[0] >= m
    assert np.array_equal(u, u.astype(np.float32).astype(np.float64))
    oracle.set_threads(16)
    try:
        ref = oracle.loglike(spec, u)
    finally:
        oracle.set_threads(1)
    bound = _fp32_logL_bound(spec, u)
    err = np.abs(got - ref)
    model = np.abs(_numpy_fp32_logL(spec, u) - ref)
    print(f"{spec_name}: {u.shape[0]} rows, max |dlogL|/bound = {np.max(err / bound):.3g}, "
          f"median |dlogL| {np.median(err):.3g} (numpy FP32 {np.median(model):.3g}), "
          f"p90 {np.quantile(err, 0.9):.3g} (numpy FP32 {np.quantile(model, 0.9):.3g})")
    assert np.all(err <= bound)
    for q in (0.5, 0.9):
        assert np.quantile(err, q) <= 4.0 * np.quantile(model, q) + 1e-9


def test_fp32_chain_kernel_runs_are_deterministic():
    spec = W.emulator(seed=3, widths=(6, 256, 256, 512), noise_frac=0.05)
    res = []
    for _ in range(2):
        s = native.Sampler(spec, 200, prec="f32", state="f32", tree_depth=1, seed=7)
        s.run(20, max_steps=40)
        res.append((s.dead()["logL"], s.dead()["u"], s.stats()["net_rows"], s.stats()["evals"]))
        s.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    assert res[0][2] == res[1][2] and res[0][3] == res[1][3]


def test_fp32_chain_kernel_complete_run_close_to_rounds_driver():
    """Same seed on both paths: the runs separate once an FP32 rounding
    difference flips a decision, so compare what the method fixes: the
    evidence within the runs' combined sigma and comparable run lengths."""
    spec = W.emulator(seed=3, widths=(6, 256, 256, 512), noise_frac=0.05)
    out = []
    for fused in (1, 0):
        s = native.Sampler(spec, 300, prec="f32", state="f32", tree_depth=1, seed=11, fused_chains=fused)
        s.run(30)
        lz, sig, H = s.logZ()
        out.append((lz, sig, s.stats()["dead"]))
        s.close()
    (za, sa, da), (zb, sb, db) = out
    print(f"fused {za:.4f} +- {sa:.4f} ({da} dead), rounds {zb:.4f} +- {sb:.4f} ({db} dead)")
    assert abs(za - zb) < 3.0 * np.hypot(sa, sb)
    assert abs(da - db) < 0.2 * db
