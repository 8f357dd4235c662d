"""The 27-d emulator workloads against the oracle's FP64 evidence reference
(tests/golden/emulator27d_reference.json: importance-sampling integral of
Eq. (1) with the oracle's FP64 likelihood, +-0.0024).

* The GPU's own likelihood arithmetic (split-bfloat16 MFMA layers, FP32
  layers) moves the evidence by little: the reference's importance samples
  re-weighted with the GPU likelihood give log Z within 0.05 of the FP64
  value.
* Complete GPU runs of workload 4 (N = 2000, m = 200; both layer
  precisions) give log Z within 2 sigma of the reference, sigma =
  sqrt(sigma_run^2 + se_ref^2), sigma_run = sqrt(H/N).  The benchmark runs
  workload 5 (N = 4000, m = 400) to the same gate.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import evidence_is as E
from paper_2608_28514_amd import native, workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
REF = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "emulator27d_reference.json")))


def test_reference_is_this_likelihood():
    spec = W.likelihood(4, seed=0)
    mode = np.array(REF["mode"])
    assert abs(float(oracle.loglike(spec, mode[None, :])[0]) - REF["logL_mode"]) < 1e-9
    assert REF["mode_to_box_edge_in_sd"] > 10


@pytest.mark.parametrize("prec", ["bf16x3", "f32"])
def test_gpu_likelihood_arithmetic_moves_the_evidence_little(prec):
    spec = W.likelihood(4, seed=0)
    mode, cov = np.array(REF["mode"]), np.array(REF["cov"])
    n, nu, scale = 20_000, 10.0, 1.2
    L = np.linalg.cholesky(cov) * scale
    rng = np.random.default_rng(12345)
    x = mode + (rng.standard_normal((n, 27)) @ L.T) / np.sqrt(rng.chisquare(nu, n) / nu)[:, None]
    x = x.astype(np.float32).astype(np.float64)       # the sampler's FP32 state
    lq = E.student_t_logpdf(x, mode, L, nu)
    oracle.set_threads(16)
    try:
        l64 = oracle.loglike(spec, x)
    finally:
        oracle.set_threads(1)
    s = native.Sampler(spec, 64, prec=prec, state="f32", tree_depth=1)
    d_u = torch.tensor(x, device=DEV)
    d_o = torch.zeros(n, dtype=torch.float64, device=DEV)
    native.ns_loglike_batch(s.ctx, d_u, d_o)
    native.ns_sync(s.ctx)
    lg = d_o.cpu().numpy()
    s.close()

    def logz(ll):
        lw = ll - lq
        mx = lw.max()
        return mx + math.log(np.mean(np.exp(lw - mx)))

    z64, zg = logz(l64), logz(lg)
    post = np.exp((l64 - lq) - (l64 - lq).max())
    post /= post.sum()
    mean_err = float(np.sum(post * (lg - l64)))
    print(f"{prec}: log Z FP64 {z64:.5f}, GPU arithmetic {zg:.5f} (shift {zg - z64:+.5f}); "
          f"posterior-mean logL error {mean_err:+.5f}; p50/p99 |dlogL| "
          f"{np.median(np.abs(lg - l64)):.4f} / {np.quantile(np.abs(lg - l64), 0.99):.4f}")
    assert abs(z64 - REF["logZ"]) < 0.05
    assert abs(zg - z64) < 0.05


@pytest.mark.parametrize("prec", ["bf16x3", "f32"])
def test_full_width_run_within_2_sigma_of_reference(prec):
    spec = W.likelihood(4, seed=0)
    s = native.Sampler(spec, 2000, prec=prec, state="f32", tree_depth=1, seed=1)
    s.run(200)
    lz, sig, H = s.logZ()
    st = s.stats()
    s.close()
    lim = 2.0 * math.sqrt(sig ** 2 + REF["logZ_se"] ** 2)
    print(f"{prec}: log Z {lz:.4f} +- {sig:.4f} (reference {REF['logZ']:.4f}), H {H:.1f}, "
          f"{st['steps']} steps, {st['net_rows']} network rows")
    assert abs(H - REF["H"]) < 15.0
    assert abs(lz - REF["logZ"]) < lim
