"""Pins of the oracle's importance-sampling evidence (oracle/evidence_is.py),
the reference for the 27-d emulator workloads, which have no closed form:

* Gaussian likelihoods on the unit box: the estimate matches the closed form
  (products of normal-CDF differences) within its standard error, also with
  a proposal that is shifted and too wide, and the standard error is
  calibrated over 20 seeds;
* a 2-d emulator (tanh network, linear output, diagonal chi^2): the numpy
  network used for the mode equals the oracle's C likelihood, its Jacobian
  equals finite differences, the mode has zero gradient, and the evidence
  matches brute-force quadrature on a fine grid;
* a box that cuts through the posterior: points outside count zero.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

import oracle
from oracle import evidence_is as E
from paper_2608_28514_amd import workloads as W


def _gauss_truth(mu, sig):
    Phi = lambda x: 0.5 * (1.0 + erf(x / math.sqrt(2.0)))
    return float(np.sum(np.log(Phi((1.0 - mu) / sig) - Phi(-mu / sig))))


def _gauss_spec(mu, sig):
    d = mu.size
    return {"kind": "mixture", "d": d, "lo": np.zeros(d), "hi": np.ones(d),
            "logw": np.array([-0.5 * float(np.sum(np.log(2 * math.pi * sig ** 2)))]),
            "mu": mu[None, :], "ivar": (1.0 / sig ** 2)[None, :]}


def test_gaussian_closed_form_and_calibrated_error():
    rng = np.random.default_rng(1)
    d = 5
    mu = rng.uniform(0.3, 0.7, d)
    sig = rng.uniform(0.02, 0.08, d)
    spec = _gauss_spec(mu, sig)
    truth = _gauss_truth(mu, sig)
    assert abs(truth) < 1e-4               # the box holds almost all the mass
    # a proposal off by half a width in every coordinate and 1.3x too wide
    mode = mu + 0.5 * sig
    cov = np.diag((1.3 * sig) ** 2)
    z = []
    for seed in range(20):
        r = E.importance_logZ(spec, mode, cov, 4000, seed)
        z.append((r["logZ"] - truth) / r["se"])
        assert r["ess"] > 200
    z = np.array(z)
    assert abs(z.mean()) < 3.0 / math.sqrt(z.size) + 0.3
    assert 0.5 < z.std(ddof=1) < 1.6
    r = E.importance_logZ(spec, mu, np.diag(sig ** 2), 100_000, 99)
    assert abs(r["logZ"] - truth) < 4 * r["se"] and r["se"] < 0.01
    # information of a normalised Gaussian: H = -d/2 - sum log(sqrt(2 pi) sig)
    Htrue = -0.5 * d - float(np.sum(np.log(math.sqrt(2 * math.pi) * sig)))
    assert abs(r["H"] - Htrue) < 0.05


def test_box_truncation_counts_outside_points_as_zero():
    mu = np.array([0.02, 0.5, 0.97])
    sig = np.array([0.03, 0.05, 0.02])
    spec = _gauss_spec(mu, sig)
    truth = _gauss_truth(mu, sig)
    assert truth < -0.3                    # a third of the mass lies outside
    r = E.importance_logZ(spec, mu, np.diag(sig ** 2), 100_000, 5)
    assert abs(r["logZ"] - truth) < 4 * r["se"]


def _tiny_emulator():
    return W.emulator(seed=2, widths=(2, 16, 16, 8), noise_frac=0.02)


def test_emulator_network_matches_the_oracle_likelihood_and_its_jacobian():
    spec = _tiny_emulator()
    rng = np.random.default_rng(3)
    for _ in range(5):
        u = rng.uniform(0.1, 0.9, 2)
        r, J = E.emulator_residual(spec, u)
        ll = float(oracle.loglike(spec, u[None, :])[0])
        assert abs(-0.5 * float(r @ r) - ll) <= 1e-12 * max(1.0, abs(ll))
        h = 1e-6
        for k in range(2):
            e = np.zeros(2)
            e[k] = h
            fd = (E.emulator_residual(spec, u + e)[0] - E.emulator_residual(spec, u - e)[0]) / (2 * h)
            assert np.allclose(J[:, k], fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max())


def test_emulator_evidence_matches_quadrature_in_2d():
    spec = _tiny_emulator()
    res = E.emulator_evidence(spec, n=60_000, seed=1)
    mode, cov = res["mode"], res["cov"]
    r, J = E.emulator_residual(spec, mode)
    g = J.T @ r
    assert np.max(np.abs(g) * np.sqrt(np.diag(cov))) < 1e-6      # stationary (in posterior widths)
    assert res["mode_to_box_edge_in_sd"] > 10
    # brute force: trapezoid rule on a grid of +-12 posterior widths
    sd = np.sqrt(np.diag(cov))
    n = 801
    xs = [np.linspace(mode[k] - 12 * sd[k], mode[k] + 12 * sd[k], n) for k in range(2)]
    X, Y = np.meshgrid(xs[0], xs[1], indexing="ij")
    ll = oracle.loglike(spec, np.stack([X.ravel(), Y.ravel()], axis=1)).reshape(n, n)
    mx = ll.max()
    Zg = np.trapezoid(np.trapezoid(np.exp(ll - mx), xs[1], axis=1), xs[0])
    truth = mx + math.log(Zg)
    assert abs(res["logZ"] - truth) < 4 * res["se"] + 1e-4, (res["logZ"], truth, res["se"])
    assert abs(res["laplace_logZ"] - truth) < 0.05
