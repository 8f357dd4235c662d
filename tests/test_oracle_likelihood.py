"""Pins of the oracle's likelihoods: special values, independent library
evaluations (scipy) and a plain numpy matrix chain for the emulator."""
import math
import numpy as np
import oracle
from scipy.stats import multivariate_normal
from scipy.special import logsumexp
from paper_2608_28514_amd import workloads as W


def test_gaussian_mode_value():
    spec = W.likelihood(1)
    # normalised 2-d Gaussian, sigma 0.1, at its mean: -log(2 pi 0.01)
    assert abs(oracle.loglike(spec, [[0.5, 0.5]])[0] - 2.76729312) < 1e-7
    assert abs(oracle.loglike(spec, [[0.5, 0.5]])[0] + math.log(2 * math.pi * 0.01)) < 1e-14


def test_rosenbrock_special_points():
    spec = W.likelihood(2)
    # theta = -5 + 10 u; theta = 1 at u = 0.6, theta = 0 at u = 0.5
    assert oracle.loglike(spec, [np.full(10, 0.6)])[0] == 0.0 or \
        abs(oracle.loglike(spec, [np.full(10, 0.6)])[0]) < 1e-24
    assert abs(oracle.loglike(spec, [np.full(10, 0.5)])[0] + 9.0) < 1e-12


def test_mixture_against_scipy():
    rng = np.random.default_rng(1)
    for i in (1, 3):
        spec = W.likelihood(i, seed=3)
        d = spec["d"]
        u = rng.uniform(0, 1, size=(200, d))
        th = spec["lo"] + (spec["hi"] - spec["lo"]) * u
        ref = logsumexp([multivariate_normal(spec["mu"][k], np.diag(1.0 / spec["ivar"][k])).logpdf(th)
                         for k in range(len(spec["logw"]))], axis=0, b=1.0 / len(spec["logw"]))
        got = oracle.loglike(spec, u)
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-10)


def test_gmm_centre_value():
    spec = W.likelihood(3, seed=0)
    c = spec["mu"][0]
    v = oracle.loglike(spec, [c])[0]
    # one component at its centre: log(1/4 (2 pi 0.0025)^{-5/2}) plus tiny cross terms
    base = math.log(0.25) - 2.5 * math.log(2 * math.pi * 0.0025)
    assert base <= v < base + 0.1


def test_shell_and_paper_problems():
    spec = W.paper_problem("test3_shell")
    u = (np.array([[5.0, 0.0], [0.0, -5.0]]) + 10.0) / 20.0
    assert np.allclose(oracle.loglike(spec, u), 0.0, atol=1e-15)
    spec = W.paper_problem("test1_array49")
    u = (np.array([[4.0, -8.0]]) + 20.0) / 40.0
    th = np.array([4.0, -8.0])
    ref = logsumexp([-0.5 * ((th - m) ** 2).sum() for m in spec["mu"]])
    assert abs(oracle.loglike(spec, u)[0] - ref) < 1e-13


def test_out_of_box_is_minus_inf():
    spec = W.likelihood(1)
    out = oracle.loglike(spec, [[1.0 + 1e-12, 0.5], [-1e-300, 0.5], [1.0, 0.0]])
    assert out[0] == -np.inf and out[1] == -np.inf and np.isfinite(out[2])


def test_emulator_matches_numpy_chain():
    spec = W.emulator(seed=0, widths=(27, 64, 64, 64, 96))
    rng = np.random.default_rng(2)
    u = rng.uniform(0, 1, size=(16, 27))
    h = u
    for l, (Wl, bl) in enumerate(zip(spec["weights"], spec["biases"])):
        h = h @ Wl + bl
        if l < 3:
            h = np.tanh(h)
    ref = -0.5 * (((h - spec["data"]) / spec["sigma"]) ** 2).sum(axis=1)
    got = oracle.loglike(spec, u)
    assert np.allclose(got, ref, rtol=1e-11)


def test_emulator_weights_are_bfloat16_values():
    spec = W.emulator(seed=0)
    for w in spec["weights"]:
        f = w.astype(np.float32)
        assert np.array_equal(f.astype(np.float64), w)
        assert np.all((f.view(np.uint32) & 0xFFFF) == 0)
