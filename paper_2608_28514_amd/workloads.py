"""Seeded synthetic workloads.

This module only *constructs inputs*: prior boxes, likelihood parameters and
the synthetic emulator network with its data vector.  It holds none of the
sampler's arithmetic and is the one module that both the GPU library's binding
and the CPU oracle's tests draw their inputs from.

A likelihood is described by a plain dict::

    {"kind": "mixture", "d": d, "lo": lo, "hi": hi,
     "logw": (K,), "mu": (K, d), "ivar": (K, d)}          # log sum_k w_k N-kernel
    {"kind": "rosenbrock", "d", "lo", "hi", "a", "b"}     # Eq. (6), chained
    {"kind": "shell", "d", "lo", "hi", "r0", "w"}         # Eq. (4)
    {"kind": "mlp", "d", "lo", "hi", "widths", "weights", "biases", "data", "sigma"}

The five benchmark workloads (``workload(i)``):

1. 2-d normalised isotropic Gaussian, mean 0.5, sigma 0.1, prior [0,1]^2,
   N=100, m=1, FP64 everywhere.
2. 10-d Rosenbrock chain, prior [-5,5]^10, N=500, m in {1,10,50}, FP64
   likelihood with FP32 sampler state, tree depth 2.
3. 5-d mixture of 4 equal-weight normalised Gaussians, sigma 0.05, centres
   uniform in [0.2,0.8]^5 (seeded), prior [0,1]^5, N=1000, m=100, depth 3.
4. 27-d emulator: random Glorot-uniform MLP 27-512-512-512-1024 with tanh
   hidden layers and a linear output, weights rounded once to bfloat16;
   data = MLP(theta0) + N(0, sigma_i^2) with sigma_i = 0.01 |MLP(theta0)_i|;
   diagonal chi^2 likelihood, prior [0,1]^27, N=2000, m=200, depth 1.
5. workload 4 with N=4000, m=400 and a learned 27-256-256-1 SiLU surrogate.

The paper's own test problems (Sec. 2.3, 3.2, 4) are available through
``paper_problem(name)``; they stand in for the paper's runs with their exact
likelihoods and boxes.
"""
import math
import numpy as np


def _round_bf16(x):
    """Round FP64 values to the nearest bfloat16 (via FP32, both ties-to-even)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16 << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def gaussian(d, mean, sigma, lo, hi, normalised=True):
    logw = -0.5 * d * math.log(2.0 * math.pi * sigma * sigma) if normalised else 0.0
    return {"kind": "mixture", "d": d, "lo": np.full(d, float(lo)), "hi": np.full(d, float(hi)),
            "logw": np.array([logw]), "mu": np.full((1, d), float(mean)),
            "ivar": np.full((1, d), 1.0 / (sigma * sigma))}


def gmm(d, n_comp, sigma, centres, lo, hi):
    logw = math.log(1.0 / n_comp) - 0.5 * d * math.log(2.0 * math.pi * sigma * sigma)
    return {"kind": "mixture", "d": d, "lo": np.full(d, float(lo)), "hi": np.full(d, float(hi)),
            "logw": np.full(n_comp, logw), "mu": np.asarray(centres, dtype=np.float64).reshape(n_comp, d),
            "ivar": np.full((n_comp, d), 1.0 / (sigma * sigma))}


def rosenbrock(d, lo, hi, a=1.0, b=100.0):
    return {"kind": "rosenbrock", "d": d, "lo": np.full(d, float(lo)), "hi": np.full(d, float(hi)),
            "a": float(a), "b": float(b)}


def glorot_mlp(widths, seed):
    """Glorot-uniform weights (drawn in FP64, rounded once to bfloat16), zero biases."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x4D4C50]))
    Ws, bs = [], []
    for l in range(len(widths) - 1):
        a = math.sqrt(6.0 / (widths[l] + widths[l + 1]))
        Ws.append(_round_bf16(rng.uniform(-a, a, size=(widths[l], widths[l + 1]))))
        bs.append(np.zeros(widths[l + 1]))
    return Ws, bs


def _forward_f64(Ws, bs, x):
    """Synthetic-data construction only: y = MLP(x) in FP64 (tanh hidden, linear out)."""
    h = np.asarray(x, dtype=np.float64)
    for l, (W, b) in enumerate(zip(Ws, bs)):
        h = h @ W + b
        if l + 1 < len(Ws):
            h = np.tanh(h)
    return h


def emulator(seed=0, widths=(27, 512, 512, 512, 1024), noise_frac=0.01):
    widths = list(widths)
    d = widths[0]
    Ws, bs = glorot_mlp(widths, seed)
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x7468]))
    theta0 = rng.uniform(0.0, 1.0, size=d)
    y0 = _forward_f64(Ws, bs, theta0)
    sigma = noise_frac * np.abs(y0)
    if not np.all(sigma > 0):
        raise ValueError("emulator data vector has a zero component; choose another seed")
    data = y0 + rng.normal(0.0, 1.0, size=y0.shape) * sigma
    return {"kind": "mlp", "d": d, "lo": np.zeros(d), "hi": np.ones(d), "widths": widths,
            "weights": Ws, "biases": bs, "data": data, "sigma": sigma, "theta0": theta0}


def gmm_centres(seed, n_comp=4, d=5, lo=0.2, hi=0.8):
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x474D4D]))
    return rng.uniform(lo, hi, size=(n_comp, d))


WORKLOADS = {
    1: {"name": "gauss2d", "n_live": 100, "m": [1], "state": "f64", "lik_prec": "f64",
        "tree_depth": 0, "desc": "d=2 normalised Gaussian, mean 0.5, sigma 0.1, prior [0,1]^2"},
    2: {"name": "rosenbrock10d", "n_live": 500, "m": [1, 10, 50], "state": "f32", "lik_prec": "f64",
        "tree_depth": 2, "desc": "d=10 Rosenbrock, prior [-5,5]^10"},
    3: {"name": "gmm5d", "n_live": 1000, "m": [100], "state": "f32", "lik_prec": "f32",
        "tree_depth": 3, "desc": "d=5 mixture of 4 Gaussians sigma 0.05, prior [0,1]^5"},
    4: {"name": "emulator27d", "n_live": 2000, "m": [200], "state": "f32", "lik_prec": "bf16",
        "tree_depth": 1, "desc": "d=27 random-MLP emulator 27-512-512-512-1024, diagonal chi^2"},
    5: {"name": "emulator27d_surrogate", "n_live": 4000, "m": [400], "state": "f32", "lik_prec": "bf16",
        "tree_depth": 1, "desc": "workload 4 + learned 27-256-256-1 SiLU surrogate pre-screen"},
}


def likelihood(i, seed=0):
    """Likelihood dict of benchmark workload i (1..5)."""
    if i == 1:
        return gaussian(2, 0.5, 0.1, 0.0, 1.0)
    if i == 2:
        return rosenbrock(10, -5.0, 5.0)
    if i == 3:
        return gmm(5, 4, 0.05, gmm_centres(seed), 0.0, 1.0)
    if i in (4, 5):
        return emulator(seed)
    raise ValueError(i)


def paper_problem(name):
    """Likelihoods of the paper's own tests."""
    if name == "eq5_gauss2d":          # Sec. 3.2, Eq. (5), box [-7,7]^2
        return gaussian(2, 0.0, 1.0, -7.0, 7.0, normalised=False)
    if name.startswith("eq5_gauss"):   # Sec. 4.1, d in {2,4,8,16,32}
        d = int(name[len("eq5_gauss"):-1])
        return gaussian(d, 0.0, 1.0, -7.0, 7.0, normalised=False)
    if name == "test1_array49":        # Eq. (2), box [-20,20]^2
        mu = np.array([[4.0 * i, 4.0 * j] for i in range(-3, 4) for j in range(-3, 4)])
        return {"kind": "mixture", "d": 2, "lo": np.full(2, -20.0), "hi": np.full(2, 20.0),
                "logw": np.zeros(49), "mu": mu, "ivar": np.ones((49, 2))}
    if name.startswith("test2_two_gauss"):  # Eq. (3), box [-20,20]^d (d=10 in the paper)
        d = int(name.split("_")[-1][:-1]) if name.endswith("d") and name[-2].isdigit() else 10
        var1 = np.array([0.1 if (i % 2 == 0) else 1.0 for i in range(d)])
        var2 = np.array([1.0 if (i % 2 == 0) else 0.1 for i in range(d)])
        return {"kind": "mixture", "d": d, "lo": np.full(d, -20.0), "hi": np.full(d, 20.0),
                "logw": np.array([math.log(0.1), 0.0]),
                "mu": np.stack([np.full(d, -10.0), np.full(d, 10.0)]),
                "ivar": np.stack([1.0 / var1, 1.0 / var2])}
    if name == "test3_shell":          # Eq. (4), box [-10,10]^2
        return {"kind": "shell", "d": 2, "lo": np.full(2, -10.0), "hi": np.full(2, 10.0),
                "r0": 5.0, "w": 1.0}
    if name == "eq6_rosenbrock2d":     # Eq. (6), box [-10,10]^2
        return rosenbrock(2, -10.0, 10.0)
    raise ValueError(name)
