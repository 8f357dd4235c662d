"""Pins of the oracle's MLP backward pass (central finite differences of its
own forward pass, FP64), of the transfer-matrix quadrature of the 10-d
Rosenbrock evidence, and of the stored oracle ensemble of that workload."""
import math
import numpy as np
import pytest
import oracle
from paper_2608_28514_amd import workloads as W


@pytest.mark.parametrize("act", [0, 1])
def test_mlp_backward_matches_finite_differences(act):
    rng = np.random.default_rng(act)
    widths = [5, 7, 6, 2]
    Ws = [rng.normal(size=(widths[l], widths[l + 1])) * 0.5 for l in range(3)]
    bs = [rng.normal(size=widths[l + 1]) * 0.1 for l in range(3)]
    X = rng.normal(size=(4, 5))
    dY = rng.normal(size=(4, 2))

    def loss(Ws_, bs_, X_):
        Y, _ = oracle.mlp_forward(widths, Ws_, bs_, act, X_)
        return float((Y * dY).sum())

    Y, acts = oracle.mlp_forward(widths, Ws, bs, act, X)
    dWs, dbs, dX = oracle.mlp_backward(widths, Ws, bs, act, X, acts, dY)
    h = 1e-6
    for l in range(3):
        for idx in [(0, 0), (widths[l] - 1, widths[l + 1] - 1), (1, 1)]:
            Wp = [w.copy() for w in Ws]; Wm = [w.copy() for w in Ws]
            Wp[l][idx] += h; Wm[l][idx] -= h
            fd = (loss(Wp, bs, X) - loss(Wm, bs, X)) / (2 * h)
            assert abs(fd - dWs[l][idx]) < 1e-7 * max(1.0, abs(fd))
        for j in (0, widths[l + 1] - 1):
            bp = [b.copy() for b in bs]; bm = [b.copy() for b in bs]
            bp[l][j] += h; bm[l][j] -= h
            fd = (loss(Ws, bp, X) - loss(Ws, bm, X)) / (2 * h)
            assert abs(fd - dbs[l][j]) < 1e-7 * max(1.0, abs(fd))
    for r, c in [(0, 0), (3, 4), (2, 1)]:
        Xp = X.copy(); Xm = X.copy()
        Xp[r, c] += h; Xm[r, c] -= h
        fd = (loss(Ws, bs, Xp) - loss(Ws, bs, Xm)) / (2 * h)
        assert abs(fd - dX[r, c]) < 1e-7 * max(1.0, abs(fd))


def rosenbrock_logZ_transfer(d=10, lo=-5.0, hi=5.0, n=4001):
    x = np.linspace(lo, hi, n)
    w = np.full(n, (hi - lo) / (n - 1)); w[0] *= 0.5; w[-1] *= 0.5
    K = np.exp(-100.0 * (x[None, :] - x[:, None] ** 2) ** 2 - (1.0 - x[:, None]) ** 2)
    f = np.ones(n)
    logscale = 0.0
    for _ in range(d - 1):
        f = (w * f) @ K
        s = f.max(); f /= s; logscale += math.log(s)
    return math.log((w * f).sum()) + logscale - d * math.log(hi - lo)


def test_rosenbrock_reference_by_quadrature():
    a = rosenbrock_logZ_transfer(n=2001)
    b = rosenbrock_logZ_transfer(n=4001)
    assert abs(a - b) < 1e-6
    assert abs(b + 43.10836) < 2e-5


def test_c2_oracle_ensemble_is_reproducible():
    """The stored ensemble of the 10-d Rosenbrock workload
    (tests/golden/c2_oracle_ensemble.json, written by c2_oracle_study.py,
    which calls only the oracle) is what the current oracle computes: two of
    its runs are repeated bit for bit, and its quadrature value is this
    file's."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c2_oracle_ensemble.json")
    ref = json.load(open(path))
    assert abs(ref["quadrature_logZ"] - rosenbrock_logZ_transfer()) < 1e-12
    row = next(r for r in ref["settings"] if (r["m"], r["n"], r["depth"]) == (50, 5, 2))
    assert len(row["seeds"]) >= 32
    oracle.set_threads(4)
    try:
        for k in (0, 7):
            o = oracle.Oracle(W.likelihood(2), ref["n_live"], seed=row["seeds"][k], tree_depth=2,
                              slice_steps_per_dim=5)
            o.run(50)
            lz, sig, H = o.logZ()
            assert lz == row["logZ"][k] and sig == row["sigma"][k] and H == row["H"][k]
    finally:
        oracle.set_threads(1)
