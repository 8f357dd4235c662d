"""Host-callback likelihoods (NS_LIK_CALLBACK) and failure handling forced
from the host.

* A callback that is the oracle's own FP64 likelihood drives the GPU sampler
  through the same run as the oracle (boxes [0,1]^d, so theta = u exactly).
* NaN and -inf injected by the callback in regions of the box: NaN counts as
  -inf and is counted exactly (with one proposal per chain per round every
  point passed is one counted evaluation), and the evidence is that of the
  likelihood restricted to the rest of the box (closed form).
* A callback that fails stops the step with NS_EINVAL.
* Coincident live points (zero cluster covariance, clipped to a positive
  definite one) run identically on the GPU and in the oracle.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

import oracle
from paper_2608_28514_amd import native, workloads as W

pytestmark = pytest.mark.gpu


def _close(got, ref, rtol):
    got, ref = np.asarray(got), np.asarray(ref)
    if not np.array_equal(np.isinf(got), np.isinf(ref)):
        return False
    f = np.isfinite(ref)
    return bool(np.all(np.abs(got[f] - ref[f]) <= rtol * np.maximum(1.0, np.abs(ref[f]))))


def _callback_spec(inner, fn):
    return {"kind": "callback", "d": inner["d"], "lo": inner["lo"], "hi": inner["hi"], "fn": fn}


@pytest.mark.parametrize("name,N,m,depth,spec_so_sh", [("c1", 100, 5, 0, (1, 1)),
                                                        ("c1", 100, 5, 0, (4, 8)),
                                                        ("c3", 400, 40, 3, (4, 8))])
def test_callback_oracle_likelihood_matches_oracle_run(name, N, m, depth, spec_so_sh):
    inner = W.likelihood(1) if name == "c1" else W.likelihood(3, seed=1)
    assert np.all(inner["lo"] == 0.0) and np.all(inner["hi"] == 1.0)
    calls = {"n": 0, "rows": 0}

    def fn(theta):
        calls["n"] += 1
        calls["rows"] += theta.shape[0]
        return oracle.loglike(inner, theta)

    so, sh = spec_so_sh
    s = native.Sampler(_callback_spec(inner, fn), N, seed=3, tree_depth=depth, stepout_spec=so,
                       shrink_spec=sh)
    o = oracle.Oracle(inner, N, seed=3, tree_depth=depth)
    s.run(m)
    o.run(m)
    g, r = s.dead(), o.dead()
    assert g["logL"].size == r["logL"].size
    assert _close(g["logL"], r["logL"], 1e-12)
    assert np.allclose(g["u"], r["u"], rtol=0, atol=1e-12)
    st, oc = s.stats(), o.counters()
    assert st["evals"] == oc["evals"] and st["oob"] == oc["oob"]
    if (so, sh) == (1, 1):
        # one proposal per chain per round: every point passed was counted
        assert calls["rows"] == st["evals"]
    assert calls["n"] > 0 and st["nan_logL"] == 0


def test_callback_nan_and_minus_inf_regions():
    inner = W.likelihood(1)                  # N((0.5, 0.5), 0.1^2 I), normalised, box [0,1]^2
    count = {"nan": 0, "rows": 0}

    def fn(theta):
        v = oracle.loglike(inner, theta)
        v[theta[:, 0] > 0.92] = np.nan
        v[theta[:, 1] < 0.07] = -np.inf
        count["nan"] += int(np.isnan(v).sum())
        count["rows"] += theta.shape[0]
        return v

    Phi = lambda x: 0.5 * (1.0 + erf(x / math.sqrt(2.0)))
    truth = math.log((Phi(4.2) - Phi(-5.0)) * (Phi(5.0) - Phi(-4.3)))
    # the zero-likelihood regions are a plateau holding a prior fraction p of
    # the box; their points die in ties, compressing log X by p/N per death
    # where the plateau shrinks by log(1 - p) in all: log Z is expected
    # high by about -p - log(1 - p)
    p = 0.08 + 0.07 - 0.08 * 0.07
    plateau = -p - math.log(1.0 - p)
    res = []
    for seed in range(16):
        count["nan"] = count["rows"] = 0
        s = native.Sampler(_callback_spec(inner, fn), 200, seed=seed, stepout_spec=1, shrink_spec=1)
        s.run(10)
        st = s.stats()
        assert st["nan_logL"] == count["nan"] and count["nan"] > 0
        assert st["evals"] == count["rows"]
        d = s.dead()
        assert np.all(np.isfinite(d["logL"][np.isfinite(d["logL"])]))
        # no point of the NaN or -inf regions survives past the first deaths
        live = s.live()
        assert np.all(live["u"][:, 0] <= 0.92) and np.all(live["u"][:, 1] >= 0.07)
        res.append(s.logZ())
        s.close()
    z = np.array([x[0] for x in res])
    sem = z.std(ddof=1) / math.sqrt(z.size)
    print(f"NaN/-inf regions: log Z {z.mean():.4f} +- {sem:.4f}, truth {truth:.5f}, plateau {plateau:.4f}")
    assert abs(z.mean() - (truth + plateau)) < 3.0 * sem + 0.01, (z.mean(), truth, sem)


def test_callback_failure_stops_with_einval():
    inner = W.likelihood(1)
    state = {"k": 0}

    def fn(theta):
        state["k"] += 1
        if state["k"] > 3:
            raise RuntimeError("likelihood unavailable")
        return oracle.loglike(inner, theta)

    s = native.Sampler(_callback_spec(inner, fn), 100, seed=0)
    with pytest.raises(native.NsError, match="NS_EINVAL.*callback"):
        s.run(5)


def test_coincident_live_points_match_oracle():
    spec = W.likelihood(1)
    N, m = 200, 10
    rng = np.random.default_rng(4)
    u = rng.uniform(0.2, 0.8, size=(N, 2))
    u[:120] = [0.5625, 0.46875]              # 120 identical points (dyadic: their mean is exact),
    #                                          a cluster with a zero covariance
    logL = oracle.loglike(spec, u)
    lab = np.zeros(N, dtype=np.int32)
    kw = dict(seed=2, tree_depth=1, recluster_every=1)
    s = native.Sampler(spec, N, **kw)
    o = oracle.Oracle(spec, N, **kw)
    s.set_live(u=u, logL=logL, label=lab)
    o.set_live(u=u, logL=logL, label=lab)
    for _ in range(30):
        s.step(m)
        o.step(m)
    g, r = s.dead(), o.dead()
    assert _close(g["logL"], r["logL"], 1e-12)
    assert np.allclose(g["u"], r["u"], rtol=0, atol=1e-12)
    t = s.tree()
    tr = o.tree()
    assert np.array_equal(t["count"], tr["count"]) and np.array_equal(t["accepted"], tr["accepted"])
    assert np.all(np.isfinite(t["chol"])) and np.all(np.isfinite(g["logL"]))
    st, oc = s.stats(), o.counters()
    assert st["evals"] == oc["evals"] and st["stepout_caps"] == oc["stepout_caps"]
