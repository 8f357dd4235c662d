"""Pins of the batch corrections (Sec. 3.1, Algorithms 1 and 2): the
hand-worked examples in tests/golden, the m = 1 reduction and the order
invariants."""
import os
import numpy as np
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
T = 8


def _golden():
    out = {}
    with open(os.path.join(HERE, "golden", "alg_worked_examples.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            out[k] = [float(x) for x in v]
    return out


def _hist(m, cols):
    H = np.full((T, m), -np.inf)
    n = np.zeros(m, dtype=np.int32)
    for j, h in cols.items():
        H[:len(h) - 0, j][:len(h)] = h
        n[j] = len(h)
        H[T - 1, j] = h[-1]
    return H, n


def test_algorithm1_worked_example():
    g = _golden()
    live = np.array([5.0, 1.0, 7.0, 3.0, 9.0, 2.0])
    order = oracle.select(live)
    W = live[order[:2]]
    assert list(order[:2]) == [1, 5]
    H, n = _hist(2, {0: [1.5], 1: [4.0]})
    r = oracle.correct(2, "sort", 1, T, W, [1.5, 4.0], W, H, n)
    assert list(r["rej_logL"]) == g["alg1_dead"]
    assert list(r["acc_logL"]) == g["alg1_live"]
    # 2 is the revived worst point (code 1), 4 the new point of chain 1
    assert list(r["acc_code"]) == [1, 3]
    assert list(r["rej_code"]) == [0, 2]


def test_algorithm2_worked_example():
    g = _golden()
    W = np.array([1.0, 2.0])
    H, n = _hist(2, {0: [1.5], 1: [0.5, 1.8, 4.0]})
    r = oracle.correct(2, "history", 1, T, W, [1.5, 4.0], W, H, n)
    assert list(r["rej_logL"]) == g["alg2_dead"]
    assert list(r["acc_logL"]) == g["alg2_live"]
    # the relaxed point is chain 1's history slot 1
    assert list(r["acc_code"]) == [3, 1] and r["acc_hslot"][0] == 1
    # a second history iteration changes nothing (J_F is empty)
    r2 = oracle.correct(2, "history", 2, T, W, [1.5, 4.0], W, H, n)
    for k in r:
        assert np.array_equal(r[k], r2[k])


def test_m1_all_corrections_identical():
    H, n = _hist(1, {0: [0.1, 0.7, 3.0]})
    outs = [oracle.correct(1, c, 1, T, [0.5], [3.0], [0.5], H, n)
            for c in ("none", "best_of_worst", "sort", "history")]
    for o in outs[1:]:
        assert o["rej_logL"][0] == outs[0]["rej_logL"][0] == 0.5
        assert o["acc_logL"][0] == outs[0]["acc_logL"][0] == 3.0


def test_sort_invariants_random():
    rng = np.random.default_rng(0)
    for trial in range(200):
        m = int(rng.integers(1, 12))
        W = np.sort(rng.normal(size=m))
        newL = W + np.abs(rng.normal(size=m)) + 1e-9        # every new point beats its threshold
        cols = {}
        for j in range(m):
            k = int(rng.integers(1, T))
            h = np.sort(rng.normal(size=k))
            h[-1] = newL[j]
            h[:-1] = np.minimum(h[:-1], W[j])               # rejected proposals lie below the threshold
            cols[j] = list(rng.permutation(h[:-1])) + [newL[j]]
        H, n = _hist(m, cols)
        for corr in ("sort", "history"):
            for K in (1, 2, 10):
                r = oracle.correct(m, corr, K, T, W, newL, W, H, n)
                assert r["rej_logL"].max() <= r["acc_logL"].min()
                assert np.all(np.diff(r["rej_logL"]) >= 0) and np.all(np.diff(r["acc_logL"]) >= 0)
                # every worst point is either dead or revived, exactly once
                codes = np.concatenate([r["rej_code"], r["acc_code"]])
                assert sorted(codes[codes < m]) == list(range(m))
