"""Pins of the oracle's selection (Algorithm 1 'sorted') and clustering
(Sec. 2.1): library sorts and decompositions, brute force, special cases."""
import itertools
import numpy as np
import oracle


def _ref_order(x):
    x = np.where(np.isnan(x), -np.inf, x)
    x = np.where(x == 0.0, 0.0, x)          # -0 -> +0
    return np.lexsort((np.arange(x.size), x))


def test_select_random_and_special_keys():
    rng = np.random.default_rng(0)
    for N in (2, 7, 100, 513, 4000):
        x = rng.normal(size=N)
        assert np.array_equal(oracle.select(x), _ref_order(x))
        y = np.round(rng.normal(size=N), 1)          # many ties
        y[rng.integers(0, N, N // 10)] = -0.0
        y[rng.integers(0, N, N // 20)] = np.nan
        y[rng.integers(0, N, N // 20)] = np.inf
        y[rng.integers(0, N, N // 20)] = -np.inf
        assert np.array_equal(oracle.select(y), _ref_order(y))


def test_jacobi_against_eigh_and_reconstruction():
    rng = np.random.default_rng(1)
    for d in (1, 2, 5, 10, 27, 32):
        A = rng.normal(size=(d, d))
        A = A @ A.T + 0.1 * np.eye(d)
        ev, Q = oracle.jacobi_eig(A)
        assert np.allclose(np.sort(ev), np.linalg.eigvalsh(A), rtol=1e-12, atol=1e-12 * np.abs(ev).max())
        assert np.allclose(Q @ np.diag(ev) @ Q.T, A, atol=1e-12 * np.abs(A).max())
        assert np.allclose(Q.T @ Q, np.eye(d), atol=1e-13)


def test_cholesky_against_numpy():
    rng = np.random.default_rng(2)
    for d in (1, 3, 27):
        A = rng.normal(size=(d, d))
        A = A @ A.T + np.eye(d)
        rc, L = oracle.cholesky(A)
        assert rc == 0
        assert np.allclose(L, np.linalg.cholesky(A), rtol=1e-12, atol=1e-13)
    rc, _ = oracle.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert rc != 0


def test_regularise_pd_unchanged_and_rank_deficient_clipped():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(6, 6))
    A = A @ A.T + np.eye(6)
    logV, L, clipped = oracle.regularise(A)
    assert not clipped
    assert np.allclose(L @ L.T, A, rtol=1e-12, atol=1e-12)
    assert abs(logV - 0.5 * np.linalg.slogdet(A)[1]) < 1e-12
    X = rng.normal(size=(3, 6))                      # 3 points in 6-d: rank 2
    S = np.cov(X.T)
    logV, L, clipped = oracle.regularise(S, eps=1e-8)
    assert clipped
    ev = np.linalg.eigvalsh(L @ L.T)
    assert abs(ev.min() / ev.max() - 1e-8) < 1e-9


def _sse(X, lab):
    return sum(((X[lab == c] - X[lab == c].mean(0)) ** 2).sum() for c in (0, 1) if np.any(lab == c))


def test_two_means_matches_brute_force_on_separated_blobs():
    rng = np.random.default_rng(4)
    for trial in range(5):
        d = 3
        X = np.concatenate([rng.normal(0.3, 0.02, size=(6, d)), rng.normal(0.7, 0.02, size=(7, d))])
        tree, labels = oracle.cluster(X, depth=1, nmin=2)
        best = min(_sse(X, np.array(bits)) for bits in itertools.product((0, 1), repeat=len(X)))
        # partition induced by the first split
        assert tree["count"][1] + tree["count"][2] == len(X)
        lab = np.array([0] * 6 + [1] * 7)
        assert abs(_sse(X, lab) - best) < 1e-15
        assert sorted([tree["count"][1], tree["count"][2]]) == [6, 7]
        assert tree["split_ok"][0] == 1
        assert set(labels[:6]) != set(labels[6:])


def test_no_split_of_one_gaussian_or_uniform_box():
    rng = np.random.default_rng(5)
    for X in (np.clip(rng.normal(0.5, 0.1, size=(2000, 3)), 0, 1), rng.uniform(size=(2000, 3))):
        tree, labels = oracle.cluster(X, depth=2)
        assert tree["accepted"][0] == 1 and tree["accepted"].sum() == 1
        assert np.all(labels == 0)


def test_four_separated_modes_give_four_clusters():
    rng = np.random.default_rng(6)
    cen = np.array([[0.2, 0.2], [0.8, 0.2], [0.2, 0.8], [0.8, 0.8]])
    X = np.concatenate([rng.normal(c, 0.03, size=(250, 2)) for c in cen])
    tree, labels = oracle.cluster(X, depth=3)
    assert tree["accepted"].sum() == 4
    for k in range(4):
        assert len(set(labels[250 * k:250 * (k + 1)])) == 1
    assert len(set(labels)) == 4
    # covariance of each cluster is the sample covariance of its points
    for k in range(4):
        n = labels[250 * k]
        S = np.cov(X[labels == n].T)
        Lc = tree["chol"][n]
        assert np.allclose(Lc @ Lc.T, S, rtol=1e-10, atol=1e-14)
        assert np.allclose(tree["centre"][n], X[labels == n].mean(0), atol=1e-14)


def test_two_means_split_of_separated_blobs():
    """The node split alone (oracle.two_means): two well separated blobs are
    recovered exactly, the first centre is the blob of the point farthest from
    the mean, and the centres are the blob means."""
    rng = np.random.default_rng(21)
    a = rng.normal(0.25, 0.03, (70, 4))
    b = rng.normal(0.75, 0.03, (50, 4))
    u = np.concatenate([a, b])
    mu = u.mean(axis=0)
    first = int(np.argmax(((u - mu) ** 2).sum(axis=1)))
    ca, cb, side = oracle.two_means(u, 20)
    truth = np.r_[np.zeros(70, dtype=int), np.ones(50, dtype=int)]
    if truth[first] == 1:
        truth = 1 - truth
    assert np.array_equal(side, truth)
    assert np.allclose(ca, u[side == 0].mean(axis=0), rtol=0, atol=1e-12)
    assert np.allclose(cb, u[side == 1].mean(axis=0), rtol=0, atol=1e-12)
