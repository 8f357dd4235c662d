"""Worst-m selection at scale (ns_select_worst): the first m of a stable sort
of (canon(logL), index), bit for bit, against numpy's lexsort on the same
keys, for sizes around the single-pass limit (8192), ties resolved through
the index digits, and the special values (NaN -> -inf, -0 = +0, +-inf)."""
import numpy as np
import pytest
import torch

from paper_2608_28514_amd import native

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _expected(x, m):
    c = np.where(np.isnan(x), -np.inf, x)
    c = np.where(c == 0.0, 0.0, c)
    return np.lexsort((np.arange(len(x)), c))[:m]


def _data(kind, N, rng):
    if kind == "normal":
        return rng.normal(-100.0, 30.0, N)
    if kind == "ties":
        return np.round(rng.normal(-10.0, 3.0, N))
    if kind == "narrow":
        return rng.uniform(-2.0, -1.0, N)
    if kind == "constant":
        return np.full(N, -7.25)
    if kind == "special":
        x = rng.normal(0.0, 1.0, N)
        pick = rng.integers(0, 6, N)
        x[pick == 0] = np.nan
        x[pick == 1] = -0.0
        x[pick == 2] = 0.0
        x[pick == 3] = -np.inf
        x[pick == 4] = np.inf
        return x
    raise ValueError(kind)


def _run(x, m):
    work = torch.empty(native.ns_select_worst_work_bytes(), dtype=torch.uint8, device=DEV)
    d_x = torch.tensor(x, dtype=torch.float64, device=DEV)
    d_s = torch.full((m,), -1, dtype=torch.int32, device=DEV)
    d_p = torch.zeros(1, dtype=torch.int32, device=DEV)
    native.ns_select_worst(d_x, m, d_s, work, d_p)
    torch.cuda.synchronize()
    return d_s.cpu().numpy(), int(d_p.item())


@pytest.mark.parametrize("kind", ["normal", "ties", "narrow", "constant", "special"])
@pytest.mark.parametrize("N", [1, 5, 8192, 8193, 50000, (1 << 20) + 3])
def test_select_worst_matches_stable_sort(kind, N):
    rng = np.random.default_rng(N + len(kind))
    x = _data(kind, N, rng)
    for m in sorted({1, min(N, 7), min(N, 1000), min(N, 4096)}):
        got, passes = _run(x, m)
        exp = _expected(x, m)
        assert np.array_equal(got, exp), (kind, N, m)
        if N <= 8192:
            assert passes == 1
        else:
            assert 2 <= passes <= 10


def test_select_worst_rejects_bad_arguments():
    x = torch.zeros(100, dtype=torch.float64, device=DEV)
    s = torch.zeros(10, dtype=torch.int32, device=DEV)
    work = torch.empty(native.ns_select_worst_work_bytes(), dtype=torch.uint8, device=DEV)
    for m in (0, 4097, 101):
        with pytest.raises(native.NsError):
            native.ns_select_worst(x, m, s, work)
    with pytest.raises(native.NsError):
        native.ns_select_worst(x[1:], 5, s, work)   # 8-byte offset: not 16-byte aligned
