"""The allocation-free selection (ns_select_worst_noalloc): the same slots as
ns_select_worst with a caller-owned workspace, bit for bit, on two calls in a
row (the second on a smaller input, so stale workspace contents from the
first call would show), and the limits of its static workspace."""
import numpy as np
import pytest
import torch

from paper_2608_28514_amd import native

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _with_workspace(x, m):
    work = torch.empty(native.ns_select_worst_work_bytes(), dtype=torch.uint8, device=DEV)
    slots = torch.full((m,), -1, dtype=torch.int32, device=DEV)
    passes = torch.zeros(1, dtype=torch.int32, device=DEV)
    native.ns_select_worst(x, m, slots, work, passes)
    torch.cuda.synchronize()
    return slots.cpu().numpy(), int(passes.item())


def _no_alloc(x, m):
    slots = torch.full((m,), -1, dtype=torch.int32, device=DEV)
    passes = torch.zeros(1, dtype=torch.int32, device=DEV)
    native.ns_select_worst_noalloc(x, m, slots, passes)
    torch.cuda.synchronize()
    return slots.cpu().numpy(), int(passes.item())


def _lexsort_first(x, m):
    c = np.where(np.isnan(x), -np.inf, x)
    c = np.where(c == 0.0, 0.0, c)
    return np.lexsort((np.arange(len(x)), c))[:m]


@pytest.mark.parametrize("sizes", [((1 << 20) + 3, 1000, 50_000, 700),
                                   (300_000, 4096, 9_000, 17),
                                   (40_000, 64, 5, 5)])
def test_noalloc_matches_workspace_entry_point_on_consecutive_calls(sizes):
    N1, m1, N2, m2 = sizes
    rng = np.random.default_rng(N1 + m1)
    x1 = np.round(rng.normal(-50.0, 20.0, N1), 2)          # ties resolved through the index
    x1[rng.integers(0, N1, N1 // 50)] = np.nan
    x2 = rng.normal(-50.0, 20.0, N2)
    x2[rng.integers(0, N2, max(1, N2 // 50))] = -0.0
    d1 = torch.tensor(x1, dtype=torch.float64, device=DEV)
    d2 = torch.tensor(x2, dtype=torch.float64, device=DEV)
    print(f"no-alloc select: N={N1}, m={m1} then N={N2}, m={m2}", flush=True)
    for x, d, m in ((x1, d1, m1), (x2, d2, m2)):
        got, gp = _no_alloc(d, m)
        ref, rp = _with_workspace(d, m)
        assert np.array_equal(got, ref)
        assert gp == rp
        assert np.array_equal(got, _lexsort_first(x, m))


def test_noalloc_rejects_sizes_beyond_its_workspace():
    x = torch.zeros(10_000, dtype=torch.float64, device=DEV)
    slots = torch.zeros(5000, dtype=torch.int32, device=DEV)
    with pytest.raises(native.NsError, match="NS_EINVAL.*4096"):
        native.ns_select_worst_noalloc(x, 4097, slots)
    with pytest.raises(native.NsError, match="NS_EINVAL"):
        native.ns_select_worst_noalloc(x[:10], 11, slots)
