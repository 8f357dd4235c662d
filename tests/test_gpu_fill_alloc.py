"""No run reads device memory it has not written.

With NS_FILL_ALLOC=255 every buffer a context allocates starts as 0xFF bytes
(NaN, -1) instead of whatever the allocator hands out; each execution path
must then give the run it gives on zeroed memory, bit for bit: the fused slice
kernel (10-d Rosenbrock of Eq. (6), FP64 likelihood, FP32 state, depth-2
trees), the batched rounds (the 49-Gaussian array of Eq. (2), FP32) and the
chain kernel with FP32 layers (a small emulator).  The split-bfloat16 chain
kernel and the emulator rounds are covered in test_gpu_emu_chains.py.
"""
import numpy as np
import pytest

from paper_2608_28514_amd import native, workloads as W

pytestmark = pytest.mark.gpu

CASES = [
    ("rosenbrock10d_fused", lambda: W.likelihood(2), 500, 50, dict(prec="f64", state="f32", tree_depth=2), 40),
    ("array49_rounds", lambda: W.likelihood(3, seed=0), 1000, 100,
     dict(prec="f32", state="f32", tree_depth=3, batch_rounds=1), 20),
    ("emulator6d_fp32_chains", lambda: W.emulator(seed=3, widths=(6, 256, 256, 512), noise_frac=0.05), 200, 20,
     dict(prec="f32", state="f32", tree_depth=1), 30),
]


def _run(spec, N, m, kw, steps):
    s = native.Sampler(spec, N, seed=5, **kw)
    s.run(m, max_steps=steps)
    out = (s.dead(), s.live(), s.stats())
    s.close()
    return out


@pytest.mark.parametrize("name,make,N,m,kw,steps", CASES, ids=[c[0] for c in CASES])
def test_filled_allocations_give_the_same_run(monkeypatch, name, make, N, m, kw, steps):
    spec = make()
    print(f"fill alloc: {name}", flush=True)
    da, la, sa = _run(spec, N, m, kw, steps)
    monkeypatch.setenv("NS_FILL_ALLOC", "255")
    db, lb, sb = _run(spec, N, m, kw, steps)
    assert sa["steps"] == steps and sb["steps"] == steps
    assert np.array_equal(da["logL"], db["logL"]) and np.array_equal(da["u"], db["u"])
    assert np.array_equal(la["u"], lb["u"]) and np.array_equal(la["logL"], lb["logL"])
    assert np.array_equal(la["label"], lb["label"])
    for k in ("evals", "dead", "clusterings"):
        assert sa[k] == sb[k], k
