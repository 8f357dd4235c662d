"""The persistent chain kernel for network likelihoods (k_emu_chains: a
workgroup takes its chains through all their rounds and evaluates their rows
through the network itself) against the batched-rounds driver: identical
runs, bit for bit (dead points, likelihoods, history, counters), for the
27-512-512-512-1024 emulator at the benchmark's shape and at small shapes, a
batch that leaves the last workgroup partly empty, and a network with
256-wide hidden layers."""
import numpy as np
import pytest

from paper_2608_28514_amd import native, workloads as W

pytestmark = pytest.mark.gpu


def _pair(spec, N, m, steps, seed=0, **kw):
    out = []
    for fused in (1, 0):
        print(f"emu chains: fused={fused} N={N} m={m} steps={steps} widths={spec['widths']}", flush=True)
        s = native.Sampler(spec, N, prec="bf16x3", state="f32", tree_depth=1, seed=seed, fused_chains=fused, **kw)
        s.run(m, max_steps=steps)
        out.append((s.dead(), s.stats(), s.last_batch(), s.live()))
        s.close()
    return out


def _same(a, b):
    (da, sa, la, va), (db, sb, lb, vb) = a, b
    assert np.array_equal(da["logL"], db["logL"])
    assert np.array_equal(da["u"], db["u"])
    assert np.array_equal(va["u"], vb["u"]) and np.array_equal(va["logL"], vb["logL"])
    for k in ("seeds", "tau", "new_u", "new_logL", "chain_evals", "hist_n"):
        assert np.array_equal(la[k], lb[k]), k
    m = la["hist_n"].size
    for j in range(m):
        n = int(la["hist_n"][j])
        assert np.array_equal(la["hist_logL"][:n, j], lb["hist_logL"][:n, j])
        assert np.array_equal(la["hist_u"][j, :n], lb["hist_u"][j, :n])
        assert la["hist_logL"][-1, j] == lb["hist_logL"][-1, j]
    for k in ("evals", "oob", "stepout_caps", "shrink_caps", "steps", "dead", "net_rows"):
        assert sa[k] == sb[k], k


@pytest.mark.parametrize("N,m,steps", [(200, 40, 30), (300, 42, 20), (4000, 400, 6)])
def test_emulator_chains_identical_to_rounds(N, m, steps):
    spec = W.likelihood(4, seed=0)
    _same(*_pair(spec, N, m, steps))


def test_runs_do_not_read_stale_device_memory(monkeypatch):
    """Device memory that earlier work released keeps its bytes, and the
    library's allocations may receive it: no run may read a buffer it has not
    written (the plain rounds once read screen flags that only a screen pass
    writes, and rejected rows wherever a stale word was nonzero).  With
    NS_FILL_ALLOC every buffer starts as 0xFF bytes (NaN, -1): both drivers
    must still give the runs they give on zeroed memory."""
    spec = W.likelihood(4, seed=0)
    clean = _pair(spec, 200, 40, 30)
    monkeypatch.setenv("NS_FILL_ALLOC", "255")
    filled = _pair(spec, 200, 40, 30)
    _same(*filled)
    _same(clean[0], filled[0])


def test_emulator_chains_256_wide_hidden_layers():
    spec = W.emulator(seed=5, widths=(12, 256, 256, 512), noise_frac=0.02)
    _same(*_pair(spec, 300, 30, 40, seed=2))


def test_emulator_chains_complete_run_identical_to_rounds():
    spec = W.emulator(seed=3, widths=(6, 256, 256, 512), noise_frac=0.05)
    res = []
    for fused in (1, 0):
        s = native.Sampler(spec, 200, prec="bf16x3", state="f32", tree_depth=1, seed=7, fused_chains=fused)
        s.run(20)
        res.append((s.dead()["logL"], s.logZ(), s.stats()["net_rows"]))
        s.close()
    assert np.array_equal(res[0][0], res[1][0])
    assert res[0][1] == res[1][1] and res[0][2] == res[1][2]
