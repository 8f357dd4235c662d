"""The learned pre-screen: the autograd wrapper of the hand-written network
kernels (finite differences and the FP64 oracle backward), on-device training
(loss falls), and the screened sampler against the plain one: equal log Z
within the combined sigma, fewer true-likelihood network rows, audited
false-screen rate within its bound."""
import math
import numpy as np
import pytest
import torch

import oracle
from paper_2608_28514_amd import native, mlp, workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_mlp_function_matches_oracle_gradients():
    torch.manual_seed(0)
    net = mlp.MLP([27, 64, 64, 1], act="silu", prec="f32", device=DEV, seed=3)
    X = torch.rand(257, 27, device=DEV)
    y = torch.randn(257, 1, device=DEV)
    out = net(X)
    loss = ((out - y) ** 2).mean()
    loss.backward()
    Ws = [w.detach().double().cpu().numpy() for w in net.W]
    bs = [b.detach().double().cpu().numpy() for b in net.b]
    Xn = X.double().cpu().numpy()
    Yr, acts = oracle.mlp_forward([27, 64, 64, 1], Ws, bs, 1, Xn)
    dY = 2.0 * (Yr - y.double().cpu().numpy()) / Yr.size
    dWr, dbr, _ = oracle.mlp_backward([27, 64, 64, 1], Ws, bs, 1, Xn, acts, dY)
    assert np.allclose(out.detach().cpu().numpy(), Yr, rtol=1e-4, atol=1e-5)
    for l in range(3):
        g = net.W[l].grad.cpu().numpy()
        assert np.max(np.abs(g - dWr[l])) <= 1e-4 * max(1e-3, np.max(np.abs(dWr[l]))), l
        g = net.b[l].grad.cpu().numpy()
        assert np.max(np.abs(g - dbr[l])) <= 1e-4 * max(1e-3, np.max(np.abs(dbr[l]))), l


def test_mlp_function_finite_differences():
    net = mlp.MLP([5, 16, 16, 1], act="silu", prec="f32", device=DEV, seed=1)
    X = torch.rand(64, 5, device=DEV, requires_grad=True)
    out = net(X).sum()
    out.backward()
    g = X.grad.detach().cpu().numpy()
    h = 1e-2
    Xd = X.detach()
    for (r, c) in [(0, 0), (5, 3), (63, 4)]:
        Xp, Xm = Xd.clone(), Xd.clone()
        Xp[r, c] += h
        Xm[r, c] -= h
        with torch.no_grad():
            fd = (net(Xp).sum() - net(Xm).sum()).item() / (2 * h)
        assert abs(fd - g[r, c]) <= 2e-3 * max(1.0, abs(fd))


def _small_emulator():
    return W.emulator(seed=3, widths=(5, 32, 32, 32, 16), noise_frac=0.05)


def _dirty_device_memory(mib=512):
    """Fill a block of device memory with NaN and hand it back to the driver,
    so that buffers allocated next are likely to start as NaN: a kernel that
    reads a slot nobody wrote then shows up as a non-finite result."""
    x = torch.full((mib << 18,), float("nan"), dtype=torch.float32, device=DEV)
    torch.cuda.synchronize()
    del x
    torch.cuda.empty_cache()


def test_screened_sampler_matches_plain_and_saves_evaluations():
    """32 screened and 32 plain runs of a small emulator: mean log Z within 3
    combined standard errors, fewer network rows with the screen, audits
    within their bound."""
    spec = _small_emulator()
    S = 32
    plain, scr = [], []
    rows_plain = rows_scr = 0
    for seed in range(S):
        if seed < 3:
            _dirty_device_memory()
        s = native.Sampler(spec, 200, prec="f32", state="f32", seed=seed, tree_depth=1)
        s.run(20)
        plain.append(s.logZ()[0])
        rows_plain += s.stats()["net_rows"]
        s.close()
        if seed < 3:
            _dirty_device_memory()
        t = native.Sampler(spec, 200, prec="f32", state="f32", seed=seed, tree_depth=1)
        t.enable_surrogate(hidden=64, batch=512, train_iters=10, min_pairs=4096, replay_cap=32768,
                           margin=3.0, floor_below=20.0, prec="f32")
        t.run(20)
        scr.append(t.logZ()[0])
        rows_scr += t.stats()["net_rows"]
        st = t.surrogate_stats()
        t.close()
        assert st["train_calls"] > 0 and st["pairs"] > 4096
        assert st["screened"] > 0 and st["audited"] > 0
        assert st["false_screens"] <= 0.05 * st["audited"] + 2
    plain, scr = np.array(plain), np.array(scr)
    sem = math.sqrt(plain.var(ddof=1) / S + scr.var(ddof=1) / S)
    print(f"logZ plain {plain.mean():.4f}, screened {scr.mean():.4f}, 3 SEM {3 * sem:.4f}; "
          f"network rows plain {rows_plain}, screened {rows_scr}")
    assert abs(plain.mean() - scr.mean()) < 3.0 * sem
    assert rows_scr < rows_plain


def test_surrogate_training_reduces_loss_and_predicts():
    spec = _small_emulator()
    t = native.Sampler(spec, 200, prec="f32", state="f32", seed=5, tree_depth=1)
    t.enable_surrogate(hidden=64, batch=512, train_iters=10, min_pairs=2048, replay_cap=32768,
                       margin=3.0, floor_below=20.0, prec="bf16")
    losses = []
    for _ in range(40):
        t.step(20)
        losses.append(t.surrogate_stats()["last_loss"])
    print("losses", losses[:3], losses[-3:], t.surrogate_stats())
    tr = [l for l in losses if l > 0]
    # the estimate tracks the true likelihood of live points near the contour
    live = t.live()
    u = torch.tensor(live["u"], dtype=torch.float32, device=DEV)
    out = torch.zeros(len(u), dtype=torch.float32, device=DEV)
    native.ns_surrogate_predict(t.ctx, u, out)
    native.ns_sync(t.ctx)
    est = out.cpu().numpy()
    err = est - live["logL"]
    print("surrogate err on live points: median", np.median(err), "abs median", np.median(np.abs(err)),
          "live logL range", live["logL"].min(), live["logL"].max())
    assert len(tr) > 10
    assert np.mean(tr[-5:]) < np.mean(tr[:5])
    # early in a run the live logL still spans a wide range; the estimate is
    # judged relative to it (the screen itself only switches on once the
    # minibatch error in nats is below half the margin)
    span = live["logL"].max() - live["logL"].min()
    assert np.median(np.abs(err)) < 0.25 * span


def test_surrogate_enabled_mid_run_trains_on_written_pairs_only():
    """Rows evaluated before the surrogate exists are not in the replay ring:
    the ring count starts at zero when it is enabled, and training on it
    stays finite even when its memory starts as NaN."""
    spec = _small_emulator()
    _dirty_device_memory()
    t = native.Sampler(spec, 200, prec="f32", state="f32", seed=11, tree_depth=1)
    t.step(20)
    t.step(20)
    rows_before = t.stats()["net_rows"]
    assert rows_before > 0
    _dirty_device_memory()
    t.enable_surrogate(hidden=32, batch=256, train_iters=4, min_pairs=1024, replay_cap=8192,
                       margin=3.0, floor_below=20.0, prec="f32")
    assert t.surrogate_stats()["pairs"] == 0
    for _ in range(6):
        t.step(20)
    st = t.surrogate_stats()
    print("mid-run surrogate:", st, "rows before", rows_before)
    assert st["train_calls"] > 0
    assert math.isfinite(st["last_loss"])
    assert st["pairs"] == t.stats()["net_rows"] - rows_before
