"""The hidden-layer tanh of the network kernels, read through ns_mlp_forward.

A 1-1-1 network with unit weights and zero biases hands every input to the
activation unchanged (d_Z returns the pre-activation the kernel used) and
returns tanh of it in d_H, so the kernels' FP32 tanh (the device math
library's tanhf) is compared here with FP64 tanh (numpy) input by input:
every FP32 value in [0.5, 1.25), where tanhf changes formula (at 0.625) and
its error peaks (1.41 ulp over all FP32 inputs), a stride through all values
up to 10, their negatives (tanh is odd, bit for bit) and the special values.
The layers' error bounds elsewhere take tanh to within 2 ulp; this pins the
function at 1.5 ulp.
"""
import numpy as np
import pytest
import torch

from paper_2608_28514_amd import native

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _inputs():
    dense = np.arange(0x3F000000, 0x3FA00000, dtype=np.uint32)        # [0.5, 1.25)
    stride = np.arange(0, 0x41200000, 97, dtype=np.uint32)             # [0, 10)
    pos = np.concatenate([dense, stride]).view(np.float32)
    special = np.array([0.0, 1e-40, 1e-30, 2.0 ** -12, 0.9, np.nextafter(np.float32(0.9), np.float32(0)),
                        9.5, 9.6, 20.0, 1e30, np.inf], dtype=np.float32)
    X = np.concatenate([pos, -pos[::7], special, -special, np.array([np.nan], np.float32)])
    return X, pos.size, special.size


def _ulp(v):
    """Spacing of FP32 numbers at |v| (that of the binade [2^e, 2^(e+1))
    holding float(|v|); subnormal spacing at the bottom)."""
    f = np.abs(v).astype(np.float32)
    m, e = np.frexp(np.maximum(f, np.float32(2.0 ** -126)).astype(np.float64))
    return np.ldexp(1.0, np.maximum(e - 24, -149))


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_hidden_tanh_within_one_and_a_half_ulp(prec):
    X, P, S = _inputs()
    B = X.size
    print(f"activation: {prec}, {B} inputs", flush=True)
    one = lambda: torch.ones((1, 1), dtype=torch.float32, device=DEV)
    zero = lambda: torch.zeros(1, dtype=torch.float32, device=DEV)
    Ws, bs = [one(), one()], [zero(), zero()]
    desc = native.mlp_desc(Ws, bs, "tanh")
    Xd = torch.tensor(X.reshape(B, 1), device=DEV)
    Yd = torch.zeros((B, 1), dtype=torch.float32, device=DEV)
    Zd = torch.zeros(2 * B, dtype=torch.float32, device=DEV)
    Hd = torch.zeros(2 * B, dtype=torch.float32, device=DEV)
    native.ns_mlp_forward(desc, prec, Xd, Yd, Zd, Hd)
    torch.cuda.synchronize()
    z = Zd[:B].cpu().numpy()
    h = Hd[:B].cpu().numpy()
    # the activation saw the input itself (the FP32 layer reproduces it; the
    # three-term split of an infinite input is NaN)
    if prec == "f32":
        assert np.array_equal(z[:-1], X[:-1])
    fin = ~np.isnan(z)
    assert fin.sum() >= B - 3
    ref = np.tanh(z[fin].astype(np.float64))
    err = np.abs(h[fin].astype(np.float64) - ref) / _ulp(ref)
    worst = int(np.argmax(err))
    print(f"{prec}: max {err.max():.4f} ulp at z = {z[fin][worst]!r}; above 1 ulp: {(err > 1).sum()}")
    assert err.max() <= 1.5
    assert np.isnan(h[~fin]).all()
    # odd, bit for bit: tanh(-z) = -tanh(z) wherever the layer passed -z on
    ip = np.arange(0, P, 7)
    ineg = P + np.arange(ip.size)
    flip = lambda a, i: a[i].view(np.uint32) ^ np.uint32(0x80000000)
    same = z[ineg].view(np.uint32) == flip(z, ip)
    assert same.mean() > 0.99
    assert np.array_equal(h[ineg][same].view(np.uint32), flip(h, ip)[same])
    sp, sn = np.arange(B - 1 - 2 * S, B - 1 - S), np.arange(B - 1 - S, B - 1)
    ok = fin[sp] & fin[sn] & (z[sn].view(np.uint32) == flip(z, sp))
    assert np.array_equal(h[sn][ok].view(np.uint32), flip(h, sp)[ok])
    assert h[sp][0] == 0.0    # (the +0 bias turns a -0 input into +0 before the activation)
    if prec == "f32":
        assert h[sp][-1] == 1.0 and h[sn][-1] == -1.0
