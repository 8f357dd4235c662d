"""Dense networks on the hand-written HIP kernels, for PyTorch users.

``MLPFunction`` is a ``torch.autograd.Function`` whose forward and backward
call ``ns_mlp_forward`` / ``ns_mlp_backward`` of libns.so (MFMA or FP32 FMA
GEMMs with fused bias and activation; the backward pass computes dW = H^T dZ,
db = column sums of dZ and dX = dZ W^T with the same kernels).  ``MLP`` wraps
the weights of such a network as ``torch.nn.Parameter``s.  This is the network
the sampler's learned pre-screen uses (SiLU hidden layers, linear output);
the sampler trains its own copy on the device, and this module exposes the
same kernels for training from PyTorch.
"""
import math
import torch

from . import native


class MLPFunction(torch.autograd.Function):
    """y = f(x; W_0, b_0, ..., W_{L-1}, b_{L-1}) on the library's kernels."""

    @staticmethod
    def forward(ctx, X, act, prec, *params):
        Ws, bs = list(params[0::2]), list(params[1::2])
        X = X.contiguous()
        Ws = [w.contiguous() for w in Ws]
        bs = [b.contiguous() for b in bs]
        B = X.shape[0]
        widths = [X.shape[1]] + [w.shape[1] for w in Ws]
        tot = B * sum(widths[1:])
        Z = torch.empty(tot, dtype=torch.float32, device=X.device)
        H = torch.empty(tot, dtype=torch.float32, device=X.device)
        Y = torch.empty((B, widths[-1]), dtype=torch.float32, device=X.device)
        desc = native.mlp_desc(Ws, bs, act)
        native.ns_mlp_forward(desc, prec, X, Y, Z, H)
        ctx.save_for_backward(X, Z, H, *Ws, *bs)
        ctx.act, ctx.prec, ctx.L, ctx.widths = act, prec, len(Ws), widths
        return Y

    @staticmethod
    def backward(ctx, dY):
        X, Z, H, *rest = ctx.saved_tensors
        L = ctx.L
        Ws, bs = rest[:L], rest[L:]
        desc = native.mlp_desc(list(Ws), list(bs), ctx.act)
        dWs = [torch.empty_like(w) for w in Ws]
        dbs = [torch.empty_like(b) for b in bs]
        dX = torch.empty_like(X) if ctx.needs_input_grad[0] else None
        work = torch.empty(2 * X.shape[0] * max(ctx.widths), dtype=torch.float32, device=X.device)
        native.ns_mlp_backward(desc, ctx.prec, X, Z, H, dY.contiguous().float(), dWs, dbs, dX, work)
        grads = []
        for dw, db in zip(dWs, dbs):
            grads += [dw, db]
        return (dX, None, None, *grads)


class MLP(torch.nn.Module):
    """widths[0] -> ... -> widths[-1], hidden activation act ('silu' or 'tanh')."""

    def __init__(self, widths, act="silu", prec="f32", device="cuda", seed=0):
        super().__init__()
        g = torch.Generator(device="cpu").manual_seed(seed)
        self.act, self.prec = act, prec
        self.W = torch.nn.ParameterList()
        self.b = torch.nn.ParameterList()
        for l in range(len(widths) - 1):
            a = math.sqrt(6.0 / (widths[l] + widths[l + 1]))
            w = (torch.rand(widths[l], widths[l + 1], generator=g, dtype=torch.float64) * 2 - 1) * a
            self.W.append(torch.nn.Parameter(w.float().to(device)))
            self.b.append(torch.nn.Parameter(torch.zeros(widths[l + 1], device=device)))

    def forward(self, X):
        params = []
        for w, b in zip(self.W, self.b):
            params += [w, b]
        return MLPFunction.apply(X, self.act, self.prec, *params)
