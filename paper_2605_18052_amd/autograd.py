"""EpipolarLoss: the epipolar-adjustment objective as a torch.autograd.Function.

forward(a6, t, logf) returns the IRLS objective of the context's current
round at those parameters; backward runs the library's hand-written adjoint
(the forward is recomputed; no per-match tensor is kept), so a torch
optimiser can drive the solve.  Parameters are float64 CUDA tensors in the
context's gauge: a6 [N,6] 6D rotations, t [N,3] translations, logf [G] log
focal length per intrinsics group.

Ordering: the library's work is queued behind everything already issued on
torch's current stream, and torch's current stream waits for the library's
work, both through device-side events; the host never waits.  Since torch's
stream waits right after each call, memory that torch later frees and hands
out again (on that stream) is reused only after the library's work: the
tensors are not marked as used on the library's stream, whose lifetime is
the context's and may end before theirs.
"""
from __future__ import annotations

import torch

from . import fastea


def _enter(fctx: fastea.Context, device):
    """(library stream, torch's current stream, whether they differ); the
    library's stream waits for torch's current one."""
    cur = torch.cuda.current_stream(device)
    lib = fctx.torch_stream()
    other = lib.cuda_stream != cur.cuda_stream
    if other:
        lib.wait_stream(cur)
    return lib, cur, other


def _leave(lib, cur, other):
    if other:
        cur.wait_stream(lib)


class EpipolarLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a6, t, logf, fctx: fastea.Context):
        for x in (a6, t, logf):
            if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
                raise ValueError("parameters must be contiguous float64 CUDA tensors")
        out = torch.empty(1, dtype=torch.float64, device=a6.device)
        lib, cur, other = _enter(fctx, a6.device)
        fctx.loss_dev(a6, t, logf, out)
        _leave(lib, cur, other)
        ctx.save_for_backward(a6, t, logf)
        ctx.fctx = fctx
        return out[0]

    @staticmethod
    def backward(ctx, gout):
        a6, t, logf = ctx.saved_tensors
        fctx = ctx.fctx
        g = gout.reshape(1).to(torch.float64).contiguous()
        ga6 = torch.empty_like(a6) if ctx.needs_input_grad[0] else None
        gt = torch.empty_like(t) if ctx.needs_input_grad[1] else None
        glogf = torch.empty_like(logf) if ctx.needs_input_grad[2] else None
        lib, cur, other = _enter(fctx, a6.device)
        fctx.adjoint_dev(a6, t, logf, g, ga6, gt, glogf)
        _leave(lib, cur, other)
        return ga6, gt, glogf, None


def epipolar_loss(a6, t, logf, fctx):
    return EpipolarLoss.apply(a6, t, logf, fctx)
