"""EpipolarLoss: the epipolar-adjustment objective as a torch.autograd.Function.

forward(a6, t, logf) returns the IRLS objective of the context's current
round at those parameters; backward runs the library's hand-written adjoint
(the forward is recomputed; no per-match tensor is kept), so a torch
optimiser can drive the solve.  Parameters are float64 CUDA tensors in the
context's gauge: a6 [N,6] 6D rotations, t [N,3] translations, logf [G] log
focal length per intrinsics group.  The torch stream is synchronised with the
library's stream around each call.
"""
from __future__ import annotations

import torch

from . import fastea


class EpipolarLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a6, t, logf, fctx: fastea.Context):
        for x in (a6, t, logf):
            if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
                raise ValueError("parameters must be contiguous float64 CUDA tensors")
        out = torch.empty(1, dtype=torch.float64, device=a6.device)
        torch.cuda.current_stream().synchronize()
        fctx.loss_dev(a6, t, logf, out)
        fctx.synchronize()
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
        torch.cuda.current_stream().synchronize()
        fctx.adjoint_dev(a6, t, logf, g, ga6, gt, glogf)
        fctx.synchronize()
        return ga6, gt, glogf, None


def epipolar_loss(a6, t, logf, fctx):
    return EpipolarLoss.apply(a6, t, logf, fctx)
