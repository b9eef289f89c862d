"""torch.autograd.Function over the zoom of one LR image.

Forward: zh_query, zh_lle_weights(lambda), zh_reconstruct and one
zh_backproject in libzoomhash. Backward: zh_backward, which returns the
gradients with respect to the dictionary's HR residual patches (the tensor
the library borrowed when its tables were built) and lambda. Neighbour
indices stay discrete; the library keeps what the backward needs from the
last forward, so a backward must follow its own forward on that engine.
"""
from __future__ import annotations

import torch


class ZoomHashFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, lr, resid, lam, engine):
        if resid.data_ptr() != engine.resid.data_ptr():
            raise ValueError("resid must be the residual tensor the engine's tables were built on")
        out = engine.forward_record(lr, float(lam))
        ctx.engine = engine
        ctx.token = engine.token
        ctx.lam_dtype = lam.dtype
        return out

    @staticmethod
    def backward(ctx, g_out):
        e = ctx.engine
        if e.token != ctx.token:
            raise RuntimeError("the engine ran another forward since this one; its record is gone")
        g_resid = torch.empty_like(e.resid)
        g_lam = torch.empty(1, dtype=torch.float32, device=g_out.device)
        e.ctx.backward(g_out.contiguous(), g_resid, g_lam)
        return None, g_resid, g_lam.reshape(()).to(ctx.lam_dtype), None


def zoom(lr, resid, lam, engine):
    """Differentiable zoom: output image [s h, s w]."""
    return ZoomHashFn.apply(lr, resid, lam, engine)
