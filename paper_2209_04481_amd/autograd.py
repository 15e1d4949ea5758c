"""torch.autograd binding of the residual: R = R(U, b) with U the state
(9, ncells) and b the inner-boundary B_r map (6N^2), both float64 CUDA.

    R = MHDResidual.apply(U, br, context)

backward returns (J_U^T g, J_b^T g) through the library's hand-written
adjoint (cfv_vjp); forward-mode AD (torch.func.jvp, torch.autograd.forward_ad)
uses the library's exact linearisation (cfv_jvp).  Every evaluation runs in
the HIP library; the wrapper only moves tensors.  The context holds one B_r
map at a time, so each call sets it from `br` before launching.  Derivatives
are first order only.
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from .binding import Context


def _plain(t):
    """The contiguous tensor under any torch.func wrappers.  The library needs
    storage, so its calls run on these with torch.func dispatch disabled
    (inside a transform, tensors created or computed would be wrapped again)."""
    if t is None:
        return None
    t = t.detach().contiguous()
    f = torch._C._functorch
    while f.is_functorch_wrapped_tensor(t):
        t = f.get_unwrapped(t)
    return t


class MHDResidual(torch.autograd.Function):
    @staticmethod
    def forward(U: torch.Tensor, br: torch.Tensor, context: Context) -> torch.Tensor:
        U, br = _plain(U), _plain(br)
        with torch._C._DisableFuncTorch():
            context.set_inner_br(br)
            return context.residual(U)

    @staticmethod
    def setup_context(ctx, inputs, output):
        U, br, context = inputs
        ctx.context = context
        ctx.save_for_backward(U, br)
        ctx.save_for_forward(U, br)

    @staticmethod
    @once_differentiable
    def backward(ctx, gR):
        U, br = (_plain(t) for t in ctx.saved_tensors)
        gR = _plain(gR)
        context = ctx.context
        want_U, want_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (want_U or want_b):
            return None, None, None
        with torch._C._DisableFuncTorch():
            context.set_inner_br(br)
            gU, gbr = context.vjp(U, gR, want_br=want_b)
        return (gU if want_U else None), (gbr if want_b else None), None

    @staticmethod
    def jvp(ctx, dU, dbr, _):
        U, br = (_plain(t) for t in ctx.saved_tensors)
        dU, dbr = _plain(dU), _plain(dbr)
        context = ctx.context
        with torch._C._DisableFuncTorch():
            if dU is None:
                dU = torch.zeros_like(U)
            context.set_inner_br(br)
            return context.jvp(U, dU, dbr=dbr)


def residual(U: torch.Tensor, br: torch.Tensor, context: Context) -> torch.Tensor:
    """R(U, br) with autograd support (see MHDResidual)."""
    return MHDResidual.apply(U, br, context)
