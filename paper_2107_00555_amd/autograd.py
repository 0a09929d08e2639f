"""RD3D: T fused reaction-diffusion steps as a torch.autograd.Function.

forward runs dcp_run with checkpoints every k steps; backward runs
dcp_adjoint_run, which recomputes each segment from its checkpoint and
applies the hand-written adjoint kernel.  Gradients are returned for u0,
alpha and beta; gamma, f, dt, h, T, the boundary and k get None.
"""
from __future__ import annotations

import torch

from . import api


def _scalar(x) -> float:
    return float(x.detach().item()) if isinstance(x, torch.Tensor) else float(x)


class RD3D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, f, alpha, beta, gamma, dt, h, T, bc, ckpt_every, tblock=2):
        coeffs = dict(alpha=_scalar(alpha), beta=_scalar(beta), gamma=_scalar(gamma),
                      h=float(h), dt=float(dt))
        k = max(1, int(ckpt_every))
        u = u0.detach().contiguous().clone()
        out = api.run(u, f.detach().contiguous(), coeffs, int(T), bc, tblock=int(tblock), norms=False,
                      ckpt_every=k)
        ctx.tblock = int(tblock)
        ctx.coeffs = coeffs
        ctx.T, ctx.bc, ctx.k = int(T), bc, k
        ctx.ckpt = out["ckpt"]
        ctx.f = f.detach().contiguous()
        ctx.alpha_is_tensor = isinstance(alpha, torch.Tensor)
        ctx.beta_is_tensor = isinstance(beta, torch.Tensor)
        ctx.alpha_meta = (alpha.dtype, alpha.device, alpha.shape) if ctx.alpha_is_tensor else None
        ctx.beta_meta = (beta.dtype, beta.device, beta.shape) if ctx.beta_is_tensor else None
        return u

    @staticmethod
    def backward(ctx, grad_uT):
        g, gab = api.adjoint_run(ctx.ckpt, ctx.k, ctx.f, grad_uT.contiguous(), ctx.coeffs,
                                 ctx.T, ctx.bc, tblock=ctx.tblock)
        ga = gb = None
        if ctx.needs_input_grad[2] and ctx.alpha_is_tensor:
            dtype, device, shape = ctx.alpha_meta
            ga = gab[0].to(dtype=dtype, device=device).reshape(shape)
        if ctx.needs_input_grad[3] and ctx.beta_is_tensor:
            dtype, device, shape = ctx.beta_meta
            gb = gab[1].to(dtype=dtype, device=device).reshape(shape)
        gu = g if ctx.needs_input_grad[0] else None
        return gu, None, ga, gb, None, None, None, None, None, None, None


def rd3d(u0, f, alpha, beta, gamma, dt, h, T, bc, ckpt_every=10, tblock=2):
    """u_T after T fused steps from u0, differentiable in u0, alpha and beta."""
    return RD3D.apply(u0, f, alpha, beta, gamma, dt, h, T, bc, ckpt_every, tblock)
