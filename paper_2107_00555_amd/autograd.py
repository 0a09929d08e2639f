"""RD3D: T fused reaction-diffusion steps as a torch.autograd.Function.

forward runs dcp_run with checkpoints every k steps; backward runs
dcp_adjoint_run, which recomputes each segment from its checkpoint and
applies the hand-written adjoint kernel.  With revolve_slots > 0 the
forward keeps that many snapshots instead (binomial checkpointing,
dcp_revolve_forward / dcp_revolve_adjoint): memory bounded for any T.  Gradients are returned for u0,
f, alpha, beta and gamma (the scalars when passed as tensors); dt, h, T,
the boundary and k get None.
"""
from __future__ import annotations

import torch

from . import api


def _scalar(x) -> float:
    return float(x.detach().item()) if isinstance(x, torch.Tensor) else float(x)


def _meta(x):
    return (x.dtype, x.device, x.shape) if isinstance(x, torch.Tensor) else None


def _as(meta, v: torch.Tensor) -> torch.Tensor:
    dtype, device, shape = meta
    return v.to(dtype=dtype, device=device).reshape(shape)


class RD3D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, f, alpha, beta, gamma, dt, h, T, bc, ckpt_every, tblock=3, revolve_slots=0):
        coeffs = dict(alpha=_scalar(alpha), beta=_scalar(beta), gamma=_scalar(gamma),
                      h=float(h), dt=float(dt))
        k = max(1, int(ckpt_every))
        u = u0.detach().contiguous().clone()
        ctx.slots = int(revolve_slots)
        if ctx.slots > 0:
            ctx.ckpt = api.revolve_forward(u, f.detach().contiguous(), coeffs, int(T), bc, ctx.slots,
                                           tblock=int(tblock), reserve_sum=True)
            # the reverse sweep reuses the snapshot slots: a second backward
            # reruns the forward from u0
            ctx.save_for_backward(u0)
            ctx.rev_fresh = True
        else:
            out = api.run(u, f.detach().contiguous(), coeffs, int(T), bc, tblock=int(tblock), norms=False,
                          ckpt_every=k)
            ctx.ckpt = out["ckpt"]
        ctx.tblock = int(tblock)
        ctx.coeffs = coeffs
        ctx.T, ctx.bc, ctx.k = int(T), bc, k
        ctx.f = f.detach().contiguous()
        ctx.metas = (_meta(alpha), _meta(beta), _meta(gamma))
        return u

    @staticmethod
    def backward(ctx, grad_uT):
        ma, mb, mg = ctx.metas
        want_f = ctx.needs_input_grad[1]
        want_gamma = ctx.needs_input_grad[4] and mg is not None
        if ctx.slots > 0:
            if not ctx.rev_fresh:
                (u0,) = ctx.saved_tensors
                ctx.ckpt = api.revolve_forward(u0.detach().contiguous().clone(), ctx.f, ctx.coeffs, ctx.T, ctx.bc,
                                               ctx.slots, tblock=ctx.tblock, reserve_sum=True)
            ctx.rev_fresh = False
            r = api.revolve_adjoint(ctx.ckpt, ctx.f, grad_uT.contiguous(), ctx.coeffs, ctx.T, ctx.bc, ctx.slots,
                                    tblock=ctx.tblock, want_f=want_f, want_gamma=want_gamma)
        else:
            r = api.adjoint_run(ctx.ckpt, ctx.k, ctx.f, grad_uT.contiguous(), ctx.coeffs, ctx.T, ctx.bc,
                                tblock=ctx.tblock, want_f=want_f, want_gamma=want_gamma)
        if not isinstance(r, dict):
            r = {"u0": r[0], "ab": r[1]}
        gu = r["u0"] if ctx.needs_input_grad[0] else None
        gf = r["f"] if want_f else None
        ga = _as(ma, r["ab"][0]) if ctx.needs_input_grad[2] and ma is not None else None
        gb = _as(mb, r["ab"][1]) if ctx.needs_input_grad[3] and mb is not None else None
        gg = _as(mg, r["gamma"]) if want_gamma else None
        return gu, gf, ga, gb, gg, None, None, None, None, None, None, None


def rd3d(u0, f, alpha, beta, gamma, dt, h, T, bc, ckpt_every=10, tblock=3, revolve_slots=0):
    """u_T after T fused steps from u0, differentiable in u0, f, alpha, beta
    and gamma.  revolve_slots > 0: binomial checkpointing with that many
    snapshots instead of a checkpoint every ckpt_every steps."""
    return RD3D.apply(u0, f, alpha, beta, gamma, dt, h, T, bc, ckpt_every, tblock, revolve_slots)
