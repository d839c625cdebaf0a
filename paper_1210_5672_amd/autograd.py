"""torch.autograd wrapper of the shooting objective (Sec. 3.1 eq. (f:phi)).

forward: f(c) = r(c).r(c)/2 by shoot_eval (base march only).
backward: df/dc by the library's discrete adjoint (shoot_adjoint: reverse sweep of
the discretised variational march with checkpointed base states).
"""
from __future__ import annotations

import torch


class ShootFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, engine, T: float, nsteps: int, ckpt_every: int = 16):
        out = engine.shoot_eval(params.detach(), T, nsteps, jacobian=False, drdT=False)
        ctx.engine, ctx.T, ctx.nsteps, ctx.ckpt = engine, T, nsteps, ckpt_every
        ctx.save_for_backward(params.detach())
        return torch.tensor(out["f"], dtype=torch.float64, device=params.device)

    @staticmethod
    def backward(ctx, grad_out):
        (params,) = ctx.saved_tensors
        res = ctx.engine.shoot_adjoint(params, ctx.T, ctx.nsteps, ctx.ckpt)
        return grad_out * res["grad"], None, None, None, None


def shoot_objective(params: torch.Tensor, engine, T: float, nsteps: int, ckpt_every: int = 16):
    return ShootFn.apply(params, engine, T, nsteps, ckpt_every)
