"""torch.autograd.Function over the backward pass: u^0 as a function of the
drift parameters and the diffusion coefficient theta = (coef..., D) of every
instance.  backward() runs the library's checkpointed adjoint (fk_adjoint)
with the incoming cotangent as dJ/du^0, so any scalar objective of u^0
differentiates through it (the exit classification of landing points is held
fixed, as in the pathwise derivative of the scheme)."""
from __future__ import annotations

from typing import Sequence

import torch

from .fkexit import Plan


def _with_theta(prob, th: Sequence[float]):
    """theta = (differentiable drift parameters..., D); coefficients past them
    (the roll count of the Section 4.2 example) are kept."""
    npar = len(th) - 1
    coef = tuple(float(v) for v in th[:npar]) + tuple(prob.coef[npar:])
    return prob.replace(coef=coef, D=float(th[npar]))


class ExitProbability(torch.autograd.Function):
    """theta: tensor [n_inst, n_theta] (any device, float64) -> packed u^0."""

    @staticmethod
    def forward(ctx, theta, problems, precision="f64", ckpt_every=64):
        th = theta.detach().double().cpu().tolist()
        probs = [_with_theta(p, t) for p, t in zip(problems, th)]
        plan = Plan(probs, precision=precision, ckpt_every=ckpt_every)
        u0 = plan.forward([0])[0]
        ctx.plan = plan
        ctx.theta_shape = theta.shape
        ctx.theta_device = theta.device
        return u0

    @staticmethod
    def backward(ctx, grad_u0):
        plan = ctx.plan
        grad, _ = plan.adjoint(grad_u0.contiguous())
        plan.close()
        g = grad[:, : ctx.theta_shape[1]].to(ctx.theta_device)
        return g, None, None, None


def exit_probability(theta, problems, precision="f64", ckpt_every=64):
    return ExitProbability.apply(theta, problems, precision, ckpt_every)
