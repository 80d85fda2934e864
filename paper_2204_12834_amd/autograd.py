"""The damped step as a differentiable PyTorch operation.

`damped_step(problem, obs_xy, intrinsics, extrinsics, lms, lam, m)` returns
the step (dx_cams, dx_lms) of eq. normal (Sec. 4.1) at the state
(extrinsics | intrinsics, lms) for the observations obs_xy, solved by the power
series of order m (eps = 0).  Gradients flow to obs_xy [n_obs, 2] and
intrinsics [n_cams, 3] (f, k1, k2) through poba_step_adjoint (implicit
differentiation at fixed lambda and damping diagonal; the adjoint reuses the
power solve).  extrinsics [n_cams, 6] and lms [n_lms, 3] are treated as
constants and must not require gradients.

Forward and backward both run in the HIP library; this module only marshals
tensors.  The handle's linearisation is redone in backward from the saved
inputs, so other calls on the same handle between forward and backward are
harmless.
"""
from __future__ import annotations

import torch

from .solver import Problem


class DampedStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, obs_xy, intrinsics, problem: Problem, extrinsics, lms, lam: float, m: int):
        if extrinsics.requires_grad or lms.requires_grad:
            raise ValueError("damped_step differentiates with respect to obs_xy and intrinsics only")
        cams = torch.cat([extrinsics.detach().to(torch.float64), intrinsics.detach().to(torch.float64)],
                         dim=1).contiguous()
        obs = obs_xy.detach().to(torch.float64).contiguous()
        lms64 = lms.detach().to(torch.float64).contiguous()
        problem.set_observations(obs)
        problem.linearize(cams, lms64)
        dxc, dxl, _ = problem.power_solve(lam, m, 0.0)
        ctx.problem, ctx.lam, ctx.m = problem, float(lam), int(m)
        ctx.dtypes = (obs_xy.dtype, intrinsics.dtype)
        ctx.save_for_backward(obs, cams, lms64, dxc, dxl)
        return dxc, dxl

    @staticmethod
    def backward(ctx, grad_dxc, grad_dxl):
        obs, cams, lms, dxc, dxl = ctx.saved_tensors
        p = ctx.problem
        if grad_dxc is None:
            grad_dxc = torch.zeros_like(dxc)
        if grad_dxl is None:
            grad_dxl = torch.zeros_like(dxl)
        p.set_observations(obs)
        p.linearize(cams, lms)
        go, gi, _, _ = p.step_adjoint(ctx.lam, ctx.m, cams, lms, dxc, dxl, grad_dxc.contiguous(),
                                      grad_dxl.contiguous())
        g_obs = go.to(ctx.dtypes[0]) if ctx.needs_input_grad[0] else None
        g_int = gi.to(ctx.dtypes[1]) if ctx.needs_input_grad[1] else None
        return g_obs, g_int, None, None, None, None, None


def damped_step(problem: Problem, obs_xy, intrinsics, extrinsics, lms, lam: float, m: int):
    """Differentiable damped step; see the module docstring."""
    return DampedStep.apply(obs_xy, intrinsics, problem, extrinsics, lms, lam, m)
