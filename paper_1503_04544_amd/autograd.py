"""torch.autograd front of the hand-written adjoint.

DragFn maps (T_w, Kn, Ma) to the drag (or torque) of a fixed-body flow after
nsteps from the inflow Maxwellian.  The library's adjoint runs the forward
sweep with checkpoints and the backward sweep with recomputation in one call
(cc_adjoint), so forward() computes the value and its gradient together and
backward() scales the stored gradient.
"""
from __future__ import annotations

import dataclasses

import torch

from .solver import Solver


def _config_with(cfg, t_wall: float, kn: float, mach: float):
    """cfg with the wall temperature, Knudsen number and inflow Mach number
    replaced (inflow along its current direction, gamma = 5/3)."""
    import math
    rho, ux, uy, uz, T = cfg.inflow
    un = math.hypot(ux, uy)
    ex, ey = (ux / un, uy / un) if un > 0 else (1.0, 0.0)
    u = mach * math.sqrt(5.0 / 3.0 * T)
    return dataclasses.replace(cfg, kn=kn, inflow=(rho, u * ex, u * ey, uz, T),
                               body=dataclasses.replace(cfg.body, t_wall=t_wall))


class DragFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, cfg, nsteps: int, ckpt_every: int = 16,
                objective: str = "drag", device: str = "cuda"):
        tw, kn, ma = (float(x) for x in params.detach().cpu().tolist())
        s = Solver(_config_with(cfg, tw, kn, ma), device=device)
        J, grad = s.adjoint(nsteps, ckpt_every, objective)
        s.close()
        ctx.save_for_backward(torch.as_tensor(grad, dtype=params.dtype, device=params.device))
        return torch.as_tensor(J, dtype=params.dtype, device=params.device)

    @staticmethod
    def backward(ctx, gJ):
        (grad,) = ctx.saved_tensors
        return gJ * grad, None, None, None, None, None


def drag(params: torch.Tensor, cfg, nsteps: int, ckpt_every: int = 16, objective: str = "drag",
         device: str = "cuda") -> torch.Tensor:
    """Differentiable drag (or torque) of cfg after nsteps; params = (T_w, Kn, Ma)."""
    return DragFn.apply(params, cfg, nsteps, ckpt_every, objective, device)
