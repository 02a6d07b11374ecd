"""One MPPI iteration as a differentiable function of the model parameters.

`MPPIStep.apply(theta, controller)` runs one iteration (noise, rollouts,
update) of a controller created with `requires_grad=True` at the parameters
theta = [MLP weights | Q diagonal | wheelbase] and returns the updated
controls U [T, m].  Its backward calls the library's adjoint
(`mppi_backward`): dL/dtheta through the softmin weights and every rollout,
with the nominal controls of the iteration held fixed.  The controller must
not run another iteration between the forward and the backward.
"""
from __future__ import annotations

import torch


class MPPIStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, controller) -> torch.Tensor:
        controller.set_theta(theta)
        controller.sample()
        controller.rollout()
        controller.update()
        controller._serial = getattr(controller, "_serial", 0) + 1
        ctx.controller = controller
        ctx.serial = controller._serial
        ctx.theta_device = theta.device
        return controller.controls().clone()

    @staticmethod
    def backward(ctx, grad_U: torch.Tensor):
        c = ctx.controller
        if getattr(c, "_serial", None) != ctx.serial:
            raise RuntimeError("the controller ran another iteration after this forward")
        g = c.backward(grad_U.contiguous())
        return g.to(ctx.theta_device), None


def mppi_step(theta: torch.Tensor, controller) -> torch.Tensor:
    """U = one MPPI iteration at parameters theta (differentiable in theta)."""
    return MPPIStep.apply(theta, controller)
