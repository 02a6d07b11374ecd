"""MPPI iterations as differentiable functions of the model parameters.

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


class MPPISteps(torch.autograd.Function):
    """`iters` warm-started iterations from u0 (the tape of the library's
    gradient mode records them); backward: dL/dtheta and dL/du0 through all of
    them (`mppi_backward_iters`)."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, u0: torch.Tensor, controller, iters: int):
        controller.set_theta(theta)
        controller.set_controls(u0.detach())
        controller.iterate(int(iters))
        controller._serial = getattr(controller, "_serial", 0) + 1
        ctx.controller = controller
        ctx.serial = controller._serial
        ctx.theta_device, ctx.u0_device = theta.device, u0.device
        return controller.controls().clone()

    @staticmethod
    def backward(ctx, grad_U: torch.Tensor):
        c = ctx.controller
        if getattr(c, "_serial", None) != ctx.serial:
            raise RuntimeError("the controller ran another iteration after this forward")
        g, du0 = c.backward_iters(grad_U.contiguous())
        return g.to(ctx.theta_device), du0.to(ctx.u0_device), None, None


def mppi_steps(theta: torch.Tensor, u0: torch.Tensor, controller, iters: int) -> torch.Tensor:
    """U after `iters` MPPI iterations from u0 at parameters theta
    (differentiable in theta and u0)."""
    return MPPISteps.apply(theta, u0, controller, iters)
