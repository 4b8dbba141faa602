"""Leave-one-slice-out loss as a torch.autograd.Function.

forward: okr_loso_forward (refined batched solves on the GPU) -> scalar loss.
backward: okr_loso_backward (adjoint of the kriging systems of Appendix A,
with the slice predictor on a drift plan) -> dL/d(nugget, sill, range). Both run entirely in the HIP library; this module
only passes the variogram parameters and device pointers.
"""
from __future__ import annotations

import torch

__all__ = ["LosoLoss", "fit_variogram"]


class LosoLoss(torch.autograd.Function):
    """loss = LosoLoss.apply(theta, plan, slices, edge, model)

    theta: float64 tensor [3] = (nugget, sill, range); plan: a Plan with
    upsample 2 over the known slices; slices: CUDA float32 [n][ny][nx].
    """

    @staticmethod
    def forward(ctx, theta, plan, slices, edge, model):
        nug, sill, rng = (float(v) for v in theta.detach().cpu().tolist())
        loss = plan.loso_forward(slices, (model, nug, sill, rng), edge)
        ctx.plan = plan
        ctx.token = plan.loso_token
        ctx.theta_device = theta.device
        return loss.clone()

    @staticmethod
    def backward(ctx, grad_out):
        if ctx.plan.loso_token != ctx.token:
            raise RuntimeError("LosoLoss.backward: the plan ran another leave-one-slice-out "
                               "forward after this loss; its adjoint would belong to that one")
        g = ctx.plan.loso_backward()
        g = g.to(ctx.theta_device) * grad_out.to(ctx.theta_device)
        return g, None, None, None, None


def fit_variogram(plan, slices, theta0, steps: int = 200, lr: float = 0.05, model: str = "exponential",
                  edge=None):
    """Adam on u = log(theta) (keeps every parameter positive). Returns the
    trajectory [(loss, theta)] evaluated at each step plus the final point."""
    u = torch.log(torch.tensor(theta0, dtype=torch.float64)).requires_grad_(True)
    opt = torch.optim.Adam([u], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    traj = []
    for _ in range(steps):
        opt.zero_grad()
        theta = torch.exp(u)
        loss = LosoLoss.apply(theta, plan, slices, edge, model)
        loss.backward()
        traj.append((float(loss.item()), theta.detach().numpy().copy()))
        opt.step()
    with torch.no_grad():
        theta = torch.exp(u)
        loss = LosoLoss.apply(theta, plan, slices, edge, model)
    traj.append((float(loss.item()), theta.detach().numpy().copy()))
    return traj
