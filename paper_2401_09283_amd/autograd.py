"""Differentiable backprojection for torch autograd (the paper's custom function, Sec. II-B.2).

``Backprojector`` owns a plan and a workspace for one geometry. ``backproject``
maps (theta [n][6] float64, mm / rad) to the volume through libgmc; its backward
runs the VJP kernel and returns dL/dtheta. Projections and calibrated matrices
are constant inputs (the paper differentiates only through the matrices).
"""
from __future__ import annotations

import torch

from . import gmc


class Backprojector:
    def __init__(self, n_views, det_w, det_h, shape, voxel_mm, origin_mm, P, weighting="fdk", grad_mode="paper",
                 flags=0, device="cuda"):
        self.geometry = gmc.make_geometry(n_views, det_w, det_h, shape, voxel_mm, origin_mm, weighting, grad_mode,
                                          flags)
        P_host = P.detach().cpu().double().numpy() if isinstance(P, torch.Tensor) else P
        self.plan = gmc.Plan(self.geometry, P_host)
        self.device = torch.device(device)
        self.workspace = self.plan.new_workspace(self.device)
        self.P = torch.as_tensor(P_host, dtype=torch.float64).reshape(n_views, 3, 4).to(self.device).contiguous()

    @classmethod
    def from_case(cls, case, weighting="fdk", grad_mode="paper", flags=0, device="cuda"):
        s, g = case.scan, case.grid
        return cls(s.n_views, s.det_w, s.det_h, g.shape, g.voxel_mm, g.origin_mm, case.P, weighting, grad_mode,
                   flags, device)

    def forward(self, proj, theta, out=None):
        vol = out if out is not None else torch.empty(self.plan.vol_shape, dtype=torch.float32, device=self.device)
        gmc.gmc_backproject(self.plan, proj, self.P, theta, vol, self.workspace)
        return vol

    def vjp(self, proj, theta, grad_vol, grad_theta=None, grad_P=None):
        n = self.geometry.n_views
        if grad_theta is None:
            grad_theta = torch.empty((n, 6), dtype=torch.float64, device=self.device)
        gmc.gmc_backproject_vjp(self.plan, proj, self.P, theta, grad_vol, grad_theta, grad_P, self.workspace)
        return grad_theta

    def check(self):
        gmc.gmc_check(self.plan, self.workspace)


class BackprojectFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, proj, bp: Backprojector):
        theta_c = theta.detach().contiguous()
        ctx.save_for_backward(theta_c, proj)
        ctx.bp = bp
        return bp.forward(proj, theta_c)

    @staticmethod
    def backward(ctx, grad_vol):
        theta, proj = ctx.saved_tensors
        g = ctx.bp.vjp(proj, theta, grad_vol.contiguous())
        return g, None, None


def backproject(theta, proj, bp: Backprojector):
    """Volume r(p(theta)) with autograd support for theta."""
    return BackprojectFn.apply(theta, proj, bp)
