"""torch.autograd.Function over rbf_eval_at / rbf_eval_adjoint_at.

RBFEval maps body-frame scan points p (Q x 3), weights w (N, f64) and a
pose increment delta = (dtheta, dt) (6, f64, on the device) to the terrain
height f and the manifold residual r at xi = R p + t, where
R = R0 Exp(dtheta), t = t0 + dt around a fixed linearisation pose (R0, t0).
The library forms the pose from delta on the device (the exponential map of
SO(3)) and maps the kernel's right-perturbation gradient back through the
right Jacobian of SO(3), so the increment and its gradient never leave the
device: the forward and the backward pass are argument marshalling only.
"""
from __future__ import annotations

import torch

from . import api


class RBFEval(torch.autograd.Function):
    """(f, r) = RBFEval.apply(ctx, params, grid, R0, t0, z_off, pts, w, delta)."""

    @staticmethod
    def forward(fctx, rctx: api.Context, params: api.Params, grid: api.Grid, R0, t0,
                z_off: float, pts: torch.Tensor, w: torch.Tensor, delta: torch.Tensor):
        d = delta.detach()
        out = rctx.eval_at(params, grid, w.detach(), pts.detach(), (R0, t0), d, z_off=z_off,
                           grad=False, jac=False)
        fctx.rctx, fctx.params, fctx.grid = rctx, params, grid
        fctx.pose0 = (R0, t0)
        fctx.save_for_backward(pts, w, d)
        return out["f"], out["resid"]

    @staticmethod
    def backward(fctx, g_f, g_r):
        pts, w, d = fctx.saved_tensors
        rctx = fctx.rctx
        dt = pts.dtype
        gf = g_f.contiguous().to(dt) if g_f is not None else None
        gr = g_r.contiguous().to(dt) if g_r is not None else None
        d_w = torch.zeros_like(w) if fctx.needs_input_grad[7] else None
        d_delta = (torch.zeros(6, dtype=torch.float64, device=w.device)
                   if fctx.needs_input_grad[8] else None)
        d_pts, _, _ = rctx.eval_adjoint_at(fctx.params, fctx.grid, w.detach(), pts.detach(),
                                           fctx.pose0, d, gbar_f=gf, gbar_r=gr,
                                           d_pts=fctx.needs_input_grad[6], d_w=d_w,
                                           d_delta=d_delta)
        return None, None, None, None, None, None, d_pts, d_w, d_delta


def rbf_eval_f_r(rctx, params, grid, R0, t0, pts, w, delta, z_off=0.0):
    """Differentiable (f, r) at every point; see RBFEval. delta is a
    6-element float64 device tensor."""
    return RBFEval.apply(rctx, params, grid, R0, t0, z_off, pts, w, delta)
