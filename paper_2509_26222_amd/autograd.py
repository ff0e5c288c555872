"""torch.autograd.Function over rbf_eval / rbf_eval_adjoint.

RBFEval maps body-frame scan points p (Q x 3), weights w (N, f64) and a
pose increment delta = (dtheta, dt) (6, f64) to the terrain height f and the
manifold residual r at xi = R p + t, where R = R0 Exp(dtheta), t = t0 + dt
around a fixed linearisation pose (R0, t0). Both the forward and the
backward pass are single launches of the library's kernels; the gradient
w.r.t. delta is the kernel's right-perturbation gradient at (R, t) mapped
through the right Jacobian of SO(3) (the identity at delta = 0, where
Gauss-Newton and LM steps evaluate it).

Only the pose is converted on the host (12 numbers to the kernel's
R, t arguments, 3 numbers back through the Jacobian).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import api


def _so3_exp(v):
    v = np.asarray(v, dtype=np.float64)
    th = float(np.linalg.norm(v))
    K = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0.0]])
    if th < 1e-8:
        return np.eye(3) + K + 0.5 * (K @ K)
    return (np.eye(3) + math.sin(th) / th * K + (1.0 - math.cos(th)) / th ** 2 * (K @ K))


def _so3_right_jacobian(v):
    """J_r(v): Exp(v + e) = Exp(v) Exp(J_r(v) e) to first order."""
    v = np.asarray(v, dtype=np.float64)
    th = float(np.linalg.norm(v))
    K = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0.0]])
    if th < 1e-8:
        return np.eye(3) - 0.5 * K + (K @ K) / 6.0
    return (np.eye(3) - (1.0 - math.cos(th)) / th ** 2 * K
            + (th - math.sin(th)) / th ** 3 * (K @ K))


class RBFEval(torch.autograd.Function):
    """(f, r) = RBFEval.apply(ctx, params, grid, R0, t0, z_off, pts, w, delta)."""

    @staticmethod
    def forward(fctx, rctx: api.Context, params: api.Params, grid: api.Grid, R0, t0,
                z_off: float, pts: torch.Tensor, w: torch.Tensor, delta: torch.Tensor):
        d = delta.detach().double().cpu().numpy()
        R = np.asarray(R0, dtype=np.float64) @ _so3_exp(d[:3])
        t = np.asarray(t0, dtype=np.float64).reshape(3) + d[3:]
        out = rctx.eval(params, grid, w.detach(), pts.detach(), pose=(R, t), z_off=z_off,
                        grad=False, jac=False)
        fctx.rctx, fctx.params, fctx.grid = rctx, params, grid
        fctx.pose = (R, t)
        fctx.delta = d
        fctx.save_for_backward(pts, w)
        return out["f"], out["resid"]

    @staticmethod
    def backward(fctx, g_f, g_r):
        pts, w = fctx.saved_tensors
        rctx = fctx.rctx
        dt = pts.dtype
        gf = g_f.contiguous().to(dt) if g_f is not None else None
        gr = g_r.contiguous().to(dt) if g_r is not None else None
        d_w = torch.zeros_like(w) if fctx.needs_input_grad[7] else None
        d_pose = torch.zeros(6, dtype=torch.float64, device=w.device)
        d_pts, _, _ = rctx.eval_adjoint(fctx.params, fctx.grid, w.detach(), pts.detach(),
                                        pose=fctx.pose, gbar_f=gf, gbar_r=gr,
                                        d_pts=fctx.needs_input_grad[6], d_w=d_w,
                                        d_pose=d_pose)
        d_delta = None
        if fctx.needs_input_grad[8]:
            gp = d_pose.cpu().numpy()
            Jr = _so3_right_jacobian(fctx.delta[:3])
            d_delta = torch.from_numpy(np.concatenate([Jr.T @ gp[:3], gp[3:]])).to(w.device)
        return None, None, None, None, None, None, d_pts, d_w, d_delta


def rbf_eval_f_r(rctx, params, grid, R0, t0, pts, w, delta, z_off=0.0):
    """Differentiable (f, r) at every point; see RBFEval."""
    return RBFEval.apply(rctx, params, grid, R0, t0, z_off, pts, w, delta)
