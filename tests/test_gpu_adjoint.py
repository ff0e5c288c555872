"""rbf_eval_adjoint and the autograd Function against the FP64 oracle.

FP64: adjoint outputs within 1e-12 (relative to the magnitude of each
output) of the oracle's adjoint, whose formulas are pinned on the CPU by
exact directional derivatives, central differences and the dot-product test.
The differentiation workload (odometry terrain, frame 50, pose perturbed by
N(0, 0.05^2) per coordinate, 200k points) is checked in FP64 by central
differences on a 2k-point subset and in FP32 (the production path) against
the FP64 oracle on 20k points with the stated 1e-3 relative bound.
"""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import dev, host
from paper_2509_26222_amd import api, synth
from paper_2509_26222_amd.autograd import rbf_eval_f_r

pytestmark = pytest.mark.gpu


def _off_cutoff(pts, R, t, centers, p, margin):
    """1.0 for body points whose world xy is farther than `margin` (m) from
    every center's cutoff circle, else 0.0."""
    xi = O.to_world(pts, R, t)
    d = np.sqrt(O.sq_dist(xi[:, :2], centers))
    return (np.abs(d - p.cutoff * p.sigma) > margin).all(1).astype(np.float64)


def _close(a, b, rel):
    scale = max(np.abs(b).max(), 1e-30)
    return np.abs(a - b).max() <= rel * scale


@pytest.fixture(scope="module")
def small(ctx):
    s = synth.small_case(0)
    p = api.Params()
    w, _ = O.ridge_batch(s.xy, s.z, s.centers, p.sigma, p.cutoff, 0.0, p.lam, p.R,
                         with_P=False)
    grid = ctx.grid(p, dev(s.centers))
    rng = np.random.default_rng(5)
    R = synth.rot_zyx(0.4, 0.05, -0.02)
    t = np.array([5.0, 5.0, 0.6])
    world = np.concatenate([rng.uniform(-0.5, 10.5, size=(3001, 2)),
                            rng.normal(0, 0.1, size=(3001, 1))], 1)
    pts = (world - t) @ R
    return s, p, w, grid, pts, R, t


def test_adjoint_pose_f64(ctx, small):
    s, p, w, grid, pts, R, t = small
    rng = np.random.default_rng(1)
    gf, gr = rng.normal(size=pts.shape[0]), rng.normal(size=pts.shape[0])
    d_w = torch.zeros(grid.N, dtype=torch.float64, device="cuda")
    d_pose = torch.zeros(6, dtype=torch.float64, device="cuda")
    d_p, _, _ = ctx.eval_adjoint(p, grid, dev(w), dev(pts), pose=(R, t), gbar_f=dev(gf),
                                 gbar_r=dev(gr), d_w=d_w, d_pose=d_pose)
    rp, rw, rpose = O.eval_adjoint_pose(pts, R, t, 0.0, s.centers, w, p.sigma, p.cutoff, gf, gr)
    assert _close(host(d_p), rp, 1e-12)
    assert _close(host(d_w), rw, 1e-12)
    assert _close(host(d_pose), rpose, 1e-12)


def test_adjoint_xy_f64_and_accumulates(ctx, small):
    s, p, w, grid, pts, R, t = small
    rng = np.random.default_rng(2)
    q = rng.uniform(0, 10, size=(1234, 2))
    gb = rng.normal(size=1234)
    d_w = torch.ones(grid.N, dtype=torch.float64, device="cuda")
    d_q, _, _ = ctx.eval_adjoint(p, grid, dev(w), dev(q), gbar_f=dev(gb), d_w=d_w)
    rq, rw = O.eval_adjoint_xy(q, s.centers, w, p.sigma, p.cutoff, gb)
    assert _close(host(d_q), rq, 1e-12)
    assert _close(host(d_w) - 1.0, rw, 1e-12)  # accumulated onto the buffer


@pytest.fixture(scope="module")
def diff_case(ctx):
    od = synth.OdometryCase()
    p = api.Params()
    allxy = np.concatenate([od.ground_xy(k) for k in range(od.N_FRAMES)])
    centers = O.select_centers(allxy, od.roi, 0.5, 0.5, 4, O.VOXEL)
    xs, zs = zip(*[od.ground(k) for k in (48, 49, 50, 51)])
    xy, z = np.concatenate(xs), np.concatenate(zs)
    H, b = O.gram(xy, z, centers, p.sigma, p.cutoff, 0.0, p.lam, sparse=True)
    w = O.spd_solve(H, b)
    pts, R, t = od.scan(50)
    Rp, tp, _ = synth.perturbed_pose(R, t, seed=2)
    grid = ctx.grid(p, dev(centers))
    return od, p, centers, w, pts, Rp, tp, grid


def test_autograd_fd_f64_subset(ctx, diff_case):
    od, p, centers, w, pts, R, t, grid = diff_case
    rng = np.random.default_rng(0)
    idx = rng.choice(pts.shape[0], 2000, replace=False)
    P = dev(pts[idx]).requires_grad_(True)
    W = dev(w).requires_grad_(True)
    D = torch.zeros(6, dtype=torch.float64, device="cuda", requires_grad=True)
    keep = _off_cutoff(pts[idx], R, t, centers, p, 1e-3)  # smooth near the base pose
    gf = dev(rng.normal(size=2000) * keep)
    gr = dev(rng.normal(size=2000) * keep)
    f, r = rbf_eval_f_r(ctx, p, grid, R, t, P, W, D)
    L = (gf * f).sum() + (gr * r).sum()
    L.backward()

    def Lval(pts_, w_, d_):
        with torch.no_grad():
            f_, r_ = rbf_eval_f_r(ctx, p, grid, R, t, pts_, w_, d_)
            return float((gf * f_).sum() + (gr * r_).sum())

    h = 1e-6
    for k in range(6):
        e = torch.zeros(6, dtype=torch.float64, device="cuda")
        e[k] = h
        fd = (Lval(P.detach(), W.detach(), e) - Lval(P.detach(), W.detach(), -e)) / (2 * h)
        assert fd == pytest.approx(float(D.grad[k]), rel=1e-5, abs=1e-6)
    v = dev(rng.normal(size=w.shape[0]))
    lin = Lval(P.detach(), W.detach() + v, D.detach()) - Lval(P.detach(), W.detach(), D.detach())
    assert lin == pytest.approx(float((W.grad * v).sum()), rel=1e-9)
    V = dev(rng.normal(size=(2000, 3)))
    fd = (Lval(P.detach() + h * V, W.detach(), D.detach())
          - Lval(P.detach() - h * V, W.detach(), D.detach())) / (2 * h)
    assert fd == pytest.approx(float((P.grad * V).sum()), rel=1e-5, abs=1e-6)


def test_autograd_f32_production_vs_oracle(ctx, diff_case):
    od, p, centers, w, pts, R, t, grid = diff_case
    rng = np.random.default_rng(3)
    # full 200k-point FP32 backward runs; 20k of them are checked
    P = dev(pts, torch.float32).requires_grad_(True)
    W = dev(w).requires_grad_(True)
    D = torch.zeros(6, dtype=torch.float64, device="cuda", requires_grad=True)
    f, r = rbf_eval_f_r(ctx, p, grid, R, t, P, W, D)
    assert f.dtype == torch.float32 and f.shape[0] == pts.shape[0]
    idx = rng.choice(pts.shape[0], 20000, replace=False)
    mask = torch.zeros(pts.shape[0], dtype=torch.float32, device="cuda")
    mask[torch.as_tensor(idx, device="cuda")] = 1.0
    gf = dev(rng.normal(size=pts.shape[0]), torch.float32) * mask
    gr = dev(rng.normal(size=pts.shape[0]), torch.float32) * mask
    ((gf * f).sum() + (gr * r).sum()).backward()
    p32 = pts[idx].astype(np.float32).astype(np.float64)
    rp, rw, rpose = O.eval_adjoint_pose(p32, R, t, 0.0, centers, w, p.sigma, p.cutoff,
                                        host(gf)[idx].astype(np.float64),
                                        host(gr)[idx].astype(np.float64))
    gp = host(P.grad)[idx].astype(np.float64)
    xi = O.to_world(p32, R, t)
    d2 = O.sq_dist(xi[:, :2], centers)
    ok = ~(np.abs(d2 - (p.cutoff * p.sigma) ** 2) <= 1e-4 * (p.cutoff * p.sigma) ** 2).any(1)
    err = np.linalg.norm(gp - rp, axis=1)[ok]
    nrm = np.maximum(np.linalg.norm(rp, axis=1)[ok], 0.01)
    print(f"f32 d_pts rel max {np.max(err / nrm):.2e}, d_w rel "
          f"{np.linalg.norm(host(W.grad) - rw) / np.linalg.norm(rw):.2e}, d_pose rel "
          f"{np.linalg.norm(host(D.grad) - rpose) / np.linalg.norm(rpose):.2e}")
    assert np.max(err / nrm) <= 1e-3
    assert np.linalg.norm(host(W.grad) - rw) / np.linalg.norm(rw) <= 1e-3
    assert np.linalg.norm(host(D.grad) - rpose) / np.linalg.norm(rpose) <= 1e-3


@pytest.mark.parametrize("scale", [1.0, 1e-3, 1e-6])
def test_eval_at_increment_matches_pose_and_fd(ctx, small, scale):
    """rbf_eval_at forms R0 Exp(dtheta), t0 + dt on the device: its outputs
    match the oracle at the pose composed on the host with scipy's rotation
    vector map, for a large increment and for small ones (the series branch
    of the exponential map), and the autograd gradient w.r.t. the increment
    (through the right Jacobian) matches central differences."""
    from scipy.spatial.transform import Rotation
    s, p, w, grid, pts, R, t = small
    d = np.array([0.3, -0.2, 0.5, 0.1, -0.05, 0.02]) * scale
    Rd = R @ Rotation.from_rotvec(d[:3]).as_matrix()
    td = t + d[3:]
    out = ctx.eval_at(p, grid, dev(w), dev(pts), (R, t), dev(d), z_off=0.02)
    f0, g0, r0, J0 = O.eval_pose(pts, Rd, td, 0.02, s.centers, w, p.sigma, p.cutoff)
    assert _close(host(out["f"]), f0, 1e-12)
    assert _close(host(out["resid"]), r0, 1e-12)
    assert _close(host(out["jac"]), J0, 1e-11)
    rng = np.random.default_rng(4)
    # the truncated kernel jumps at the cutoff circle: points within 1 mm
    # of it (a perturbation of h moves a point by ~1e-5 m) get zero weight,
    # so that the central differences see a smooth function
    keep = _off_cutoff(pts, Rd, td, s.centers, p, 1e-3)
    gf = dev(rng.normal(size=pts.shape[0]) * keep)
    gr = dev(rng.normal(size=pts.shape[0]) * keep)
    D = dev(d).requires_grad_(True)
    f, r = rbf_eval_f_r(ctx, p, grid, R, t, dev(pts), dev(w), D)
    ((gf * f).sum() + (gr * r).sum()).backward()

    def L(dd):
        with torch.no_grad():
            f_, r_ = rbf_eval_f_r(ctx, p, grid, R, t, dev(pts), dev(w), dd)
            return float((gf * f_).sum() + (gr * r_).sum())

    h = 1e-6
    for k in range(6):
        e = torch.zeros(6, dtype=torch.float64, device="cuda")
        e[k] = h
        fd = (L(D.detach() + e) - L(D.detach() - e)) / (2 * h)
        assert fd == pytest.approx(float(D.grad[k]), rel=1e-5, abs=1e-6)
