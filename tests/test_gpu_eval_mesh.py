"""Mesh form of the evaluation (rbf_grid_set_mesh): the centers are nodes of
a square mesh (the paper's candidate-center mesh), the weights sit in a
dense node array and a point reads a fixed window of nodes, with the
Gaussian factored over the axes.

Against the FP64 oracle with the bounds of the binned form: FP64
|f - f0| <= 1e-13 sum_j |w_j phi_j| (and the gradient likewise); FP32
1e-4 m and 1e-3 relative gradient over points not within 1e-4 rc^2 of a
cutoff circle. Windows of 4, 8 and 12 nodes (8 is the odometry map's:
sigma 0.5, cutoff 3, 0.5 m mesh), the xy and the pose form, a pose
increment, the fused Gauss-Newton sums, and the odometry frame at full
size (200k points on 10k centers) on sampled points. set_mesh refuses
centers off the mesh, two centers on one node and a window over 12 nodes;
res = 0 restores the binned form bit for bit."""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import dev, host
from paper_2509_26222_amd import api, synth

pytestmark = pytest.mark.gpu


def abs_sums(q, c, w, sigma, cutoff):
    Phi = O.phi_dense(q, c, sigma, cutoff)
    A = np.abs(Phi * w[None, :])
    dx = np.abs(q[:, 0:1] - c[None, :, 0])
    dy = np.abs(q[:, 1:2] - c[None, :, 1])
    return A.sum(1), (A * (dx + dy)).sum(1) / sigma ** 2


def ambiguous(q, c, sigma, cutoff, rel=1e-4):
    rc2 = (cutoff * sigma) ** 2
    d2 = O.sq_dist(q, c)
    return (np.abs(d2 - rc2) <= rel * rc2).any(axis=1)


def mesh_case(seed, nx, ny, res, x0=-3.0, y0=2.0, keep=0.8):
    """Nodes (x0 + (i + 1/2) res, y0 + (j + 1/2) res) of an nx x ny mesh, a
    random subset kept (holes in the node array), random weights; query
    points over the mesh and a rim of 2 m around it."""
    rng = np.random.default_rng(seed)
    c = synth.grid_centers(rng, nx, ny, res, x0, y0, jitter=0.0)
    c = c[rng.uniform(size=c.shape[0]) < keep]
    c = np.ascontiguousarray(c[rng.permutation(c.shape[0])])
    w = rng.normal(0.0, 0.3, c.shape[0])
    lo, hi = c.min(0) - 2.0, c.max(0) + 2.0
    q = rng.uniform(lo, hi, size=(6000, 2))
    return c, w, q, (x0, y0, x0 + nx * res, y0 + ny * res)


def check_f64(out, q, c, w, p):
    f0, g0 = O.eval_height_grad(q, c, w, p.sigma, p.cutoff)
    af, ag = abs_sums(q, c, w, p.sigma, p.cutoff)
    assert np.all(np.abs(host(out["f"]) - f0) <= 1e-13 * af + 1e-300)
    assert np.all(np.abs(host(out["grad"]) - g0).max(1) <= 1e-13 * ag + 1e-300)


def check_f32(out, q32, c, w, p):
    f0, g0 = O.eval_height_grad(q32, c, w, p.sigma, p.cutoff)
    ok = ~ambiguous(q32, c, p.sigma, p.cutoff)
    assert ok.sum() > 0.99 * len(ok)
    ef = np.abs(host(out["f"]).astype(np.float64) - f0)[ok]
    eg = np.linalg.norm(host(out["grad"]).astype(np.float64) - g0, axis=1)[ok]
    gn = np.maximum(np.linalg.norm(g0, axis=1)[ok], 0.01)
    assert ef.max() <= 1e-4
    assert np.max(eg / gn) <= 1e-3


# (res, window): sigma 0.5, cutoff 3 -> support radius 1.5 m = R nodes
WINDOWS = [(1.1, 4), (1.0, 4), (0.5, 8), (0.43, 8), (0.3, 12)]


@pytest.mark.parametrize("res,window", WINDOWS)
def test_mesh_xy_matches_oracle(ctx, res, window):
    p = api.Params()
    nx = int(12.0 / res)
    c, w, q, roi = mesh_case(int(res * 100), nx, nx - 3, res)
    grid = ctx.grid(p, dev(c)).set_mesh_roi(roi, res)
    print(f"mesh xy: res {res} window {window} N {c.shape[0]}", flush=True)
    check_f64(ctx.eval(p, grid, dev(w), dev(q)), q, c, w, p)
    q32 = q.astype(np.float32).astype(np.float64)
    check_f32(ctx.eval(p, grid, dev(w), dev(q, torch.float32)), q32, c, w, p)


def test_mesh_far_nan_and_empty(ctx):
    p = api.Params()
    c, w, q, roi = mesh_case(3, 20, 17, 0.5)
    grid = ctx.grid(p, dev(c)).set_mesh_roi(roi, 0.5)
    far = np.array([[-1e3, 5.0], [5.0, 1e6], [1e30, -1e30], [-3.1, 2.1], [6.9, 10.6]])
    qq = np.concatenate([q[:100], far])
    for dt in (torch.float64, torch.float32):
        out = ctx.eval(p, grid, dev(w), dev(qq, dt))
        f = host(out["f"])
        assert np.all(f[100:103] == 0.0)
        qn = qq.copy()
        qn[7] = [np.nan, 1.0]
        fn = host(ctx.eval(p, grid, dev(w), dev(qn, dt))["f"])
        assert fn[7] == 0.0
        keep = np.arange(qq.shape[0]) != 7
        assert np.array_equal(fn[keep], f[keep])
    check_f64(ctx.eval(p, grid, dev(w), dev(qq)), qq, c, w, p)
    out = ctx.eval(p, grid, dev(w), torch.zeros((0, 2), dtype=torch.float64, device="cuda"))
    assert out["f"].numel() == 0


def _pose_points(c, n, seed):
    rng = np.random.default_rng(seed)
    R = synth.rot_zyx(0.4, 0.06, -0.03)
    lo, hi = c.min(0) - 1.0, c.max(0) + 1.0
    t = np.array([(lo[0] + hi[0]) / 2, (lo[1] + hi[1]) / 2, 0.6])
    xy = rng.uniform(lo, hi, size=(n, 2))
    z = rng.normal(0, 0.05, size=n)
    world = np.concatenate([xy, z[:, None]], 1)
    return np.ascontiguousarray((world - t) @ R), R, t


@pytest.mark.parametrize("n", [1, 63, 5003])
def test_mesh_pose_f64(ctx, n):
    p = api.Params()
    c, w, _, roi = mesh_case(21, 30, 24, 0.5)
    grid = ctx.grid(p, dev(c)).set_mesh_roi(roi, 0.5)
    pts, R, t = _pose_points(c, n, 5 + n)
    out = ctx.eval(p, grid, dev(w), dev(pts), pose=(R, t), z_off=0.03)
    f0, g0, r0, J0 = O.eval_pose(pts, R, t, 0.03, c, w, p.sigma, p.cutoff)
    xi = O.to_world(pts, R, t)
    af, ag = abs_sums(xi[:, :2], c, w, p.sigma, p.cutoff)
    assert np.all(np.abs(host(out["f"]) - f0) <= 1e-13 * af + 1e-14)
    assert np.all(np.abs(host(out["resid"]) - r0) <= 1e-13 * af + 1e-14)
    assert np.all(np.abs(host(out["grad"]) - g0).max(1) <= 1e-13 * ag + 1e-14)
    scale = 1.0 + np.abs(pts).max(1)
    assert np.all(np.abs(host(out["jac"]) - J0).max(1) <= 1e-13 * scale * (ag + 1.0))


def test_mesh_pose_f32(ctx):
    p = api.Params()
    c, w, _, roi = mesh_case(22, 30, 24, 0.5)
    grid = ctx.grid(p, dev(c)).set_mesh_roi(roi, 0.5)
    pts, R, t = _pose_points(c, 20000, 9)
    out = ctx.eval(p, grid, dev(w), dev(pts, torch.float32), pose=(R, t))
    p32 = pts.astype(np.float32).astype(np.float64)
    f0, g0, r0, J0 = O.eval_pose(p32, R, t, 0.0, c, w, p.sigma, p.cutoff)
    xi = O.to_world(p32, R, t)
    ok = ~ambiguous(xi[:, :2], c, p.sigma, p.cutoff)
    ef = np.abs(host(out["f"]).astype(np.float64) - f0)[ok]
    er = np.abs(host(out["resid"]).astype(np.float64) - r0)[ok]
    eg = np.linalg.norm(host(out["grad"]).astype(np.float64) - g0, axis=1)[ok]
    gn = np.maximum(np.linalg.norm(g0, axis=1)[ok], 0.01)
    print(f"mesh f32 pose: max|df| {ef.max():.2e}, grad rel {np.max(eg / gn):.2e}")
    assert ef.max() <= 1e-4 and er.max() <= 1e-4
    assert np.max(eg / gn) <= 1e-3


def test_mesh_against_binned_and_back(ctx):
    """The same grid in both forms: equal to rounding; res = 0 restores the
    binned results bit for bit; a pose increment agrees in both forms."""
    p = api.Params()
    c, w, q, roi = mesh_case(31, 26, 22, 0.5)
    grid = ctx.grid(p, dev(c))
    wt = dev(w)
    bins = {dt: ctx.eval(p, grid, wt, dev(q, dt)) for dt in (torch.float64, torch.float32)}
    pts, R, t = _pose_points(c, 3001, 4)
    delta = torch.tensor([0.01, -0.02, 0.015, 0.05, -0.03, 0.01], dtype=torch.float64,
                         device="cuda")
    at_bins = ctx.eval_at(p, grid, wt, dev(pts), (R, t), delta)
    grid.set_mesh_roi(roi, 0.5)
    assert grid.mesh is not None
    m64 = ctx.eval(p, grid, wt, dev(q))
    af, _ = abs_sums(q, c, w, p.sigma, p.cutoff)
    assert np.all(np.abs(host(m64["f"]) - host(bins[torch.float64]["f"])) <= 2e-13 * af + 1e-300)
    at_mesh = ctx.eval_at(p, grid, wt, dev(pts), (R, t), delta)
    assert np.abs(host(at_mesh["f"]) - host(at_bins["f"])).max() <= 1e-12
    assert np.abs(host(at_mesh["jac"]) - host(at_bins["jac"])).max() <= 1e-11
    grid.set_mesh(0, 0, 0)
    assert grid.mesh is None
    for dt in (torch.float64, torch.float32):
        again = ctx.eval(p, grid, wt, dev(q, dt))
        assert torch.equal(again["f"], bins[dt]["f"])
        assert torch.equal(again["grad"], bins[dt]["grad"])


def test_set_mesh_refusals(ctx):
    p = api.Params()
    rng = np.random.default_rng(2)
    c, w, q, roi = mesh_case(41, 16, 14, 0.5)
    wt = dev(w)
    # off the mesh: one center moved by 1e-9 m
    bad = c.copy()
    bad[5, 0] += 1e-9
    g = ctx.grid(p, dev(bad))
    before = ctx.eval(p, g, wt, dev(q))
    with pytest.raises(api.RbfError, match="not a node"):
        g.set_mesh_roi(roi, 0.5)
    assert g.mesh is None
    assert torch.equal(ctx.eval(p, g, wt, dev(q))["f"], before["f"])
    # jittered centers
    cj = synth.grid_centers(rng, 10, 10, 0.5, jitter=0.1)
    with pytest.raises(api.RbfError, match="not a node"):
        ctx.grid(p, dev(cj)).set_mesh(0.25, 0.25, 0.5)
    # two centers on one node
    dup = np.concatenate([c, c[3:4]])
    with pytest.raises(api.RbfError, match="same node"):
        ctx.grid(p, dev(dup)).set_mesh_roi(roi, 0.5)
    # a window of 13 nodes (support radius 6 nodes)
    with pytest.raises(api.RbfError, match="nodes per axis"):
        ctx.grid(p, dev(c)).set_mesh_roi(roi, 0.25)
    # the refusals left nothing behind: the same centers take the mesh
    g2 = ctx.grid(p, dev(c)).set_mesh_roi(roi, 0.5)
    assert g2.mesh is not None


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_mesh_gn_and_full_size_odometry(ctx, dt):
    """The odometry map (10k voxel-selected centers: nodes of the 0.5 m
    mesh over the 50 m square) in the mesh form: fused Gauss-Newton sums of
    20k scan points against the oracle's J and r, and 200k scan points in
    the benchmark's launch against the oracle on 2000 sampled points."""
    od = synth.OdometryCase()
    p = api.Params()
    allxy = np.concatenate([od.ground_xy(k) for k in range(od.N_FRAMES)])
    centers = O.select_centers(allxy, od.roi, 0.5, 0.5, 4, O.VOXEL)
    rng = np.random.default_rng(5)
    w = rng.normal(0, 0.3, size=centers.shape[0])
    grid = ctx.grid(p, dev(centers)).set_mesh_roi(od.roi, 0.5)
    pts, R, t = od.scan(12, n=20000)
    f0, g0, r0, J0 = O.eval_pose(pts, R, t, 0.1, centers, w, p.sigma, p.cutoff)
    JtJ0, Jtr0, rtr0 = J0.T @ J0, J0.T @ r0, r0 @ r0
    JtJ, Jtr, rtr = ctx.eval_gn(p, grid, dev(w), dev(pts, dt), pose=(R, t), z_off=0.1)
    JtJ, Jtr, rtr = host(JtJ), host(Jtr), float(rtr)
    tol = 1e-10 if dt == torch.float64 else 2e-4
    scale = np.abs(JtJ0).max()
    assert np.abs(JtJ - JtJ0).max() <= tol * scale
    assert np.array_equal(JtJ, JtJ.T)
    assert np.abs(Jtr - Jtr0).max() <= tol * (np.abs(Jtr0).max() + np.sqrt(scale * rtr0))
    assert abs(rtr - rtr0) <= tol * rtr0
    pts, R, t = od.scan(10)
    idx = rng.choice(pts.shape[0], 2000, replace=False)
    f0, g0, r0, J0 = O.eval_pose(pts[idx], R, t, 0.0, centers, w, p.sigma, p.cutoff)
    out = ctx.eval(p, grid, dev(w), dev(pts, dt), pose=(R, t))
    f = host(out["f"]).astype(np.float64)[idx]
    r = host(out["resid"]).astype(np.float64)[idx]
    if dt == torch.float64:
        assert np.abs(f - f0).max() <= 1e-12
        assert np.abs(r - r0).max() <= 1e-12
    else:
        xi = O.to_world(pts[idx].astype(np.float32).astype(np.float64), R, t)
        ok = ~ambiguous(xi[:, :2], centers, p.sigma, p.cutoff)
        assert np.abs(f - f0)[ok].max() <= 1e-4
