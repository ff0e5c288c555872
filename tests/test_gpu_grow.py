"""Growing center set: rbf_select_centers_grow (running counts, new
centers per frame) bit for bit against the oracle's select_centers_grow,
rbf_state_grow exactly, and the grown recursion (dense and active-rows)
against the oracle's chain to the FP64 bound (||dw|| / ||w|| <= 1e-9,
max |dP| <= 1e-9 max |P|). The deviation of the grown map from one with all
centers present from the start is printed (a measured property)."""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import dev, host
from paper_2509_26222_amd import _lib as L
from paper_2509_26222_amd import api, synth

pytestmark = pytest.mark.gpu

TOL = 1e-9
MODES = {O.RADIUS: L.SELECT_RADIUS, O.VOXEL: L.SELECT_VOXEL}


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("mode,r_kd,thr", [(O.RADIUS, 0.5, 4), (O.VOXEL, 0.5, 4),
                                           (O.RADIUS, 1.3, 40)])
def test_select_grow_matches_oracle(ctx, mode, r_kd, thr):
    od = synth.OdometryCase()
    G, nx, ny = O.candidate_mesh(od.roi, 0.5)
    counts_o = np.zeros(nx * ny, dtype=np.int64)
    counts_g = torch.zeros(nx * ny, dtype=torch.int32, device="cuda")
    sizes = []
    for k in (0, 1, 2, 40):
        xy = od.ground_xy(k)
        new_g = ctx.select_centers_grow(dev(xy), od.roi, 0.5, r_kd, thr, counts_g,
                                        mode=MODES[mode])
        counts_o, new_o = O.select_centers_grow(counts_o, xy, od.roi, 0.5, r_kd, thr, mode)
        assert np.array_equal(host(new_g), new_o)
        assert np.array_equal(host(counts_g).astype(np.int64), counts_o)
        sizes.append(new_o.shape[0])
    print(f"grow mode {mode} r_kd {r_kd} thr {thr}: new centers per frame {sizes}")
    assert sizes[0] > 0 and sizes[-1] > 0


def test_select_grow_capacity_leaves_counts(ctx):
    od = synth.OdometryCase()
    _, nx, ny = O.candidate_mesh(od.roi, 0.5)
    counts = torch.zeros(nx * ny, dtype=torch.int32, device="cuda")
    xy = dev(od.ground_xy(0))
    with pytest.raises(api.RbfError) as e:
        ctx.select_centers_grow(xy, od.roi, 0.5, 0.5, 4, counts, cap=10)
    assert e.value.status == 6  # RBF_E_CAPACITY
    assert int(counts.abs().sum()) == 0
    ctx.sync_status()
    new = ctx.select_centers_grow(xy, od.roi, 0.5, 0.5, 4, counts)
    assert new.shape[0] > 10
    assert ctx.select_centers_grow(xy[:0], od.roi, 0.5, 0.5, 4, counts).shape[0] == 0


def test_state_grow_exact(ctx):
    p = api.Params()
    cap = 300
    rng = np.random.default_rng(0)
    A = rng.normal(size=(cap, cap))
    Pc = dev(A @ A.T)
    wc = dev(rng.normal(size=cap))
    P0, w0 = host(Pc).copy(), host(wc).copy()
    ctx.state_grow(p, wc, Pc, 130, 257)
    P1, w1 = host(Pc), host(wc)
    pr = p.R / p.lam
    assert np.array_equal(P1[:130, :130], P0[:130, :130])
    assert not P1[:130, 130:257].any() and not P1[130:257, :130].any()
    assert np.array_equal(P1[130:257, 130:257], pr * np.eye(127))
    assert np.array_equal(P1[:, 257:], P0[:, 257:]) and np.array_equal(P1[257:], P0[257:])
    assert np.array_equal(w1[:130], w0[:130]) and not w1[130:257].any()
    assert np.array_equal(w1[257:], w0[257:])
    ctx.state_grow(p, wc, Pc, 257, 257)  # nothing to do
    with pytest.raises(api.RbfError):
        ctx.state_grow(p, wc, Pc, 200, 100)


def _path(s, n=6, seed=5):
    rng = np.random.default_rng(seed)
    frames = []
    for k in range(n):
        ctr = (1.5 + 1.4 * k, 5.0 + 1.5 * np.sin(k))
        r = 2.2 * np.sqrt(rng.uniform(0, 1, 1500))
        t = rng.uniform(0, 2 * np.pi, 1500)
        xy = np.clip(np.stack([ctr[0] + r * np.cos(t), ctr[1] + r * np.sin(t)], 1), 0, 9.99)
        frames.append((xy, s.terrain.height(xy) + rng.normal(0, 0.02, 1500)))
    return frames


@pytest.mark.parametrize("active", [False, True])
def test_grown_chain_matches_oracle(ctx, active):
    s = synth.small_case(0)
    p = api.Params()
    roi = (0.0, 0.0, 10.0, 10.0)
    frames = _path(s)
    _, nx, ny = O.candidate_mesh(roi, 0.5)
    cap = nx * ny
    counts = torch.zeros(cap, dtype=torch.int32, device="cuda")
    wc = torch.zeros(cap, dtype=torch.float64, device="cuda")
    Pc = torch.zeros((cap, cap), dtype=torch.float64, device="cuda")
    centers = torch.zeros((0, 2), dtype=torch.float64, device="cuda")
    counts_o = np.zeros(cap, dtype=np.int64)
    c_o = np.zeros((0, 2))
    w_o, P_o = np.zeros(0), np.zeros((0, 0))
    Ns = []
    for xy, z in frames:
        new = ctx.select_centers_grow(dev(xy), roi, 0.5, 0.5, 6, counts)
        n_old = centers.shape[0]
        centers = torch.cat([centers, new]).contiguous()
        N = centers.shape[0]
        ctx.state_grow(p, wc, Pc, n_old, N)
        grid = ctx.grid(p, centers)
        w, P = wc[:N], Pc[:N, :N]
        if active:
            ctx.update_active(p, grid, w, P, dev(xy), dev(z), batch=512)
        else:
            ctx.update(p, grid, w, P, dev(xy), dev(z), batch=512)
        counts_o, new_o = O.select_centers_grow(counts_o, xy, roi, 0.5, 0.5, 6, O.RADIUS)
        w_o, P_o = O.grow_state(w_o, P_o, new_o.shape[0], p.lam, p.R)
        c_o = np.concatenate([c_o, new_o])
        if active:
            w_o, P_o, _ = O.kalman_update_active(w_o, P_o, xy, z, c_o, p.sigma, p.cutoff, 0.0,
                                                 p.R, batch=512)
        else:
            w_o, P_o = O.kalman_update(w_o, P_o, xy, z, c_o, p.sigma, p.cutoff, 0.0, p.R,
                                       batch=512)
        Ns.append(N)
    assert np.array_equal(host(centers), c_o)
    N = centers.shape[0]
    assert _rel(host(wc[:N]), w_o) <= TOL
    assert np.abs(host(Pc[:N, :N]) - P_o).max() <= TOL * np.abs(P_o).max()
    assert len(set(Ns)) >= 4  # the set really grew
    print(f"grown chain ({'active rows' if active else 'dense'}): centers per frame {Ns}")


def test_grown_vs_all_centers_odometry(ctx):
    """Eight odometry frames: centers grown frame by frame against the
    same frames absorbed with the final center set present from the start;
    heights at the last frame's points (printed). Points absorbed before a
    center existed do not inform it, so the two differ near the edges of
    earlier frames."""
    od = synth.OdometryCase()
    p = api.Params()
    _, nx, ny = O.candidate_mesh(od.roi, 0.5)
    cap = nx * ny
    counts = torch.zeros(cap, dtype=torch.int32, device="cuda")
    wc = torch.zeros(cap, dtype=torch.float64, device="cuda")
    Pc = torch.zeros((cap, cap), dtype=torch.float64, device="cuda")
    centers = torch.zeros((0, 2), dtype=torch.float64, device="cuda")
    frames = [od.ground(k) for k in range(8)]
    for xy, z in frames:
        new = ctx.select_centers_grow(dev(xy), od.roi, 0.5, 0.5, 4, counts, mode=L.SELECT_VOXEL)
        n_old = centers.shape[0]
        centers = torch.cat([centers, new]).contiguous()
        N = centers.shape[0]
        ctx.state_grow(p, wc, Pc, n_old, N)
        grid = ctx.grid(p, centers)
        xs, zs, _ = ctx.sort_points(grid, dev(xy), dev(z))
        ctx.update(p, grid, wc[:N], Pc[:N, :N], xs, zs, batch=1024)
    N = centers.shape[0]
    grid = ctx.grid(p, centers)
    wf = torch.zeros(N, dtype=torch.float64, device="cuda")
    Pf = Pc[:N, :N]
    Pf.zero_()
    Pf.diagonal().fill_(p.R / p.lam)
    for xy, z in frames:
        xs, zs, _ = ctx.sort_points(grid, dev(xy), dev(z))
        ctx.update(p, grid, wf, Pf, xs, zs, batch=1024)
    xy_last = dev(frames[-1][0])
    dh = (ctx.eval(p, grid, wc[:N], xy_last)["f"] - ctx.eval(p, grid, wf, xy_last)["f"]).abs()
    print(f"grown vs all centers from the start, 8 odometry frames, {N} centers: heights at "
          f"the last frame's points max dev {float(dh.max()):.2e} m, mean "
          f"{float(dh.mean()):.2e} m, w rel dev {_rel(host(wc[:N]), host(wf)):.2e}")
    assert bool(torch.isfinite(dh).all())
