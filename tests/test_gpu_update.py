"""rbf_update (recursive Kalman-form ridge update) against the FP64 oracle.

The FP64 target for weights is ||w_gpu - w|| / ||w|| <= 1e-9. P is compared
elementwise against R calH^{-1} with the same relative bound, scaled by the
largest entry of P; it must also be exactly symmetric.
"""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import dev, host
from paper_2509_26222_amd import api, synth

pytestmark = pytest.mark.gpu

TOL_W = 1e-9


def _state(N, p):
    w = torch.zeros(N, dtype=torch.float64, device="cuda")
    P = torch.eye(N, dtype=torch.float64, device="cuda") * (p.R / p.lam)
    return w, P


@pytest.fixture(scope="module")
def small(ctx):
    s = synth.small_case(0)
    p = api.Params()
    grid = ctx.grid(p, dev(s.centers))
    wb, Pb = O.ridge_batch(s.xy, s.z, s.centers, p.sigma, p.cutoff, 0.0, p.lam, p.R)
    return s, p, grid, wb, Pb


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("batch", [1, 7, 64, 65, 150, 200, 300, 1024, 2000, 0])
def test_update_chain_equals_batch_ridge(ctx, small, batch):
    s, p, grid, wb, Pb = small
    xy, z = s.xy, s.z
    if batch == 1:  # keep the 1-point chain short
        xy, z = xy[:150], z[:150]
        wb, Pb = O.ridge_batch(xy, z, s.centers, p.sigma, p.cutoff, 0.0, p.lam, p.R)
    w, P = _state(grid.N, p)
    nd = ctx.update(p, grid, w, P, dev(xy), dev(z), batch=batch)
    assert nd == xy.shape[0]
    wg, Pg = host(w), host(P)
    print(f"batch {batch}: w rel {_rel(wg, wb):.2e}, P rel {np.abs(Pg - Pb).max() / np.abs(Pb).max():.2e}")
    assert _rel(wg, wb) <= TOL_W
    assert np.abs(Pg - Pb).max() <= TOL_W * np.abs(Pb).max()
    assert np.array_equal(Pg, Pg.T)


def test_update_matches_oracle_recursion_and_sorted_order(ctx, small):
    s, p, grid, wb, Pb = small
    w, P = _state(grid.N, p)
    xs, zs, perm = ctx.sort_points(grid, dev(s.xy), dev(s.z))
    ctx.update(p, grid, w, P, xs, zs, batch=300)
    w0, P0 = O.initial_state(grid.N, p.lam, p.R)
    pm = host(perm)
    wk, Pk = O.kalman_update(w0, P0, s.xy[pm], s.z[pm], s.centers, p.sigma, p.cutoff, 0.0,
                             p.R, batch=300)
    assert _rel(host(w), wk) <= TOL_W
    assert np.abs(host(P) - Pk).max() <= TOL_W * np.abs(Pk).max()


def test_update_two_calls_equal_one(ctx, small):
    s, p, grid, wb, Pb = small
    w, P = _state(grid.N, p)
    ctx.update(p, grid, w, P, dev(s.xy[:900]), dev(s.z[:900]), batch=256)
    ctx.update(p, grid, w, P, dev(s.xy[900:]), dev(s.z[900:]), batch=256)
    assert _rel(host(w), wb) <= TOL_W


def test_update_moment_regressor(ctx):
    s = synth.small_case(1)
    p = api.Params(sigma_eps=0.1)
    grid = ctx.grid(p, dev(s.centers))
    w, P = _state(grid.N, p)
    ctx.update(p, grid, w, P, dev(s.xy), dev(s.z), batch=512)
    wb, Pb = O.ridge_batch(s.xy, s.z, s.centers, p.sigma, p.cutoff, p.sigma_eps, p.lam, p.R)
    assert _rel(host(w), wb) <= TOL_W
    assert np.abs(host(P) - Pb).max() <= TOL_W * np.abs(Pb).max()


def test_update_nonfinite_commits_earlier_batches(ctx, small):
    s, p, grid, wb, Pb = small
    B = 256
    z = s.z.copy()
    z[3 * B + 17] = np.nan
    w, P = _state(grid.N, p)
    with pytest.raises(api.RbfError) as e:
        ctx.update(p, grid, w, P, dev(s.xy), dev(z), batch=B)
    assert e.value.status == 4
    assert e.value.index == 3
    w3, P3 = O.ridge_batch(s.xy[:3 * B], s.z[:3 * B], s.centers, p.sigma, p.cutoff, 0.0,
                           p.lam, p.R)
    assert _rel(host(w), w3) <= TOL_W
    assert np.abs(host(P) - P3).max() <= TOL_W * np.abs(P3).max()
    ctx.sync_status()  # cleared


def test_update_not_spd_leaves_state(ctx, small):
    s, p, grid, wb, Pb = small
    w = torch.zeros(grid.N, dtype=torch.float64, device="cuda")
    P = -torch.eye(grid.N, dtype=torch.float64, device="cuda") * (p.R / p.lam)
    P0 = P.clone()
    with pytest.raises(api.RbfError) as e:
        ctx.update(p, grid, w, P, dev(s.xy), dev(s.z), batch=128)
    assert e.value.status == 3 and e.value.index == 0
    assert torch.equal(P, P0) and torch.count_nonzero(w) == 0


def test_update_empty(ctx, small):
    s, p, grid, wb, Pb = small
    w, P = _state(grid.N, p)
    e = torch.zeros((0, 2), dtype=torch.float64, device="cuda")
    assert ctx.update(p, grid, w, P, e, torch.zeros(0, dtype=torch.float64, device="cuda")) == 0


def test_update_full_size_odometry_frame(ctx):
    """One 20k-point frame on 10k centers with dense P (800 MB), batch 1024:
    w vs the batch ridge solution (sparse LU) and 32 sampled columns of P vs
    R calH^{-1} e_j."""
    od = synth.OdometryCase()
    p = api.Params()
    allxy = np.concatenate([od.ground_xy(k) for k in range(od.N_FRAMES)])
    centers = O.select_centers(allxy, od.roi, 0.5, 0.5, 4, O.VOXEL)
    grid = ctx.grid(p, dev(centers))
    xy, z = od.ground(10)
    w, P = _state(grid.N, p)
    xs, zs, _ = ctx.sort_points(grid, dev(xy), dev(z))
    nd = ctx.update(p, grid, w, P, xs, zs, batch=1024)
    assert nd == xy.shape[0]
    H, b = O.gram(xy, z, centers, p.sigma, p.cutoff, 0.0, p.lam, sparse=True)
    wb = O.spd_solve(H, b)
    assert _rel(host(w), wb) <= TOL_W
    rng = np.random.default_rng(0)
    cols = rng.choice(grid.N, 32, replace=False)
    E = np.zeros((grid.N, 32))
    E[cols, np.arange(32)] = 1.0
    Pc = p.R * O.spd_solve(H, E)
    Pg = host(P[:, torch.as_tensor(cols, device="cuda")])
    assert np.abs(Pg - Pc).max() <= TOL_W * (p.R / p.lam)
    assert torch.equal(P, P.T)


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_update_two_streams_bitwise_equal(ctx, small, prec):
    """The two-stream schedule (next batch's chain beside the split
    covariance product) computes the same arithmetic in the same order."""
    s, p, grid, wb, Pb = small
    out = []
    for streams in (1, 2):
        ctx.set_update_streams(streams)
        try:
            w, P = _state(grid.N, p)
            ctx.update(p, grid, w, P, dev(s.xy), dev(s.z), batch=128, gemm_prec=prec)
            out.append((w, P))
        finally:
            ctx.set_update_streams(1)
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])


def test_update_two_streams_failure_commits_earlier_batches(ctx, small):
    """A failure in batch k+1's chain (on the second stream) must not cut
    short batch k's covariance product running beside it."""
    s, p, grid, wb, Pb = small
    B = 128
    z = s.z.copy()
    z[5 * B + 3] = np.inf
    ctx.set_update_streams(2)
    try:
        w, P = _state(grid.N, p)
        with pytest.raises(api.RbfError) as e:
            ctx.update(p, grid, w, P, dev(s.xy), dev(z), batch=B)
    finally:
        ctx.set_update_streams(1)
    assert e.value.status == 4 and e.value.index == 5
    w5, P5 = O.ridge_batch(s.xy[:5 * B], s.z[:5 * B], s.centers, p.sigma, p.cutoff, 0.0,
                           p.lam, p.R)
    assert _rel(host(w), w5) <= TOL_W
    assert np.abs(host(P) - P5).max() <= TOL_W * np.abs(P5).max()
    ctx.sync_status()


def test_update_unsorted_and_sorted_points_large_grid(ctx):
    """2,500 centers (25 x 25 m at 0.5 m) and 3,000 points: in their given
    (random) order each 64-point group touches many more rows of P than the
    grouped gather takes, so U = P H^T and S come from the per-point kernels;
    in bin order they come from the grouped MFMA products. Both against the
    oracle's batch ridge solution."""
    s = synth.small_case(7, n_points=3000, n_queries=10, side=25.0, spacing=0.5)
    p = api.Params()
    grid = ctx.grid(p, dev(s.centers))
    assert grid.N == 2500
    wb, Pb = O.ridge_batch(s.xy, s.z, s.centers, p.sigma, p.cutoff, 0.0, p.lam, p.R)
    for sort in (False, True):
        w, P = _state(grid.N, p)
        xy, z = dev(s.xy), dev(s.z)
        if sort:
            xy, z, _ = ctx.sort_points(grid, xy, z)
        ctx.update(p, grid, w, P, xy, z, batch=1024)
        assert _rel(host(w), wb) <= TOL_W, sort
        assert np.abs(host(P) - Pb).max() <= TOL_W * np.abs(Pb).max(), sort
        assert torch.equal(P, P.T)


def test_update_with_pending_error_absorbs_nothing(ctx, small):
    """A device error left pending by an earlier asynchronous call (here a
    capacity error of the regressor rows, kmax too small) makes every batch
    of the next update skip: the synchronous call returns that error, w and
    P are unchanged, and the following update runs normally."""
    s, p, grid, wb, Pb = small
    ctx.sync_status()
    ctx.assemble_phi(p, grid, dev(s.xy[:50]), kmax=2)  # records RBF_E_CAPACITY
    w, P = _state(grid.N, p)
    w0, P0 = w.clone(), P.clone()
    with pytest.raises(api.RbfError) as e:
        ctx.update(p, grid, w, P, dev(s.xy), dev(s.z), batch=256)
    assert e.value.status == 6  # RBF_E_CAPACITY, from the earlier call
    assert torch.equal(w, w0) and torch.equal(P, P0)
    assert ctx.update(p, grid, w, P, dev(s.xy), dev(s.z), batch=256) == s.xy.shape[0]
    assert _rel(host(w), wb) <= TOL_W


def test_two_stream_update_refused_under_capture(small):
    """The two-stream schedule is not captured into graphs: on a capturing
    stream rbf_update returns RBF_E_INVALID_ARG before enqueuing anything,
    and (w, P) are untouched; the one-stream schedule is unaffected."""
    s, p, grid, wb, Pb = small
    side = torch.cuda.Stream()
    c2 = api.Context(0, stream=side)
    c2.set_update_streams(2)
    w, P = _state(grid.N, p)
    w0, P0 = w.clone(), P.clone()
    xy, z = dev(s.xy), dev(s.z)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        with pytest.raises(api.RbfError) as e:
            c2.update(p, grid, w, P, xy, z, batch=256, sync=False)
    assert e.value.status == 1  # RBF_E_INVALID_ARG
    torch.cuda.synchronize()
    assert torch.equal(w, w0) and torch.equal(P, P0)
    c2.set_update_streams(1)
    with torch.cuda.stream(side):
        assert c2.update(p, grid, w, P, xy, z, batch=256) == s.xy.shape[0]
    torch.cuda.synchronize()
    assert _rel(host(w), wb) <= TOL_W
    c2.close()
