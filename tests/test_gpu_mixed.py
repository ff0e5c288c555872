"""Mixed-precision covariance product (FP32 / split-BF16 operands, FP32
accumulation into the FP64 P) against the FP64 oracle.

Bound (stated target of the mixed path): heights of the fitted terrain within
1e-4 m of the FP64 oracle's at the queries, and the weights error is
reported. P stays exactly symmetric and S stays positive definite."""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import dev, host
from paper_2509_26222_amd import api, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("batch", [128, 1024])
def test_mixed_update_heights(ctx, prec, batch):
    s = synth.small_case(0)
    p = api.Params()
    grid = ctx.grid(p, dev(s.centers))
    N = grid.N
    w = torch.zeros(N, dtype=torch.float64, device="cuda")
    P = torch.eye(N, dtype=torch.float64, device="cuda") * (p.R / p.lam)
    ctx.update(p, grid, w, P, dev(s.xy), dev(s.z), batch=batch, gemm_prec=prec)
    wb, Pb = O.ridge_batch(s.xy, s.z, s.centers, p.sigma, p.cutoff, 0.0, p.lam, p.R)
    f_gpu, _ = O.eval_height_grad(s.queries, s.centers, host(w), p.sigma, p.cutoff)
    f_ref, _ = O.eval_height_grad(s.queries, s.centers, wb, p.sigma, p.cutoff)
    ew = np.linalg.norm(host(w) - wb) / np.linalg.norm(wb)
    ef = np.abs(f_gpu - f_ref).max()
    eP = np.abs(host(P) - Pb).max() / np.abs(Pb).max()
    print(f"{prec} batch {batch}: w rel {ew:.2e}, max |df| {ef:.2e} m, P rel {eP:.2e}")
    assert ef <= 1e-4
    assert torch.equal(P, P.T)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mixed_update_odometry_frame(ctx, prec):
    od = synth.OdometryCase()
    p = api.Params()
    allxy = np.concatenate([od.ground_xy(k) for k in range(od.N_FRAMES)])
    centers = O.select_centers(allxy, od.roi, 0.5, 0.5, 4, O.VOXEL)
    grid = ctx.grid(p, dev(centers))
    N = grid.N
    w = torch.zeros(N, dtype=torch.float64, device="cuda")
    P = torch.eye(N, dtype=torch.float64, device="cuda") * (p.R / p.lam)
    frames = [od.ground(k) for k in (10, 11)]
    for xy, z in frames:
        xs, zs, _ = ctx.sort_points(grid, dev(xy), dev(z))
        ctx.update(p, grid, w, P, xs, zs, batch=1024, gemm_prec=prec)
    xy = np.concatenate([f[0] for f in frames])
    z = np.concatenate([f[1] for f in frames])
    H, b = O.gram(xy, z, centers, p.sigma, p.cutoff, 0.0, p.lam, sparse=True)
    wb = O.spd_solve(H, b)
    q = np.random.default_rng(0).uniform(0, 50, size=(5000, 2))
    f_gpu, _ = O.eval_height_grad(q, centers, host(w), p.sigma, p.cutoff)
    f_ref, _ = O.eval_height_grad(q, centers, wb, p.sigma, p.cutoff)
    ef = np.abs(f_gpu - f_ref).max()
    print(f"{prec} odometry 2 frames: w rel "
          f"{np.linalg.norm(host(w) - wb) / np.linalg.norm(wb):.2e}, max |df| {ef:.2e} m")
    assert ef <= 1e-4
