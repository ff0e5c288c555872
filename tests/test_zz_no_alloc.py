"""rbf_eval_noalloc (the evaluation entry point that allocates no device
memory, for callers that cannot allocate) against rbf_eval: same kernels,
so the outputs must be bitwise equal. Two calls in a row on one context,
the second on a smaller center set and fewer points, in FP64 and FP32, in
the world-xy and the pose form, with the binned and the mesh form of the
evaluation; a grid above the stated maximum is refused before any launch."""
import numpy as np
import pytest
import torch

from paper_2509_26222_amd import api, synth

pytestmark = pytest.mark.gpu


def _case(seed, nx, ny, q, mesh=False):
    rng = np.random.default_rng(seed)
    centers = synth.grid_centers(rng, nx, ny, 0.5, jitter=0.0 if mesh else 0.1)
    w = rng.normal(0.0, 0.3, centers.shape[0])
    lo = centers.min(0) - 1.0
    hi = centers.max(0) + 1.0
    xy = rng.uniform(lo, hi, size=(q, 2))
    z = rng.normal(0.0, 0.05, q)
    return centers, w, xy, z


def _outputs(ctx, p, grid, w, pts, pose, noalloc):
    out = ctx.eval(p, grid, w, pts, pose=pose, noalloc=noalloc)
    torch.cuda.synchronize()
    return {k: v.cpu() for k, v in out.items() if v is not None}


@pytest.mark.parametrize("mesh", [False, True])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("form", ["xy", "pose"])
def test_noalloc_matches_rbf_eval_two_calls(dtype, form, mesh):
    d = torch.device("cuda:0")
    p = api.Params()
    ctx = api.Context(0)
    R = synth.rot_zyx(0.4, 0.03, -0.02)
    # first call: 100 x 90 centers, 70,001 points; second: 23 x 31, 3,001
    for seed, nx, ny, q in ((11, 100, 90, 70_001), (12, 23, 31, 3_001)):
        centers, w_np, xy, z = _case(seed, nx, ny, q, mesh)
        grid = ctx.grid(p, torch.from_numpy(centers).to(d))
        if mesh:  # nodes (i + 1/2) 0.5: the mesh form of the evaluation
            grid.set_mesh(0.25, 0.25, 0.5)
        w = torch.from_numpy(w_np).to(d)
        if form == "xy":
            pts = torch.from_numpy(xy).to(d).to(dtype).contiguous()
            pose = None
        else:
            t = np.array([xy[:, 0].mean(), xy[:, 1].mean(), 0.6])
            world = np.concatenate([xy, z[:, None]], 1)
            pts = torch.from_numpy((world - t) @ R).to(d).to(dtype).contiguous()
            pose = (R, t)
        print(f"noalloc case: {form} {dtype} mesh={mesh} N={grid.N} Q={q}", flush=True)
        ref = _outputs(ctx, p, grid, w, pts, pose, noalloc=False)
        got = _outputs(ctx, p, grid, w, pts, pose, noalloc=True)
        assert set(got) == set(ref)
        for k in ref:
            assert torch.equal(got[k], ref[k]), k
        # the plain entry point is unaffected by a no-alloc call before it
        again = _outputs(ctx, p, grid, w, pts, pose, noalloc=False)
        for k in ref:
            assert torch.equal(again[k], ref[k]), k
        ctx.sync_status()
        grid.close()
    ctx.close()


def test_noalloc_refuses_grid_above_maximum():
    d = torch.device("cuda:0")
    p = api.Params()
    ctx = api.Context(0)
    n_side = int(np.ceil(np.sqrt(131072 + 1)))
    rng = np.random.default_rng(5)
    centers = synth.grid_centers(rng, n_side, n_side, 0.5)
    assert centers.shape[0] > 131072
    grid = ctx.grid(p, torch.from_numpy(centers).to(d))
    w = torch.zeros(grid.N, dtype=torch.float64, device=d)
    pts = torch.zeros((16, 2), dtype=torch.float64, device=d)
    with pytest.raises(api.RbfError) as e:
        ctx.eval(p, grid, w, pts, noalloc=True)
    assert e.value.status == 6  # RBF_E_CAPACITY
    assert "maximum" in str(e.value)
    # the plain entry point still evaluates the same grid
    out = ctx.eval(p, grid, w, pts)
    torch.cuda.synchronize()
    assert torch.all(out["f"] == 0)
    ctx.sync_status()
    grid.close()
    ctx.close()
