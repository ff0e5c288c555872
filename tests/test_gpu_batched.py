"""Batched form: many patches of uneven size updated and evaluated by one
hipGraph launch, each stage of the recursion one launch over all patches.
The kernels are deterministic (no atomics on this path) and every patch runs
the same kernel bodies on the same arguments as a plain call, so the
batched results must equal the sequential plain calls bit for bit; the
plain calls are themselves parity-tested against the oracle, and two
patches are also checked directly against the oracle here."""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import dev, host
from paper_2509_26222_amd import api, synth

pytestmark = pytest.mark.gpu


def make_patches(ctx, p, count, seed=4, n_range=(200, 1200), m_range=(1000, 5000),
                 nan_patch=None):
    _, raw = synth.patches_case(seed=seed, count=count, n_range=n_range, m_range=m_range)
    out = []
    for i, r in enumerate(raw):
        grid = ctx.grid(p, dev(r.centers))
        N = grid.N
        z = r.z.copy()
        if i == nan_patch:
            z[len(z) // 2] = np.nan
        pts = np.concatenate([r.xy, z[:, None]], 1)
        Q = pts.shape[0]
        out.append(dict(
            grid=grid, raw=r,
            w=torch.zeros(N, dtype=torch.float64, device="cuda"),
            P=torch.eye(N, dtype=torch.float64, device="cuda") * (p.R / p.lam),
            xy=dev(r.xy), z=dev(z),
            pts=dev(pts, torch.float32), pose=(np.eye(3), np.zeros(3)),
            f=torch.empty(Q, dtype=torch.float32, device="cuda"),
            grad=torch.empty((Q, 2), dtype=torch.float32, device="cuda"),
            resid=torch.empty(Q, dtype=torch.float32, device="cuda"),
            jac=torch.empty((Q, 6), dtype=torch.float32, device="cuda"),
            batch=512 if i % 2 else 0))
    return out


def run_sequential(ctx, p, patches, gemm_prec="f64", default_batch=1024):
    for q in patches:
        ctx.update(p, q["grid"], q["w"], q["P"], q["xy"], q["z"],
                   batch=q["batch"] or default_batch, gemm_prec=gemm_prec, sync=False)
        o = ctx.eval(p, q["grid"], q["w"], q["pts"], pose=q["pose"])
        for k in ("f", "grad", "resid", "jac"):
            q[k].copy_(o[k])
    torch.cuda.synchronize()


@pytest.mark.parametrize("tile,chains", [("auto", 1), ("128", 2), ("sub", 4)])
def test_batched_equals_sequential(ctx, tile, chains):
    p = api.Params()
    A = make_patches(ctx, p, 12)
    B = make_patches(ctx, p, 12)
    plan = api.Batched(ctx, p, A, dim=3, eval_prec="f32", gemm_prec="f64", tile=tile,
                       chains=chains)
    for rep in range(2):  # capture, then replay on the updated state
        plan.run()
        assert plan.sync() == -1
        run_sequential(ctx, p, B)
        for a, b in zip(A, B):
            for k in ("w", "P", "f", "grad", "resid", "jac"):
                assert torch.equal(a[k], b[k]), (rep, k)
    plan.close()
    # direct oracle check of two patches after the first run's state: redo one run
    C = make_patches(ctx, p, 12)
    plan = api.Batched(ctx, p, C, dim=3, eval_prec="f32", gemm_prec="f64", tile=tile,
                       chains=chains)
    plan.run()
    plan.sync()
    for q in (C[0], C[7]):
        r = q["raw"]
        wb, _ = O.ridge_batch(r.xy, r.z, r.centers, p.sigma, p.cutoff, 0.0, p.lam, p.R,
                              with_P=False)
        assert np.linalg.norm(host(q["w"]) - wb) / np.linalg.norm(wb) <= 1e-9
    plan.close()


@pytest.mark.parametrize("gemm_prec", ["f32", "bf16"])
def test_batched_mixed_products_equal_sequential(ctx, gemm_prec):
    """The FP32 and split-BF16 covariance products, batched across patches,
    against the plain calls with the same products (bit for bit)."""
    p = api.Params()
    A = make_patches(ctx, p, 10, seed=6)
    B = make_patches(ctx, p, 10, seed=6)
    plan = api.Batched(ctx, p, A, dim=3, eval_prec="f32", gemm_prec=gemm_prec)
    plan.run()
    assert plan.sync() == -1
    plan.close()
    run_sequential(ctx, p, B, gemm_prec=gemm_prec)
    for a, b in zip(A, B):
        for k in ("w", "P", "f", "grad", "resid", "jac"):
            assert torch.equal(a[k], b[k]), k


def test_grid_fixed_while_a_plan_evaluates_on_it(ctx):
    """A batched plan's captured launches keep its grids' tables: while the
    plan exists a grid's form cannot change and the grid is not destroyed
    (both refused, nothing changed); after the plan is closed both work."""
    p = api.Params()
    A = make_patches(ctx, p, 2)
    plan = api.Batched(ctx, p, A, dim=3)
    g = A[0]["grid"]
    with pytest.raises(api.RbfError, match="batched plan"):
        g.set_mesh(0.25, 0.25, 0.5)
    assert g.mesh is None
    h = g.h
    g.close()  # refused: the handle stays
    assert g.h is h
    plan.run()
    assert plan.sync() == -1
    plan.close()
    g.set_mesh(0, 0, 0)  # allowed again (already binned: no change)
    g.close()
    assert g.h is None
    ctx.sync_status()


def test_batched_reports_failed_patch(ctx):
    """A non-finite height in patch 5 stops patch 5 at its failing batch;
    every other patch completes as its plain calls do."""
    p = api.Params()
    A = make_patches(ctx, p, 8, nan_patch=5)
    plan = api.Batched(ctx, p, A, dim=3, chains=3)
    plan.run()
    with pytest.raises(api.RbfError) as e:
        plan.sync()
    assert e.value.status == 4 and e.value.index == 5
    B = make_patches(ctx, p, 8, nan_patch=5)
    run_sequential(ctx, p, [q for i, q in enumerate(B) if i != 5])
    for i in range(8):
        if i != 5:
            assert torch.equal(A[i]["w"], B[i]["w"]) and torch.equal(A[i]["P"], B[i]["P"]), i
    # the failed patch kept the state of the batches before the failing one
    q = B[5]
    M = q["xy"].shape[0]
    bad = (M // 2) // 512 * 512  # batch 512 (odd index): start of the failing batch
    ctx.update(p, q["grid"], q["w"], q["P"], q["xy"][:bad], q["z"][:bad], batch=512)
    assert torch.equal(A[5]["w"], q["w"]) and torch.equal(A[5]["P"], q["P"])
    plan.close()
    ctx.sync_status()


def test_batched_full_size_patches(ctx):
    """Eight patches of the full 256-patch workload (centers up to 8000, scans
    up to 40k points): its four costliest (N_p^2 M_p) and four drawn at
    random, batched against the sequential plain calls bit for bit, and the largest and one random patch against the oracle's
    sparse batch ridge solution (weights within 1e-9)."""
    p = api.Params()
    _, sizes = synth.patches_case(seed=4, count=256, only=set())
    cost = np.array([r.centers.shape[0] ** 2 * r.xy.shape[0] for r in sizes])
    rng = np.random.default_rng(11)
    top = list(np.argsort(cost)[-4:])
    rest = [i for i in range(256) if i not in top]
    sel = sorted(top + list(rng.choice(rest, 4, replace=False)))
    _, raw = synth.patches_case(seed=4, count=256, only=set(sel))
    assert max(raw[i].centers.shape[0] for i in sel) > 7000
    assert max(raw[i].xy.shape[0] for i in sel) > 30000

    def build():
        out = []
        for i in sel:
            r = raw[i]
            grid = ctx.grid(p, dev(r.centers))
            N = grid.N
            xs, zs, _ = ctx.sort_points(grid, dev(r.xy), dev(r.z))
            pts = torch.cat([xs, zs[:, None]], 1).float().contiguous()
            Q = pts.shape[0]
            out.append(dict(
                grid=grid, raw=r, w=torch.zeros(N, dtype=torch.float64, device="cuda"),
                P=torch.eye(N, dtype=torch.float64, device="cuda") * (p.R / p.lam),
                xy=xs, z=zs, pts=pts, pose=(np.eye(3), np.zeros(3)),
                f=torch.empty(Q, dtype=torch.float32, device="cuda"),
                grad=torch.empty((Q, 2), dtype=torch.float32, device="cuda"),
                resid=torch.empty(Q, dtype=torch.float32, device="cuda"),
                jac=torch.empty((Q, 6), dtype=torch.float32, device="cuda"), batch=0))
        return out

    A = build()
    plan = api.Batched(ctx, p, A, dim=3, eval_prec="f32", gemm_prec="f64", tile="auto",
                       default_batch=1024)
    plan.run()
    assert plan.sync() == -1
    plan.close()
    B = build()
    run_sequential(ctx, p, B, default_batch=1024)
    for a, b in zip(A, B):
        for k in ("w", "P", "f", "grad", "resid", "jac"):
            assert torch.equal(a[k], b[k]), k
    largest = int(np.argmax([cost[i] for i in sel]))
    drawn = next(j for j, i in enumerate(sel) if i not in top)
    for j in (largest, drawn):
        r = A[j]["raw"]
        wb, _ = O.ridge_batch(r.xy, r.z, r.centers, p.sigma, p.cutoff, 0.0, p.lam, p.R,
                              sparse=True, with_P=False)
        err = np.linalg.norm(host(A[j]["w"]) - wb) / np.linalg.norm(wb)
        print(f"patch {sel[j]}: N {r.centers.shape[0]}, M {r.xy.shape[0]}, w rel {err:.2e}")
        assert err <= 1e-9
    del A, B
    torch.cuda.empty_cache()
    ctx.sync_status()
