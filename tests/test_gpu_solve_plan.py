"""rbf_solve_plan (nested dissection with dense fronts + FP64 refinement).

The same bounds as rbf_solve: the returned relative residual, recomputed on
the host in FP64 from the same CSR matrix, must be <= rtol, and the forward
error against the oracle's sparse solve is bounded by cond(calH) * relres.
Covered: one and many right-hand sides, the inverse (P = R calH^{-1}
against the oracle's batch ridge covariance), reuse of a plan with new
values, a disconnected pattern (a front without unknowns at the root), the
40k-center map (against the banded solver too), and errors."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle as O
from helpers import dev, host
from paper_2509_26222_amd import api, synth

pytestmark = pytest.mark.gpu


def csr_dev(H):
    H = sp.csr_matrix(H)
    H.sort_indices()
    return (dev(H.indptr.astype(np.int64)), dev(H.indices.astype(np.int32)),
            dev(H.data.astype(np.float64)))


@pytest.fixture(scope="module")
def small():
    s = synth.small_case(0)
    p = api.Params()
    H, b = O.gram(s.xy, s.z, s.centers, p.sigma, p.cutoff, 0.0, p.lam, sparse=True)
    return s, p, H, b


@pytest.mark.parametrize("leaf", [64, 0])
def test_plan_small_rhs_and_inverse(ctx, small, leaf):
    s, p, H, b = small
    rp, ci, v = csr_dev(H)
    plan = ctx.solve_plan(rp, ci, leaf=leaf)
    info = plan.info()
    assert info["nodes"] >= 1 and info["front_bytes"] > 0
    x, rel, it, st = plan.run(v, dev(b), rtol=1e-12, max_iter=5)
    assert st == 0 and it >= 1 and rel[0] <= 1e-12
    xg = host(x)
    assert O.relres(H, xg, b) <= 1e-12
    xo = O.spd_solve(H, b)
    cond = np.linalg.cond(H.toarray())
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 10 * cond * max(rel[0], 1e-16)
    # the inverse: P = R calH^{-1} is the batch ridge covariance
    N = H.shape[0]
    X, rel, it, st = plan.run(v, dev(np.eye(N)), rtol=1e-11, max_iter=5)
    Xg = host(X)
    assert np.abs(H.toarray() @ Xg - np.eye(N)).max() <= 1e-9
    w, P = O.ridge_batch(s.xy, s.z, s.centers, p.sigma, p.cutoff, 0.0, p.lam, p.R)
    assert np.abs(p.R * Xg - P).max() <= 1e-9 * np.abs(P).max()
    # ragged multi-RHS
    Bm = np.random.default_rng(2).normal(size=(N, 37))
    X, rel, it, st = plan.run(v, dev(Bm), rtol=1e-11, max_iter=5)
    for k in range(37):
        assert O.relres(H, host(X)[:, k], Bm[:, k]) <= 1e-11
    plan.close()


def test_plan_reuse_new_values(ctx, small):
    """One plan, two matrices on the same pattern (the Gram matrix of two
    different point sets), each solved to the bound."""
    s, p, H, b = small
    H2, b2 = O.gram(s.xy[::2] + 0.01, s.z[::2], s.centers, p.sigma, p.cutoff, 0.0, p.lam,
                    sparse=True)
    pat = (H != 0).astype(np.float64) + (H2 != 0).astype(np.float64)
    pat = sp.csr_matrix(pat)
    pat.sort_indices()
    rp, ci = dev(pat.indptr.astype(np.int64)), dev(pat.indices.astype(np.int32))
    plan = ctx.solve_plan(rp, ci, leaf=128)
    rows, cols = pat.nonzero()  # CSR order (indices sorted)
    for Hk, bk in ((H, b), (H2, b2)):
        vals = np.asarray(Hk.tocsr()[rows, cols]).ravel()
        Hp = sp.csr_matrix((vals, pat.indices, pat.indptr), shape=pat.shape)
        x, rel, it, st = plan.run(dev(vals), dev(bk), rtol=1e-12, max_iter=5)
        assert st == 0 and O.relres(Hp, host(x), bk) <= 1e-12
    plan.close()


def test_plan_disconnected(ctx):
    """Two far-apart center clusters: the root front has no unknowns and
    only joins the two components; the solve is exact to the bound."""
    p = api.Params()
    rng = np.random.default_rng(4)
    c = np.concatenate([rng.uniform(0, 12, size=(600, 2)),
                        rng.uniform(0, 12, size=(500, 2)) + np.array([60.0, 0.0])])
    xy = np.concatenate([rng.uniform(0, 12, size=(3000, 2)),
                         rng.uniform(0, 12, size=(3000, 2)) + np.array([60.0, 0.0])])
    z = np.sin(xy[:, 0]) + 0.1 * rng.normal(size=xy.shape[0])
    H, b = O.gram(xy, z, c, p.sigma, p.cutoff, 0.0, p.lam, sparse=True)
    rp, ci, v = csr_dev(H)
    plan = ctx.solve_plan(rp, ci, leaf=128)
    x, rel, it, st = plan.run(v, dev(b), rtol=1e-12, max_iter=5)
    assert st == 0 and O.relres(H, host(x), b) <= 1e-12
    xo = O.spd_solve(H, b)
    assert np.linalg.norm(host(x) - xo) / np.linalg.norm(xo) <= 1e-8
    plan.close()


@pytest.mark.parametrize("inner", ["f64"])
def test_plan_large_grid_40k(ctx, inner):
    """40,000 centers, calH from 800k points assembled on the GPU, solved to
    relres 1e-10; relres recomputed on the host."""
    case = synth.large_case(3)
    p = api.Params()
    grid = ctx.grid(p, dev(case.centers))
    xy, z = synth.large_points(case, 800_000)
    rowptr, colidx = ctx.gram_pattern(p, grid)
    vals, b = ctx.assemble_gram(p, grid, dev(xy), dev(z), rowptr, colidx)
    plan = ctx.solve_plan(rowptr, colidx)
    x, rel, it, st = plan.run(vals, b, rtol=1e-10, max_iter=20, inner=inner)
    assert st == 0
    H = sp.csr_matrix((host(vals), host(colidx), host(rowptr)), shape=(grid.N, grid.N))
    assert O.relres(H, host(x), host(b)) <= 1e-10
    # the banded solver's answer agrees
    xb, relb, _, _ = ctx.solve(rowptr, colidx, vals, b, rtol=1e-12, max_iter=10, inner="f64")
    assert np.linalg.norm(host(x) - host(xb)) / np.linalg.norm(host(xb)) <= 1e-7
    print(f"40k plan ({inner}): {plan.info()}, sweeps {it}, relres {rel[0]:.2e}")
    plan.close()


def test_plan_errors(ctx, small):
    s, p, H, b = small
    rp, ci, v = csr_dev(H)
    plan = ctx.solve_plan(rp, ci, leaf=64)
    x, rel, it, st = plan.run(v, dev(b), rtol=1e-300, max_iter=1)
    assert st == 5 and it == 1  # RBF_E_NO_CONVERGE, result still returned
    with pytest.raises(api.RbfError) as e:
        plan.run(dev(-H.tocsr().sorted_indices().data), dev(b), rtol=1e-10, max_iter=3)
    assert e.value.status == 3
    for inner in ("f32", "bf16"):  # the factor is FP64 only
        with pytest.raises(api.RbfError) as e:
            plan.run(v, dev(b), rtol=1e-10, max_iter=3, inner=inner)
        assert e.value.status == 1
    # the plan still solves after the failures
    x, rel, it, st = plan.run(v, dev(b), rtol=1e-12, max_iter=5)
    assert st == 0 and O.relres(H, host(x), b) <= 1e-12
    plan.close()
    ctx.sync_status()


def test_context_outlives_its_plans(small):
    """A plan uses its context's device and stream until it is destroyed:
    rbf_ctx_destroy refuses while a plan is alive (and destroys nothing),
    Context.close() destroys the context's plans first."""
    s, p, H, b = small
    c = api.Context(0)
    rp, ci, v = csr_dev(H)
    plan = c.solve_plan(rp, ci, leaf=64)
    assert c.lib.rbf_ctx_destroy(c.h) == 1  # RBF_E_INVALID_ARG
    x, rel, it, st = plan.run(v, dev(b), rtol=1e-12, max_iter=5)  # context intact
    assert st == 0 and O.relres(H, host(x), b) <= 1e-12
    c.close()
    assert plan.h is None and c.h is None
