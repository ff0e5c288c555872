"""Pins of the FP64 oracle against facts that do not come from the oracle:
closed forms, invariants, special cases, finite differences and independent
library routines (scipy cKDTree, least squares via SVD, sparse LU)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp
from scipy.spatial import cKDTree

import oracle as O
from paper_2509_26222_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
SIG, CUT, LAM, RV = 0.5, 3.0, 1e-3, 4e-4


def small(seed=0, M=600, side=4.0):
    rng = np.random.default_rng(seed)
    c = synth.grid_centers(rng, int(side / 0.5), int(side / 0.5), 0.5)
    x = rng.uniform(0, side, size=(M, 2))
    z = np.sin(x[:, 0]) * 0.2 + 0.1 * np.cos(2 * x[:, 1]) + rng.normal(0, 0.02, M)
    return c, x, z


# ---------------------------------------------------------------- kernel

def test_kernel_special_values_fixture():
    rows = np.loadtxt(os.path.join(GOLD, "kernel_special_values.txt"))
    c = np.zeros((1, 2))
    for d_over_s, phi in rows:
        x = np.array([[d_over_s * SIG * 0.6, d_over_s * SIG * 0.8]])
        got = O.phi_dense(x, c, SIG, CUT)[0, 0]
        assert got == pytest.approx(phi, rel=1e-15, abs=0)


def test_kernel_cutoff_is_hard_and_inclusive():
    c = np.zeros((1, 2))
    rc = CUT * SIG
    assert O.phi_dense(np.array([[rc, 0.0]]), c, SIG, CUT)[0, 0] == \
        pytest.approx(math.exp(-4.5), rel=1e-15)
    assert O.phi_dense(np.array([[rc * (1 + 1e-9), 0.0]]), c, SIG, CUT)[0, 0] == 0.0
    # the regressor truncates at cutoff * sigma_t (sigma_t > sigma)
    se = 0.3
    s_m, st = O.regressor_scale(SIG, se)
    x_in = np.array([[CUT * st * (1 - 1e-9), 0.0]])
    assert O.regressor_dense(x_in, c, SIG, CUT, se)[0, 0] > 0.0
    x_out = np.array([[CUT * st * (1 + 1e-9), 0.0]])
    assert O.regressor_dense(x_out, c, SIG, CUT, se)[0, 0] == 0.0
    assert O.regressor_dense(np.zeros((1, 2)), c, SIG, CUT, se)[0, 0] == \
        pytest.approx(SIG ** 2 / (SIG ** 2 + se ** 2), rel=1e-15)


def test_regressor_reduces_to_kernel_without_xy_noise():
    c, x, _ = small()
    assert np.array_equal(O.regressor_dense(x, c, SIG, CUT, 0.0),
                          O.phi_dense(x, c, SIG, CUT))


def test_moment_identity_monte_carlo():
    """m(x) = E[phi(xbar) | x] with xbar = x - eps, eps ~ N(0, se^2 I):
    Monte Carlo of the conditional expectation vs the closed form
    (sigma^2/sigma_t^2) kappa_{sigma_t} (untruncated: cutoff 50)."""
    rng = np.random.default_rng(7)
    se = 0.1
    c = np.array([[0.2, -0.1]])
    n = 2_000_000
    for x in ([0.0, 0.0], [0.45, 0.3], [0.9, -0.6]):
        x = np.array([x])
        eps = rng.normal(0.0, se, size=(n, 2))
        samples = O.phi_dense(x - eps, c, SIG, 50.0)[:, 0]
        mc = samples.mean()
        se_mc = samples.std() / math.sqrt(n)
        exact = O.regressor_dense(x, c, SIG, 50.0, se)[0, 0]
        assert abs(mc - exact) < 5 * se_mc + 1e-12


# ------------------------------------------------------- center selection

@pytest.mark.parametrize("r_kd,thr", [(0.5, 4), (0.8, 10), (0.35, 0)])
def test_select_radius_matches_kdtree(r_kd, thr):
    rng = np.random.default_rng(11)
    xy = rng.uniform(-0.3, 7.3, size=(3000, 2))
    xy[:500] = rng.normal(3.0, 0.5, size=(500, 2))
    roi = (0.0, 0.0, 7.0, 6.0)
    got = O.select_centers(xy, roi, 0.5, r_kd, thr, O.RADIUS)
    # independent: mesh built by hand, counts by k-d tree
    gx = np.arange(14) * 0.5 + 0.25
    gy = np.arange(12) * 0.5 + 0.25
    G = np.array([(a, b) for b in gy for a in gx])
    cnt = cKDTree(xy).query_ball_point(G, r_kd, return_length=True)
    ref = G[np.asarray(cnt) > thr]
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


def test_select_voxel_matches_histogram():
    rng = np.random.default_rng(12)
    xy = rng.uniform(-1.0, 11.0, size=(20000, 2))
    roi = (0.0, 0.0, 10.0, 10.0)
    got = O.select_centers(xy, roi, 0.5, 0.5, 48, O.VOXEL)
    H, _, _ = np.histogram2d(xy[:, 1], xy[:, 0], bins=[20, 20],
                             range=[[0, 10], [0, 10]])
    gx = np.arange(20) * 0.5 + 0.25
    ref = np.array([(gx[i], gx[j]) for j in range(20) for i in range(20)
                    if H[j, i] > 48])
    assert np.array_equal(got, ref)


def test_select_mesh_sizes_cell_centers():
    # cell-center nodes: 10 m at 0.5 m -> 20 x 20 = 400; 50 m -> 10,000
    assert O.candidate_mesh((0, 0, 10, 10), 0.5)[0].shape[0] == 400
    assert O.candidate_mesh((0, 0, 50, 50), 0.5)[0].shape[0] == 10000


def test_select_strictly_exceeds():
    xy = np.array([[0.25, 0.25]] * 4 + [[0.75, 0.25]] * 5)
    got = O.select_centers(xy, (0, 0, 1, 0.5), 0.5, 0.1, 4, O.VOXEL)
    assert np.array_equal(got, np.array([[0.75, 0.25]]))


# ------------------------------------------------------------ ridge / gram

def test_gram_equals_sum_of_outer_products():
    c, x, z = small(M=120, side=2.0)
    H, b = O.gram(x, z, c, SIG, CUT, 0.0, LAM)
    Href = LAM * np.eye(c.shape[0])
    bref = np.zeros(c.shape[0])
    for i in range(x.shape[0]):  # definition: sum_i m_i m_i^T, sum_i m_i z_i
        m = np.array([math.exp(-((x[i, 0] - cc[0]) ** 2 + (x[i, 1] - cc[1]) ** 2)
                               / (2 * SIG ** 2))
                      if (x[i, 0] - cc[0]) ** 2 + (x[i, 1] - cc[1]) ** 2
                      <= (CUT * SIG) ** 2 else 0.0 for cc in c])
        Href += np.outer(m, m)
        bref += m * z[i]
    assert np.allclose(H, Href, rtol=1e-13, atol=1e-15)
    assert np.allclose(b, bref, rtol=1e-13, atol=1e-15)


def test_gram_sparse_equals_dense():
    c, x, z = small()
    Hd, bd = O.gram(x, z, c, SIG, CUT, 0.0, LAM)
    Hs, bs = O.gram(x, z, c, SIG, CUT, 0.0, LAM, sparse=True)
    assert np.allclose(Hs.toarray(), Hd, rtol=1e-14, atol=1e-15)
    assert np.allclose(bs, bd, rtol=1e-14, atol=1e-15)


def test_gram_pattern_covers_nonzeros():
    c, x, z = small()
    H, _ = O.gram(x, z, c, SIG, CUT, 0.0, LAM)
    pat = O.gram_pattern(c, SIG, CUT, 0.0)
    for j in range(c.shape[0]):
        nz = set(np.flatnonzero(H[j]).tolist())
        assert nz <= set(pat[j].tolist())


@pytest.mark.parametrize("seps", [0.0, 0.1])
def test_gram_pattern_equals_kdtree_pairs(seps):
    """Exact row-by-row equality with scipy's k-d tree pair search at the
    radius 2 * cutoff * sqrt(sigma^2 + sigma_eps^2) (diagonal included), on
    jittered centers (no pair distance sits on the radius)."""
    rng = np.random.default_rng(11)
    c = synth.grid_centers(rng, 24, 20, 0.5)
    r = 2.0 * CUT * math.sqrt(SIG * SIG + seps * seps)
    pairs = cKDTree(c).query_pairs(r, output_type="ndarray")
    N = c.shape[0]
    ref = [{j} for j in range(N)]
    for a, b in pairs:
        ref[a].add(int(b))
        ref[b].add(int(a))
    pat = O.gram_pattern(c, SIG, CUT, seps)
    assert len(pat) == N
    for j in range(N):
        assert pat[j].tolist() == sorted(ref[j])
    # sigma_eps widens the pattern: the sigma_t radius, not sigma's
    if seps > 0.0:
        narrow = O.gram_pattern(c, SIG, CUT, 0.0)
        assert sum(len(a) for a in pat) > sum(len(a) for a in narrow)


@pytest.mark.parametrize("seps,bound", [(0.0, 36), (0.1, 37)])
def test_gram_pattern_on_lattice_is_integer_disc(seps, bound):
    """Unjittered 0.5 m lattice: centers (a, b) and (a', b') pair iff
    (a-a')^2 + (b-b')^2 <= (2 cutoff sigma_t / 0.5)^2, i.e. <= 36 at
    sigma_eps = 0 (the tie at exactly 3 m kept: hard inclusive cutoff) and
    <= 37 at sigma_eps = 0.1 (37.44). Integer arithmetic only."""
    nx, ny = 17, 15
    c = synth.grid_centers(None, nx, ny, 0.5, jitter=0.0)
    pat = O.gram_pattern(c, SIG, CUT, seps)
    for j in range(nx * ny):
        aj, bj = j % nx, j // nx
        ref = [k for k in range(nx * ny)
               if (k % nx - aj) ** 2 + (k // nx - bj) ** 2 <= bound]
        assert pat[j].tolist() == ref


@pytest.mark.parametrize("seps", [0.0, 0.1])
def test_gram_pattern_is_tight(seps):
    """Every pair of the pattern can be nonzero in calH: one point at the
    midpoint of the two centers has both regressor entries nonzero (so the
    pattern is exactly the set of reachable entries, not a wider one)."""
    rng = np.random.default_rng(12)
    c = synth.grid_centers(rng, 12, 10, 0.5)
    pat = O.gram_pattern(c, SIG, CUT, seps)
    for j in range(c.shape[0]):
        for k in pat[j]:
            mid = 0.5 * (c[j] + c[k])
            m = O.regressor_dense(mid[None, :], c[[j, k]], SIG, CUT, seps)
            assert (m > 0.0).all()


def test_ridge_matches_augmented_least_squares():
    c, x, z = small()
    w, _ = O.ridge_batch(x, z, c, SIG, CUT, 0.0, LAM, RV, with_P=False)
    Phi = O.regressor_dense(x, c, SIG, CUT, 0.0)
    A = np.vstack([Phi, math.sqrt(LAM) * np.eye(c.shape[0])])
    rhs = np.concatenate([z, np.zeros(c.shape[0])])
    wl = scipy.linalg.lstsq(A, rhs, lapack_driver="gelsd")[0]
    assert np.linalg.norm(w - wl) / np.linalg.norm(wl) < 1e-9


def test_scalar_closed_form_fixture():
    g = json.load(open(os.path.join(GOLD, "scalar_ridge.json")))
    c = np.array([g["center"]])
    x = np.array([g["point"]])
    z = np.array([g["z"]])
    d2 = sum((a - b) ** 2 for a, b in zip(g["point"], g["center"]))
    phi = math.exp(-d2 / (2 * g["sigma"] ** 2))
    w_ref = phi * g["z"] / (phi * phi + g["lambda"])
    P_ref = g["R"] / (phi * phi + g["lambda"])
    w, P = O.ridge_batch(x, z, c, g["sigma"], g["cutoff"], 0.0, g["lambda"], g["R"])
    assert w[0] == pytest.approx(w_ref, rel=1e-14)
    assert P[0, 0] == pytest.approx(P_ref, rel=1e-14)
    w0, P0 = O.initial_state(1, g["lambda"], g["R"])
    wk, Pk = O.kalman_update(w0, P0, x, z, c, g["sigma"], g["cutoff"], 0.0, g["R"])
    assert wk[0] == pytest.approx(w_ref, rel=1e-14)
    assert Pk[0, 0] == pytest.approx(P_ref, rel=1e-14)


@pytest.mark.parametrize("batch", [1, 7, 64, None])
def test_kalman_chain_equals_batch_ridge(batch):
    c, x, z = small(M=300)
    w0, P0 = O.initial_state(c.shape[0], LAM, RV)
    wk, Pk = O.kalman_update(w0, P0, x, z, c, SIG, CUT, 0.0, RV, batch=batch)
    wb, Pb = O.ridge_batch(x, z, c, SIG, CUT, 0.0, LAM, RV)
    # forward error of two backward-stable routes: c * cond(calH) * u
    H, _ = O.gram(x, z, c, SIG, CUT, 0.0, LAM)
    tol = 100 * np.linalg.cond(H) * np.finfo(float).eps
    assert np.linalg.norm(wk - wb) / np.linalg.norm(wb) < tol
    assert np.abs(Pk - Pb).max() / np.abs(Pb).max() < tol
    assert np.array_equal(Pk, Pk.T)


def test_kalman_chain_with_moment_regressor():
    c, x, z = small(M=300)
    se = 0.1
    w0, P0 = O.initial_state(c.shape[0], LAM, RV)
    wk, Pk = O.kalman_update(w0, P0, x, z, c, SIG, CUT, se, RV, batch=50)
    wb, Pb = O.ridge_batch(x, z, c, SIG, CUT, se, LAM, RV)
    assert np.linalg.norm(wk - wb) / np.linalg.norm(wb) < 1e-10
    assert np.abs(Pk - Pb).max() / np.abs(Pb).max() < 1e-10


def test_kalman_equals_information_form_and_order_free():
    c, x, z = small(M=400)
    N = c.shape[0]
    w0, P0 = O.initial_state(N, LAM, RV)
    wk, Pk = O.kalman_update(w0, P0, x, z, c, SIG, CUT, 0.0, RV, batch=100)
    H = LAM * np.eye(N)
    w = np.zeros(N)
    for s in range(0, 400, 133):
        H, w = O.information_update(H, w, x[s:s + 133], z[s:s + 133], c, SIG, CUT, 0.0)
    assert np.linalg.norm(wk - w) / np.linalg.norm(w) < 1e-10
    assert np.abs(Pk - RV * np.linalg.inv(H)).max() / np.abs(Pk).max() < 1e-10
    perm = np.random.default_rng(3).permutation(400)
    wp, Pp = O.kalman_update(w0, P0, x[perm], z[perm], c, SIG, CUT, 0.0, RV, batch=64)
    assert np.linalg.norm(wk - wp) / np.linalg.norm(wk) < 1e-10


def test_weights_independent_of_R():
    c, x, z = small(M=200)
    N = c.shape[0]
    outs = []
    for R in (1.0, 4e-4):
        w0, P0 = O.initial_state(N, LAM, R)
        outs.append(O.kalman_update(w0, P0, x, z, c, SIG, CUT, 0.0, R, batch=37))
    assert np.linalg.norm(outs[0][0] - outs[1][0]) / np.linalg.norm(outs[0][0]) < 1e-11
    assert np.allclose(outs[0][1] * 4e-4, outs[1][1], rtol=1e-10, atol=1e-18)


def test_planted_weights_bias_is_linear_in_lambda():
    """z = Phi w0 exactly: w_lambda - w0 = -lambda calH^{-1} w0 (closed form),
    so the recovery error scales with lambda and vanishes as lambda -> 0."""
    rng = np.random.default_rng(5)
    c = synth.grid_centers(rng, 5, 5, 0.5, x0=1.0, y0=1.0)
    x = rng.uniform(0.5, 4.0, size=(1500, 2))
    Phi = O.regressor_dense(x, c, SIG, CUT, 0.0)
    w0 = rng.normal(0, 0.3, size=c.shape[0])
    z = Phi @ w0
    errs = []
    for lam in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10):
        w, _ = O.ridge_batch(x, z, c, SIG, CUT, 0.0, lam, RV, with_P=False)
        errs.append(np.linalg.norm(w - w0) / np.linalg.norm(w0))
        H = Phi.T @ Phi + lam * np.eye(c.shape[0])
        bias = -lam * np.linalg.solve(H, w0)
        assert np.linalg.norm((w - w0) - bias) <= 1e-6 * np.linalg.norm(w0) + 1e-3 * np.linalg.norm(bias)
    assert errs[-1] < 1e-6
    for a, b in zip(errs[1:-1], errs[2:]):
        assert 30 < a / b < 300  # ~100x per 100x in lambda


# ------------------------------------------------------- active-rows form

def _disc_scan(rng, center, radius, M):
    r = radius * np.sqrt(rng.uniform(0, 1, M))
    t = rng.uniform(0, 2 * np.pi, M)
    x = np.stack([center[0] + r * np.cos(t), center[1] + r * np.sin(t)], 1)
    z = 0.2 * np.sin(x[:, 0]) + 0.1 * np.cos(2 * x[:, 1]) + rng.normal(0, 0.02, M)
    return x, z


def _scan_world(seed=11):
    rng = np.random.default_rng(seed)
    c = synth.grid_centers(rng, 16, 16, 0.5)  # 8 x 8 m
    return rng, c


def _tol(xs, c):
    """100 cond(calH) u for the information matrix of the points xs (the
    forward error bound of two backward-stable routes, as for chain = batch)."""
    x = np.concatenate(xs)
    H, _ = O.gram(x, np.zeros(x.shape[0]), c, SIG, CUT, 0.0, LAM)
    return 100 * np.linalg.cond(H) * np.finfo(float).eps


@pytest.mark.parametrize("se", [0.0, 0.1])
def test_active_set_matches_kdtree(se):
    rng, c = _scan_world()
    x, _ = _disc_scan(rng, (3.0, 4.0), 1.2, 300)
    rad = CUT * math.sqrt(SIG ** 2 + se ** 2)
    hits = cKDTree(x).query_ball_point(c, rad)
    ref = np.array([j for j, h in enumerate(hits) if len(h) > 0])
    A = O.active_set(x, c, SIG, CUT, se)
    assert np.array_equal(A, ref)
    assert 0 < A.size < c.shape[0]


def test_active_update_from_prior_equals_dense():
    """From P_0 = (R/lambda) I nothing couples A to the other centers, so the
    active-rows form equals the dense recursion (and the batch ridge
    solution of the scan) everywhere."""
    rng, c = _scan_world()
    N = c.shape[0]
    x, z = _disc_scan(rng, (3.0, 4.0), 1.2, 300)
    w0, P0 = O.initial_state(N, LAM, RV)
    wa, Pa, A = O.kalman_update_active(w0, P0, x, z, c, SIG, CUT, 0.0, RV, batch=64)
    wd, Pd = O.kalman_update(w0, P0, x, z, c, SIG, CUT, 0.0, RV, batch=64)
    wb, Pb = O.ridge_batch(x, z, c, SIG, CUT, 0.0, LAM, RV)
    tol = _tol([x], c)
    assert np.linalg.norm(wa - wd) / np.linalg.norm(wd) < tol
    assert np.abs(Pa - Pd).max() / np.abs(Pd).max() < tol
    assert np.linalg.norm(wa - wb) / np.linalg.norm(wb) < tol
    out = np.setdiff1d(np.arange(N), A)
    assert np.array_equal(wa[out], w0[out])
    assert np.array_equal(Pa[np.ix_(out, out)], P0[np.ix_(out, out)])
    assert not Pa[np.ix_(A, out)].any()


def test_active_update_disjoint_scans_equal_dense():
    rng, c = _scan_world()
    N = c.shape[0]
    w, P = O.initial_state(N, LAM, RV)
    wd, Pd = w.copy(), P.copy()
    xs = []
    for ctr in ((1.5, 1.5), (6.5, 6.5), (1.5, 6.5)):
        x, z = _disc_scan(rng, ctr, 0.6, 200)
        xs.append(x)
        w, P, _ = O.kalman_update_active(w, P, x, z, c, SIG, CUT, 0.0, RV, batch=50)
        wd, Pd = O.kalman_update(wd, Pd, x, z, c, SIG, CUT, 0.0, RV, batch=50)
    tol = _tol(xs, c)
    assert np.linalg.norm(w - wd) / np.linalg.norm(wd) < tol
    assert np.abs(P - Pd).max() / np.abs(Pd).max() < tol


def test_active_update_is_dense_update_of_block_diagonal_part():
    """Overlapping scans: the active-rows result equals, everywhere, the
    dense recursion applied to P with its A-to-rest coupling removed (the
    block-diagonal form of eq. H_inverse_update), stays positive definite,
    and differs from the exact dense recursion on the unmodified P."""
    rng, c = _scan_world()
    N = c.shape[0]
    w, P = O.initial_state(N, LAM, RV)
    x1, z1 = _disc_scan(rng, (3.0, 4.0), 1.5, 300)
    w, P, _ = O.kalman_update_active(w, P, x1, z1, c, SIG, CUT, 0.0, RV)
    x2, z2 = _disc_scan(rng, (4.5, 4.0), 1.5, 300)  # overlaps the first scan
    wa, Pa, A = O.kalman_update_active(w, P, x2, z2, c, SIG, CUT, 0.0, RV, batch=100)
    out = np.setdiff1d(np.arange(N), A)
    Pblk = P.copy()
    Pblk[np.ix_(A, out)] = 0.0
    Pblk[np.ix_(out, A)] = 0.0
    assert np.abs(P[np.ix_(A, out)]).max() > 1e-6  # the scans really are coupled
    wd, Pd = O.kalman_update(w, Pblk, x2, z2, c, SIG, CUT, 0.0, RV, batch=100)
    tol = _tol([x1, x2], c)
    assert np.linalg.norm(wa - wd) / np.linalg.norm(wd) < tol
    assert np.abs(Pa - Pd).max() / np.abs(Pd).max() < tol
    assert not Pa[np.ix_(A, out)].any() and not Pa[np.ix_(out, A)].any()
    assert np.array_equal(Pa[np.ix_(out, out)], P[np.ix_(out, out)])
    assert np.array_equal(Pa, Pa.T)
    assert np.linalg.eigvalsh(Pa).min() > 0
    we, _ = O.kalman_update(w, P, x2, z2, c, SIG, CUT, 0.0, RV)
    assert np.linalg.norm(wa - we) / np.linalg.norm(we) > 1e3 * tol


# ------------------------------------------------------ growing center set

def _path_frames(seed=12, n=5):
    rng = np.random.default_rng(seed)
    frames = []
    for k in range(n):
        ctr = (1.5 + 1.2 * k, 4.0 + 0.5 * math.sin(k))
        x, z = _disc_scan(rng, ctr, 1.6, 400)
        frames.append((np.clip(x, 0.0, 8.0), z))
    return frames


@pytest.mark.parametrize("mode,r_kd,thr", [(O.RADIUS, 0.5, 6), (O.VOXEL, 0.5, 3)])
def test_select_grow_union_equals_batch_selection(mode, r_kd, thr):
    roi = (0.0, 0.0, 8.0, 8.0)
    frames = _path_frames()
    G, nx, ny = O.candidate_mesh(roi, 0.5)
    counts = np.zeros(nx * ny, dtype=np.int64)
    got = []
    for x, _ in frames:
        counts, new = O.select_centers_grow(counts, x, roi, 0.5, r_kd, thr, mode)
        # mesh order within the frame
        lin = np.round((new[:, 1] - 0.25) / 0.5) * nx + np.round((new[:, 0] - 0.25) / 0.5)
        assert np.all(np.diff(lin) > 0)
        got.append(new)
    allx = np.concatenate([f[0] for f in frames])
    if mode == O.RADIUS:  # independent count: k-d tree over all points
        ref_cnt = np.array([len(h) for h in cKDTree(allx).query_ball_point(G, r_kd)])
    else:
        ref_cnt, _, _ = np.histogram2d(allx[:, 1], allx[:, 0], bins=[ny, nx],
                                       range=[[0, 8], [0, 8]])
        ref_cnt = ref_cnt.ravel().astype(np.int64)
    assert np.array_equal(counts, ref_cnt)
    grown = np.concatenate(got)
    batch = G[ref_cnt > thr]
    assert grown.shape == batch.shape and len({tuple(c) for c in grown}) == grown.shape[0]
    key = lambda a: a[np.lexsort((a[:, 0], a[:, 1]))]
    assert np.array_equal(key(grown), batch)
    assert sum(g.shape[0] > 0 for g in got) >= 3  # the set really grows


def test_grown_chain_equals_masked_batch_ridge():
    """Growing centers with the recursion equals the ridge estimator in
    which each point's regressor keeps only the centers that existed when
    the point was absorbed (closed form: calH = lambda I + sum m^ m^T,
    b = sum m^ z, with m^ the masked regressor)."""
    roi = (0.0, 0.0, 8.0, 8.0)
    frames = _path_frames()
    G, nx, ny = O.candidate_mesh(roi, 0.5)
    counts = np.zeros(nx * ny, dtype=np.int64)
    c = np.zeros((0, 2))
    w, P = np.zeros(0), np.zeros((0, 0))
    born = []
    for x, z in frames:
        counts, new = O.select_centers_grow(counts, x, roi, 0.5, 0.5, 6, O.RADIUS)
        w, P = O.grow_state(w, P, new.shape[0], LAM, RV)
        c = np.concatenate([c, new])
        born.append(c.shape[0])
        w, P = O.kalman_update(w, P, x, z, c, SIG, CUT, 0.0, RV, batch=128)
    N = c.shape[0]
    H = LAM * np.eye(N)
    b = np.zeros(N)
    for (x, z), nb in zip(frames, born):
        m = np.zeros((x.shape[0], N))
        m[:, :nb] = O.regressor_dense(x, c[:nb], SIG, CUT, 0.0)
        H += m.T @ m
        b += m.T @ z
    w_ref = scipy.linalg.solve(H, b, assume_a="pos")
    tol = 100 * np.linalg.cond(H) * np.finfo(float).eps
    assert np.linalg.norm(w - w_ref) / np.linalg.norm(w_ref) < tol
    assert np.abs(P - RV * np.linalg.inv(H)).max() / np.abs(P).max() < tol
    # the late centers miss earlier points: not the batch ridge of all points
    allx = np.concatenate([f[0] for f in frames])
    allz = np.concatenate([f[1] for f in frames])
    wb, _ = O.ridge_batch(allx, allz, c, SIG, CUT, 0.0, LAM, RV, with_P=False)
    assert np.linalg.norm(w - wb) / np.linalg.norm(wb) > 1e3 * tol


# ------------------------------------------------------------- evaluation

def test_eval_single_center_closed_form():
    c = np.array([[1.0, 2.0]])
    w = np.array([0.7])
    q = np.array([[1.3, 2.1], [1.0, 2.0], [3.0, 2.0]])
    f, g = O.eval_height_grad(q, c, w, SIG, CUT)
    e = math.exp(-(0.09 + 0.01) / (2 * SIG ** 2))
    assert f[0] == pytest.approx(0.7 * e, rel=1e-15)
    assert g[0, 0] == pytest.approx(-0.7 * e * 0.3 / SIG ** 2, rel=1e-14)
    assert g[0, 1] == pytest.approx(-0.7 * e * 0.1 / SIG ** 2, rel=1e-13)
    assert f[1] == 0.7 and g[1, 0] == 0.0
    assert f[2] == 0.0 and g[2, 1] == 0.0  # beyond the cutoff


def _far_from_cutoff(q, c, h):
    d = np.sqrt(O.sq_dist(q, c))
    return (np.abs(d - CUT * SIG) > 4 * h).all(axis=1)


def test_gradient_matches_central_differences():
    c, x, z = small()
    w, _ = O.ridge_batch(x, z, c, SIG, CUT, 0.0, LAM, RV, with_P=False)
    rng = np.random.default_rng(9)
    q = rng.uniform(0.5, 3.5, size=(400, 2))
    h = 1e-6
    q = q[_far_from_cutoff(q, c, h)]
    _, g = O.eval_height_grad(q, c, w, SIG, CUT)
    for k in range(2):
        e = np.zeros(2)
        e[k] = h
        fp, _ = O.eval_height_grad(q + e, c, w, SIG, CUT)
        fm, _ = O.eval_height_grad(q - e, c, w, SIG, CUT)
        fd = (fp - fm) / (2 * h)
        assert np.max(np.abs(fd - g[:, k])) <= 1e-7 * max(1.0, np.abs(g).max())


def _pose_case(seed=21, Q=60):
    c, x, z = small(seed=seed)
    w, _ = O.ridge_batch(x, z, c, SIG, CUT, 0.0, LAM, RV, with_P=False)
    rng = np.random.default_rng(seed)
    R = synth.rot_zyx(0.7, 0.05, -0.04)
    t = np.array([2.0, 2.0, 0.6])
    world = np.concatenate([rng.uniform(0.8, 3.2, size=(Q, 2)),
                            rng.normal(0, 0.1, size=(Q, 1))], 1)
    p = (world - t) @ R
    return c, w, p, R, t


def test_pose_jacobian_matches_se3_central_differences():
    c, w, p, R, t = _pose_case()
    h = 1e-6
    _, _, r, J = O.eval_pose(p, R, t, 0.05, c, w, SIG, CUT)
    fd = np.zeros_like(J)
    for k in range(6):
        d = np.zeros(6)
        d[k] = h
        Rp, tp = R @ synth.so3_exp(d[:3]), t + d[3:]
        Rm, tm = R @ synth.so3_exp(-d[:3]), t - d[3:]
        rp = O.eval_pose(p, Rp, tp, 0.05, c, w, SIG, CUT)[2]
        rm = O.eval_pose(p, Rm, tm, 0.05, c, w, SIG, CUT)[2]
        fd[:, k] = (rp - rm) / (2 * h)
    xi = O.to_world(p, R, t)
    ok = _far_from_cutoff(xi[:, :2], c, 1e-4)
    assert ok.sum() > 40
    assert np.max(np.abs(fd[ok] - J[ok])) < 1e-7


def test_residual_vanishes_on_fitted_surface():
    c, w, p, R, t = _pose_case()
    xi = O.to_world(p, R, t)
    f, _ = O.eval_height_grad(xi[:, :2], c, w, SIG, CUT)
    world = np.concatenate([xi[:, :2], (f + 0.05)[:, None]], 1)
    p2 = (world - t) @ R
    _, _, r, _ = O.eval_pose(p2, R, t, 0.05, c, w, SIG, CUT)
    assert np.abs(r).max() < 1e-13


def test_adjoint_pose_dot_product_and_fd():
    c, w, p, R, t = _pose_case(Q=40)
    rng = np.random.default_rng(4)
    gf = rng.normal(size=p.shape[0])
    gr = rng.normal(size=p.shape[0])
    zo = 0.02
    d_p, d_w, d_pose = O.eval_adjoint_pose(p, R, t, zo, c, w, SIG, CUT, gf, gr)

    def L(p_, w_, R_, t_):
        f, _, r, _ = O.eval_pose(p_, R_, t_, zo, c, w_, SIG, CUT)
        return gf @ f + gr @ r

    # weights enter linearly: exact directional derivative
    v = rng.normal(size=w.shape[0])
    assert (L(p, w + v, R, t) - L(p, w, R, t)) == pytest.approx(d_w @ v, rel=1e-10)
    # pose: right perturbation, central differences
    h = 1e-6
    for k in range(6):
        d = np.zeros(6)
        d[k] = h
        lp = L(p, w, R @ synth.so3_exp(d[:3]), t + d[3:])
        lm = L(p, w, R @ synth.so3_exp(-d[:3]), t - d[3:])
        assert (lp - lm) / (2 * h) == pytest.approx(d_pose[k], rel=1e-6, abs=1e-7)
    # points: dot-product test <d_p, v> = dL along v
    V = rng.normal(size=p.shape)
    fd = (L(p + h * V, w, R, t) - L(p - h * V, w, R, t)) / (2 * h)
    assert fd == pytest.approx(np.sum(d_p * V), rel=1e-6, abs=1e-7)
    # L = gf f + gr r and f = xi_z - z_off - r, so the pose adjoint is
    # J^T (gr - gf) + (d xi_z / d pose)^T gf with J the residual Jacobian
    _, _, _, J = O.eval_pose(p, R, t, zo, c, w, SIG, CUT)
    dxi_z = np.zeros((p.shape[0], 6))
    dxi_z[:, :3] = (-R @ np.stack([O.skew(pi) for pi in p]))[:, 2, :]
    dxi_z[:, 5] = 1.0
    ref = J.T @ (gr - gf) + dxi_z.T @ gf
    assert np.allclose(d_pose, ref, rtol=1e-12, atol=1e-12)


def test_adjoint_xy():
    c, x, z = small()
    w, _ = O.ridge_batch(x, z, c, SIG, CUT, 0.0, LAM, RV, with_P=False)
    rng = np.random.default_rng(8)
    q = rng.uniform(0.5, 3.5, size=(100, 2))
    gb = rng.normal(size=100)
    d_q, d_w = O.eval_adjoint_xy(q, c, w, SIG, CUT, gb)
    v = rng.normal(size=w.shape[0])
    f0, _ = O.eval_height_grad(q, c, w, SIG, CUT)
    f1, _ = O.eval_height_grad(q, c, w + v, SIG, CUT)
    assert gb @ (f1 - f0) == pytest.approx(d_w @ v, rel=1e-10)
    _, g = O.eval_height_grad(q, c, w, SIG, CUT)
    assert np.array_equal(d_q, gb[:, None] * g)


# ------------------------------------------------------------------ solve

def test_solve_inverse_identity_and_sparse_vs_dense():
    c, x, z = small(M=500, side=3.0)
    H, b = O.gram(x, z, c, SIG, CUT, 0.0, LAM)
    Hs, _ = O.gram(x, z, c, SIG, CUT, 0.0, LAM, sparse=True)
    N = c.shape[0]
    X = O.spd_solve(Hs, np.eye(N))  # sparse LU
    cond = np.linalg.cond(H)
    assert np.abs(H @ X - np.eye(N)).max() <= 50 * cond * np.finfo(float).eps
    xd = O.spd_solve(H, b)  # dense LAPACK
    assert np.linalg.norm(X @ b - xd) / np.linalg.norm(xd) < 50 * cond * 1e-16
    assert O.relres(H, xd, b) < 1e-14
    assert O.relres(Hs, xd, b) < 1e-14
