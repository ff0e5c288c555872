"""Plain FP64 CPU oracle for the RBF terrain hot path.

TEST INFRASTRUCTURE ONLY. This module is the reference the GPU library is
checked against. Only the tests, the smoke check and the benchmark's CPU
baseline leg may import it; the library and its Python binding never do.
It shares no code with the HIP path.

Every function computes the plain definition of a step of the method in
float64, in the order and notation of the paper ("Terrain-Awared LiDAR-
Inertial Odometry for Legged-Wheel Robots Based on Radial Basis Function
Approximation"). Library primitives (matrix products, dense/sparse direct
solves) are used as single steps; there is no blocking or fusion.

Notation: centers c_j (N x 2), weights w (N), bandwidth sigma, points
x_i (M x 2) with heights z_i, ridge penalty lambda, and the covariance
P = R * inv(calH) with calH = lambda*I + sum_i m(x_i) m(x_i)^T.

Readings of the paper that these definitions fix (each is stated where it
is used):
  * hard kernel truncation at d <= cutoff*sigma (tie kept);
  * the regressor uses sigma_t = sqrt(sigma^2 + sigma_eps^2) inside the
    kernel, as in its definition in the ridge-regression subsection;
  * b_k = calH_k w_k and calH_{k+1} - m m^T in the Kalman-style rewrite;
  * P = R * inv(calH), so the paper's identity in (I + m^T calH^-1 m)
    becomes R*I + m^T P m;
  * the gradient of f carries a minus sign;
  * the pose Jacobian uses a right perturbation R <- R Exp(dtheta) and the
    body-frame point, ordered [rotation, translation].
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

RADIUS = 0
VOXEL = 1


# ---------------------------------------------------------------------------
# Kernel and regressor (eq. RBF_def; moment regressor m(x) in the ridge
# regression subsection; truncation per the compact-support remark of the
# GPU section)
# ---------------------------------------------------------------------------

def regressor_scale(sigma, sigma_eps):
    """(s_m, sigma_t): m(x) = s_m * kappa_{sigma_t}(x; c), 2-D Gaussian
    convolution of the kernel with the xy noise N(0, sigma_eps^2 I)."""
    sigma_t = math.sqrt(sigma * sigma + sigma_eps * sigma_eps)
    return (sigma * sigma) / (sigma_t * sigma_t), sigma_t


def sq_dist(x, c):
    """d^2 = dx*dx + dy*dy, products rounded separately (M x N)."""
    dx = x[:, 0:1] - c[None, :, 0]
    dy = x[:, 1:2] - c[None, :, 1]
    return dx * dx + dy * dy


def kernel_block(x, c, bw, cutoff, scale=1.0):
    """scale * exp(-d^2 / (2 bw^2)) where d <= cutoff*bw, else 0 (M x N)."""
    rc = cutoff * bw
    d2 = sq_dist(x, c)
    out = scale * np.exp(-d2 / (2.0 * bw * bw))
    out[d2 > rc * rc] = 0.0
    return out


def phi_dense(x, c, sigma, cutoff):
    """Kernel matrix of eq. RBF_def evaluated at x: Phi[i, j] = phi(x_i, c_j)."""
    return kernel_block(np.asarray(x, np.float64), np.asarray(c, np.float64),
                        sigma, cutoff)


def regressor_dense(x, c, sigma, cutoff, sigma_eps):
    """Rows m(x_i)^T of the moment-corrected regressor (M x N)."""
    s_m, sigma_t = regressor_scale(sigma, sigma_eps)
    return kernel_block(np.asarray(x, np.float64), np.asarray(c, np.float64),
                        sigma_t, cutoff, s_m)


def regressor_csr(x, c, sigma, cutoff, sigma_eps, chunk=2048):
    """Same as regressor_dense but returned as scipy CSR (for large N)."""
    x = np.asarray(x, np.float64)
    c = np.asarray(c, np.float64)
    blocks = []
    for s in range(0, x.shape[0], chunk):
        blocks.append(sp.csr_matrix(
            regressor_dense(x[s:s + chunk], c, sigma, cutoff, sigma_eps)))
    if not blocks:
        return sp.csr_matrix((0, c.shape[0]))
    return sp.vstack(blocks, format="csr")


# ---------------------------------------------------------------------------
# Adaptive center selection (subsection "The RBF Approximation Model")
# ---------------------------------------------------------------------------

def candidate_mesh(roi, res):
    """Candidate nodes at the cell centers of a res-mesh over the ROI,
    row-major with y outer: node (i, j) = (x0 + (i+1/2)res, y0 + (j+1/2)res)."""
    x0, y0, x1, y1 = roi
    nx = int(math.ceil((x1 - x0) / res))
    ny = int(math.ceil((y1 - y0) / res))
    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)
    gx = x0 + (i + 0.5) * res
    gy = y0 + (j + 0.5) * res
    G = np.stack([np.tile(gx, ny), np.repeat(gy, nx)], axis=1)
    return G, nx, ny


def candidate_counts(xy, roi, res, r_kd, mode):
    """Number of terrain points supporting each candidate node.

    RADIUS: points with ||p - g||^2 <= r_kd^2 (the k-d-tree radius count).
    VOXEL : points whose mesh cell (floor((p - origin)/res)) is the node's.
    """
    xy = np.asarray(xy, np.float64)
    G, nx, ny = candidate_mesh(roi, res)
    if mode == RADIUS:
        r2 = r_kd * r_kd
        cnt = np.zeros(G.shape[0], dtype=np.int64)
        for s in range(0, G.shape[0], 256):
            d2 = sq_dist(G[s:s + 256], xy)
            cnt[s:s + 256] = (d2 <= r2).sum(axis=1)
        return cnt
    x0, y0 = roi[0], roi[1]
    ix = np.floor((xy[:, 0] - x0) / res)
    iy = np.floor((xy[:, 1] - y0) / res)
    ok = (ix >= 0) & (ix < nx) & (iy >= 0) & (iy < ny)
    lin = (iy[ok] * nx + ix[ok]).astype(np.int64)
    return np.bincount(lin, minlength=nx * ny).astype(np.int64)


def select_centers(xy, roi, res, r_kd, thr, mode=RADIUS):
    """Accept a candidate node iff its point count exceeds thr (strict >).
    Accepted nodes keep mesh order (y outer, x inner)."""
    G, _, _ = candidate_mesh(roi, res)
    cnt = candidate_counts(xy, roi, res, r_kd, mode)
    return np.ascontiguousarray(G[cnt > thr])


def select_centers_grow(counts, xy, roi, res, r_kd, thr, mode=RADIUS):
    """Center selection applied frame by frame (a growing center set).

    Reading: the support count of a candidate node is over every terrain
    point seen so far, so a frame adds its own counts to the running ones
    (counts: one integer per node, zeros before the first frame). A node
    becomes a center in the frame whose points take its count past thr;
    the frame's new centers are appended in mesh order. Over all frames the
    centers are those of select_centers on all the points together.
    Returns (counts after the frame, the frame's new centers)."""
    G, _, _ = candidate_mesh(roi, res)
    old = np.asarray(counts, dtype=np.int64)
    new = old + candidate_counts(xy, roi, res, r_kd, mode)
    return new, np.ascontiguousarray(G[(old <= thr) & (new > thr)])


def grow_state(w, P, n_new, lam, R):
    """Append n_new centers to the state: their weights start at the prior
    w = 0 with the prior covariance (R/lambda) I and no coupling to the
    existing centers, i.e. calH gains lambda on the new diagonal entries."""
    N = w.shape[0]
    w2 = np.zeros(N + n_new)
    w2[:N] = w
    P2 = np.zeros((N + n_new, N + n_new))
    P2[:N, :N] = P
    P2[np.arange(N, N + n_new), np.arange(N, N + n_new)] = R / lam
    return w2, P2


# ---------------------------------------------------------------------------
# Ridge estimator (eq. RBF_estimator with the ridge term)
# ---------------------------------------------------------------------------

def gram(x, z, c, sigma, cutoff, sigma_eps, lam, sparse=False):
    """calH = lambda*I + sum_i m(x_i) m(x_i)^T and b = sum_i m(x_i) z_i."""
    N = c.shape[0]
    if sparse:
        Phi = regressor_csr(x, c, sigma, cutoff, sigma_eps)
        H = (Phi.T @ Phi + lam * sp.identity(N, format="csr")).tocsr()
        b = Phi.T @ np.asarray(z, np.float64)
        return H, b
    Phi = regressor_dense(x, c, sigma, cutoff, sigma_eps)
    return Phi.T @ Phi + lam * np.eye(N), Phi.T @ np.asarray(z, np.float64)


def spd_solve(H, B):
    """X = calH^{-1} B (dense LAPACK or sparse LU as one library step)."""
    if sp.issparse(H):
        lu = spla.splu(sp.csc_matrix(H))
        return lu.solve(np.asarray(B, np.float64))
    return np.linalg.solve(H, B)


def ridge_batch(x, z, c, sigma, cutoff, sigma_eps, lam, R, sparse=False,
                with_P=True):
    """Batch ridge solution w = calH^{-1} b and its covariance P = R calH^{-1}."""
    H, b = gram(x, z, c, sigma, cutoff, sigma_eps, lam, sparse=sparse)
    w = spd_solve(H, b)
    if not with_P:
        return w, None
    N = c.shape[0]
    P = R * spd_solve(H, np.eye(N))
    return w, P


# ---------------------------------------------------------------------------
# Recursive update (eqs. weights_update / H_update, kf_w_update and
# H_inverse_update of the recursive-update subsection)
# ---------------------------------------------------------------------------

def information_update(Hk, wk, x, z, c, sigma, cutoff, sigma_eps):
    """eqs. weights_update and H_update: calH_{k+1} = calH_k + m m^T and
    w_{k+1} = calH_{k+1}^{-1} (b_k + m p_z), with b_k = calH_k w_k."""
    m = regressor_dense(x, c, sigma, cutoff, sigma_eps).T  # N x M
    H1 = Hk + m @ m.T
    b = Hk @ wk + m @ np.asarray(z, np.float64)
    return H1, np.linalg.solve(H1, b)


def kalman_update(w, P, x, z, c, sigma, cutoff, sigma_eps, R, batch=None):
    """Kalman-style recursion over consecutive batches of points.

    Per batch (m = [m(x_1) ... m(x_B)], N x B), in the paper's order:
      calH^{-1} <- calH^{-1} - calH^{-1} m (I + m^T calH^{-1} m)^{-1} m^T calH^{-1}
                                                     (eq. H_inverse_update)
      w <- w + calH_{new}^{-1} m (p_z - m^T w)       (eq. kf_w_update)
    with calH^{-1} = P / R on entry and P = R calH^{-1} on exit. The inverse
    is symmetrised after each batch.
    """
    x = np.asarray(x, np.float64)
    z = np.asarray(z, np.float64)
    w = np.array(w, dtype=np.float64, copy=True)
    Hinv = np.array(P, dtype=np.float64, copy=True) / R
    M = x.shape[0]
    B = M if not batch else int(batch)
    for s in range(0, M, max(B, 1)):
        m = regressor_dense(x[s:s + B], c, sigma, cutoff, sigma_eps).T
        nu = z[s:s + B] - m.T @ w
        Hm = Hinv @ m
        S = np.eye(m.shape[1]) + m.T @ Hm
        Hinv = Hinv - Hm @ np.linalg.solve(S, Hm.T)
        Hinv = 0.5 * (Hinv + Hinv.T)
        w = w + Hinv @ (m @ nu)
    return w, R * Hinv


def active_set(x, c, sigma, cutoff, sigma_eps):
    """Active rows of a scan (eq. mfk_m_approx and the remark after it): the
    centers whose regressor entry is non-zero at one or more of the scan's
    points, in ascending index order. With the hard truncation the other
    rows of m are exactly zero. The paper draws them as one contiguous run
    j1..j2; the set itself is used here, whatever its order."""
    m = regressor_dense(x, c, sigma, cutoff, sigma_eps)  # M x N
    return np.flatnonzero((m != 0.0).any(axis=0))


def kalman_update_active(w, P, x, z, c, sigma, cutoff, sigma_eps, R, batch=None):
    """Active-rows form of the recursive update (eqs.
    active_rows_weights_update and H_inverse_update).

    With A the scan's active set, the Kalman recursion runs on w_A and the
    A x A block of calH^{-1} (P / R) with the regressor m~ restricted to A.
    Eq. H_inverse_update gives the new inverse in block-diagonal form: the
    A x A block updated, the blocks of the other centers as before, and
    nothing coupling A to the other centers. Reading: the coupling blocks
    (rows A, columns outside A, and their mirror) are set to zero by the
    update; w outside A and P outside the rows and columns of A are
    unchanged. This keeps P positive semi-definite (block diagonal with PSD
    blocks), so the S of a later scan stays positive definite. When P has no
    such coupling (e.g. the prior (R/lambda) I), the result equals the dense
    update. Returns (w, P, A)."""
    w = np.array(w, dtype=np.float64, copy=True)
    P = np.array(P, dtype=np.float64, copy=True)
    A = active_set(x, c, sigma, cutoff, sigma_eps)
    if A.size == 0:
        return w, P, A
    wA, PA = kalman_update(w[A], P[np.ix_(A, A)], x, z, np.asarray(c)[A], sigma, cutoff,
                           sigma_eps, R, batch=batch)
    out = np.setdiff1d(np.arange(P.shape[0]), A)
    w[A] = wA
    P[np.ix_(A, A)] = PA
    P[np.ix_(A, out)] = 0.0
    P[np.ix_(out, A)] = 0.0
    return w, P, A


def initial_state(N, lam, R):
    """Prior before any scan: w_0 = 0, calH_0 = lambda*I, so P_0 = (R/lambda) I."""
    return np.zeros(N), (R / lam) * np.eye(N)


# ---------------------------------------------------------------------------
# Evaluation (eqs. RBF_fml, manifold_derivative, manidolf_grad_detail,
# residual_manifold_left_wheel, manifold_grad_2)
# ---------------------------------------------------------------------------

def eval_height_grad(q, c, w, sigma, cutoff, chunk=4096):
    """f(x) = sum_j w_j phi(x, c_j) and grad f = -sum_j w_j phi (x - c_j)/sigma^2."""
    q = np.asarray(q, np.float64)
    c = np.asarray(c, np.float64)
    w = np.asarray(w, np.float64)
    Q = q.shape[0]
    f = np.empty(Q)
    g = np.empty((Q, 2))
    for s in range(0, Q, chunk):
        qs = q[s:s + chunk]
        Phi = phi_dense(qs, c, sigma, cutoff)
        Pw = Phi * w[None, :]
        f[s:s + chunk] = Pw.sum(axis=1)
        dx = qs[:, 0:1] - c[None, :, 0]
        dy = qs[:, 1:2] - c[None, :, 1]
        g[s:s + chunk, 0] = -(Pw * dx).sum(axis=1) / (sigma * sigma)
        g[s:s + chunk, 1] = -(Pw * dy).sum(axis=1) / (sigma * sigma)
    return f, g


def skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def skew_rows(p):
    """[p_i]x for every row of p (Q x 3 x 3)."""
    p = np.asarray(p, np.float64)
    K = np.zeros((p.shape[0], 3, 3))
    K[:, 0, 1], K[:, 0, 2] = -p[:, 2], p[:, 1]
    K[:, 1, 0], K[:, 1, 2] = p[:, 2], -p[:, 0]
    K[:, 2, 0], K[:, 2, 1] = -p[:, 1], p[:, 0]
    return K


def to_world(p, Rs, t):
    """xi = R_s p + t for body-frame points p (Q x 3)."""
    return np.asarray(p, np.float64) @ np.asarray(Rs, np.float64).T + t


def eval_pose(p, Rs, t, z_off, c, w, sigma, cutoff):
    """Residual r = xi_z - z_off - f(xi_x, xi_y) at xi = R_s p + t, and its
    Jacobian w.r.t. a right perturbation (R_s Exp(dtheta), t + dt):
    J = [ g^T (-R_s [p]x),  g^T ],  g = (-f_x, -f_y, 1)."""
    p = np.asarray(p, np.float64)
    Rs = np.asarray(Rs, np.float64)
    xi = to_world(p, Rs, t)
    f, grad = eval_height_grad(xi[:, :2], c, w, sigma, cutoff)
    r = xi[:, 2] - z_off - f
    g = np.stack([-grad[:, 0], -grad[:, 1], np.ones_like(f)], axis=1)
    J = np.empty((p.shape[0], 6))
    # row i: g_i^T (-R_s [p_i]x), then g_i^T
    J[:, :3] = np.einsum("qa,ab,qbc->qc", g, -Rs, skew_rows(p))
    J[:, 3:] = g
    return f, grad, r, J


def eval_adjoint_xy(q, c, w, sigma, cutoff, gbar_f):
    """Adjoint of f at world queries for L = sum_i gbar_i f_i:
    dL/dq_i = gbar_i grad f(q_i),  dL/dw = Phi(q)^T gbar."""
    f, grad = eval_height_grad(q, c, w, sigma, cutoff)
    Phi = phi_dense(q, c, sigma, cutoff)
    return gbar_f[:, None] * grad, Phi.T @ gbar_f


def eval_adjoint_pose(p, Rs, t, z_off, c, w, sigma, cutoff, gbar_f, gbar_r):
    """Adjoint of (f, r) of the pose form for L = sum_i gf_i f_i + gr_i r_i.

    Returns dL/dp (Q x 3, body frame), dL/dw (N) and dL/d(dtheta, dt) (6),
    the latter for the same right perturbation as eval_pose."""
    p = np.asarray(p, np.float64)
    Rs = np.asarray(Rs, np.float64)
    gf = np.asarray(gbar_f, np.float64)
    gr = np.asarray(gbar_r, np.float64)
    xi = to_world(p, Rs, t)
    f, grad = eval_height_grad(xi[:, :2], c, w, sigma, cutoff)
    a = gf - gr  # coefficient of f in L
    d_xi = np.zeros_like(xi)
    d_xi[:, 0] = a * grad[:, 0]
    d_xi[:, 1] = a * grad[:, 1]
    d_xi[:, 2] = gr
    d_p = d_xi @ Rs
    Phi = phi_dense(xi[:, :2], c, sigma, cutoff)
    d_w = Phi.T @ a
    d_pose = np.zeros(6)
    # sum_i dL/dxi_i^T (-R_s [p_i]x) and sum_i dL/dxi_i
    d_pose[:3] = np.einsum("qa,ab,qbc->c", d_xi, -Rs, skew_rows(p))
    d_pose[3:] = d_xi.sum(axis=0)
    return d_p, d_w, d_pose


# ---------------------------------------------------------------------------
# Sparse solve with the stated stopping rule (GPU section, "sparse kernel
# matrix inversion")
# ---------------------------------------------------------------------------

def relres(H, x, b):
    """||b - calH x||_2 / ||b||_2 in float64."""
    r = np.asarray(b, np.float64) - H @ np.asarray(x, np.float64)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def gram_pattern(c, sigma, cutoff, sigma_eps):
    """Structural nonzeros of calH: pairs of centers whose regressor supports
    overlap, i.e. ||c_j - c_k|| <= 2 * cutoff * sigma_t, columns ascending."""
    _, sigma_t = regressor_scale(sigma, sigma_eps)
    r = 2.0 * cutoff * sigma_t
    c = np.asarray(c, np.float64)
    rows = []
    for s in range(0, c.shape[0], 1024):
        d2 = sq_dist(c[s:s + 1024], c)
        rows.extend(np.flatnonzero(row) for row in (d2 <= r * r))
    return rows
