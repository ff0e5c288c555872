/*
 * rbf.h -- C ABI of librbf, the gfx950 (MI355X) RBF terrain hot path.
 *
 * The method (Liu & Zhang, "Terrain-Awared LiDAR-Inertial Odometry for
 * Legged-Wheel Robots Based on Radial Basis Function Approximation"):
 *   f(x; w) = sum_j w_j phi(||x - c_j||),  phi(r) = exp(-r^2 / (2 sigma^2))
 * (eqs. RBF_fml, RBF_def), centers chosen adaptively on a mesh (subsection
 * "The RBF Approximation Model"), weights estimated by ridge regression on
 * the moment-corrected regressor m(x) (eq. RBF_estimator and the ridge
 * estimator after it) and updated recursively scan by scan (eqs.
 * weights_update, H_update, kf_w_update, H_inverse_update), then evaluated
 * with its gradient and the manifold residual / Jacobian (eqs.
 * residual_manifold_left_wheel, manifold_derivative, manidolf_grad_detail,
 * manifold_grad_2).
 *
 * Conventions (all entry points)
 *   - Every array argument is a DEVICE pointer owned by the caller, unless
 *     the comment says "host". The library never frees or retains caller
 *     memory after a call returns.
 *   - Matrices are row-major. Sizes are int64_t.
 *   - Work is enqueued on the context's HIP stream and is asynchronous,
 *     except where an argument is documented as a host output (the call
 *     then synchronises the stream before returning).
 *   - Argument errors are detected on the host and returned before any
 *     launch. Errors found by kernels (non-positive Cholesky pivot,
 *     non-finite input, capacity overflow) are recorded in a device status
 *     word; rbf_sync_status() returns and clears it.
 *   - A context is bound to one device and one stream; it is not
 *     thread-safe. No C++ exception crosses this ABI.
 *   - Kernel truncation: phi is taken as exactly zero for r > cutoff*sigma
 *     and kept for r == cutoff*sigma (the paper calls the kernel compactly
 *     supported without giving the radius; cutoff = 3 is the default).
 */
#ifndef RBF_H
#define RBF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RBF_OK = 0,
  RBF_E_INVALID_ARG = 1,  /* bad pointer, size, layout or parameter       */
  RBF_E_NOMEM = 2,        /* workspace allocation failed                  */
  RBF_E_NOT_SPD = 3,      /* non-positive pivot in a Cholesky factor      */
  RBF_E_NONFINITE = 4,    /* NaN/Inf in an input or an innovation         */
  RBF_E_NO_CONVERGE = 5,  /* iterative refinement did not reach rtol      */
  RBF_E_CAPACITY = 6,     /* output capacity (cap, kmax, nnz) exceeded     */
  RBF_E_HIP = 7           /* a HIP runtime call failed                    */
} rbf_status;

typedef enum { RBF_F64 = 0, RBF_F32 = 1, RBF_BF16 = 2 } rbf_prec;

enum { RBF_SELECT_RADIUS = 0, RBF_SELECT_VOXEL = 1 };

/* Model and filter parameters.
 *   sigma     Gaussian bandwidth of phi (eq. RBF_def), metres.
 *   cutoff    truncation radius in units of sigma (3.0 by default).
 *   sigma_eps std of the isotropic xy point noise; the regressor is then
 *             m(x) = (sigma^2/sigma_t^2) kappa_{sigma_t}(x; c) with
 *             sigma_t^2 = sigma^2 + sigma_eps^2 (moment regressor in the
 *             ridge-regression subsection), truncated at cutoff*sigma_t.
 *   lambda    ridge penalty; calH = lambda I + sum_i m(x_i) m(x_i)^T.
 *   R         height-measurement variance. The paper writes the Woodbury
 *             update with R = 1; here the covariance is P = R calH^{-1},
 *             so w does not depend on R and P scales with it. */
typedef struct {
  double sigma;
  double cutoff;
  double sigma_eps;
  double lambda;
  double R;
} rbf_params;

typedef struct rbf_ctx rbf_ctx;   /* device, stream, status word, workspace */
typedef struct rbf_grid rbf_grid; /* neighbour-binned copy of a center set  */

/* ------------------------------------------------------------------ ctx */

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the null stream). *out receives the handle. */
rbf_status rbf_ctx_create(rbf_ctx** out, int device, void* hip_stream);
/* Destroy a context and free its workspace (synchronises its stream).
 * Batched and solve plans made on the context use its device and stream
 * until they are destroyed: while any is alive the call returns
 * RBF_E_INVALID_ARG and destroys nothing. */
rbf_status rbf_ctx_destroy(rbf_ctx* ctx);
/* Re-bind the context to another stream of the same device. */
rbf_status rbf_ctx_set_stream(rbf_ctx* ctx, void* hip_stream);
/* Schedule of rbf_update on this context: streams = 1 (the default) runs
 * everything on the context's stream; streams = 2 runs each batch's
 * covariance product on the context's stream while the next batch's
 * regressor rows, gather, Cholesky and triangular solve run on a second
 * stream of the library's. Results are bitwise the same. (On one MI355X
 * the two streams contend for CUs and the two-stream schedule measured
 * slower.) The two-stream schedule cannot be captured into a graph:
 * rbf_update and rbf_update_active on a capturing stream return
 * RBF_E_INVALID_ARG, before any launch, while streams = 2. */
rbf_status rbf_ctx_set_update_streams(rbf_ctx* ctx, int32_t streams);
/* Form of the covariance update of rbf_update on this context (mixed form
 * with FP32 products only). on = 0 (the default): P -= V V^T. on != 0: the
 * Joseph form P <- (I - K H) P (I - K H)^T + K R K^T of the Kalman update
 * (eq. H_inverse_update written for the covariance), expanded as
 * P - K U^T - U K^T + K S K^T with the gain K = U S^{-1} formed in FP64 and
 * the three products on FP32 MFMA accumulated into the FP64 P (lower tiles,
 * mirrored, so P stays exactly symmetric). Equal to the default in exact
 * arithmetic; with rounded products its terms are larger than V V^T and
 * cancel. rbf_update with the Joseph form on returns RBF_E_INVALID_ARG unless
 * gemm_prec is RBF_F32 and the context uses one stream. */
rbf_status rbf_ctx_set_update_joseph(rbf_ctx* ctx, int32_t on);
/* Synchronise the stream, return the first device-side error recorded
 * since the last call (RBF_OK if none) and clear it. */
rbf_status rbf_sync_status(rbf_ctx* ctx);
/* Index attached to the last device error returned by rbf_sync_status
 * (the batch index for rbf_update, the row for capacity errors), or -1. */
int64_t rbf_last_error_index(const rbf_ctx* ctx);
/* Human-readable text of the last error seen by this context (static
 * storage inside the context; valid until the next call). */
const char* rbf_last_error(const rbf_ctx* ctx);
const char* rbf_status_string(rbf_status s);

/* ------------------------------------------------------ center selection */

/* Adaptive center selection (subsection "The RBF Approximation Model").
 * Candidate nodes are the cell centers of a `res` mesh over the ROI
 * roi = {x0, y0, x1, y1} (host array): nx = ceil((x1-x0)/res),
 * ny = ceil((y1-y0)/res), node (i, j) = (x0+(i+1/2)res, y0+(j+1/2)res).
 * A node is accepted iff its support count is strictly greater than thr
 * ("exceeds"):
 *   RBF_SELECT_RADIUS  points with ||p - node||^2 <= r_kd^2 (the k-d tree
 *                      radius count of the paper, done exactly by binning),
 *   RBF_SELECT_VOXEL   points with floor((p - (x0,y0)) / res) == (i, j).
 * xy: M x 2 f64. centers_out: cap x 2 f64, accepted nodes in mesh order
 * (y outer, x inner). *n_out (host) receives the number accepted; the call
 * synchronises. Returns RBF_E_CAPACITY (and writes the first cap) if more
 * than cap nodes are accepted. */
rbf_status rbf_select_centers(rbf_ctx* ctx, const double* xy, int64_t M,
                              const double* roi, double res, double r_kd,
                              int32_t thr, int32_t mode, double* centers_out,
                              int64_t cap, int64_t* n_out);

/* The same selection applied frame by frame, for a growing center set.
 * counts (device, nx * ny int32, zero before the first frame, kept by the
 * caller between frames) holds each node's support count over every point
 * passed so far; this call adds the M points' counts. A node becomes a
 * center in the call whose points take its count past thr; those nodes are
 * written to centers_out (cap x 2 f64) in mesh order and *n_new (host)
 * receives their number. Over all calls the centers are exactly those of
 * rbf_select_centers on all the points together. Synchronises. If more
 * than cap nodes would be new, returns RBF_E_CAPACITY and leaves counts
 * unchanged. Counts are int32 (at most 2^31 - 1 points per node). */
rbf_status rbf_select_centers_grow(rbf_ctx* ctx, const double* xy, int64_t M,
                                   const double* roi, double res, double r_kd,
                                   int32_t thr, int32_t mode, int32_t* counts,
                                   double* centers_out, int64_t cap,
                                   int64_t* n_new);

/* Grow the state of the recursive update from n_old to n_new centers (the
 * new centers appended after the old ones): the new weights start at 0 and
 * the new rows and columns of P at the prior (R/lambda) I with no coupling
 * to the old centers (calH gains lambda on the new diagonal entries; the
 * ridge estimator's prior, subsection "The RBF Weight Estimate by Ridge
 * Regression"). In place: w (device, capacity >= n_new) and P (device,
 * row-major, leading dimension ldp >= n_new) already hold the old state in
 * their first n_old entries / n_old x n_old block; only the new rows and
 * columns are written. Asynchronous. Points absorbed before a center
 * existed do not inform its weight (the recursion then equals the ridge
 * estimator with each point's regressor restricted to the centers that
 * existed when it was absorbed). */
rbf_status rbf_state_grow(rbf_ctx* ctx, const rbf_params* params, double* w,
                          double* P, int64_t ldp, int64_t n_old,
                          int64_t n_new);

/* --------------------------------------------------------------- binning */

/* Build the neighbour-binned center table used by every kernel below:
 * square bins of side slightly above cutoff*max(sigma, sigma_t), so all
 * centers within the kernel support of a point lie in its 3x3 bins, and,
 * for the evaluation kernels, a second sorted copy over bins of side
 * 1.01*cutoff*sigma/3 (at most 16384 of them per axis; more returns
 * RBF_E_INVALID_ARG). The centers (N x 2 f64, device) are copied; the
 * caller may free them after the call. The grid owns its device memory
 * until rbf_grid_destroy. The call synchronises (it reads the centers'
 * bounding box). */
rbf_status rbf_grid_create(rbf_ctx* ctx, const rbf_params* params,
                           const double* centers, int64_t N, rbf_grid** out);
rbf_status rbf_grid_destroy(rbf_grid* grid);
/* The same call with the argument order of the center-binning step of the
 * evaluation path (centers, N, then the parameters): bins the centers the
 * kernel matrix and its evaluation are built on (eq. rbf_kernel, compact
 * support; subsection "The RBF Approximation Model"). */
rbf_status rbf_bin_centers(rbf_ctx* ctx, const double* centers, int64_t N,
                           const rbf_params* params, rbf_grid** out);
/* Declare the grid's centers nodes of a square mesh: node (i, j) at
 * (x0 + i res, y0 + j res) for integers i, j. This is how the paper places
 * centers: candidate nodes of a mesh of given resolution over the region
 * of interest (section on center selection); rbf_select_centers returns
 * such nodes with x0 = roi[0] + res/2, y0 = roi[1] + res/2. Every center
 * must lie on a node (up to the rounding of that formula) and no two on
 * the same node. Afterwards rbf_eval, rbf_eval_at, rbf_eval_gn and
 * rbf_eval_noalloc on this grid use the mesh form: the Gaussian factors
 * over the axes, so a point's support is a fixed window of nodes read from
 * a dense node array, with one exponential per window row and column
 * instead of one per candidate. Results equal the binned form up to
 * rounding (the support test is taken on the same scaled squared
 * distance). rbf_eval_adjoint and the assembly keep the binned form.
 * res = 0 returns the grid to the binned form. The dense node array covers
 * the centers' node range plus a margin of the window width: at most
 * 16384 nodes per axis and 2^26 in all; the support may span at most 12
 * nodes per axis (2 (cutoff sigma / res + 1/64) < 12). The grid holds the
 * node map (4 bytes per node) until rbf_grid_destroy; the evaluations keep
 * the node weights in the context's workspace (8 or 4 bytes per node).
 * Set the mesh before a batched plan that evaluates on the grid is made:
 * while such a plan exists (its captured launches keep the node map's
 * address and the form) this call returns RBF_E_INVALID_ARG, and so does
 * rbf_grid_destroy on the grid.
 * Errors: RBF_E_INVALID_ARG (a center off the mesh, two on one node, too
 * many nodes or too wide a window; the grid then keeps its previous form),
 * RBF_E_NOMEM. Synchronises the context's stream. */
rbf_status rbf_grid_set_mesh(rbf_ctx* ctx, rbf_grid* grid, double x0, double y0,
                             double res);
/* Host outputs: number of centers, bins in x and y, and the largest number
 * of centers that can lie within one point's 3x3 bins (an upper bound on
 * the nonzeros of one regressor row). Any pointer may be NULL. */
rbf_status rbf_grid_info(const rbf_grid* grid, int64_t* N, int32_t* nbx,
                         int32_t* nby, int32_t* max_candidates);

/* Spatially sort points by the grid's bins (a counting sort; points in one
 * bin keep their input order). xy: M x 2 f64 and z: M f64 (z may be NULL).
 * Writes xy_out, z_out (if z != NULL) and perm (M int32, perm[k] = input
 * index of output k). Sorting is optional: every entry point accepts any
 * point order; compact batches make the covariance update cheaper. */
rbf_status rbf_sort_points(rbf_ctx* ctx, const rbf_grid* grid,
                           const double* xy, const double* z, int64_t M,
                           double* xy_out, double* z_out, int32_t* perm);

/* -------------------------------------------------------------- assembly */

/* Regressor rows m(x_i)^T (eq. rbf_kernel, the columns of the kernel matrix
 * of one scan) in point-major ELL form. Row i holds nnz[i] <= kmax entries
 * (cols[i*kmax + k], vals[i*kmax + k]) with distinct column indices into the
 * original center order, in a fixed order; entries k >= nnz[i] are zero with
 * column 0. prec: RBF_F64 (vals double) or RBF_F32 (vals float).
 * Rows with more than kmax nonzeros are truncated and recorded as
 * RBF_E_CAPACITY (index = row). */
rbf_status rbf_assemble_phi(rbf_ctx* ctx, const rbf_params* params,
                            const rbf_grid* grid, const double* xy, int64_t M,
                            rbf_prec prec, void* vals, int32_t* cols,
                            int32_t* nnz, int32_t kmax);

/* Structural pattern of calH: row j lists the centers k whose regressor
 * supports overlap j's (||c_j - c_k|| <= 2 cutoff sigma_t), in ascending
 * order. rowptr: N+1 int64, colidx: cap int32. *nnz_out (host) receives the
 * total; the call synchronises. RBF_E_CAPACITY if nnz > cap (rowptr is
 * still complete, so the call can be repeated with a larger buffer). */
rbf_status rbf_gram_pattern(rbf_ctx* ctx, const rbf_params* params,
                            const rbf_grid* grid, int64_t* rowptr,
                            int32_t* colidx, int64_t cap, int64_t* nnz_out);

/* Accumulate the information matrix and right-hand side of the ridge
 * estimator: vals += sum_i m(x_i) m(x_i)^T (on the pattern above, CSR with
 * the same rowptr/colidx) and b += sum_i m(x_i) z_i; with add_lambda != 0
 * also vals += lambda on the diagonal (the ridge term, added once).
 * xy: M x 2, z: M, both f64. Deterministic (no atomics). */
rbf_status rbf_assemble_gram(rbf_ctx* ctx, const rbf_params* params,
                             const rbf_grid* grid, const double* xy,
                             const double* z, int64_t M,
                             const int64_t* rowptr, const int32_t* colidx,
                             double* vals, double* b, int32_t add_lambda);

/* Sparse symmetric matrix in CSR form (device arrays; both triangles). */
typedef struct {
  int64_t n;        /* rows (and columns)                                  */
  int64_t nnz;      /* stored entries                                      */
  int64_t* rowptr;  /* n + 1 offsets                                       */
  int32_t* colidx;  /* nnz column indices, ascending within a row          */
  double* vals;     /* nnz values                                          */
} rbf_csr;

enum { RBF_ASSEMBLE_PHI = 1, RBF_ASSEMBLE_GRAM = 2 };

/* Kernel-matrix assembly in one call (eq. rbf_kernel; ridge estimator eq.
 * RBF_estimator with calH = lambda I + sum m m^T, b = sum m z). `what` is
 * RBF_ASSEMBLE_PHI, RBF_ASSEMBLE_GRAM or both or-ed:
 *   PHI   the regressor rows of the M points, as rbf_assemble_phi (prec
 *         RBF_F64 or RBF_F32; phi_val, phi_col, phi_nnz, kmax as there);
 *   GRAM  accumulate the information matrix into H (the pattern of
 *         rbf_gram_pattern in H->rowptr / H->colidx, H->n == N, values
 *         added to H->vals) and b (N) as rbf_assemble_gram (z required,
 *         prec must be RBF_F64; add_lambda adds the ridge term once).
 * Arguments a part does not use may be NULL / 0. Errors as in the two
 * calls it makes (the PHI part runs first). */
rbf_status rbf_assemble(rbf_ctx* ctx, const rbf_params* params, const rbf_grid* grid,
                        const double* xy, const double* z, int64_t M, int32_t what,
                        rbf_prec prec, void* phi_val, int32_t* phi_col, int32_t* phi_nnz,
                        int32_t kmax, rbf_csr* H, double* b, int32_t add_lambda);

/* ------------------------------------------------------ recursive update */

/* Absorb M points into (w, P) by the Kalman-style recursion of eqs.
 * kf_w_update and H_inverse_update, in consecutive batches of `batch`
 * points (0 = library default) taken in the given order. Per batch, with
 * H the B x N regressor block and y = z - H w:
 *   U = P H^T,  S = H U + R I,  L L^T = S (FP64),  V = U L^{-T},
 *   t = L^{-1} y,  w += V t,  P -= V V^T.
 * P is N x N with leading dimension ldp >= N, symmetric in full storage;
 * it is kept exactly symmetric (each lower tile is written to both
 * triangles). gemm_prec selects the operand precision of the covariance
 * product V V^T (RBF_F64: FP64 MFMA; RBF_F32 / RBF_BF16: low-precision
 * operands with FP32 accumulation subtracted from the FP64 P).
 * Batches are committed one at a time: if a batch fails (RBF_E_NOT_SPD,
 * RBF_E_NONFINITE) no later batch runs, and (w, P) is the state after the
 * batches before it. n_done (host, may be NULL): if non-NULL the call
 * synchronises and stores the number of points absorbed; if NULL the call
 * is asynchronous and errors are read with rbf_sync_status. A device error
 * still pending from an earlier asynchronous call (not yet read by
 * rbf_sync_status) makes every batch skip: (w, P) is unchanged, and with
 * n_done the call returns that error with *n_done = 0. */
rbf_status rbf_update(rbf_ctx* ctx, const rbf_params* params,
                      const rbf_grid* grid, double* w, double* P, int64_t ldp,
                      const double* xy, const double* z, int64_t M,
                      int64_t batch, rbf_prec gemm_prec, int64_t* n_done);

/* Active-rows form of the update (eqs. active_rows_weights_update and
 * H_inverse_update, with the active rows of eq. mfk_m_approx): the M points
 * are one scan, and its active set A is every center whose regressor entry
 * is non-zero at one or more of the points (ascending center index). The
 * recursion of rbf_update (same batches, same arithmetic, same gemm_prec)
 * runs on w_A and the A x A block of P only. Afterwards the entries of P
 * coupling A to the other centers (rows A / columns not in A, and the
 * mirror) are zero: the block-diagonal result of eq. H_inverse_update,
 * which keeps P positive semi-definite. w outside A and P outside the rows
 * and columns of A are neither read nor written. This equals rbf_update
 * whenever P couples no center of A to a center outside it (e.g. from the
 * prior (R/lambda) I); otherwise it is the paper's approximation, which
 * drops that coupling. Arguments as for rbf_update, plus: active (device,
 * capacity N int32, may be NULL) receives A; n_active (host, may be NULL)
 * receives |A|. The call synchronises once to size the compact block
 * (|A| x |A| FP64 workspace, grown as needed and kept by the context), so
 * it cannot be captured in a graph. Batches commit one by one as in
 * rbf_update: after a failing batch, w_A and the A x A block hold the
 * state after the batches before it, and the coupling is cleared only if
 * at least one batch was absorbed. */
rbf_status rbf_update_active(rbf_ctx* ctx, const rbf_params* params,
                             const rbf_grid* grid, double* w, double* P,
                             int64_t ldp, const double* xy, const double* z,
                             int64_t M, int64_t batch, rbf_prec gemm_prec,
                             int32_t* active, int64_t* n_active,
                             int64_t* n_done);

/* ----------------------------------------------------------------- solve */

/* Solve calH X = B for the sparse SPD matrix in CSR (rowptr N+1 int64,
 * colidx int32, vals f64; both triangles stored), the "sparse kernel
 * matrix inversion" of the GPU-acceleration section. B and X are N x nrhs
 * (leading dimensions ldb, ldx >= nrhs). The matrix is reordered into
 * dense diagonal / sub-diagonal blocks of its bandwidth, factored in FP64
 * (`inner` must be RBF_F64; any other value returns RBF_E_INVALID_ARG:
 * the factor's time is in dependent latency-bound block steps, which a
 * lower precision would not shorten), and refined in FP64 until
 * ||B_k - calH X_k||_2 <= rtol ||B_k||_2 for every column k, or max_iter
 * sweeps. relres (host, nrhs doubles, may be NULL) and iters (host, may be
 * NULL) report the result; the call synchronises. Returns
 * RBF_E_NO_CONVERGE if rtol was not met, RBF_E_NOT_SPD if the factor
 * broke down. With B = I it returns calH^{-1} (so P = R X). */
rbf_status rbf_solve(rbf_ctx* ctx, int64_t N, const int64_t* rowptr,
                     const int32_t* colidx, const double* vals,
                     const double* B, int64_t ldb, double* X, int64_t ldx,
                     int64_t nrhs, double rtol, int32_t max_iter,
                     rbf_prec inner, double* relres, int32_t* iters);

/* The same solve for repeated use on one sparsity pattern (the Gram
 * pattern of a center set), by nested dissection with dense frontal
 * matrices. rbf_solve_plan_create copies the pattern (rowptr N+1 int64,
 * colidx int32, device, both triangles) to the host once and analyses it:
 * each set of unknowns is cut by the level of a breadth-first search from a
 * pseudo-peripheral unknown (disconnected sets by their components) until
 * at most `leaf` unknowns remain (0: 256); the tree is numbered in
 * postorder. It reserves the fronts' device memory (rbf_solve_plan_info:
 * front_bytes) and synchronises; the plan keeps the device pattern
 * pointers, which must stay valid and unchanged while it lives.
 * rbf_solve_plan_run factors calH (vals, nnz f64, device) front height by
 * front height from the leaves up, every front of a height in one launch
 * per stage: assembly from calH and the children's update matrices, the
 * blocked FP64 Cholesky of the front's own block, the gain on FP64 MFMA and
 * the update matrix by the FP64 covariance product; then solves and refines
 * in FP64 as rbf_solve (same arguments, nrhs <= 65535, same return codes;
 * inner must be RBF_F64: with FP32 products in the update matrices the
 * refinement of the 40k-center map stalls near relres 1e-3; a factor
 * breakdown returns RBF_E_NOT_SPD with the front's node as index).
 * The run synchronises; runs on one plan must not overlap. */
typedef struct rbf_solve_plan rbf_solve_plan;
rbf_status rbf_solve_plan_create(rbf_ctx* ctx, int64_t N, const int64_t* rowptr,
                                 const int32_t* colidx, int32_t leaf,
                                 rbf_solve_plan** out);
rbf_status rbf_solve_plan_run(rbf_solve_plan* plan, const double* vals,
                              const double* B, int64_t ldb, double* X,
                              int64_t ldx, int64_t nrhs, double rtol,
                              int32_t max_iter, rbf_prec inner,
                              double* relres, int32_t* iters);
/* nodes of the dissection tree, front heights, bytes of the fronts and
 * factors, and the largest front (kp + m); any pointer may be NULL. */
rbf_status rbf_solve_plan_info(const rbf_solve_plan* plan, int32_t* nodes,
                               int32_t* levels, int64_t* front_bytes,
                               int32_t* max_front);
rbf_status rbf_solve_plan_destroy(rbf_solve_plan* plan);

/* The dissection alone, on HOST arrays (no device, no context): new2old
 * (N int32) receives the elimination order, node_of (N int32) the tree
 * node of each unknown, parent (cap int32) the parent of each node (-1: the
 * root); *n_nodes the node count (RBF_E_CAPACITY if above cap). For
 * checks of the ordering. */
rbf_status rbf_solve_order_host(int64_t N, const int64_t* rowptr,
                                const int32_t* colidx, int32_t leaf,
                                int32_t* new2old, int32_t* node_of,
                                int32_t* parent, int32_t cap,
                                int32_t* n_nodes);

/* FP64 iterative refinement of the weights of the recursive update against
 * the information form of the ridge estimator (subsection "The RBF Weight
 * Estimate by Ridge Regression", eqs. RBF_estimator, H_update and
 * H_inverse_update: after any sequence of batches the recursion's weights
 * equal calH^{-1} b, calH = lambda I + sum m m^T, b = sum m z, and its
 * covariance is P = R calH^{-1}). Conjugate gradients (Hestenes-Stiefel) on
 * calH w = b from the given w, preconditioned by the recursion's P / R
 * (from covariance products of any precision): per iteration one FP64 CSR
 * product with calH, one FP64 pass over P and three dot products; the
 * residual r = b - calH w is recomputed from w before the result is
 * accepted. Stops when ||r||_2 <= rtol ||b||_2 or after max_iter iterations
 * (0 = only report). rowptr (N+1 int64), colidx (int32), vals (f64): calH
 * in CSR with both triangles and lambda on the diagonal, as
 * rbf_gram_pattern + rbf_assemble_gram (add_lambda once) build it over all
 * absorbed points; b: N f64; P: N x N f64, leading dimension ldp >= N,
 * symmetric positive definite; w: N f64, refined in place. relres (host,
 * may be NULL) receives the final ||r|| / ||b||, iters (host, may be NULL)
 * the iterations done; the call synchronises. Returns RBF_E_NO_CONVERGE (w
 * holds the last iterate) if rtol was not met, also when P / R or calH
 * showed a non-positive curvature. */
rbf_status rbf_refine(rbf_ctx* ctx, int64_t N, const int64_t* rowptr,
                      const int32_t* colidx, const double* vals, const double* b,
                      const double* P, int64_t ldp, double R, double* w, double rtol,
                      int32_t max_iter, double* relres, int32_t* iters);

/* ------------------------------------------------------------ evaluation */

/* Evaluate the terrain model at Q points.
 *   dim == 2: pts are world xy (Q x 2); outputs f (Q) and grad (Q x 2):
 *             f = sum_j w_j phi, grad f = -sum_j w_j phi (x - c_j)/sigma^2
 *             (eqs. RBF_fml, manidolf_grad_detail with the sign of the
 *             derivative of exp restored). pose must be NULL.
 *   dim == 3: pts are body-frame points p (Q x 3) and pose (host, 12
 *             doubles: R row-major then t) maps them to xi = R p + t.
 *             Outputs f, grad at xi_xy, the residual
 *             r = xi_z - z_off - f(xi_x, xi_y) (eq.
 *             residual_manifold_left_wheel, z_off = wheel radius or 0), and
 *             its Jacobian J (Q x 6) for the right perturbation
 *             R <- R Exp(dtheta), t <- t + dt, ordered [dtheta, dt]:
 *             J = [ (p x R^T g)^T, g^T ], g = (-f_x, -f_y, 1)
 *             (eqs. manifold_derivative, manifold_grad_2 with the body
 *             point in the skew matrix).
 * prec RBF_F64: pts and outputs are double; RBF_F32: float (w stays f64
 * and is rounded once per call). Any output pointer except f may be NULL.
 * xy points (dim 2), grad and jac are read and written two elements at a
 * time and must be aligned to two elements (16 bytes in FP64, 8 in FP32);
 * a misaligned pointer returns RBF_E_INVALID_ARG. Candidate centers come
 * from the grid's evaluation bins (side about cutoff*sigma/3): each bin row
 * within the support radius is read only over the bins that meet the
 * support circle. */
rbf_status rbf_eval(rbf_ctx* ctx, const rbf_params* params,
                    const rbf_grid* grid, const double* w, const void* pts,
                    int64_t Q, int32_t dim, const double* pose, double z_off,
                    rbf_prec prec, void* f, void* grad, void* resid,
                    void* jac);

/* Evaluation at a pose increment, for differentiation with respect to the
 * pose (form 3): as rbf_eval in the pose form (dim 3), at
 *   R = R0 Exp(delta[0:3]),  t = t0 + delta[3:6],
 * around a linearisation pose pose0 (host, 12 doubles: R0 row-major then
 * t0), with the increment delta (DEVICE, 6 f64) read on the device, so that
 * it never travels to the host. Exp is the exponential map of SO(3)
 * (Rodrigues' formula), formed by a one-thread kernel in FP64. */
rbf_status rbf_eval_at(rbf_ctx* ctx, const rbf_params* params, const rbf_grid* grid,
                       const double* w, const void* pts, int64_t Q, const double* pose0,
                       const double* delta, double z_off, rbf_prec prec, void* f,
                       void* grad, void* resid, void* jac);

/* Adjoint of rbf_eval_at: as rbf_eval_adjoint in the pose form, with the
 * pose gradient taken with respect to the increment: d_delta (device, 6
 * f64, may be NULL) is ACCUMULATED with
 *   d_delta[0:3] += J_r(delta[0:3])^T dL/dtheta,  d_delta[3:6] += dL/dt,
 * where dL/dtheta is the gradient for the right perturbation
 * R <- R Exp(theta) at the evaluated pose and J_r is the right Jacobian of
 * SO(3) (Exp(v + e) = Exp(v) Exp(J_r(v) e) to first order). */
rbf_status rbf_eval_adjoint_at(rbf_ctx* ctx, const rbf_params* params, const rbf_grid* grid,
                               const double* w, const void* pts, int64_t Q,
                               const double* pose0, const double* delta, rbf_prec prec,
                               const void* gbar_f, const void* gbar_r, void* d_pts,
                               double* d_w, double* d_delta);

/* Largest center count (grid N) that rbf_eval_noalloc accepts. */
#define RBF_EVAL_NOALLOC_MAX_CENTERS 131072

/* rbf_eval for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results as rbf_eval (bitwise), but the call
 * allocates nothing: its packed center table (x, y, w and index per
 * center, 32 bytes in FP64, 16 in FP32) lives in a device array of the
 * library of RBF_EVAL_NOALLOC_MAX_CENTERS x 32 bytes (4 MiB), one per GPU,
 * held until the process ends. The caller still passes the inputs and
 * outputs. Returns
 * RBF_E_CAPACITY, before any launch, if the grid holds more than
 * RBF_EVAL_NOALLOC_MAX_CENTERS centers. On a grid in the mesh form
 * (rbf_grid_set_mesh) the array holds the dense node weights instead (8 or
 * 4 bytes per node of the padded mesh), and a mesh whose node weights
 * exceed the 4 MiB returns RBF_E_CAPACITY. Every call on one GPU, from any
 * context, shares that GPU's array and rewrites its first entries, so
 * calls that overlap on one GPU (on different streams, or from several
 * threads) race and must be ordered by the caller. */
rbf_status rbf_eval_noalloc(rbf_ctx* ctx, const rbf_params* params,
                            const rbf_grid* grid, const double* w, const void* pts,
                            int64_t Q, int32_t dim, const double* pose, double z_off,
                            rbf_prec prec, void* f, void* grad, void* resid,
                            void* jac);

/* Gauss-Newton terms of the manifold residual, fused into the evaluation:
 * the Levenberg-Marquardt minimisation of eq. cost_fn (subsection "The
 * Manifold Constraints") takes the manifold term's normal-equation blocks
 * sum_i J_i^T J_i and sum_i J_i^T r_i (eqs. residual_manifold_left_wheel,
 * manifold_derivative, manifold_grad_2; the penalty weight is applied by
 * the caller):
 * with r_i and J_i as rbf_eval computes them in the pose form (dim 3),
 * writes JtJ = sum_i J_i^T J_i (device, 6 x 6 f64, both triangles),
 * Jtr = sum_i J_i^T r_i (device, 6 f64) and, if rtr is not NULL,
 * sum_i r_i^2 (device, 1 f64), without writing per-point outputs. Points
 * in prec (F32: Q x 3 float, F64: Q x 3 double); the sums are formed in
 * FP64 in a fixed order (per-block partials, then blocks in order), so
 * results are reproducible. Q = 0 writes zeros. */
rbf_status rbf_eval_gn(rbf_ctx* ctx, const rbf_params* params, const rbf_grid* grid,
                       const double* w, const void* pts, int64_t Q, const double* pose,
                       double z_off, rbf_prec prec, double* JtJ, double* Jtr, double* rtr);

/* Adjoint of rbf_eval for L = sum_i gbar_f[i] f_i + gbar_r[i] r_i
 * (gbar_r only for dim == 3; either gbar may be NULL = zero).
 *   d_pts  (Q x dim, same precision as pts, may be NULL): dL/dpts,
 *   d_w    (N f64, may be NULL): dL/dw, ACCUMULATED (+=) into the buffer,
 *   d_pose (6 f64, device, may be NULL, dim == 3): dL/d[dtheta, dt],
 *          ACCUMULATED (+=).
 * Accumulations use atomics, so d_w and d_pose are reproducible only up to
 * the order of floating-point additions. */
rbf_status rbf_eval_adjoint(rbf_ctx* ctx, const rbf_params* params,
                            const rbf_grid* grid, const double* w,
                            const void* pts, int64_t Q, int32_t dim,
                            const double* pose, rbf_prec prec,
                            const void* gbar_f, const void* gbar_r,
                            void* d_pts, double* d_w, double* d_pose);

/* -------------------------------------------------------- many patches */

/* One independent terrain patch for the batched form: its own centers
 * (grid), weights and covariance, a scan of update points and a set of
 * evaluation points. All pointers are device pointers except `pose`
 * (host values, R row-major then t, read when the plan is built). */
typedef struct {
  const rbf_grid* grid;
  double* w;            /* N_p, in/out                                    */
  double* P;            /* N_p x ldp, in/out, symmetric                   */
  int64_t ldp;
  const double* xy;     /* M x 2 update points                            */
  const double* z;      /* M heights                                      */
  int64_t M;
  const void* pts;      /* Q x dim evaluation points (plan's precision)   */
  int64_t Q;
  double pose[12];      /* dim == 3 only                                  */
  void* f;              /* Q, required                                    */
  void* grad;           /* Q x 2 or NULL                                  */
  void* resid;          /* Q or NULL (dim == 3)                           */
  void* jac;            /* Q x 6 or NULL (dim == 3)                       */
  int64_t batch;        /* Kalman batch of this patch, 0 = plan default   */
} rbf_patch;

typedef struct rbf_batched rbf_batched;

/* Tile shape of the batched covariance products (FP64; the FP32 and BF16
 * products always use 128x128 tiles). */
enum {
  RBF_TILE_AUTO = 0, /* per patch: whole rounds of 128x128 tiles, the rest as
                        32x64 sub-tiles (the rule of rbf_update)            */
  RBF_TILE_128 = 1,  /* 128x128 tiles, 8 waves each                         */
  RBF_TILE_SUB = 2   /* every tile as 32x64 sub-tiles (more, shorter groups) */
};

/* Plan the recursive update (as rbf_update, eqs. kf_w_update and
 * H_inverse_update) followed by the evaluation (as rbf_eval) of n
 * independent patches (n <= 65535), to be run as ONE hipGraph launch. The
 * patches advance in lockstep over their Kalman batches: round t absorbs
 * batch t of every patch that has one, and each stage of a round (regressor
 * rows, U, S, every Cholesky step, the gain, w, the covariance product) is
 * one kernel launch over all of the round's patches. Each patch gets its own
 * device workspace, reserved here (about 16 (N_p + 32) B_p + 24 B_p^2 bytes
 * plus the grouped-gather blocks, B_p its batch rounded up to 64), so a run
 * allocates nothing. Results equal those of rbf_update and rbf_eval called
 * on each patch, bit for bit. The patches are split into `chains` (1..4)
 * sets of about equal cost (longest processing time first on N_p^2 M_p);
 * each set advances through its own rounds on its own stream of the graph,
 * so the latency-bound stages of one set run beside the covariance
 * products of another. `tile` is one of RBF_TILE_*; `default_batch`
 * (0: 1024) is the batch of patches whose own `batch` is 0. The patch table
 * is copied; the buffers it points to must stay valid while the plan lives.
 * Calls on `ctx` must not run concurrently with the plan's runs. The Joseph
 * option of the context does not apply to the plan. */
rbf_status rbf_batched_plan(rbf_ctx* ctx, const rbf_params* params,
                            const rbf_patch* patches, int32_t n, int32_t dim,
                            rbf_prec eval_prec, rbf_prec gemm_prec,
                            int32_t tile, int32_t chains,
                            int64_t default_batch, double z_off,
                            rbf_batched** out);
/* Enqueue one run of the plan on the context's stream (ordered after its
 * earlier work, and before its later work): the first call captures the
 * graph on the plan's own stream, later calls relaunch it. Asynchronous. */
rbf_status rbf_batched_run(rbf_batched* b);
/* Synchronise; return the device error of the last run (RBF_OK if none)
 * and, in *failed_patch (host, may be NULL), the lowest index of a patch
 * whose update failed (-1 if none). A failed patch keeps the state of the
 * batch before its failing one (its later batches are skipped, its
 * evaluation still runs on that state); the other patches are not
 * affected. */
rbf_status rbf_batched_sync(rbf_batched* b, int32_t* failed_patch);
rbf_status rbf_batched_destroy(rbf_batched* b);

/* ----------------------------------------------------------- diagnostics */

/* Kernel timing with HIP events recorded on the context stream around each
 * launch of a kernel family (for roofline figures). Off by default; do not
 * enable while the stream is being captured into a graph. */
enum {
  RBF_PROF_SYRK = 0,   /* covariance product P -= V V^T                   */
  RBF_PROF_EVAL = 1,   /* evaluation kernel of rbf_eval                   */
  RBF_PROF_TRSM = 2,   /* V^T = L^{-1} U^T of rbf_update                  */
  RBF_PROF_CHOL = 3,   /* Cholesky of S (all launches of one batch)       */
  RBF_PROF_GATHER = 4, /* U^T = H P gather of rbf_update                  */
  RBF_PROF_KINDS = 5
};
/* Enable (non-zero) or disable timing; enabling clears the accumulators. */
rbf_status rbf_profile_enable(rbf_ctx* ctx, int32_t enable);
/* Synchronise, then report the summed elapsed time (ms, host) and the
 * number of timed launches (host) of one kind since the last read, and
 * reset that kind. */
rbf_status rbf_profile_read(rbf_ctx* ctx, int32_t kind, double* total_ms,
                            int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* RBF_H */
