// Internal interface between the update orchestration and the covariance
// product kernels.
#pragma once

#include <cmath>

#include "internal.hpp"

namespace rbf {

// Points absorbed per Kalman batch when the caller passes batch = 0.
constexpr int64_t UPDATE_DEFAULT_BATCH = 1024;

// Regressor m(x, c) = scale * exp(-d^2 / den) for d^2 <= rc2 (moment
// regressor with sigma_t^2 = sigma^2 + sigma_eps^2, cut at cutoff sigma_t).
struct RegKU {
  double rc2, den, scale;
};
inline RegKU regku(const rbf_params* p) {
  const double st = std::sqrt(p->sigma * p->sigma + p->sigma_eps * p->sigma_eps);
  RegKU k;
  k.rc2 = (p->cutoff * st) * (p->cutoff * st);
  k.den = 2.0 * st * st;
  k.scale = (p->sigma * p->sigma) / (st * st);
  return k;
}

// Output tile of the covariance product (rows and columns of P).
constexpr int SYRK_TILE = 128;

// P -= V V^T for V^T = Ut[0:Bc, 0:N] (row-major, leading dimension ldu);
// lower tiles are computed and written to both triangles of P, so P stays
// exactly symmetric. prec selects the operand precision of the product.
// part 0 computes every tile; part 1 only the tiles (I, J) with flags[I] or
// flags[J] set (flags per SYRK_TILE block of rows), part 2 the others, with
// the low-precision operand copy made by part 1 and reused by part 2.
// Launches belong to launch group seq.
rbf_status syrk_update(rbf_ctx* ctx, double* P, int64_t ldp, int64_t N, const double* Ut,
                       int64_t ldu, int32_t Bc, rbf_prec prec, const int32_t* flags,
                       int part, int64_t seq);

// Joseph form of the same update with FP32 products: with the gain
// K = U S^{-1} = V L^{-1} formed in FP64 (K^T = L^{-T} V^T from LiT, the
// rows of L^{-1} transposed, n = Bpc), P += -(K U^T + U K^T) + K S K^T,
// K S K^T = V V^T, each product on FP32 MFMA from FP32-rounded operands and
// accumulated into the FP64 P with the mirrored write. Ut: U^T of the batch.
rbf_status syrk_update_joseph(rbf_ctx* ctx, double* P, int64_t ldp, int64_t N, const double* Vt,
                              const double* Ut, const double* LiT, int64_t ldu, int32_t Bc,
                              int32_t Bpc, int64_t seq);

// Device workspace of rbf_update for N centers, kmax candidates per point
// and batches of at most Bmax points (all slots grown up front, so later
// calls with these sizes allocate nothing).
struct UpdWs {
  double* vals;
  int32_t* cols;
  int32_t* nnz;
  double* Ut;
  double* Ut2;     // second U^T buffer (consecutive batches alternate)
  double* Vt;      // V^T = L^{-1} U^T, two buffers (consecutive batches alternate)
  double* Vt2;
  double* LiT;     // L^{-1} transposed (Bp x Bp)
  int32_t* flags;  // 2 x ceil(N / SYRK_TILE) touched-block flags
  double* S;
  double* Lb;
  double* Linv;
  double* wpart;
  // gather by groups of 64 batch rows (when N <= GATHER_GROUP_NMAX): per
  // group the distinct rows of P its points touch (glist, Rcap entries),
  // their count rounded up to 4 (gR), and the dense block of H over those
  // rows (gH, Rcap x 64, rank-major)
  int32_t* glist;
  int32_t* gR;
  double* gH;
  int64_t Rcap;
};

// Largest N for the grouped gather (its LDS bitmap has one bit per center).
constexpr int64_t GATHER_GROUP_NMAX = (int64_t)1 << 17;

// A group of 64 batch rows whose points touch more distinct rows of P than
// this (points not in spatial order) takes the per-point gather and S
// kernels instead of the dense group products, whose work grows with the
// number of distinct rows.
constexpr int32_t GATHER_GROUP_RMAX = 512;
rbf_status update_workspace(rbf_ctx* ctx, int64_t N, int32_t kmax, int64_t Bmax,
                            rbf_prec gemm_prec, UpdWs* ws);

// FP64 blocked Cholesky of the n x n (n a multiple of 64, row-major,
// leading dimension n) symmetric matrix S, lower triangle used. S is
// overwritten with intermediate trailing blocks; the factor is returned as
// its off-diagonal 64x64 blocks in Lb (n x n, leading dimension n) and the
// inverses of its diagonal blocks in Linv ((n/64) x 64 x 64). A breakdown
// records RBF_E_NOT_SPD with `index` in the status word. Launches belong to
// launch group seq.
rbf_status chol_blocked(rbf_ctx* ctx, double* S, int32_t n, double* Lb, double* Linv,
                        int64_t index, int64_t seq, double* LiT = nullptr);

// With LiT (n x n, leading dimension n, zero above the diagonal blocks on
// entry), chol_blocked also forms X = L^{-1} transposed: LiT[c][r] = X[r][c].
// linv_apply then computes V^T = X U^T (n x ncols, rows of U^T with leading
// dimension ldu) into Vt (leading dimension ldu) on FP64 MFMA: the block
// triangular solve as one product (FP64 in every form: the gain V feeds the
// weight update w += V t directly).
rbf_status linv_apply(rbf_ctx* ctx, const double* LiT, int32_t n, const double* Ut,
                      int64_t ldu, int64_t ncols, double* Vt, int64_t seq);

// X := L^{-1} X (trans = false) or X := L^{-T} X (trans = true) in place for
// X with nblk*64 rows, ncols columns and leading dimension ldx, with L given
// as by chol_blocked (Lb with leading dimension ldl, Linv).
rbf_status trsm_blocks(rbf_ctx* ctx, double* X, int64_t ldx, int64_t ncols, int32_t nblk,
                       const double* Lb, int64_t ldl, const double* Linv, bool trans,
                       int64_t seq);

// Argument checks shared by rbf_update and rbf_update_active.
rbf_status update_check(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g, const double* w,
                        const double* P, int64_t ldp, const double* xy, const double* z,
                        int64_t M, int64_t batch, rbf_prec gemm_prec);

// Enqueue the recursive update of (w, P) (N x N, leading dimension ldp) by
// the M points xy, z in batches of B. colmap (device, one int32 per center
// of g, or null) maps a center to its column: the active-rows form runs the
// update on its compact block with colmap = compact index of each active
// center. Only enqueues; update_done reads the outcome.
rbf_status update_run(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                      const int32_t* colmap, int64_t N, double* w, double* P, int64_t ldp,
                      const double* xy, const double* z, int64_t M, int64_t B,
                      rbf_prec gemm_prec);

// Wait for the context's stream and report the points absorbed: M, or the
// points of the batches before the first failing one (whose error is
// returned and cleared). seq0 is the launch group of the call's first
// batch; an error recorded before it leaves n_done = 0.
rbf_status update_done(rbf_ctx* ctx, int64_t M, int64_t B, int64_t seq0, int64_t* n_done);

}  // namespace rbf
