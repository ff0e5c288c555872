// Internal interface between the update orchestration and the covariance
// product kernels.
#pragma once

#include <cmath>
#include <vector>

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

// Threads of a grouped-gather workgroup (one group of 64 batch rows), and
// its dynamic LDS for N centers: the bitmap, the word ranks and one count
// per wave.
constexpr int GATHER_GROUP_NT = 1024;
inline int32_t gather_group_words(int64_t N) { return (int32_t)((N + 31) / 32); }
inline size_t gather_group_lds(int32_t words) {
  return sizeof(uint32_t) * (2 * (size_t)words + GATHER_GROUP_NT / 64);
}

// k extent step of the BF16 operands (their k extent is Bc rounded up to it).
constexpr int SYRK_BF16_KSTEP = 64;

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

// ------------------------------------------------ grouped (many patches)
//
// The batched form runs the recursion of many independent patches in
// lockstep: round t absorbs batch t of every patch that has one, and each
// stage of the round (regressor rows, U, S, Cholesky steps, V, w, the
// covariance product) is ONE launch over all of the round's jobs. A job is
// one patch's batch; its workgroups take it from blockIdx.z (the grid is the
// largest job's, the others' surplus workgroups return at once) or, for the
// covariance products, from a prefix of per-job workgroup counts. Each job
// runs the same bodies, with the same arguments, as the single-patch
// launches, so a patch's results are the same bit for bit.
struct GJob {
  double* P;  // patch state
  int64_t ldp, N;
  double* w;
  const double* xy;  // this batch's points and heights
  const double* z;
  const double* cxy;  // the patch's center grid
  const int32_t* idx;
  const int32_t* start;
  GridGeom g;
  RegKU rk;
  double R;  // noise variance of the heights
  int32_t kmax;
  int32_t Bc, Bp;  // points of the batch, and padded to a multiple of 64
  int64_t index;   // status index (patch << 32) + batch
  int64_t seq;     // launch group (batch + 1) of the patch's status words
  int32_t* status;
  double* vals;  // workspace of the patch (as UpdWs)
  int32_t* cols;
  int32_t* nnz;
  double* Ut;
  int64_t ldu;
  double* S;
  double* Lb;
  double* LiT;
  double* Linv;
  double* Vt;
  double* wpart;
  int32_t* glist;  // null: no grouped gather for this patch
  int32_t* gR;
  double* gH;
  int64_t Rcap;
  int32_t words;   // 32-bit words of the grouped gather's bitmap
  int64_t ncols;   // columns of U^T in the gain product V^T = L^{-1} U^T
                   // (N + 1 in the recursion: U and the innovation)
  int32_t Kp;      // k extent of the BF16 operands
  void* vlo;       // low-precision copy of V^T (FP32 / BF16 products)
  int64_t T, per_xcd, main_per_xcd;  // covariance product: tiles, per XCD,
                                     // of which as 128x128 tiles
};

// Launch shapes of one round (largest job per stage, grouped covariance
// product prefixes), computed on the host from the round's jobs.
struct GRound {
  const GJob* jobs;  // device array of the round's jobs
  int32_t n;
  int32_t rows_x, gg_x, gm_x, gm_y, gu_x, gu_y, sg_x, s_x, s_y, zero_x;
  size_t gg_lds;
  int32_t nsteps;                 // Cholesky step launches (largest nblk - 1)
  const int32_t* step_x;          // host: workgroups of step kb, kb < nsteps
  int32_t lr_x, la_x, wp_x, wp_y, ws_x, cvt_x, cvt_y;
  const int64_t* pre_main;        // device: prefix of 128x128-tile workgroups
  const int64_t* pre_tail;        // device: prefix of sub-tile workgroups
  int64_t n_main, n_tail;         // total workgroups of each
  // Cholesky steps in the split form (a panel launch, then a trailing
  // launch: throughput over many factors) instead of one launch per step
  // (the critical path of few factors)
  int32_t chol_split;
};

// Workgroups of Cholesky step kb for a batch of Bp rows (0: no such step).
__host__ __device__ inline int32_t chol_step_groups(int32_t Bp, int32_t kb) {
  const int32_t nblk = Bp / 64, m = nblk - kb - 1;
  if (m <= 0) return 0;
  return m + m * (m + 1) / 2 + kb + kb * (nblk - 1 - kb);
}

// Job of workgroup b of a prefix-mapped launch: the last j with pre[j] <= b
// (jobs without workgroups have pre[j] == pre[j + 1] and are passed over).
// The search is uniform across the workgroup.
__device__ inline int32_t job_of(const int64_t* __restrict__ pre, int32_t n, int64_t b) {
  int32_t lo = 0, hi = n;  // pre[lo] <= b < pre[hi]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Enqueue round r on the context's stream: every stage of the recursion
// for all of its jobs, covariance product (prec) included.
rbf_status update_round_grouped(rbf_ctx* ctx, const GRound& r, rbf_prec prec);

// The blocked Cholesky of every job's S (Bp x Bp, leading dimension Bp)
// with L^{-1} transposed in LiT, as chol_blocked does for one matrix (uses
// the jobs' S, Bp, Lb, Linv, LiT, status, index and seq; the round's
// zero_x, nsteps, step_x and lr_x).
rbf_status chol_grouped(rbf_ctx* ctx, const GRound& r);

// The covariance products of a round, and its V^T = L^{-1} U^T (syrk.hip).
rbf_status syrk_grouped(rbf_ctx* ctx, const GRound& r, rbf_prec prec);
rbf_status linv_apply_grouped(rbf_ctx* ctx, const GRound& r);

// Covariance product tiles of N rows: T lower 128x128 tiles, per_xcd of
// them per XCD, main_per_xcd of those computed whole and the rest as
// 32x64 sub-tiles (the single-call rule: whole rounds of two workgroups per
// CU as 128x128 tiles).
void syrk_tiles(int64_t N, int32_t cu_count, int64_t* T, int64_t* per_xcd,
                int64_t* main_per_xcd);
constexpr int SYRK_SUB_PER_TILE = 8;

// Sparse solve helpers (solve.hip): R (N x nrhs, leading dimension nrhs)
// = B - calH X for calH in CSR; the 2-norms of the nrhs columns of A (N
// rows, leading dimension lda) in `host` (synchronises).
rbf_status solve_residual(rbf_ctx* ctx, const int64_t* rowptr, const int32_t* colidx,
                          const double* vals, int64_t N, const double* B, int64_t ldb,
                          const double* X, int64_t ldx, int64_t nrhs, double* R);
rbf_status solve_col_norms(rbf_ctx* ctx, const double* A, int64_t lda, int64_t N, int64_t nrhs,
                           std::vector<double>& host);

}  // namespace rbf
