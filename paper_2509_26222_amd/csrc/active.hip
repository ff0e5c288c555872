// Active-rows form of the recursive update (eqs. active_rows_weights_update
// and H_inverse_update; active rows per eq. mfk_m_approx).
//
// A scan touches only the centers within the regressor's support of its
// points (the active set A). Treating calH^{-1} as block diagonal with A as
// one block, the scan's Kalman update runs on w_A and P_AA alone:
//   mark A          flags[c] = 1 for every center in a point's support
//   compact map     exclusive scan of the flags: colmap[c] = rank of c in A
//   gather          Pc = P[A, A], wc = w[A]   (compact, |A| x ldc)
//   update          the dense recursive update on (wc, Pc) with the
//                   regressor columns mapped through colmap
//   scatter         P[A, A] = Pc, w[A] = wc
//   decouple        P[A, not A] = P[not A, A] = 0
// The last step is the block-diagonal result of eq. H_inverse_update: the
// scan's block is updated and nothing couples it to the other centers,
// which keeps P positive semi-definite for later scans. w outside A and P
// outside the rows and columns of A are neither read nor written. The
// update costs |A|^2 B per batch instead of N^2 B, the decoupling |A| N
// flag tests and at most 2 |A| (N - |A|) stores.
#include <cmath>

#include "internal.hpp"
#include "update.hpp"

namespace rbf {

// flags[c] = 1 for every center c with a non-zero regressor entry at one of
// the points: the same support test, in the same arithmetic, as the rows of
// the update (k_upd_rows), so every column the update forms is in A.
__global__ void __launch_bounds__(256) k_act_mark(const double* __restrict__ xy, int64_t M,
                                                  const double* __restrict__ cxy,
                                                  const int32_t* __restrict__ idx,
                                                  const int32_t* __restrict__ start, GridGeom g,
                                                  double rc2, int32_t kmax,
                                                  int32_t* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const double x = xy[2 * i], y = xy[2 * i + 1];
  int bx0, bx1, by0, by1;
  if (!bin_range(x, g.x0, g.inv_h, g.nbx, &bx0, &bx1) ||
      !bin_range(y, g.y0, g.inv_h, g.nby, &by0, &by1))
    return;
  int n = 0;
  for (int by = by0; by <= by1; ++by) {
    const int row = by * g.nbx;
    const int s0 = start[row + bx0], s1 = start[row + bx1 + 1];
    for (int s = s0; s < s1; ++s) {
      const double dx = __dsub_rn(x, cxy[2 * s]), dy = __dsub_rn(y, cxy[2 * s + 1]);
      const double d2 = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
      if (d2 <= rc2 && n < kmax) {
        flags[idx[s]] = 1;  // every writer stores the same value
        ++n;
      }
    }
  }
}

// act[rank] = c for every active center c; F holds the exclusive scan of
// the flags (F[N] = |A|).
__global__ void __launch_bounds__(256) k_act_list(const int32_t* __restrict__ F, int64_t N,
                                                  int32_t* __restrict__ act) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c < N && F[c + 1] > F[c]) act[F[c]] = (int32_t)c;
}

// Pc[i][j] = P[act[i]][act[j]] (TO_COMPACT) or the reverse, and the same for
// w. One row per blockIdx.x, 1024 columns per blockIdx.y, 4 per thread.
template <bool TO_COMPACT>
__global__ void __launch_bounds__(256) k_act_move(double* __restrict__ P, int64_t ldp,
                                                  double* __restrict__ w,
                                                  const int32_t* __restrict__ act, int32_t NA,
                                                  double* __restrict__ Pc, int64_t ldc,
                                                  double* __restrict__ wc) {
  const int32_t i = blockIdx.x;
  const int64_t r = act[i];
  double* prow = P + r * ldp;
  double* crow = Pc + (int64_t)i * ldc;
  const int32_t j0 = blockIdx.y * 1024 + threadIdx.x;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int32_t j = j0 + 256 * u;
    if (j < NA) {
      if (TO_COMPACT)
        crow[j] = prow[act[j]];
      else
        prow[act[j]] = crow[j];
    }
  }
  if (blockIdx.y == 0 && threadIdx.x == 0) {
    if (TO_COMPACT)
      wc[i] = w[r];
    else
      w[r] = wc[i];
  }
}

// P[r][c] = 0 where exactly one of r, c is active. Row r per blockIdx.x;
// an active row clears its inactive columns (1024 columns per blockIdx.y),
// an inactive row its active columns (1024 compact indices per blockIdx.y).
// Skipped when the scan's first batch (launch group seq) failed, since
// then no batch was absorbed.
__global__ void __launch_bounds__(256) k_act_decouple(double* __restrict__ P, int64_t ldp,
                                                      int64_t N, const int32_t* __restrict__ F,
                                                      const int32_t* __restrict__ act,
                                                      int32_t NA,
                                                      const int32_t* __restrict__ status,
                                                      int64_t seq) {
  if (seq_skip(status, seq)) return;
  const int64_t r = blockIdx.x;
  double* prow = P + r * ldp;
  const bool r_act = F[r + 1] > F[r];
  const int64_t j0 = (int64_t)blockIdx.y * 1024 + threadIdx.x;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t j = j0 + 256 * u;
    if (r_act) {
      if (j < N && F[j + 1] == F[j]) prow[j] = 0.0;
    } else {
      if (j < NA) prow[act[j]] = 0.0;
    }
  }
}

}  // namespace rbf

using namespace rbf;

extern "C" rbf_status rbf_update_active(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                                        double* w, double* P, int64_t ldp, const double* xy,
                                        const double* z, int64_t M, int64_t batch,
                                        rbf_prec gemm_prec, int32_t* active,
                                        int64_t* n_active, int64_t* n_done) {
  if (!ctx) return RBF_E_INVALID_ARG;
  if (n_done) *n_done = 0;
  if (n_active) *n_active = 0;
  RBF_TRY(update_check(ctx, p, g, w, P, ldp, xy, z, M, batch, gemm_prec));
  if (M == 0) return RBF_OK;
  RBF_TRY(set_device(ctx));
  const int64_t N = g->N;
  const int64_t B = batch > 0 ? batch : UPDATE_DEFAULT_BATCH;
  rbf_status st;
  // F: N + 1 flags, then their exclusive scan (the compact map); act: N
  // indices; wc: N doubles
  const size_t off_w = ((2 * (size_t)N + 1) * sizeof(int32_t) + 7) / 8 * 8;
  char* base = (char*)ws_get(ctx, WS_ACT_IDX, off_w + sizeof(double) * (size_t)N, &st);
  if (!base) return st;
  int32_t* F = (int32_t*)base;
  int32_t* act = F + (N + 1);
  double* wc = (double*)(base + off_w);
  RBF_TRY(fill_zero(ctx, F, sizeof(int32_t) * (size_t)(N + 1)));
  const RegKU rk = regku(p);
  const int32_t kmax = g->max_cand > 0 ? g->max_cand : 1;
  k_act_mark<<<ceil_div(M, 256), 256, 0, ctx->stream>>>(xy, M, g->d_cxy, g->d_idx, g->d_start,
                                                        geom(g), rk.rc2, kmax, F);
  RBF_LAUNCHED(ctx, "k_act_mark");
  k_scan_excl_i32<<<1, 1024, 0, ctx->stream>>>(F, N);
  RBF_LAUNCHED(ctx, "k_scan_excl_i32");
  k_act_list<<<ceil_div(N, 256), 256, 0, ctx->stream>>>(F, N, act);
  RBF_LAUNCHED(ctx, "k_act_list");
  int32_t na32 = 0;
  RBF_HIP(ctx, hipMemcpyAsync(&na32, F + N, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const int32_t NA = na32;
  if (NA < 0 || NA > N) return fail(ctx, RBF_E_HIP, "rbf_update_active: bad active count");
  if (n_active) *n_active = NA;
  if (active && NA > 0)
    RBF_HIP(ctx, hipMemcpyAsync(active, act, sizeof(int32_t) * (size_t)NA,
                                hipMemcpyDeviceToDevice, ctx->stream));
  if (NA == 0) {  // no point near any center: nothing to update
    if (n_done) *n_done = M;
    return RBF_OK;
  }
  const int64_t ldc = ceil_div(NA, 32) * 32;
  double* Pc = (double*)ws_get(ctx, WS_ACT_P, sizeof(double) * (size_t)NA * ldc, &st);
  if (!Pc) return st;
  const dim3 gm((unsigned)NA, (unsigned)ceil_div(NA, 1024));
  k_act_move<true><<<gm, 256, 0, ctx->stream>>>(P, ldp, w, act, NA, Pc, ldc, wc);
  RBF_LAUNCHED(ctx, "k_act_move");
  // Batches commit one by one; whatever update_run enqueued (up to a failing
  // batch, or an early host-side error) is written back.
  const int64_t seq0 = ctx->seq;  // launch group of the scan's first batch
  const rbf_status rs = update_run(ctx, p, g, F, NA, wc, Pc, ldc, xy, z, M, B, gemm_prec);
  k_act_move<false><<<gm, 256, 0, ctx->stream>>>(P, ldp, w, act, NA, Pc, ldc, wc);
  RBF_LAUNCHED(ctx, "k_act_move");
  if (rs == RBF_OK) {
    const dim3 gd((unsigned)N, (unsigned)ceil_div(N, 1024));
    k_act_decouple<<<gd, 256, 0, ctx->stream>>>(P, ldp, N, F, act, NA, ctx->d_status, seq0);
    RBF_LAUNCHED(ctx, "k_act_decouple");
  }
  if (rs != RBF_OK) return rs;
  if (!n_done) return RBF_OK;
  return update_done(ctx, M, B, seq0, n_done);
}
