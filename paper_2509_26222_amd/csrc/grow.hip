// Growing center set: new centers join the state with the prior of the
// ridge estimator (subsection "The RBF Weight Estimate by Ridge
// Regression": calH_0 = lambda I, w_0 = 0), i.e. w = 0, P = (R/lambda) I on
// their rows and columns, and no coupling to the existing centers. The
// caller's buffers hold the larger state already (P with leading dimension
// >= the new size), so growing writes only the new rows and columns.
#include <cmath>

#include "internal.hpp"

namespace rbf {

// Rows r < n_old: columns [n_old, n_new) = 0. Rows r >= n_old: columns
// [0, n_new) = (r == c) ? p0 : 0, and w[r] = 0. One row per blockIdx.x,
// 1024 columns per blockIdx.y.
__global__ void __launch_bounds__(256) k_grow_state(double* __restrict__ P, int64_t ldp,
                                                    int64_t n_old, int64_t n_new, double p0,
                                                    double* __restrict__ w) {
  const int64_t r = blockIdx.x;
  const int64_t c0 = (r < n_old ? n_old : 0) + (int64_t)blockIdx.y * 1024 + threadIdx.x;
  double* prow = P + r * ldp;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t c = c0 + 256 * u;
    if (c < n_new) prow[c] = (c == r) ? p0 : 0.0;
  }
  if (r >= n_old && blockIdx.y == 0 && threadIdx.x == 0) w[r] = 0.0;
}

}  // namespace rbf

using namespace rbf;

extern "C" rbf_status rbf_state_grow(rbf_ctx* ctx, const rbf_params* p, double* w, double* P,
                                     int64_t ldp, int64_t n_old, int64_t n_new) {
  if (!ctx) return RBF_E_INVALID_ARG;
  if (!p || !w || !P || n_old < 0 || n_new < n_old || ldp < n_new ||
      n_new >= ((int64_t)1 << 31))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_state_grow: bad pointer or size");
  if (!(p->R > 0) || !(p->lambda > 0) || !std::isfinite(p->R / p->lambda))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_state_grow: R and lambda must be > 0");
  if (n_new == n_old) return RBF_OK;
  RBF_TRY(set_device(ctx));
  const dim3 gg((unsigned)n_new, (unsigned)ceil_div(n_new, 1024));
  k_grow_state<<<gg, 256, 0, ctx->stream>>>(P, ldp, n_old, n_new, p->R / p->lambda, w);
  RBF_LAUNCHED(ctx, "k_grow_state");
  return RBF_OK;
}
