// Recursive covariance update (eqs. kf_w_update, H_inverse_update).
#include "internal.hpp"

extern "C" rbf_status rbf_update(rbf_ctx* ctx, const rbf_params*, const rbf_grid*, double*,
                                 double*, int64_t, const double*, const double*, int64_t,
                                 int64_t, rbf_prec, int64_t*) {
  return rbf::fail(ctx, RBF_E_INVALID_ARG, "rbf_update: not built yet");
}
