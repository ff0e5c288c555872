// Sparse solve with FP64 iterative refinement.
#include "internal.hpp"

extern "C" rbf_status rbf_solve(rbf_ctx* ctx, int64_t, const int64_t*, const int32_t*,
                                const double*, const double*, int64_t, double*, int64_t,
                                int64_t, double, int32_t, rbf_prec, double*, int32_t*) {
  return rbf::fail(ctx, RBF_E_INVALID_ARG, "rbf_solve: not built yet");
}
