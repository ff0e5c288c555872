// Internal interface between the update orchestration and the covariance
// product kernels.
#pragma once

#include "internal.hpp"

namespace rbf {

// Points absorbed per Kalman batch when the caller passes batch = 0.
constexpr int64_t UPDATE_DEFAULT_BATCH = 1024;

// P -= V V^T for V^T = Ut[0:Bc, 0:N] (row-major, leading dimension ldu);
// lower tiles are computed and written to both triangles of P, so P stays
// exactly symmetric. prec selects the operand precision of the product.
rbf_status syrk_update(rbf_ctx* ctx, double* P, int64_t ldp, int64_t N, const double* Ut,
                       int64_t ldu, int32_t Bc, rbf_prec prec);

}  // namespace rbf
