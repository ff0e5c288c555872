// Covariance product P -= V V^T on MFMA (the dominant step of the recursive
// update, eq. H_inverse_update in Kalman form).
//
// V^T (Bc x N) is read as two 128-column panels per 128x128 output tile;
// only tiles on or below the diagonal are computed and each result is
// written to both triangles, which keeps P exactly symmetric. Tiles are
// assigned so that each XCD works through a contiguous run of the tile
// list (neighbouring tiles share V^T panels in that XCD's L2).
//
// Lane layouts (v_mfma_f64_16x16x4_f64, checked on gfx950):
//   A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
//   D[i][j] in lane j + 16 (i % 4), item i / 4.
#include "update.hpp"

namespace rbf {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int ST = 128;     // output tile
constexpr int SKC = 16;     // rows of V^T per LDS stage
constexpr int SLD = ST + 8; // LDS pitch (doubles)

__device__ inline void tile_of(int64_t t, int* I, int* J) {
  int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(i + 1) * (i + 2) / 2 <= t) ++i;
  while ((int64_t)i * (i + 1) / 2 > t) --i;
  *I = i;
  *J = (int)(t - (int64_t)i * (i + 1) / 2);
}

__device__ inline int64_t xcd_tile(int64_t per_xcd) {
  const int64_t bid = blockIdx.x;
  return (bid & 7) * per_xcd + (bid >> 3);
}

// Load 8 consecutive doubles of row r of V^T starting at column c (zero
// outside [0, N) x [0, K)).
__device__ inline void load8(const double* __restrict__ Ut, int64_t ldu, int64_t N, int r, int K,
                             int64_t c, double v[8]) {
  if (r < K && c + 7 < N) {
    const double2* p = reinterpret_cast<const double2*>(Ut + (int64_t)r * ldu + c);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double2 q = p[u];
      v[2 * u] = q.x;
      v[2 * u + 1] = q.y;
    }
  } else {
#pragma unroll
    for (int u = 0; u < 8; ++u)
      v[u] = (r < K && c + u < N) ? Ut[(int64_t)r * ldu + c + u] : 0.0;
  }
}

__global__ void __launch_bounds__(256, 2) k_syrk_f64(double* __restrict__ P, int64_t ldp,
                                                     int64_t N, const double* __restrict__ Ut,
                                                     int64_t ldu, int32_t K, int64_t T,
                                                     int64_t per_xcd,
                                                     const int32_t* __restrict__ status) {
  if (*(volatile const int32_t*)status != 0) return;
  const int64_t t = xcd_tile(per_xcd);
  if (t >= T) return;
  int I, J;
  tile_of(t, &I, &J);
  const int64_t I0 = (int64_t)I * ST, J0 = (int64_t)J * ST;
  __shared__ double As[2][SKC][SLD];
  __shared__ double Bs[2][SKC][SLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = tid >> 4, lc = (tid & 15) * 8;  // loader: row, first column
  v4d acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  const int nch = (K + SKC - 1) / SKC;
  double ra[8], rb[8];
  load8(Ut, ldu, N, lr, K, I0 + lc, ra);
  load8(Ut, ldu, N, lr, K, J0 + lc, rb);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    As[0][lr][lc + u] = ra[u];
    Bs[0][lr][lc + u] = rb[u];
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) {
      const int r = (ch + 1) * SKC + lr;
      load8(Ut, ldu, N, r, K, I0 + lc, ra);
      load8(Ut, ldu, N, r, K, J0 + lc, rb);
    }
#pragma unroll
    for (int kk = 0; kk < SKC; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[buf][kr][wm * 64 + q * 16 + (lane & 15)];
        b[q] = Bs[buf][kr][wn * 64 + q * 16 + (lane & 15)];
      }
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
    if (ch + 1 < nch) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        As[buf ^ 1][lr][lc + u] = ra[u];
        Bs[buf ^ 1][lr][lc + u] = rb[u];
      }
    }
    __syncthreads();
  }
  // epilogue: P[gi][gj] -= C and mirror (lower tiles; diagonal tiles keep
  // gi >= gj so each element is written once)
  const bool diag = (I == J);
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = I0 + wm * 64 + mi * 16 + 4 * v + (lane >> 4);
        const int64_t gj = J0 + wn * 64 + ni * 16 + (lane & 15);
        if (gi < N && gj < N && (!diag || gi >= gj)) {
          const double nv = P[gi * ldp + gj] - acc[mi][ni][v];
          P[gi * ldp + gj] = nv;
          if (gi != gj) P[gj * ldp + gi] = nv;
        }
      }
}

rbf_status syrk_update(rbf_ctx* ctx, double* P, int64_t ldp, int64_t N, const double* Ut,
                       int64_t ldu, int32_t Bc, rbf_prec prec) {
  if (prec != RBF_F64)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_update: gemm_prec %d not available", (int)prec);
  const int64_t nt = ceil_div(N, ST);
  const int64_t T = nt * (nt + 1) / 2;
  const int64_t per_xcd = ceil_div(T, 8);
  prof_begin(ctx, RBF_PROF_SYRK);
  k_syrk_f64<<<(unsigned)(per_xcd * 8), 256, 0, ctx->stream>>>(P, ldp, N, Ut, ldu, Bc, T,
                                                               per_xcd, ctx->d_status);
  RBF_LAUNCHED(ctx, "k_syrk_f64");
  prof_end(ctx, RBF_PROF_SYRK);
  return RBF_OK;
}

}  // namespace rbf
