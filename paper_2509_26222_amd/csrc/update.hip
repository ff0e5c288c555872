// Recursive covariance update (eqs. kf_w_update and H_inverse_update).
//
// With P = R calH^{-1}, a batch of B points with regressor block H (B x N)
// and heights z is absorbed by the Kalman form of the Woodbury update:
//   y = z - H w                 innovation
//   U = P H^T                   (stored transposed, U^T: B x ldu, plus y)
//   S = H U + R I               B x B, FP64
//   L L^T = S                   FP64 blocked Cholesky
//   V^T = L^{-1} U^T, t = L^{-1} y   (y rides along as column N of U^T)
//   w += V t,  P -= V V^T       (SYRK on MFMA, both triangles written)
// This equals calH^{-1} <- calH^{-1} - calH^{-1} m (I + m^T calH^{-1} m)^{-1}
// m^T calH^{-1} and w <- w + calH_new^{-1} m (p_z - m^T w) with m = H^T.
//
// Every kernel returns at once if the context's status word holds an error,
// so a failed batch leaves (w, P) as they were after the previous batch.
#include <cmath>

#include "internal.hpp"
#include "update.hpp"

namespace rbf {

constexpr int NB = 64;       // Cholesky / TRSM block size
constexpr int LDT = NB + 1;  // padded LDS row of a 64x64 tile

struct RegKU {
  double rc2, den, scale;
};

__device__ inline bool failed(const int32_t* st) { return *(volatile const int32_t*)st != 0; }

// ------------------------------------------------------------ batch rows

// Regressor rows of the batch (ELL), innovation y = z - H w into U^T[:, N].
__global__ void __launch_bounds__(256) k_upd_rows(
    const double* __restrict__ xy, const double* __restrict__ z, int32_t Bc, int32_t Bp,
    const double* __restrict__ cxy, const int32_t* __restrict__ idx,
    const int32_t* __restrict__ start, GridGeom g, RegKU k, int32_t kmax,
    const double* __restrict__ w, double* __restrict__ vals, int32_t* __restrict__ cols,
    int32_t* __restrict__ nnz, double* __restrict__ Ut, int64_t ldu, int64_t N,
    int32_t* __restrict__ status, int64_t batch) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= Bp || failed(status)) return;
  if (b >= Bc) {
    nnz[b] = 0;
    Ut[(int64_t)b * ldu + N] = 0.0;
    return;
  }
  const double x = xy[2 * b], y = xy[2 * b + 1];
  double* vrow = vals + (int64_t)b * kmax;
  int32_t* crow = cols + (int64_t)b * kmax;
  int n = 0;
  double hw = 0.0;
  int bx0, bx1, by0, by1;
  if (bin_range(x, g.x0, g.inv_h, g.nbx, &bx0, &bx1) &&
      bin_range(y, g.y0, g.inv_h, g.nby, &by0, &by1)) {
    for (int by = by0; by <= by1; ++by) {
      const int row = by * g.nbx;
      const int s0 = start[row + bx0], s1 = start[row + bx1 + 1];
      for (int s = s0; s < s1; ++s) {
        const double dx = __dsub_rn(x, cxy[2 * s]), dy = __dsub_rn(y, cxy[2 * s + 1]);
        const double d2 = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
        if (d2 <= k.rc2 && n < kmax) {
          const double v = k.scale * exp(-d2 / k.den);
          const int32_t c = idx[s];
          vrow[n] = v;
          crow[n] = c;
          hw += v * w[c];
          ++n;
        }
      }
    }
  }
  nnz[b] = n;
  const double zb = z[b];
  const double yb = zb - hw;
  if (!isfinite(zb) || !isfinite(yb) || !isfinite(x) || !isfinite(y))
    set_status(status, RBF_E_NONFINITE, batch);
  Ut[(int64_t)b * ldu + N] = yb;
}

// U^T[b, n] = sum_k vals[b,k] P[cols[b,k], n]  (P symmetric: rows of P).
// Block: 8 batch rows x 1024 columns; each thread 4 columns.
__global__ void __launch_bounds__(256) k_upd_gather_u(
    const double* __restrict__ P, int64_t ldp, int64_t N, int32_t Bc,
    const double* __restrict__ vals, const int32_t* __restrict__ cols,
    const int32_t* __restrict__ nnz, int32_t kmax, double* __restrict__ Ut, int64_t ldu,
    const int32_t* __restrict__ status) {
  if (failed(status)) return;
  const int64_t n0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const int b0 = blockIdx.y * 8;
  for (int r = 0; r < 8; ++r) {
    const int b = b0 + r;
    double acc[4] = {0, 0, 0, 0};
    if (b < Bc) {
      const int nz = nnz[b];
      const double* vr = vals + (int64_t)b * kmax;
      const int32_t* cr = cols + (int64_t)b * kmax;
      for (int q = 0; q < nz; ++q) {
        const double v = vr[q];
        const double* prow = P + (int64_t)cr[q] * ldp;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t n = n0 + 256 * u;
          if (n < N) acc[u] += v * prow[n];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t n = n0 + 256 * u;
      if (n < N) Ut[(int64_t)b * ldu + n] = acc[u];
    }
  }
}

// S[a][b] (a >= b) = sum_k vals[a,k] U^T[b, cols[a,k]] + R delta_ab; the
// padding rows a >= Bc carry the identity.
__global__ void __launch_bounds__(256) k_upd_S(const double* __restrict__ vals,
                                               const int32_t* __restrict__ cols,
                                               const int32_t* __restrict__ nnz, int32_t kmax,
                                               const double* __restrict__ Ut, int64_t ldu,
                                               int32_t Bc, int32_t Bp, double R,
                                               double* __restrict__ S,
                                               const int32_t* __restrict__ status) {
  if (failed(status)) return;
  const int b = blockIdx.y;
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= Bp || a < b) return;
  double s;
  if (a < Bc && b < Bc) {
    s = (a == b) ? R : 0.0;
    const double* ub = Ut + (int64_t)b * ldu;
    const int nz = nnz[a];
    const double* vr = vals + (int64_t)a * kmax;
    const int32_t* cr = cols + (int64_t)a * kmax;
    for (int q = 0; q < nz; ++q) s += vr[q] * ub[cr[q]];
  } else {
    s = (a == b) ? 1.0 : 0.0;
  }
  S[(int64_t)a * Bp + b] = s;
}

// ------------------------------------------------------------- Cholesky

// Load a 64x64 block of a row-major matrix into an LDS tile.
__device__ inline void load_tile(double (*T)[LDT], const double* __restrict__ A, int64_t lda) {
  for (int e = threadIdx.x; e < NB * NB; e += 256) T[e >> 6][e & 63] = A[(int64_t)(e >> 6) * lda + (e & 63)];
}

__device__ inline void store_tile(const double (*T)[LDT], double* __restrict__ A, int64_t lda) {
  for (int e = threadIdx.x; e < NB * NB; e += 256) A[(int64_t)(e >> 6) * lda + (e & 63)] = T[e >> 6][e & 63];
}

// acc (4x4 micro-tile at rows r0.., cols c0..) = X Y^T over 64 (both LDS).
__device__ inline void mm_nt(const double (*X)[LDT], const double (*Y)[LDT], double acc[4][4],
                             int r0, int c0) {
  for (int q = 0; q < NB; ++q) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = X[r0 + u][q];
      b[u] = Y[c0 + u][q];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
  }
}

// In-place Cholesky of the lower triangle of T (64x64), then Tinv = L^{-1}
// (lower). Upper parts of both are set to zero. A non-positive or non-finite
// pivot records RBF_E_NOT_SPD with `index`.
__device__ void chol64(double (*T)[LDT], double (*Tinv)[LDT], int32_t* status, int64_t index) {
  const int tid = threadIdx.x;
  __shared__ double piv;
  __shared__ int bad;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    if (tid == 0) {
      double d = T[j][j];
      if (!(d > 0.0) || !isfinite(d)) {
        bad = 1;
        d = 1.0;
      }
      piv = sqrt(d);
      T[j][j] = piv;
    }
    __syncthreads();
    const double inv = 1.0 / piv;
    for (int i = j + 1 + tid; i < NB; i += 256) T[i][j] *= inv;
    __syncthreads();
    // trailing update of the lower triangle
    const int m = NB - j - 1;
    for (int e = tid; e < m * m; e += 256) {
      const int i = j + 1 + e / m, c = j + 1 + e % m;
      if (c <= i) T[i][c] -= T[i][j] * T[c][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e >> 6, c = e & 63;
    if (c > i) T[i][c] = 0.0;
  }
  __syncthreads();
  // Tinv: forward substitution L X = I, one column per thread (64 columns)
  if (tid < NB) {
    const int c = tid;
    for (int i = 0; i < NB; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int q = c; q < i; ++q) s -= T[i][q] * Tinv[q][c];
      Tinv[i][c] = (i < c) ? 0.0 : s / T[i][i];
    }
  }
  __syncthreads();
  if (tid == 0 && bad) set_status(status, RBF_E_NOT_SPD, index);
}

// Factor diagonal block 0.
__global__ void __launch_bounds__(256) k_chol_first(const double* __restrict__ S, int32_t Bp,
                                                    double* __restrict__ Lb,
                                                    double* __restrict__ Linv,
                                                    int32_t* __restrict__ status, int64_t batch) {
  if (failed(status)) return;
  __shared__ double T[NB][LDT], Ti[NB][LDT];
  load_tile(T, S, Bp);
  __syncthreads();
  chol64(T, Ti, status, batch);
  store_tile(T, Lb, Bp);
  store_tile(Ti, Linv, NB);
}

// Step kb of the right-looking blocked Cholesky, one launch per block
// column. Tiles t < m are panel tiles (i = kb+1+t): L_ik = A_ik Linv_kk^T.
// The rest are trailing tiles (i, j), kb < j <= i: they recompute L_ik and
// L_jk from A and Linv_kk (read-only in this launch) and update A_ij; tile
// (kb+1, kb+1) then factors itself, ready for step kb+1.
__global__ void __launch_bounds__(256) k_chol_step(double* __restrict__ S, int32_t Bp,
                                                   int32_t nblk, int32_t kb,
                                                   double* __restrict__ Lb,
                                                   double* __restrict__ Linv,
                                                   int32_t* __restrict__ status, int64_t batch) {
  if (failed(status)) return;
  __shared__ double Li[NB][LDT], T1[NB][LDT], T2[NB][LDT];
  const int m = nblk - kb - 1;
  const int t = blockIdx.x;
  int i, j;
  bool panel;
  if (t < m) {
    panel = true;
    i = kb + 1 + t;
    j = kb;
  } else {
    panel = false;
    const int u = t - m;
    int ii = (int)((sqrt(8.0 * u + 1.0) - 1.0) * 0.5);
    while ((ii + 1) * (ii + 2) / 2 <= u) ++ii;
    while (ii * (ii + 1) / 2 > u) --ii;
    i = kb + 1 + ii;
    j = kb + 1 + (u - ii * (ii + 1) / 2);
  }
  const int tid = threadIdx.x;
  const int r0 = (tid >> 4) * 4, c0 = (tid & 15) * 4;
  const double* Lkk_inv = Linv + (int64_t)kb * NB * NB;
  load_tile(Li, Lkk_inv, NB);
  load_tile(T1, S + (int64_t)i * NB * Bp + (int64_t)kb * NB, Bp);
  __syncthreads();
  double acc[4][4] = {};
  mm_nt(T1, Li, acc, r0, c0);  // L_ik
  if (panel) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Lb[(int64_t)(i * NB + r0 + u) * Bp + kb * NB + c0 + v] = acc[u][v];
    return;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) T2[r0 + u][c0 + v] = acc[u][v];  // T2 = L_ik
  if (j != i) {
    __syncthreads();
    load_tile(T1, S + (int64_t)j * NB * Bp + (int64_t)kb * NB, Bp);
    __syncthreads();
    double bcc[4][4] = {};
    mm_nt(T1, Li, bcc, r0, c0);  // L_jk
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) T1[r0 + u][c0 + v] = bcc[u][v];
  }
  __syncthreads();
  double (*Lj)[LDT] = (j != i) ? T1 : T2;
  double upd[4][4] = {};
  mm_nt(T2, Lj, upd, r0, c0);  // L_ik L_jk^T
  double* Aij = S + (int64_t)i * NB * Bp + (int64_t)j * NB;
  if (i == kb + 1 && j == kb + 1) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Li[r0 + u][c0 + v] = Aij[(int64_t)(r0 + u) * Bp + c0 + v] - upd[u][v];
    __syncthreads();
    chol64(Li, T1, status, batch);
    store_tile(Li, Lb + (int64_t)i * NB * Bp + (int64_t)i * NB, Bp);
    store_tile(T1, Linv + (int64_t)i * NB * NB, NB);
    return;
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) Aij[(int64_t)(r0 + u) * Bp + c0 + v] -= upd[u][v];
}

// ----------------------------------------------------------------- TRSM

// V^T = L^{-1} U^T in place on a slab of TW columns per workgroup:
// X_i = Linv_ii (U_i - sum_{j<i} L_ij X_j), block rows in order.
constexpr int TW = 16;
__global__ void __launch_bounds__(256) k_upd_trsm(double* __restrict__ Ut, int64_t ldu,
                                                  int64_t ncols, int32_t nblk,
                                                  const double* __restrict__ Lb, int32_t Bp,
                                                  const double* __restrict__ Linv,
                                                  const int32_t* __restrict__ status) {
  if (failed(status)) return;
  __shared__ double Lt[NB][LDT];
  __shared__ double X[NB][TW + 1];
  const int tid = threadIdx.x;
  const int64_t col0 = (int64_t)blockIdx.x * TW;
  const int r = tid >> 2;          // row within the block (0..63)
  const int cq = (tid & 3) * 4;    // 4 columns per thread
  for (int i = 0; i < nblk; ++i) {
    double acc[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t c = col0 + cq + v;
      acc[v] = c < ncols ? Ut[(int64_t)(i * NB + r) * ldu + c] : 0.0;
    }
    for (int j = 0; j < i; ++j) {
      __syncthreads();
      load_tile(Lt, Lb + (int64_t)i * NB * Bp + (int64_t)j * NB, Bp);
      for (int e = tid; e < NB * TW; e += 256) {
        const int rr = e / TW, cc = e % TW;
        const int64_t c = col0 + cc;
        X[rr][cc] = c < ncols ? Ut[(int64_t)(j * NB + rr) * ldu + c] : 0.0;
      }
      __syncthreads();
      for (int q = 0; q < NB; ++q) {
        const double l = Lt[r][q];
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] -= l * X[q][cq + v];
      }
    }
    __syncthreads();
    load_tile(Lt, Linv + (int64_t)i * NB * NB, NB);
#pragma unroll
    for (int v = 0; v < 4; ++v) X[r][cq + v] = acc[v];
    __syncthreads();
    double out[4] = {0, 0, 0, 0};
    for (int q = 0; q <= r; ++q) {
      const double l = Lt[r][q];
#pragma unroll
      for (int v = 0; v < 4; ++v) out[v] += l * X[q][cq + v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t c = col0 + cq + v;
      if (c < ncols) Ut[(int64_t)(i * NB + r) * ldu + c] = out[v];
    }
  }
}

// w[n] += sum_b V^T[b, n] t[b], t = V^T[:, N].
__global__ void __launch_bounds__(256) k_upd_w(double* __restrict__ w,
                                               const double* __restrict__ Ut, int64_t ldu,
                                               int64_t N, int32_t Bc,
                                               const int32_t* __restrict__ status) {
  if (failed(status)) return;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  double s = 0.0;
  for (int b = 0; b < Bc; ++b) s += Ut[(int64_t)b * ldu + n] * Ut[(int64_t)b * ldu + N];
  w[n] += s;
}

}  // namespace rbf

using namespace rbf;

extern "C" rbf_status rbf_update(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                                 double* w, double* P, int64_t ldp, const double* xy,
                                 const double* z, int64_t M, int64_t batch, rbf_prec gemm_prec,
                                 int64_t* n_done) {
  if (!ctx) return RBF_E_INVALID_ARG;
  if (n_done) *n_done = 0;
  if (!p || !g || !w || !P)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_update: null params/grid/w/P");
  if (g->device != ctx->device)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_update: grid on another device");
  if (p->sigma != g->sigma || p->cutoff != g->cutoff || p->sigma_eps != g->sigma_eps)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_update: params differ from the grid's");
  const int64_t N = g->N;
  if (ldp < N || M < 0 || (M > 0 && (!xy || !z)) || batch < 0 || batch > (1 << 16))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_update: bad ldp/M/batch");
  if (!(p->R > 0) || !std::isfinite(p->R))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_update: R must be > 0");
  if (gemm_prec != RBF_F64 && gemm_prec != RBF_F32 && gemm_prec != RBF_BF16)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_update: unknown gemm_prec");
  if (M == 0) return RBF_OK;
  RBF_TRY(set_device(ctx));
  const int64_t B = batch > 0 ? batch : UPDATE_DEFAULT_BATCH;
  const int32_t Bmax = (int32_t)(B < M ? B : M);
  const int32_t Bp = (int32_t)ceil_div(Bmax, NB) * NB;
  const int32_t nblk_max = Bp / NB;
  const int64_t ldu = ceil_div(N + 1, 32) * 32;
  const int32_t kmax = g->max_cand > 0 ? g->max_cand : 1;
  rbf_status st;
  char* ell = (char*)ws_get(ctx, WS_UPD_ELL, (size_t)Bp * kmax * 12 + (size_t)Bp * 4 + 256, &st);
  if (!ell) return st;
  double* vals = (double*)ell;
  int32_t* cols = (int32_t*)(ell + (size_t)Bp * kmax * 8);
  int32_t* nnz = cols + (size_t)Bp * kmax;
  double* Ut = (double*)ws_get(ctx, WS_UPD_UT, sizeof(double) * (size_t)Bp * ldu, &st);
  if (!Ut) return st;
  double* S = (double*)ws_get(ctx, WS_UPD_S, sizeof(double) * (size_t)Bp * Bp * 2, &st);
  if (!S) return st;
  double* Lb = S + (size_t)Bp * Bp;
  double* Linv = (double*)ws_get(ctx, WS_UPD_LINV, sizeof(double) * (size_t)nblk_max * NB * NB,
                                 &st);
  if (!Linv) return st;
  const double st_ = std::sqrt(p->sigma * p->sigma + p->sigma_eps * p->sigma_eps);
  RegKU rk;
  rk.rc2 = (p->cutoff * st_) * (p->cutoff * st_);
  rk.den = 2.0 * st_ * st_;
  rk.scale = (p->sigma * p->sigma) / (st_ * st_);
  const int64_t nb_total = ceil_div(M, B);
  for (int64_t bi = 0; bi < nb_total; ++bi) {
    const int64_t s0 = bi * B;
    const int32_t Bc = (int32_t)((M - s0) < B ? (M - s0) : B);
    const int32_t Bpc = (int32_t)ceil_div(Bc, NB) * NB;
    const int32_t nblk = Bpc / NB;
    k_upd_rows<<<ceil_div(Bpc, 256), 256, 0, ctx->stream>>>(
        xy + 2 * s0, z + s0, Bc, Bpc, g->d_cxy, g->d_idx, g->d_start, geom(g), rk, kmax, w,
        vals, cols, nnz, Ut, ldu, N, ctx->d_status, bi);
    RBF_LAUNCHED(ctx, "k_upd_rows");
    dim3 gg((unsigned)ceil_div(N, 1024), (unsigned)ceil_div(Bpc, 8));
    k_upd_gather_u<<<gg, 256, 0, ctx->stream>>>(P, ldp, N, Bc, vals, cols, nnz, kmax, Ut, ldu,
                                                 ctx->d_status);
    RBF_LAUNCHED(ctx, "k_upd_gather_u");
    dim3 gs((unsigned)ceil_div(Bpc, 256), (unsigned)Bpc);
    k_upd_S<<<gs, 256, 0, ctx->stream>>>(vals, cols, nnz, kmax, Ut, ldu, Bc, Bpc, p->R, S,
                                         ctx->d_status);
    RBF_LAUNCHED(ctx, "k_upd_S");
    k_chol_first<<<1, 256, 0, ctx->stream>>>(S, Bpc, Lb, Linv, ctx->d_status, bi);
    RBF_LAUNCHED(ctx, "k_chol_first");
    for (int32_t kb = 0; kb + 1 < nblk; ++kb) {
      const int m = nblk - kb - 1;
      k_chol_step<<<m + m * (m + 1) / 2, 256, 0, ctx->stream>>>(S, Bpc, nblk, kb, Lb, Linv,
                                                               ctx->d_status, bi);
      RBF_LAUNCHED(ctx, "k_chol_step");
    }
    k_upd_trsm<<<ceil_div(N + 1, TW), 256, 0, ctx->stream>>>(Ut, ldu, N + 1, nblk, Lb, Bpc,
                                                             Linv, ctx->d_status);
    RBF_LAUNCHED(ctx, "k_upd_trsm");
    k_upd_w<<<ceil_div(N, 256), 256, 0, ctx->stream>>>(w, Ut, ldu, N, Bc, ctx->d_status);
    RBF_LAUNCHED(ctx, "k_upd_w");
    RBF_TRY(syrk_update(ctx, P, ldp, N, Ut, ldu, Bc, gemm_prec));
  }
  if (n_done) {
    int32_t h[4];
    RBF_HIP(ctx, hipMemcpyAsync(h, ctx->d_status, sizeof(h), hipMemcpyDeviceToHost,
                                ctx->stream));
    RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (h[0] != 0) {
      int64_t idx;
      memcpy(&idx, h + 2, sizeof(idx));
      const int64_t done = idx * B;
      *n_done = done < M ? done : M;
      return rbf_sync_status(ctx);
    }
    *n_done = M;
  }
  return RBF_OK;
}
