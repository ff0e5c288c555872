// Sparse solve calH X = B (the "sparse kernel matrix inversion" of the GPU
// section), with iterative refinement in FP64.
//
// calH couples only centers closer than 2 cutoff sigma_t, so with centers in
// a spatial (mesh) order its bandwidth bw is small against N. The rows are
// cut into blocks of s >= bw (a multiple of 64): calH is then block
// tridiagonal with dense s x s diagonal blocks D_i and super-diagonal blocks
// U_i = E_i^T. Block Cholesky:
//   D_0 = L_0 L_0^T;  G_i = L_i^{-1} U_i;  D_{i+1} - G_i^T G_i = L_{i+1} L_{i+1}^T
// so calH = L L^T with L block bidiagonal (diagonal L_i, sub-diagonal
// G_i^T). A solve is a forward sweep y_i = L_i^{-1} (r_i - G_{i-1}^T y_{i-1})
// and a backward sweep x_i = L_i^{-T} (y_i - G_i x_{i+1}). Refinement:
// x += solve(b - calH x) until ||b - calH x|| <= rtol ||b|| per column.
// Dense blocks use the FP64 MFMA kernels of the covariance update.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "update.hpp"

namespace rbf {

typedef double v4d __attribute__((ext_vector_type(4)));


__global__ void __launch_bounds__(256) k_csr_bandwidth(const int64_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ colidx,
                                                       int64_t N, int32_t* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  int64_t bw = 0;
  bool bad = false;
  for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
    const int64_t c = colidx[e];
    if (c < 0 || c >= N) bad = true;
    const int64_t d = c > r ? c - r : r - c;
    bw = d > bw ? d : bw;
  }
  atomicMax(out, bad ? INT32_MAX : (int32_t)bw);
}

// D_i[a][b] and U_i[a][b] from the CSR rows; padding rows get D = I.
__global__ void __launch_bounds__(256) k_csr_to_blocks(const int64_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ colidx,
                                                       const double* __restrict__ vals,
                                                       int64_t N, int32_t s, int32_t nblk,
                                                       double* __restrict__ D,
                                                       double* __restrict__ U) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= (int64_t)nblk * s) return;
  const int64_t i = r / s, a = r % s;
  const int64_t ss = (int64_t)s * s;
  if (r >= N) {
    D[i * ss + a * s + a] = 1.0;
    return;
  }
  for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
    const int64_t c = colidx[e];
    const int64_t bi = c / s, b = c % s;
    if (bi == i)
      D[i * ss + a * s + b] = vals[e];
    else if (bi == i + 1)
      U[i * ss + a * s + b] = vals[e];
  }
}

// C[m][n] -= sum_k op(A)[m][k] B[k][n] on FP64 MFMA; op(A) = A (M x K) or
// A^T (A is K x M). 64x64 output tile per workgroup, K in chunks of 16.
constexpr int GT = 64, GK = 16;

template <bool TA>
__global__ void __launch_bounds__(256) k_gemm_sub(int64_t M, int64_t Nc, int64_t K,
                                                  const double* __restrict__ A, int64_t lda,
                                                  const double* __restrict__ B, int64_t ldb,
                                                  double* __restrict__ C, int64_t ldc,
                                                  const int32_t* __restrict__ status,
                                                  int64_t seq) {
  if (seq_skip(status, seq)) return;
  __shared__ double As[GK][GT + 1];  // As[k][m]
  __shared__ double Bs[GK][GT + 1];  // Bs[k][n]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.y * GT, n0 = (int64_t)blockIdx.x * GT;
  const int rb = 32 * (wave >> 1), cb = 32 * (wave & 1);
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = 0; k0 < K; k0 += GK) {
    // 16 x 64 elements of each operand: 4 per thread
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      const int kk = e >> 6, mm = e & 63;
      const int64_t gk = k0 + kk, gm = m0 + mm, gn = n0 + mm;
      double av = 0.0, bv = 0.0;
      if (gk < K && gm < M) av = TA ? A[gk * lda + gm] : A[gm * lda + gk];
      if (gk < K && gn < Nc) bv = B[gk * ldb + gn];
      As[kk][mm] = av;
      Bs[kk][mm] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GK; k += 4) {
      const int kk = k + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        a[u] = As[kk][rb + 16 * u + (lane & 15)];
        b[u] = Bs[kk][cb + 16 * u + (lane & 15)];
      }
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gm = m0 + rb + 16 * mi + 4 * v + (lane >> 4);
        const int64_t gn = n0 + cb + 16 * ni + (lane & 15);
        if (gm < M && gn < Nc) C[gm * ldc + gn] -= acc[mi][ni][v];
      }
}

// Matrix-vector products of the one-right-hand-side sweeps, n x n blocks
// (leading dimension lda), deterministic:
//   k_mv_cols: out[j] = base[j] + sgn sum_k A[k][j] x[k]   (A^T x)
//   k_mv_rows: out[c] = base[c] + sgn sum_r A[c][r] x[r]   (A x)
// base may be null (0) or equal to out; x must not overlap out.
// k_mv_cols: 64 outputs per workgroup, 16 slices of k summed in order.
__global__ void __launch_bounds__(1024) k_mv_cols(const double* __restrict__ A, int64_t lda,
                                                  int32_t n, const double* __restrict__ x,
                                                  const double* base, double sgn, double* out) {
  __shared__ double part[16][64];
  const int tid = threadIdx.x, jl = tid & 63, sl = tid >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + jl;
  const int per = (n + 15) / 16;
  const int k0 = sl * per, k1 = min(n, k0 + per);
  double s0 = 0.0, s1 = 0.0;
  if (j < n) {
    int k = k0;
    for (; k + 1 < k1; k += 2) {
      s0 += A[(int64_t)k * lda + j] * x[k];
      s1 += A[(int64_t)(k + 1) * lda + j] * x[k + 1];
    }
    if (k < k1) s0 += A[(int64_t)k * lda + j] * x[k];
  }
  part[sl][jl] = s0 + s1;
  __syncthreads();
  if (sl == 0 && j < n) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += part[q][jl];
    out[j] = (base ? base[j] : 0.0) + sgn * t;
  }
}

// k_mv_rows: one wave per output, a fixed-order butterfly over the lanes.
__global__ void __launch_bounds__(256) k_mv_rows(const double* __restrict__ A, int64_t lda,
                                                 int32_t n, const double* __restrict__ x,
                                                 const double* base, double sgn, double* out) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  const double* row = A + c * lda;
  double s0 = 0.0, s1 = 0.0;
  int r = lane;
  for (; r + 64 < n; r += 128) {
    s0 += row[r] * x[r];
    s1 += row[r + 64] * x[r + 64];
  }
  if (r < n) s0 += row[r] * x[r];
  double t = s0 + s1;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  if (lane == 0) out[c] = (base ? base[c] : 0.0) + sgn * t;
}

static rbf_status mv_cols(rbf_ctx* ctx, const double* A, int64_t lda, int64_t n,
                          const double* x, const double* base, double sgn, double* out) {
  k_mv_cols<<<(unsigned)ceil_div(n, 64), 1024, 0, ctx->stream>>>(A, lda, (int32_t)n, x, base,
                                                                  sgn, out);
  RBF_LAUNCHED(ctx, "k_mv_cols");
  return RBF_OK;
}

static rbf_status mv_rows(rbf_ctx* ctx, const double* A, int64_t lda, int64_t n,
                          const double* x, const double* base, double sgn, double* out) {
  k_mv_rows<<<(unsigned)ceil_div(n, 4), 256, 0, ctx->stream>>>(A, lda, (int32_t)n, x, base, sgn,
                                                                out);
  RBF_LAUNCHED(ctx, "k_mv_rows");
  return RBF_OK;
}

static rbf_status gemm_sub(rbf_ctx* ctx, bool ta, int64_t M, int64_t Nc, int64_t K,
                           const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                           int64_t ldc, int64_t seq) {
  dim3 grid((unsigned)ceil_div(Nc, GT), (unsigned)ceil_div(M, GT));
  if (ta)
    k_gemm_sub<true><<<grid, 256, 0, ctx->stream>>>(M, Nc, K, A, lda, B, ldb, C, ldc,
                                                    ctx->d_status, seq);
  else
    k_gemm_sub<false><<<grid, 256, 0, ctx->stream>>>(M, Nc, K, A, lda, B, ldb, C, ldc,
                                                     ctx->d_status, seq);
  RBF_LAUNCHED(ctx, "k_gemm_sub");
  return RBF_OK;
}

// Y (padded rows, ld nrhs) = R (N rows, ld ldr); padding rows zero.
__global__ void __launch_bounds__(256) k_pad_copy(const double* __restrict__ R, int64_t ldr,
                                                  int64_t N, int64_t Np, int64_t nrhs,
                                                  double* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= Np * nrhs) return;
  const int64_t r = e / nrhs, c = e % nrhs;
  Y[e] = r < N ? R[r * ldr + c] : 0.0;
}

// X (ld ldx) (+)= Y[:N]
__global__ void __launch_bounds__(256) k_accum(double* __restrict__ X, int64_t ldx,
                                               const double* __restrict__ Y, int64_t N,
                                               int64_t nrhs, int32_t first) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= N * nrhs) return;
  const int64_t r = e / nrhs, c = e % nrhs;
  X[r * ldx + c] = first ? Y[e] : X[r * ldx + c] + Y[e];
}

// R = B - calH X (FP64); one thread per (row, column).
__global__ void __launch_bounds__(256) k_residual(const int64_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colidx,
                                                  const double* __restrict__ vals, int64_t N,
                                                  const double* __restrict__ B, int64_t ldb,
                                                  const double* __restrict__ X, int64_t ldx,
                                                  int64_t nrhs, double* __restrict__ R) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= N * nrhs) return;
  const int64_t r = e / nrhs, c = e % nrhs;
  double s = B[r * ldb + c];
  for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) s -= vals[k] * X[(int64_t)colidx[k] * ldx + c];
  R[r * nrhs + c] = s;
}

// Dot product in two fixed-order stages: part[g] over 2048-element group g,
// then out = sum_g part[g] (one workgroup).
constexpr int DOT_G = 2048;
__device__ inline double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) sh[tid] += sh[tid + o];
    __syncthreads();
  }
  return sh[0];
}

__global__ void __launch_bounds__(256) k_dot_part(const double* __restrict__ x,
                                                  const double* __restrict__ y, int64_t N,
                                                  double* __restrict__ part) {
  __shared__ double sh[256];
  const int64_t g0 = (int64_t)blockIdx.x * DOT_G;
  double v = 0.0;
  for (int u = 0; u < DOT_G / 256; ++u) {
    const int64_t e = g0 + u * 256 + threadIdx.x;
    if (e < N) v += x[e] * y[e];
  }
  const double t = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) k_dot_sum(const double* __restrict__ part, int32_t ng,
                                                 double* __restrict__ out) {
  __shared__ double sh[256];
  double v = 0.0;
  for (int g = threadIdx.x; g < ng; g += 256) v += part[g];
  const double t = block_sum(v, sh);
  if (threadIdx.x == 0) *out = t;
}

// Column sums of squares: part[g][c] over row group g (1024 rows), then
// out[c] = sum_g part[g][c] in order.
constexpr int NRG = 1024;
__global__ void __launch_bounds__(256) k_colsq_part(const double* __restrict__ A, int64_t lda,
                                                    int64_t N, int64_t nrhs,
                                                    double* __restrict__ part) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= nrhs) return;
  const int64_t r0 = (int64_t)blockIdx.y * NRG;
  const int64_t r1 = r0 + NRG < N ? r0 + NRG : N;
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const double v = A[r * lda + c];
    s += v * v;
  }
  part[(int64_t)blockIdx.y * nrhs + c] = s;
}

__global__ void __launch_bounds__(256) k_colsq_sum(const double* __restrict__ part, int64_t nrhs,
                                                   int32_t ngroups, double* __restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= nrhs) return;
  double s = 0.0;
  for (int g = 0; g < ngroups; ++g) s += part[(int64_t)g * nrhs + c];
  out[c] = s;
}

static rbf_status col_norms(rbf_ctx* ctx, const double* A, int64_t lda, int64_t N, int64_t nrhs,
                            double* part, double* dout, std::vector<double>& host) {
  if (nrhs == 1 && lda == 1) {  // one column: a two-stage dot product over many groups
    const int32_t g = (int32_t)ceil_div(N, DOT_G);
    k_dot_part<<<g, 256, 0, ctx->stream>>>(A, A, N, part);
    RBF_LAUNCHED(ctx, "k_dot_part");
    k_dot_sum<<<1, 256, 0, ctx->stream>>>(part, g, dout);
    RBF_LAUNCHED(ctx, "k_dot_sum");
    host.resize(1);
    RBF_HIP(ctx, hipMemcpyAsync(host.data(), dout, sizeof(double), hipMemcpyDeviceToHost,
                                ctx->stream));
    RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    host[0] = std::sqrt(host[0]);
    return RBF_OK;
  }
  const int32_t ng = (int32_t)ceil_div(N, NRG);
  dim3 g1((unsigned)ceil_div(nrhs, 256), (unsigned)ng);
  k_colsq_part<<<g1, 256, 0, ctx->stream>>>(A, lda, N, nrhs, part);
  RBF_LAUNCHED(ctx, "k_colsq_part");
  k_colsq_sum<<<ceil_div(nrhs, 256), 256, 0, ctx->stream>>>(part, nrhs, ng, dout);
  RBF_LAUNCHED(ctx, "k_colsq_sum");
  host.resize(nrhs);
  RBF_HIP(ctx, hipMemcpyAsync(host.data(), dout, sizeof(double) * nrhs, hipMemcpyDeviceToHost,
                              ctx->stream));
  RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& v : host) v = std::sqrt(v);
  return RBF_OK;
}

// ---- refinement of the recursive update's weights (rbf_refine): conjugate
// gradients on calH w = b preconditioned by P / R, the Hestenes-Stiefel
// method with the preconditioner applied as z = M r.

// y_i = s sum_j P_ij x_j: one wave per row of P (coalesced row reads, four
// loads in flight per lane), fixed-order shuffle reduction.
__global__ void __launch_bounds__(256) k_pcg_symv(const double* __restrict__ P, int64_t ldp,
                                                  int64_t N, const double* __restrict__ x,
                                                  double s, double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= N) return;
  const double* __restrict__ row = P + i * ldp;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t j = lane;
  for (; j + 192 < N; j += 256) {
    s0 += row[j] * x[j];
    s1 += row[j + 64] * x[j + 64];
    s2 += row[j + 128] * x[j + 128];
    s3 += row[j + 192] * x[j + 192];
  }
  for (; j < N; j += 64) s0 += row[j] * x[j];
  double t = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  if (lane == 0) y[i] = s * t;
}

// y = b - A x (b may be null: y = A x) for the CSR matrix: 16 lanes per row
// (rows of ~100 entries), lane partial sums combined in a fixed order.
__global__ void __launch_bounds__(256) k_csr_mv16(const int64_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colidx,
                                                  const double* __restrict__ vals, int64_t N,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ b,
                                                  double* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  const int sub = threadIdx.x & 15;
  if (r >= N) return;  // the 16 lanes of a row leave together
  double t = 0.0;
  for (int64_t k = rowptr[r] + sub; k < rowptr[r + 1]; k += 16) t += vals[k] * x[colidx[k]];
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) t += __shfl_xor(t, o, 16);
  if (sub == 0) y[r] = b ? b[r] - t : t;
}

// Scalars of the iteration (device): rz = r.z, rz_new, pq = p.(calH p), rr.
enum { SC_RZ = 0, SC_RZN = 1, SC_PQ = 2, SC_RR = 3, SC_N = 4 };

// A step is taken only with positive curvature of both the preconditioner
// (r.z > 0) and calH (p.calH p > 0) and a finite step length; the host
// applies the same test to stop the iteration.
__host__ __device__ inline bool pcg_step_ok(double rz, double pq) {
  // a <= DBL_MAX is false for NaN and infinity
  return rz > 0.0 && pq > 0.0 && rz / pq <= DBL_MAX;
}

// w += alpha p, r -= alpha q, alpha = rz / pq; nothing is written unless
// pcg_step_ok holds, so w keeps the last accepted iterate.
__global__ void __launch_bounds__(256) k_pcg_step(double* __restrict__ w, double* __restrict__ r,
                                                  const double* __restrict__ p,
                                                  const double* __restrict__ q, int64_t N,
                                                  const double* __restrict__ sc) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= N) return;
  if (!pcg_step_ok(sc[SC_RZ], sc[SC_PQ])) return;
  const double alpha = sc[SC_RZ] / sc[SC_PQ];
  w[e] += alpha * p[e];
  r[e] -= alpha * q[e];
}

// p = z + beta p with beta = rz_new / rz (p = z when first != 0)
__global__ void __launch_bounds__(256) k_pcg_dir(double* __restrict__ p,
                                                 const double* __restrict__ z, int64_t N,
                                                 const double* __restrict__ sc, int first) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= N) return;
  p[e] = first ? z[e] : z[e] + (sc[SC_RZN] / sc[SC_RZ]) * p[e];
}

__global__ void k_pcg_shift(double* __restrict__ sc) { sc[SC_RZ] = sc[SC_RZN]; }

// ---- shared with the nested-dissection solver (ndsolve.hip)

rbf_status solve_residual(rbf_ctx* ctx, const int64_t* rowptr, const int32_t* colidx,
                          const double* vals, int64_t N, const double* B, int64_t ldb,
                          const double* X, int64_t ldx, int64_t nrhs, double* R) {
  if (nrhs == 1 && ldb == 1 && ldx == 1) {
    k_csr_mv16<<<(unsigned)ceil_div(N, 16), 256, 0, ctx->stream>>>(rowptr, colidx, vals, N, X,
                                                                    B, R);
    RBF_LAUNCHED(ctx, "k_csr_mv16");
    return RBF_OK;
  }
  k_residual<<<ceil_div(N * nrhs, 256), 256, 0, ctx->stream>>>(rowptr, colidx, vals, N, B, ldb,
                                                               X, ldx, nrhs, R);
  RBF_LAUNCHED(ctx, "k_residual");
  return RBF_OK;
}

rbf_status solve_col_norms(rbf_ctx* ctx, const double* A, int64_t lda, int64_t N, int64_t nrhs,
                           std::vector<double>& host) {
  rbf_status st;
  const int32_t ngroups = (int32_t)ceil_div(N, NRG);
  double* part = (double*)ws_get(ctx, WS_TMP3, sizeof(double) * (ngroups + 1) * nrhs, &st);
  if (!part) return st;
  double* dnorm = (double*)ws_get(ctx, WS_TMP2, sizeof(double) * nrhs, &st);
  if (!dnorm) return st;
  return col_norms(ctx, A, lda, N, nrhs, part, dnorm, host);
}

}  // namespace rbf

using namespace rbf;

extern "C" rbf_status rbf_refine(rbf_ctx* ctx, int64_t N, const int64_t* rowptr,
                                 const int32_t* colidx, const double* vals, const double* b,
                                 const double* P, int64_t ldp, double R, double* w, double rtol,
                                 int32_t max_iter, double* relres, int32_t* iters) {
  if (!ctx) return RBF_E_INVALID_ARG;
  if (iters) *iters = 0;
  if (relres) *relres = NAN;
  if (N <= 0 || !rowptr || !colidx || !vals || !b || !P || !w || ldp < N || !(R > 0) ||
      !(rtol > 0) || max_iter < 0)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_refine: bad arguments");
  RBF_TRY(set_device(ctx));
  RBF_TRY(rbf_sync_status(ctx));
  rbf_status st;
  double* vec = (double*)ws_get(ctx, WS_SOLVE5, sizeof(double) * 4 * (size_t)N, &st);
  if (!vec) return st;
  double *r = vec, *z = vec + N, *pd = vec + 2 * N, *q = vec + 3 * N;
  const int32_t ng = (int32_t)ceil_div(N, DOT_G);
  double* part = (double*)ws_get(ctx, WS_TMP3, sizeof(double) * (ng + 1), &st);
  if (!part) return st;
  double* sc = (double*)ws_get(ctx, WS_TMP2, sizeof(double) * 8, &st);
  if (!sc) return st;
  const unsigned gN = (unsigned)ceil_div(N, 256);
  auto dot = [&](const double* x, const double* y, int slot) -> rbf_status {
    k_dot_part<<<ng, 256, 0, ctx->stream>>>(x, y, N, part);
    RBF_LAUNCHED(ctx, "k_dot_part");
    k_dot_sum<<<1, 256, 0, ctx->stream>>>(part, ng, sc + slot);
    RBF_LAUNCHED(ctx, "k_dot_sum");
    return RBF_OK;
  };
  double h[SC_N];
  auto read = [&]() -> rbf_status {
    RBF_HIP(ctx, hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return RBF_OK;
  };
  // ||b||
  RBF_TRY(dot(b, b, SC_RR));
  RBF_TRY(read());
  const double bn = std::sqrt(h[SC_RR]);
  auto rel_of = [&](double rr) { return bn > 0 ? std::sqrt(rr) / bn : std::sqrt(rr); };
  // true residual r = b - calH w and its norm
  auto residual = [&](double* rel) -> rbf_status {
    k_csr_mv16<<<(unsigned)ceil_div(N, 16), 256, 0, ctx->stream>>>(rowptr, colidx, vals, N, w,
                                                                    b, r);
    RBF_LAUNCHED(ctx, "k_csr_mv16");
    RBF_TRY(dot(r, r, SC_RR));
    RBF_TRY(read());
    *rel = rel_of(h[SC_RR]);
    return RBF_OK;
  };
  double rel = 0.0;
  RBF_TRY(residual(&rel));
  int32_t it = 0;
  bool breakdown = false;
  // restart from the true residual whenever the recursive one says done
  while (!(rel <= rtol) && it < max_iter && std::isfinite(rel) && !breakdown) {
    k_pcg_symv<<<(unsigned)ceil_div(N, 4), 256, 0, ctx->stream>>>(P, ldp, N, r, 1.0 / R, z);
    RBF_LAUNCHED(ctx, "k_pcg_symv");
    RBF_TRY(dot(r, z, SC_RZN));
    k_pcg_dir<<<gN, 256, 0, ctx->stream>>>(pd, z, N, sc, 1);
    RBF_LAUNCHED(ctx, "k_pcg_dir");
    k_pcg_shift<<<1, 1, 0, ctx->stream>>>(sc);
    RBF_LAUNCHED(ctx, "k_pcg_shift");
    double rec = rel;
    while (it < max_iter) {
      k_csr_mv16<<<(unsigned)ceil_div(N, 16), 256, 0, ctx->stream>>>(rowptr, colidx, vals, N,
                                                                      pd, nullptr, q);
      RBF_LAUNCHED(ctx, "k_csr_mv16");
      RBF_TRY(dot(pd, q, SC_PQ));
      k_pcg_step<<<gN, 256, 0, ctx->stream>>>(w, r, pd, q, N, sc);
      RBF_LAUNCHED(ctx, "k_pcg_step");
      ++it;
      RBF_TRY(dot(r, r, SC_RR));
      RBF_TRY(read());
      if (!pcg_step_ok(h[SC_RZ], h[SC_PQ])) {  // P / R or calH not positive definite
        breakdown = true;
        break;
      }
      rec = rel_of(h[SC_RR]);
      if (rec <= rtol || !std::isfinite(rec)) break;
      k_pcg_symv<<<(unsigned)ceil_div(N, 4), 256, 0, ctx->stream>>>(P, ldp, N, r, 1.0 / R, z);
      RBF_LAUNCHED(ctx, "k_pcg_symv");
      RBF_TRY(dot(r, z, SC_RZN));
      k_pcg_dir<<<gN, 256, 0, ctx->stream>>>(pd, z, N, sc, 0);
      RBF_LAUNCHED(ctx, "k_pcg_dir");
      k_pcg_shift<<<1, 1, 0, ctx->stream>>>(sc);
      RBF_LAUNCHED(ctx, "k_pcg_shift");
    }
    RBF_TRY(residual(&rel));
  }
  if (iters) *iters = it;
  if (relres) *relres = rel;
  if (!(rel <= rtol))
    return fail(ctx, RBF_E_NO_CONVERGE, "rbf_refine: relres %g above %g after %d iterations%s",
                rel, rtol, it, breakdown ? " (lost positive definiteness)" : "");
  return RBF_OK;
}

extern "C" rbf_status rbf_solve(rbf_ctx* ctx, int64_t N, const int64_t* rowptr,
                                const int32_t* colidx, const double* vals, const double* B,
                                int64_t ldb, double* X, int64_t ldx, int64_t nrhs, double rtol,
                                int32_t max_iter, rbf_prec inner, double* relres,
                                int32_t* iters) {
  if (!ctx) return RBF_E_INVALID_ARG;
  if (iters) *iters = 0;
  if (N <= 0 || N >= ((int64_t)1 << 31) || !rowptr || !colidx || !vals || !B || !X ||
      nrhs <= 0 || ldb < nrhs || ldx < nrhs || !(rtol > 0) || max_iter < 1)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_solve: bad arguments");
  if (inner != RBF_F64)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_solve: inner precision %d not available",
                (int)inner);
  RBF_TRY(set_device(ctx));
  const int64_t seq = ctx->seq++;  // one launch group for the whole solve
  rbf_status st;
  // ---- bandwidth -> block size
  int32_t* d_bw = (int32_t*)ws_get(ctx, WS_SOLVE6, 256, &st);
  if (!d_bw) return st;
  RBF_TRY(fill_zero(ctx, d_bw, sizeof(int32_t)));
  k_csr_bandwidth<<<ceil_div(N, 256), 256, 0, ctx->stream>>>(rowptr, colidx, N, d_bw);
  RBF_LAUNCHED(ctx, "k_csr_bandwidth");
  int32_t bw = 0;
  RBF_HIP(ctx, hipMemcpyAsync(&bw, d_bw, sizeof(bw), hipMemcpyDeviceToHost, ctx->stream));
  RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (bw == INT32_MAX) return fail(ctx, RBF_E_INVALID_ARG, "rbf_solve: column index out of range");
  const int64_t s = ceil_div(bw > 0 ? bw : 1, 64) * 64;
  const int64_t nblk = ceil_div(N, s);
  const int64_t Np = nblk * s;
  const int64_t ss = s * s;
  if (s > 16384)
    return fail(ctx, RBF_E_INVALID_ARG,
                "rbf_solve: bandwidth %d too large (order the centers spatially)", bw);
  // ---- workspace
  double* D = (double*)ws_get(ctx, WS_SOLVE0, sizeof(double) * nblk * ss, &st);
  if (!D) return st;
  double* Ub = (double*)ws_get(ctx, WS_SOLVE1, sizeof(double) * nblk * ss, &st);
  if (!Ub) return st;
  double* Lb = (double*)ws_get(ctx, WS_SOLVE2, sizeof(double) * nblk * ss, &st);
  if (!Lb) return st;
  const int64_t nsub = s / 64;
  double* Linv = (double*)ws_get(ctx, WS_SOLVE3, sizeof(double) * nblk * nsub * 4096, &st);
  if (!Linv) return st;
  double* Y = (double*)ws_get(ctx, WS_SOLVE4, sizeof(double) * Np * nrhs, &st);
  if (!Y) return st;
  double* Rr = (double*)ws_get(ctx, WS_SOLVE5, sizeof(double) * N * nrhs, &st);
  if (!Rr) return st;
  const int32_t ngroups = (int32_t)ceil_div(N, NRG);
  double* part = (double*)ws_get(ctx, WS_TMP3, sizeof(double) * (ngroups + 1) * nrhs, &st);
  if (!part) return st;
  double* dnorm = (double*)ws_get(ctx, WS_TMP2, sizeof(double) * nrhs, &st);
  if (!dnorm) return st;
  // L^{-1} of every diagonal block (transposed), kept for the sweeps
  double* LiT = (double*)ws_get(ctx, WS_SOLVE7, sizeof(double) * nblk * ss, &st);
  if (!LiT) return st;
  // one block for the out-of-place product, then the forward sweep's vector
  double* Tmp = (double*)ws_get(ctx, WS_SOLVE8, sizeof(double) * std::max(ss, Np), &st);
  if (!Tmp) return st;
  const bool vec1 = nrhs == 1;
  // ---- blocks
  RBF_TRY(fill_zero(ctx, D, sizeof(double) * nblk * ss));
  RBF_TRY(fill_zero(ctx, Ub, sizeof(double) * nblk * ss));
  k_csr_to_blocks<<<ceil_div(Np, 256), 256, 0, ctx->stream>>>(rowptr, colidx, vals, N, (int32_t)s,
                                                              (int32_t)nblk, D, Ub);
  RBF_LAUNCHED(ctx, "k_csr_to_blocks");
  // ---- block Cholesky: D_i -= U_{i-1}^T U_{i-1} (the covariance product's
  // kernel, V^T = U_{i-1}), L_i L_i^T = D_i with X_i = L_i^{-1}, and
  // U_i = X_i A_{i,i+1} as one product
  RBF_TRY(fill_zero(ctx, LiT, sizeof(double) * nblk * ss));
  for (int64_t i = 0; i < nblk; ++i) {
    double* Di = D + i * ss;
    if (i > 0)
      RBF_TRY(syrk_update(ctx, Di, s, s, Ub + (i - 1) * ss, s, (int32_t)s, RBF_F64, nullptr, 0,
                          seq));
    RBF_TRY(chol_blocked(ctx, Di, (int32_t)s, Lb + i * ss, Linv + i * nsub * 4096, i, seq,
                         LiT + i * ss));
    if (i + 1 < nblk) {
      RBF_TRY(linv_apply(ctx, LiT + i * ss, (int32_t)s, Ub + i * ss, s, s, Tmp, seq));
      RBF_HIP(ctx, hipMemcpyAsync(Ub + i * ss, Tmp, sizeof(double) * ss, hipMemcpyDeviceToDevice,
                                  ctx->stream));
    }
  }
  {
    int32_t h[4];
    RBF_HIP(ctx, hipMemcpyAsync(h, ctx->d_status, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (h[0] != 0) return rbf_sync_status(ctx);
  }
  // ---- refinement
  std::vector<double> bn, rn;
  RBF_TRY(col_norms(ctx, B, ldb, N, nrhs, part, dnorm, bn));
  const double* R = B;
  int64_t ldr = ldb;
  int32_t it = 0;
  bool conv = false;
  for (it = 0; it < max_iter && !conv; ++it) {
    k_pad_copy<<<ceil_div(Np * nrhs, 256), 256, 0, ctx->stream>>>(R, ldr, N, Np, nrhs, Y);
    RBF_LAUNCHED(ctx, "k_pad_copy");
    if (vec1) {
      // L y = r by blocks: Z_i = X_i (r_i - U_{i-1}^T Z_{i-1}) into Tmp; then
      // L^T y = z: Y_i = X_i^T (Z_i - U_i Y_{i+1})
      for (int64_t i = 0; i < nblk; ++i) {
        double* Yi = Y + i * s;
        if (i > 0) RBF_TRY(mv_cols(ctx, Ub + (i - 1) * ss, s, s, Tmp + (i - 1) * s, Yi, -1.0, Yi));
        RBF_TRY(mv_cols(ctx, LiT + i * ss, s, s, Yi, nullptr, 1.0, Tmp + i * s));
      }
      for (int64_t i = nblk - 1; i >= 0; --i) {
        double* Zi = Tmp + i * s;
        if (i + 1 < nblk) RBF_TRY(mv_rows(ctx, Ub + i * ss, s, s, Y + (i + 1) * s, Zi, -1.0, Zi));
        RBF_TRY(mv_rows(ctx, LiT + i * ss, s, s, Zi, nullptr, 1.0, Y + i * s));
      }
    }
    for (int64_t i = 0; !vec1 && i < nblk; ++i) {
      double* Yi = Y + i * s * nrhs;
      if (i > 0)
        RBF_TRY(gemm_sub(ctx, true, s, nrhs, s, Ub + (i - 1) * ss, s, Yi - s * nrhs, nrhs, Yi,
                         nrhs, seq));
      RBF_TRY(trsm_blocks(ctx, Yi, nrhs, nrhs, (int32_t)nsub, Lb + i * ss, s,
                          Linv + i * nsub * 4096, false, seq));
    }
    for (int64_t i = nblk - 1; !vec1 && i >= 0; --i) {
      double* Yi = Y + i * s * nrhs;
      if (i + 1 < nblk)
        RBF_TRY(gemm_sub(ctx, false, s, nrhs, s, Ub + i * ss, s, Yi + s * nrhs, nrhs, Yi, nrhs,
                         seq));
      RBF_TRY(trsm_blocks(ctx, Yi, nrhs, nrhs, (int32_t)nsub, Lb + i * ss, s,
                          Linv + i * nsub * 4096, true, seq));
    }
    k_accum<<<ceil_div(N * nrhs, 256), 256, 0, ctx->stream>>>(X, ldx, Y, N, nrhs, it == 0);
    RBF_LAUNCHED(ctx, "k_accum");
    if (nrhs == 1 && ldb == 1 && ldx == 1) {
      k_csr_mv16<<<(unsigned)ceil_div(N, 16), 256, 0, ctx->stream>>>(rowptr, colidx, vals, N, X,
                                                                      B, Rr);
      RBF_LAUNCHED(ctx, "k_csr_mv16");
    } else {
      k_residual<<<ceil_div(N * nrhs, 256), 256, 0, ctx->stream>>>(rowptr, colidx, vals, N, B,
                                                                   ldb, X, ldx, nrhs, Rr);
      RBF_LAUNCHED(ctx, "k_residual");
    }
    R = Rr;
    ldr = nrhs;
    RBF_TRY(col_norms(ctx, Rr, nrhs, N, nrhs, part, dnorm, rn));
    conv = true;
    for (int64_t c = 0; c < nrhs; ++c) {
      const double rel = bn[c] > 0 ? rn[c] / bn[c] : rn[c];
      if (relres) relres[c] = rel;
      if (!(rel <= rtol)) conv = false;
    }
  }
  if (iters) *iters = it;
  RBF_TRY(rbf_sync_status(ctx));
  if (!conv)
    return fail(ctx, RBF_E_NO_CONVERGE, "rbf_solve: relres above %g after %d sweeps", rtol, it);
  return RBF_OK;
}
