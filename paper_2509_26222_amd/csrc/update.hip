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
#include <algorithm>
#include <cmath>

#include "internal.hpp"
#include "update.hpp"

namespace rbf {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int NB = 64;       // Cholesky / TRSM block size
constexpr int LDT = NB + 1;  // padded LDS row of a 64x64 tile


// ------------------------------------------------------------ batch rows

// Regressor rows of the batch in column-major ELL (entry q of row b at
// q * Bp + b), and the innovation y = z - H w into U^T[:, N]. With colmap,
// a center's column is colmap[center] (the compact index of an active
// center), else the center's own index. 16 lanes per point test the
// candidates 16 at a time; a ballot and popcount prefix keep the entries in
// candidate order (the order of a serial scan), capped at kmax.
__device__ __forceinline__ void upd_rows_body(const double* __restrict__ xy,
    const double* __restrict__ z, int32_t Bc, int32_t Bp, const double* __restrict__ cxy,
    const int32_t* __restrict__ idx, const int32_t* __restrict__ colmap,
    const int32_t* __restrict__ start, GridGeom g, RegKU k, int32_t kmax,
    const double* __restrict__ w, double* __restrict__ vals, int32_t* __restrict__ cols,
    int32_t* __restrict__ nnz, double* __restrict__ Ut, int64_t ldu, int64_t N,
    int32_t* __restrict__ status, int64_t batch, int64_t seq) {
  const int tid = threadIdx.x, l = tid & 15, gshift = tid & 48;
  const int b = blockIdx.x * 16 + (tid >> 4);
  if (b >= Bp || seq_skip(status, seq)) return;
  if (b >= Bc) {
    if (l == 0) {
      nnz[b] = 0;
      Ut[(int64_t)b * ldu + N] = 0.0;
    }
    return;
  }
  const double x = xy[2 * b], y = xy[2 * b + 1];
  int n = 0;
  double hw = 0.0;
  int bx0, bx1, by0, by1;
  if (bin_range(x, g.x0, g.inv_h, g.nbx, &bx0, &bx1) &&
      bin_range(y, g.y0, g.inv_h, g.nby, &by0, &by1)) {
    for (int by = by0; by <= by1; ++by) {
      const int row = by * g.nbx;
      const int s0 = start[row + bx0], s1 = start[row + bx1 + 1];
      for (int base = s0; base < s1; base += 16) {
        const int s = base + l;
        bool ok = false;
        double d2 = 0.0;
        if (s < s1) {
          const double dx = __dsub_rn(x, cxy[2 * s]), dy = __dsub_rn(y, cxy[2 * s + 1]);
          d2 = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
          ok = d2 <= k.rc2;
        }
        const uint32_t gm = (uint32_t)(__ballot(ok) >> gshift) & 0xFFFFu;
        const int pos = n + __popc(gm & ((1u << l) - 1u));
        if (ok && pos < kmax) {
          const double v = k.scale * exp(-d2 / k.den);
          const int32_t c = colmap ? colmap[idx[s]] : idx[s];
          vals[(int64_t)pos * Bp + b] = v;
          cols[(int64_t)pos * Bp + b] = c;
          hw += v * w[c];
        }
        n = min(n + __popc(gm), kmax);
      }
    }
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) hw += __shfl_xor(hw, off, 16);
  if (l == 0) {
    nnz[b] = n;
    const double zb = z[b];
    const double yb = zb - hw;
    if (!isfinite(zb) || !isfinite(yb) || !isfinite(x) || !isfinite(y))
      set_status(status, RBF_E_NONFINITE, batch, seq);
    Ut[(int64_t)b * ldu + N] = yb;
  }
}

__global__ void __launch_bounds__(256) k_upd_rows(const double* __restrict__ xy,
    const double* __restrict__ z, int32_t Bc, int32_t Bp, const double* __restrict__ cxy,
    const int32_t* __restrict__ idx, const int32_t* __restrict__ colmap,
    const int32_t* __restrict__ start, GridGeom g, RegKU k, int32_t kmax,
    const double* __restrict__ w, double* __restrict__ vals, int32_t* __restrict__ cols,
    int32_t* __restrict__ nnz, double* __restrict__ Ut, int64_t ldu, int64_t N,
    int32_t* __restrict__ status, int64_t batch, int64_t seq) {
  upd_rows_body(xy, z, Bc, Bp, cxy, idx, colmap, start, g, k, kmax, w, vals, cols, nnz, Ut, ldu, N,
    status, batch, seq);
}

// U^T[b, n] = sum_k vals[b,k] P[cols[b,k], n]  (P symmetric: rows of P).
// Block: 8 batch rows x 1024 columns; each thread 4 columns. With gR, only
// the rows of groups the grouped kernels leave (more than
// GATHER_GROUP_RMAX distinct rows of P).
__device__ __forceinline__ void upd_gather_u_body(const double* __restrict__ P, int64_t ldp,
    int64_t N, int32_t Bc, int32_t Bp, const double* __restrict__ vals,
    const int32_t* __restrict__ cols, const int32_t* __restrict__ nnz, double* __restrict__ Ut,
    int64_t ldu, const int32_t* __restrict__ gR, const int32_t* __restrict__ status, int64_t seq) {
  if (seq_skip(status, seq)) return;
  const int64_t n0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const int b0 = blockIdx.y * 8;
  if (gR && gR[b0 / 64] <= GATHER_GROUP_RMAX) return;
  for (int r = 0; r < 8; ++r) {
    const int b = b0 + r;
    double acc[4] = {0, 0, 0, 0};
    if (b < Bc) {
      const int nz = nnz[b];
      for (int q = 0; q < nz; ++q) {
        const double v = vals[(int64_t)q * Bp + b];
        const double* prow = P + (int64_t)cols[(int64_t)q * Bp + b] * ldp;
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

__global__ void __launch_bounds__(256) k_upd_gather_u(const double* __restrict__ P, int64_t ldp,
    int64_t N, int32_t Bc, int32_t Bp, const double* __restrict__ vals,
    const int32_t* __restrict__ cols, const int32_t* __restrict__ nnz, double* __restrict__ Ut,
    int64_t ldu, const int32_t* __restrict__ gR, const int32_t* __restrict__ status, int64_t seq) {
  upd_gather_u_body(P, ldp, N, Bc, Bp, vals, cols, nnz, Ut, ldu, gR, status, seq);
}

// Grouped gather, step 1 (one workgroup per group of 64 batch rows): the
// distinct columns of the group's regressor rows (the rows of P it needs)
// by an LDS bitmap over the N centers, ranked in ascending order by a
// popcount scan. Writes the list (padded to a multiple of 4 with row 0) and
// the dense block H_g[rank][row] (zero where a row has no entry).
constexpr int GG_NT = GATHER_GROUP_NT;  // threads per group of 64 batch rows

__device__ __forceinline__ void gather_groups_body(const double* __restrict__ vals,
    const int32_t* __restrict__ cols, const int32_t* __restrict__ nnz, int32_t Bc, int32_t Bp,
    int32_t kmax, int32_t words, int64_t Rcap, int32_t* __restrict__ glist,
    int32_t* __restrict__ gR, double* __restrict__ gH, const int32_t* __restrict__ status,
    int64_t seq) {
  if (seq_skip(status, seq)) return;
  extern __shared__ uint32_t gsm[];
  uint32_t* bits = gsm;
  int32_t* wbase = (int32_t*)(gsm + words);
  int32_t* tsum = wbase + words;  // one per wave
  const int tid = threadIdx.x;
  const int g = blockIdx.x, b0 = 64 * g;
  int32_t* L = glist + (int64_t)g * Rcap;
  double* H = gH + (int64_t)g * Rcap * 64;
  for (int w = tid; w < words; w += GG_NT) bits[w] = 0u;
  __syncthreads();
  const int ne = 64 * kmax;
  for (int e = tid; e < ne; e += GG_NT) {
    const int b = b0 + (e & 63), q = e >> 6;
    if (b < Bc && q < nnz[b]) {
      const int32_t c = cols[(int64_t)q * Bp + b];
      atomicOr(&bits[c >> 5], 1u << (c & 31));
    }
  }
  __syncthreads();
  const int per = (words + GG_NT - 1) / GG_NT;
  const int w0 = tid * per, w1 = min(w0 + per, words);
  int cnt = 0;
  for (int w = w0; w < w1; ++w) cnt += __popc(bits[w]);
  // exclusive scan of the counts in thread order: a shuffle scan in each
  // wave, then the totals of the waves before
  const int lane = tid & 63, wv = tid >> 6;
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) tsum[wv] = incl;
  __syncthreads();
  int base = incl - cnt;
  int R = 0;
  for (int w = 0; w < GG_NT / 64; ++w) {
    if (w < wv) base += tsum[w];
    R += tsum[w];
  }
  for (int w = w0; w < w1; ++w) {
    wbase[w] = base;
    uint32_t m = bits[w];
    while (m) {
      L[base++] = 32 * w + (__ffs(m) - 1);
      m &= m - 1u;
    }
  }
  const int R4 = (R + 3) & ~3;
  if (tid < R4 - R) L[R + tid] = 0;  // padding ranks: a valid row, zero H
  if (tid == 0) gR[g] = R4;
  for (int e = tid; e < R4 * 64; e += GG_NT) H[e] = 0.0;
  __syncthreads();  // zeros stored before the values below
  for (int e = tid; e < ne; e += GG_NT) {
    const int bl = e & 63, b = b0 + bl, q = e >> 6;
    if (b < Bc && q < nnz[b]) {
      const int32_t c = cols[(int64_t)q * Bp + b];
      const int r = wbase[c >> 5] + __popc(bits[c >> 5] & ((1u << (c & 31)) - 1u));
      H[(int64_t)r * 64 + bl] = vals[(int64_t)q * Bp + b];
    }
  }
}

__global__ void __launch_bounds__(GG_NT) k_gather_groups(const double* __restrict__ vals,
    const int32_t* __restrict__ cols, const int32_t* __restrict__ nnz, int32_t Bc, int32_t Bp,
    int32_t kmax, int32_t words, int64_t Rcap, int32_t* __restrict__ glist,
    int32_t* __restrict__ gR, double* __restrict__ gH, const int32_t* __restrict__ status,
    int64_t seq) {
  gather_groups_body(vals, cols, nnz, Bc, Bp, kmax, words, Rcap, glist, gR, gH, status, seq);
}

// Grouped gather, step 2: U^T[b0 + i][n] = sum_r H_g[r][i] P[list[r]][n]
// on FP64 MFMA, one workgroup per (128 columns, group); wave w owns columns
// 32w..32w+31 and all 64 rows (4 x 2 blocks of 16 x 16). Rows b >= Bc have
// no entries and get 0.
__device__ __forceinline__ void gather_mfma_body(const double* __restrict__ P, int64_t ldp,
    int64_t N, const int32_t* __restrict__ glist, const int32_t* __restrict__ gR,
    const double* __restrict__ gH, int64_t Rcap, double* __restrict__ Ut, int64_t ldu,
    const int32_t* __restrict__ status, int64_t seq) {
  if (seq_skip(status, seq)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = blockIdx.y;
  const int64_t c0 = (int64_t)blockIdx.x * 128 + wave * 32;
  const int32_t* L = glist + (int64_t)g * Rcap;
  const double* H = gH + (int64_t)g * Rcap * 64;
  const int R4 = gR[g];
  if (R4 > GATHER_GROUP_RMAX) return;  // left to k_upd_gather_u
  v4d acc[4][2];
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = (v4d){0.0, 0.0, 0.0, 0.0};
  const int kq = lane >> 4, li = lane & 15;
  int64_t colv[2];
  bool okc[2];
#pragma unroll
  for (int ni = 0; ni < 2; ++ni) {
    colv[ni] = c0 + 16 * ni + li;
    okc[ni] = colv[ni] < N;
    if (!okc[ni]) colv[ni] = 0;  // clamped: a valid address, value masked
  }
  // four k-steps at a time: all their loads are issued before the MFMAs
  int r = 0;
  for (; r + 16 <= R4; r += 16) {
    double a[4][4], bv[4][2];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int kr = r + 4 * st + kq;
      const double* prow = P + (int64_t)L[kr] * ldp;
#pragma unroll
      for (int mi = 0; mi < 4; ++mi) a[st][mi] = H[(int64_t)kr * 64 + 16 * mi + li];
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) {
        const double v = prow[colv[ni]];
        bv[st][ni] = okc[ni] ? v : 0.0;
      }
    }
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          acc[mi][ni] =
              __builtin_amdgcn_mfma_f64_16x16x4f64(a[st][mi], bv[st][ni], acc[mi][ni], 0, 0, 0);
  }
  for (; r < R4; r += 4) {
    const int kr = r + kq;
    const double* prow = P + (int64_t)L[kr] * ldp;
    double a[4], bv[2];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) a[mi] = H[(int64_t)kr * 64 + 16 * mi + li];
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
      const double v = prow[colv[ni]];
      bv[ni] = okc[ni] ? v : 0.0;
    }
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
        acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mi], bv[ni], acc[mi][ni], 0, 0, 0);
  }
  const int64_t b0 = 64 * (int64_t)g;
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
      if (okc[ni])
#pragma unroll
        for (int v = 0; v < 4; ++v)
          Ut[(b0 + 16 * mi + 4 * v + kq) * ldu + colv[ni]] = acc[mi][ni][v];
}

__global__ void __launch_bounds__(256) k_gather_mfma(const double* __restrict__ P, int64_t ldp,
    int64_t N, const int32_t* __restrict__ glist, const int32_t* __restrict__ gR,
    const double* __restrict__ gH, int64_t Rcap, double* __restrict__ Ut, int64_t ldu,
    const int32_t* __restrict__ status, int64_t seq) {
  gather_mfma_body(P, ldp, N, glist, gR, gH, Rcap, Ut, ldu, status, seq);
}

// S[a][b] (a >= b) = sum_k vals[a,k] U^T[b, cols[a,k]] + R delta_ab; the
// padding rows a >= Bc carry the identity. With gR, only the rows a of
// groups the grouped kernel leaves.
__device__ __forceinline__ void upd_S_body(const double* __restrict__ vals,
    const int32_t* __restrict__ cols, const int32_t* __restrict__ nnz,
    const double* __restrict__ Ut, int64_t ldu, int32_t Bc, int32_t Bp, double R,
    double* __restrict__ S, const int32_t* __restrict__ gR, const int32_t* __restrict__ status,
    int64_t seq) {
  if (seq_skip(status, seq)) return;
  const int b = blockIdx.y;
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= Bp || a < b) return;
  if (gR && gR[a / 64] <= GATHER_GROUP_RMAX) return;
  double s;
  if (a < Bc && b < Bc) {
    s = (a == b) ? R : 0.0;
    const double* ub = Ut + (int64_t)b * ldu;
    const int nz = nnz[a];
    for (int q = 0; q < nz; ++q) s += vals[(int64_t)q * Bp + a] * ub[cols[(int64_t)q * Bp + a]];
  } else {
    s = (a == b) ? 1.0 : 0.0;
  }
  S[(int64_t)a * Bp + b] = s;
}

__global__ void __launch_bounds__(256) k_upd_S(const double* __restrict__ vals,
    const int32_t* __restrict__ cols, const int32_t* __restrict__ nnz,
    const double* __restrict__ Ut, int64_t ldu, int32_t Bc, int32_t Bp, double R,
    double* __restrict__ S, const int32_t* __restrict__ gR, const int32_t* __restrict__ status,
    int64_t seq) {
  upd_S_body(vals, cols, nnz, Ut, ldu, Bc, Bp, R, S, gR, status, seq);
}

// The same lower triangle of S from the grouped gather's data: workgroup
// (ga, gb), gb <= ga, computes S[a][b] for the 64 rows a of group ga and the
// 64 columns b of block gb as sum_r H_ga[r][a] U^T[b][list_ga[r]] on FP64
// MFMA (wave w: columns 16w..16w+15, all 64 rows).
__device__ __forceinline__ void upd_S_groups_body(const int32_t* __restrict__ glist,
    const int32_t* __restrict__ gR, const double* __restrict__ gH, int64_t Rcap,
    const double* __restrict__ Ut, int64_t ldu, int32_t Bc, int32_t Bp, double R,
    double* __restrict__ S, const int32_t* __restrict__ status, int64_t seq) {
  if (seq_skip(status, seq)) return;
  const int t = blockIdx.x;
  int ga = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((ga + 1) * (ga + 2) / 2 <= t) ++ga;
  while (ga * (ga + 1) / 2 > t) --ga;
  const int gb = t - ga * (ga + 1) / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = lane >> 4, li = lane & 15;
  const int32_t* L = glist + (int64_t)ga * Rcap;
  const double* H = gH + (int64_t)ga * Rcap * 64;
  const int R4 = gR[ga];
  if (R4 > GATHER_GROUP_RMAX) return;  // left to k_upd_S (uniform per workgroup)
  // the group's row list in LDS, so that the value loads of four k-steps
  // can be issued together below (each step's value load needs its index)
  __shared__ int32_t Ls[GATHER_GROUP_RMAX];
  for (int e = threadIdx.x; e < R4; e += 256) Ls[e] = L[e];
  __syncthreads();
  const int bcol = gb * 64 + wave * 16 + li;  // < Bp
  const double* urow = Ut + (int64_t)bcol * ldu;
  v4d acc[4];
#pragma unroll
  for (int mi = 0; mi < 4; ++mi) acc[mi] = (v4d){0.0, 0.0, 0.0, 0.0};
  int r = 0;
  for (; r + 16 <= R4; r += 16) {
    double bv[4], hv[4][4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int kr = r + 4 * st + kq;
      bv[st] = urow[Ls[kr]];
#pragma unroll
      for (int mi = 0; mi < 4; ++mi) hv[st][mi] = H[(int64_t)kr * 64 + 16 * mi + li];
    }
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
        acc[mi] = __builtin_amdgcn_mfma_f64_16x16x4f64(hv[st][mi], bv[st], acc[mi], 0, 0, 0);
  }
  for (; r < R4; r += 4) {
    const int kr = r + kq;
    const double bv = urow[Ls[kr]];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
      acc[mi] = __builtin_amdgcn_mfma_f64_16x16x4f64(H[(int64_t)kr * 64 + 16 * mi + li], bv,
                                                     acc[mi], 0, 0, 0);
  }
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = ga * 64 + 16 * mi + 4 * v + kq;
      if (a < bcol) continue;
      double sv;
      if (a < Bc && bcol < Bc)
        sv = acc[mi][v] + ((a == bcol) ? R : 0.0);
      else
        sv = (a == bcol) ? 1.0 : 0.0;
      S[(int64_t)a * Bp + bcol] = sv;
    }
}

__global__ void __launch_bounds__(256) k_upd_S_groups(const int32_t* __restrict__ glist,
    const int32_t* __restrict__ gR, const double* __restrict__ gH, int64_t Rcap,
    const double* __restrict__ Ut, int64_t ldu, int32_t Bc, int32_t Bp, double R,
    double* __restrict__ S, const int32_t* __restrict__ status, int64_t seq) {
  upd_S_groups_body(glist, gR, gH, Rcap, Ut, ldu, Bc, Bp, R, S, status, seq);
}

// ------------------------------------------------------------- 64x64 tiles

// All 16 loads of a thread are issued before the first LDS store, so a tile
// costs one memory latency rather than sixteen.
__device__ inline void load_tile(double (*T)[LDT], const double* __restrict__ A, int64_t lda) {
  double v[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = threadIdx.x + 256 * u;
    v[u] = A[(int64_t)(e >> 6) * lda + (e & 63)];
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = threadIdx.x + 256 * u;
    T[e >> 6][e & 63] = v[u];
  }
}

__device__ inline void store_tile(const double (*T)[LDT], double* __restrict__ A, int64_t lda) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = threadIdx.x + 256 * u;
    A[(int64_t)(e >> 6) * lda + (e & 63)] = T[e >> 6][e & 63];
  }
}

// C = X Y^T for 64x64 LDS tiles on FP64 MFMA. Wave w owns the 32x32
// quadrant (w >> 1, w & 1); acc[mi][ni][v] is element
// (32 (w>>1) + 16 mi + 4 v + lane/16, 32 (w&1) + 16 ni + lane%16).
struct Acc64 {
  v4d c[2][2];
};

__device__ inline int acc_row(int mi, int v) {
  return 32 * ((threadIdx.x >> 6) >> 1) + 16 * mi + 4 * v + ((threadIdx.x & 63) >> 4);
}
__device__ inline int acc_col(int ni) {
  return 32 * ((threadIdx.x >> 6) & 1) + 16 * ni + (threadIdx.x & 15);
}

// A += X Y^T
__device__ inline void mm_nt_acc(const double (*X)[LDT], const double (*Y)[LDT], Acc64& A) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rb = 32 * (wave >> 1), cb = 32 * (wave & 1);
#pragma unroll 4
  for (int k = 0; k < NB; k += 4) {
    const int kk = k + (lane >> 4);
    double a[2], b[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      a[u] = X[rb + 16 * u + (lane & 15)][kk];
      b[u] = Y[cb + 16 * u + (lane & 15)][kk];
    }
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
        A.c[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mi], b[ni], A.c[mi][ni], 0, 0, 0);
  }
}

// A = X Y^T
__device__ inline void mm_nt(const double (*X)[LDT], const double (*Y)[LDT], Acc64& A) {
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) A.c[mi][ni] = (v4d){0.0, 0.0, 0.0, 0.0};
  mm_nt_acc(X, Y, A);
}

// A (64x64, leading dimension lda) = T^T: column-ordered walk, so the
// global stores are coalesced and the LDS reads go down a padded column.
__device__ inline void store_tile_t(const double (*T)[LDT], double* __restrict__ A, int64_t lda) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = threadIdx.x + 256 * u;
    A[(int64_t)(e >> 6) * lda + (e & 63)] = T[e & 63][e >> 6];
  }
}

__device__ inline void acc_to_lds(const Acc64& A, double (*T)[LDT]) {
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) T[acc_row(mi, v)][acc_col(ni)] = A.c[mi][ni][v];
}

// In-place Cholesky of the lower triangle of T (64x64) and Tinv = L^{-1}:
// chol64() in chol64.hpp.
#include "chol64.hpp"

// Blocks of the inverse X = L^{-1} of the blocked factor, row by row:
//   X_kj = -Linv_kk Y_kj,   Y_kj = sum_{m=j}^{k-1} L_km X_mj   (j < k).
// X is held transposed in LiT (LiT[c][r] = X[r][c], leading dimension Bp,
// zeroed before the factorization): the k-major operand of V^T = X U^T.
// The sums are spread over the launches so no workgroup walks a whole row:
// launch kb adds the term m = kb - 1 to the partial sums Y_kj of the rows
// k > kb (kept, transposed, in LiT's block of X_kj) and finishes row kb
// with its own last term. Every term is added in order of m.

// Y_kj^T (block (j, k) of LiT) += (L_km X_mj)^T, m = kb - 1, k > kb.
__device__ inline void linv_accum(int m, int k, int j, int32_t Bp, const double* __restrict__ Lb,
                                  double* __restrict__ LiT, double (*T1)[LDT],
                                  double (*T2)[LDT]) {
  load_tile(T1, Lb + (int64_t)k * NB * Bp + (int64_t)m * NB, Bp);  // L_km
  load_tile(T2, LiT + (int64_t)j * NB * Bp + (int64_t)m * NB, Bp);  // X_mj^T
  double* blk = LiT + (int64_t)j * NB * Bp + (int64_t)k * NB;       // Y_kj^T
  Acc64 Y;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Y.c[mi][ni][v] = blk[(int64_t)acc_col(ni) * Bp + acc_row(mi, v)];
  __syncthreads();
  mm_nt_acc(T1, T2, Y);  // Y += L_km X_mj
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        blk[(int64_t)acc_col(ni) * Bp + acc_row(mi, v)] = Y.c[mi][ni][v];
}

// X_kj (k = kb > j): Y_kj = (partial sum in LiT) + L_k,k-1 X_k-1,j, then
// X_kj = -Linv_kk Y_kj, written transposed over the partial sum.
__device__ inline void linv_finish(int kb, int j, int32_t Bp, const double* __restrict__ Lb,
                                   const double* __restrict__ Linv, double* __restrict__ LiT,
                                   double (*T1)[LDT], double (*T2)[LDT]) {
  const int m = kb - 1;
  load_tile(T1, Lb + (int64_t)kb * NB * Bp + (int64_t)m * NB, Bp);  // L_km
  load_tile(T2, LiT + (int64_t)j * NB * Bp + (int64_t)m * NB, Bp);  // X_mj^T
  double* blk = LiT + (int64_t)j * NB * Bp + (int64_t)kb * NB;
  Acc64 Y;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Y.c[mi][ni][v] = blk[(int64_t)acc_col(ni) * Bp + acc_row(mi, v)];
  __syncthreads();
  mm_nt_acc(T1, T2, Y);
  __syncthreads();  // T1, T2 free
  load_tile(T1, Linv + (int64_t)kb * NB * NB, NB);  // Linv_kk
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) T2[acc_col(ni)][acc_row(mi, v)] = Y.c[mi][ni][v];  // Y^T
  __syncthreads();
  Acc64 Z;
  mm_nt(T2, T1, Z);  // Z = Y^T Linv_kk^T = (Linv_kk Y)^T = -X_kj^T
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        blk[(int64_t)acc_row(mi, v) * Bp + acc_col(ni)] = -Z.c[mi][ni][v];
}

// The inverse's workgroups of launch kb (kb >= 1): u < kb finishes X_kb,u;
// the rest add term kb - 1 to the rows below.
__device__ inline void linv_work(int u, int kb, int32_t Bp, const double* __restrict__ Lb,
                                 const double* __restrict__ Linv, double* __restrict__ LiT,
                                 double (*T1)[LDT], double (*T2)[LDT]) {
  if (u < kb) {
    linv_finish(kb, u, Bp, Lb, Linv, LiT, T1, T2);
    return;
  }
  u -= kb;
  linv_accum(kb - 1, kb + 1 + u / kb, u % kb, Bp, Lb, LiT, T1, T2);
}

// The last block row of L^{-1} (kb = nblk - 1), after the final step.
__device__ __forceinline__ void linv_row_body(int32_t Bp, int32_t kb, const double* __restrict__ Lb,
    const double* __restrict__ Linv, double* __restrict__ LiT, const int32_t* __restrict__ status,
    int64_t seq) {
  if (seq_skip(status, seq)) return;
  __shared__ double T1[NB][LDT], T2[NB][LDT];
  linv_finish(kb, blockIdx.x, Bp, Lb, Linv, LiT, T1, T2);
}

__global__ void __launch_bounds__(256) k_linv_row(int32_t Bp, int32_t kb,
    const double* __restrict__ Lb, const double* __restrict__ Linv, double* __restrict__ LiT,
    const int32_t* __restrict__ status, int64_t seq) {
  linv_row_body(Bp, kb, Lb, Linv, LiT, status, seq);
}

// Factor diagonal block 0.
__device__ __forceinline__ void chol_first_body(const double* __restrict__ S, int32_t Bp,
    double* __restrict__ Lb, double* __restrict__ Linv, double* __restrict__ LiT,
    int32_t* __restrict__ status, int64_t batch, int64_t seq) {
  if (seq_skip(status, seq)) return;
  __shared__ double T[NB][LDT], Ti[NB][LDT];
  load_tile(T, S, Bp);
  __syncthreads();
  chol64(T, Ti, status, batch, seq);
  store_tile(T, Lb, Bp);
  store_tile(Ti, Linv, NB);
  if (LiT) store_tile_t(Ti, LiT, Bp);
}

__global__ void __launch_bounds__(256) k_chol_first(const double* __restrict__ S, int32_t Bp,
    double* __restrict__ Lb, double* __restrict__ Linv, double* __restrict__ LiT,
    int32_t* __restrict__ status, int64_t batch, int64_t seq) {
  chol_first_body(S, Bp, Lb, Linv, LiT, status, batch, seq);
}

// The diagonal workgroup of step kb (the launch's critical path), with Ta =
// Linv_kk and Tb = A_ik (i = kb + 1) loaded: L_ik = A_ik Linv_kk^T, then
// A_ii - L_ik L_ik^T factored in place. The two products use their zero
// structure with the work balanced over the four waves, each element
// keeping the MFMA sequence over k of the full product: wave w forms row
// block w of L_ik, where column block n needs k < 16 (n + 1) only (Linv_kk
// is lower triangular; 40 k-steps per wave instead of 64); the lower 16x16
// blocks of L_ik L_ik^T, the only ones the factor reads, are dealt round
// robin (at most 3 blocks, 48 k-steps, per wave).
// This wave's entries of A_ii in the lower blocks it updates (block b =
// wave + 4 q, see below), loaded before the workgroup's tiles so that their
// latency overlaps the tile loads.
__device__ inline void chol_diag_prefetch(const double* __restrict__ S, int32_t Bp, int i,
                                          double (&aii)[3][4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const double* Aii = S + (int64_t)i * NB * Bp + (int64_t)i * NB;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int b = wave + 4 * q;
    const int r = b < 1 ? 0 : b < 3 ? 1 : b < 6 ? 2 : 3;
    const int n = b - r * (r + 1) / 2;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      aii[q][v] = b < 10 ? Aii[(int64_t)(16 * r + 4 * v + kq) * Bp + 16 * n + li] : 0.0;
  }
}

__device__ inline void chol_step_diag(const double (&aii)[3][4], int32_t Bp, int i,
                                      double* __restrict__ Lb, double* __restrict__ Linv,
                                      double* __restrict__ LiT, double (*Ta)[LDT],
                                      double (*Tb)[LDT], int32_t* __restrict__ status,
                                      int64_t batch, int64_t seq) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, kq = lane >> 4;
  v4d l[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    l[n] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 16 * (n + 1); k += 4)
      l[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(Tb[16 * wave + li][k + kq],
                                                  Ta[16 * n + li][k + kq], l[n], 0, 0, 0);
  }
  __syncthreads();  // every wave is done with Linv_kk
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int v = 0; v < 4; ++v) Ta[16 * wave + 4 * v + kq][16 * n + li] = l[n][v];
  __syncthreads();
  // lower blocks (r, n), n <= r, in order 0:(0,0) 1:(1,0) 2:(1,1) 3:(2,0)
  // 4:(2,1) 5:(2,2) 6:(3,0) 7:(3,1) 8:(3,2) 9:(3,3); wave w takes w, w+4, w+8
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int b = wave + 4 * q;
    if (b < 10) {
      const int r = b < 1 ? 0 : b < 3 ? 1 : b < 6 ? 2 : 3;
      const int n = b - r * (r + 1) / 2;
      v4d u = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < NB; k += 4)
        u = __builtin_amdgcn_mfma_f64_16x16x4f64(Ta[16 * r + li][k + kq],
                                                 Ta[16 * n + li][k + kq], u, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = 16 * r + 4 * v + kq, cc = 16 * n + li;
        Tb[rr][cc] = aii[q][v] - u[v];
      }
    }
  }
  __syncthreads();
  // the strictly upper blocks of Tb still hold A_ik; the factor clears them
  // without reading them
  chol64(Tb, Ta, status, batch, seq);
  store_tile(Tb, Lb + (int64_t)i * NB * Bp + (int64_t)i * NB, Bp);
  store_tile(Ta, Linv + (int64_t)i * NB * NB, NB);
  if (LiT) store_tile_t(Ta, LiT + (int64_t)i * NB * Bp + (int64_t)i * NB, Bp);
}

// Step kb of the right-looking blocked Cholesky, one launch per block
// column. Tiles t < m are panel tiles (i = kb+1+t): L_ik = A_ik Linv_kk^T.
// Then come the trailing tiles (i, j), kb < j <= i: they recompute L_ik and
// L_jk from A and Linv_kk (read-only in this launch) and update A_ij; tile
// (kb+1, kb+1) then factors itself, ready for step kb+1. With LiT, the
// launch also carries the inverse's work of step kb (linv_work: kb + kb *
// (nblk - 1 - kb) workgroups of one or two block products), beside the
// critical path of the factor.
__device__ __forceinline__ void chol_step_body(double* __restrict__ S, int32_t Bp, int32_t nblk,
    int32_t kb, double* __restrict__ Lb, double* __restrict__ Linv, double* __restrict__ LiT,
    int32_t* __restrict__ status, int64_t batch, int64_t seq) {
  if (seq_skip(status, seq)) return;
  // two 64x64 tiles of LDS (67 KB) in every role, so a step workgroup fits
  // on a CU beside one covariance-product workgroup
  __shared__ double Ta[NB][LDT], Tb[NB][LDT];
  const int m = nblk - kb - 1;
  const int t = blockIdx.x;
  const int nfac = m + m * (m + 1) / 2;
  if (t >= nfac) {
    linv_work(t - nfac, kb, Bp, Lb, Linv, LiT, Ta, Tb);
    return;
  }
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
  const bool diag = !panel && i == kb + 1 && j == kb + 1;
  double aii[3][4];
  if (diag) chol_diag_prefetch(S, Bp, i, aii);
  load_tile(Ta, Linv + (int64_t)kb * NB * NB, NB);
  load_tile(Tb, S + (int64_t)i * NB * Bp + (int64_t)kb * NB, Bp);
  __syncthreads();
  if (diag) {
    chol_step_diag(aii, Bp, i, Lb, Linv, LiT, Ta, Tb, status, batch, seq);
    return;
  }
  Acc64 A;
  mm_nt(Tb, Ta, A);  // L_ik = A_ik Linv_kk^T
  if (panel) {
    double* out = Lb + (int64_t)i * NB * Bp + (int64_t)kb * NB;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          out[(int64_t)acc_row(mi, v) * Bp + acc_col(ni)] = A.c[mi][ni][v];
    return;
  }
  Acc64 Bq;
  if (j != i) {
    // L_jk = A_jk Linv_kk^T, with A_jk loaded over A_ik (now in registers)
    __syncthreads();
    load_tile(Tb, S + (int64_t)j * NB * Bp + (int64_t)kb * NB, Bp);
    __syncthreads();
    mm_nt(Tb, Ta, Bq);
  }
  __syncthreads();
  // Linv_kk is no longer needed: Ta = L_ik, Tb = L_jk
  acc_to_lds(A, Ta);
  if (j != i) acc_to_lds(Bq, Tb);
  __syncthreads();
  Acc64 U;
  mm_nt(Ta, (j != i) ? Tb : Ta, U);  // L_ik L_jk^T
  double* Aij = S + (int64_t)i * NB * Bp + (int64_t)j * NB;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Aij[(int64_t)acc_row(mi, v) * Bp + acc_col(ni)] -= U.c[mi][ni][v];
}

__global__ void __launch_bounds__(256, 2) k_chol_step(double* __restrict__ S, int32_t Bp,
    int32_t nblk, int32_t kb, double* __restrict__ Lb, double* __restrict__ Linv,
    double* __restrict__ LiT, int32_t* __restrict__ status, int64_t batch, int64_t seq) {
  chol_step_body(S, Bp, nblk, kb, Lb, Linv, LiT, status, batch, seq);
}

// ----------------------------------------------------------------- TRSM

// Blocked triangular solve in place on a slab of TW = 32 columns per
// workgroup, on FP64 MFMA, for a lower-triangular L held as off-diagonal
// 64x64 blocks (Lb, leading dimension ldl) and inverses of its diagonal
// blocks (Linv):
//   TRANS = false: X := L^{-1} X,   X_i = Linv_ii (X_i - sum_{j<i} L_ij X_j),
//                  block rows i = 0, 1, ...
//   TRANS = true : X := L^{-T} X,   X_i = Linv_ii^T (X_i - sum_{j>i} L_ji^T X_j),
//                  block rows i = nblk-1, ..., 0.
// The work of a slab is a sequence of tile pairs (i, j) ending each block
// row with (i, i), which applies the diagonal inverse; the next pair's tiles
// are loaded into registers while the current pair computes. Wave w owns
// rows 16w..16w+15 of a block row and both 16-column halves of the slab.
constexpr int TW = 32;
constexpr int LDX = TW + 1;

struct TrsmPre {
  double l[16];  // 64x64 tile: element (e >> 6, e & 63), e = tid + 256 u
  double x[8];   // 64x32 tile (e / 32, e % 32), e = tid + 256 u; or X_i values
};

template <bool TRANS>
__device__ inline void trsm_fetch(TrsmPre& pf, int i, int j, const double* __restrict__ Ut,
                                  int64_t ldu, int64_t ncols, int64_t col0,
                                  const double* __restrict__ Lb, int64_t ldl,
                                  const double* __restrict__ Linv) {
  const int tid = threadIdx.x, lane = tid & 63, rr = 16 * (tid >> 6);
  const double* src;
  int64_t lds;
  if (j != i) {
    src = TRANS ? Lb + (int64_t)j * NB * ldl + (int64_t)i * NB
                : Lb + (int64_t)i * NB * ldl + (int64_t)j * NB;
    lds = ldl;
  } else {
    src = Linv + (int64_t)i * NB * NB;
    lds = NB;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = tid + 256 * u;
    pf.l[u] = src[(int64_t)(e >> 6) * lds + (e & 63)];
  }
  if (j != i) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + 256 * u;
      const int64_t gc = col0 + (e & 31);
      pf.x[u] = gc < ncols ? Ut[(int64_t)(j * NB + (e >> 5)) * ldu + gc] : 0.0;
    }
  } else {
    // X_i in the MFMA accumulator layout of this lane
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rr + 4 * v + (lane >> 4), c = 16 * n + (lane & 15);
        const int64_t gc = col0 + c;
        pf.x[4 * n + v] = gc < ncols ? Ut[(int64_t)(i * NB + r) * ldu + gc] : 0.0;
      }
  }
}

template <bool TRANS>
__device__ inline void trsm_next(int i, int j, int nblk, int* ni, int* nj) {
  if (!TRANS) {
    *ni = i;
    *nj = j + 1;
    if (*nj > i) {
      *ni = i + 1;
      *nj = 0;
    }
  } else {
    if (j > i) {
      *ni = i;
      *nj = j - 1;
    } else {
      *ni = i - 1;
      *nj = nblk - 1;
    }
  }
}

template <bool TRANS>
__global__ void __launch_bounds__(256) k_trsm_blocks(double* __restrict__ Ut, int64_t ldu,
                                                     int64_t ncols, int32_t nblk,
                                                     const double* __restrict__ Lb, int64_t ldl,
                                                     const double* __restrict__ Linv,
                                                     const int32_t* __restrict__ status,
                                                     int64_t seq) {
  if (seq_skip(status, seq)) return;
  __shared__ double Lt[NB][LDT];
  __shared__ double X[NB][LDX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t col0 = (int64_t)blockIdx.x * TW;
  const int rr = 16 * wave;
  TrsmPre pf;
  int i = TRANS ? nblk - 1 : 0, j = i;  // current pair
  trsm_fetch<TRANS>(pf, i, j, Ut, ldu, ncols, col0, Lb, ldl, Linv);
  v4d acc[2] = {(v4d){0.0, 0.0, 0.0, 0.0}, (v4d){0.0, 0.0, 0.0, 0.0}};
  while (i >= 0 && i < nblk) {
    const bool diag = (j == i);
    __syncthreads();  // previous pair done with LDS (and its X_i stores)
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u;
      Lt[e >> 6][e & 63] = pf.l[u];
    }
    if (!diag) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = tid + 256 * u;
        X[e >> 5][e & 31] = pf.x[u];
      }
    } else {
      // R_i = X_i - sum_j (off-diagonal block) X_j, in the accumulator layout
#pragma unroll
      for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          X[rr + 4 * v + (lane >> 4)][16 * n + (lane & 15)] = pf.x[4 * n + v] - acc[n][v];
    }
    __syncthreads();
    // Next pair. Its X_j blocks were finished by earlier diagonal steps,
    // except right after the first diagonal step, whose successor needs the
    // block just solved: that fetch waits for the stores below.
    int ni, nj;
    trsm_next<TRANS>(i, j, nblk, &ni, &nj);
    const bool nvalid = ni >= 0 && ni < nblk;
    const bool late = diag && nj == i;
    if (nvalid && !late) trsm_fetch<TRANS>(pf, ni, nj, Ut, ldu, ncols, col0, Lb, ldl, Linv);
    if (!diag) {
#pragma unroll 4
      for (int k = 0; k < NB; k += 4) {
        const int kk = k + (lane >> 4);
        const double a = TRANS ? Lt[kk][rr + (lane & 15)] : Lt[rr + (lane & 15)][kk];
#pragma unroll
        for (int n = 0; n < 2; ++n)
          acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, X[kk][16 * n + (lane & 15)], acc[n],
                                                        0, 0, 0);
      }
    } else {
      v4d out[2] = {(v4d){0.0, 0.0, 0.0, 0.0}, (v4d){0.0, 0.0, 0.0, 0.0}};
#pragma unroll 4
      for (int k = 0; k < NB; k += 4) {
        const int kk = k + (lane >> 4);
        const double a = TRANS ? Lt[kk][rr + (lane & 15)] : Lt[rr + (lane & 15)][kk];
#pragma unroll
        for (int n = 0; n < 2; ++n)
          out[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, X[kk][16 * n + (lane & 15)], out[n],
                                                        0, 0, 0);
      }
#pragma unroll
      for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = rr + 4 * v + (lane >> 4), c = 16 * n + (lane & 15);
          const int64_t gc = col0 + c;
          if (gc < ncols) Ut[(int64_t)(i * NB + r) * ldu + gc] = out[n][v];
        }
      acc[0] = (v4d){0.0, 0.0, 0.0, 0.0};
      acc[1] = (v4d){0.0, 0.0, 0.0, 0.0};
      if (late && nvalid) {
        __syncthreads();  // X_i stored by all waves before it is read back
        trsm_fetch<TRANS>(pf, ni, nj, Ut, ldu, ncols, col0, Lb, ldl, Linv);
      }
    }
    i = ni;
    j = nj;
  }
}

// w[n] += sum_b V^T[b, n] t[b], t = V^T[:, N]; stage 1 sums groups of 64
// rows into part[g][n], stage 2 adds the groups in order (deterministic).
__device__ __forceinline__ void upd_w_part_body(const double* __restrict__ Ut, int64_t ldu,
    int64_t N, int32_t Bc, double* __restrict__ part, const int32_t* __restrict__ status,
    int64_t seq) {
  if (seq_skip(status, seq)) return;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const int b0 = blockIdx.y * 64;
  const int b1 = b0 + 64 < Bc ? b0 + 64 : Bc;
  double s0 = 0.0, s1 = 0.0;
  int b = b0;
  for (; b + 1 < b1; b += 2) {
    s0 += Ut[(int64_t)b * ldu + n] * Ut[(int64_t)b * ldu + N];
    s1 += Ut[(int64_t)(b + 1) * ldu + n] * Ut[(int64_t)(b + 1) * ldu + N];
  }
  if (b < b1) s0 += Ut[(int64_t)b * ldu + n] * Ut[(int64_t)b * ldu + N];
  part[(int64_t)blockIdx.y * N + n] = s0 + s1;
}

__global__ void __launch_bounds__(256) k_upd_w_part(const double* __restrict__ Ut, int64_t ldu,
    int64_t N, int32_t Bc, double* __restrict__ part, const int32_t* __restrict__ status,
    int64_t seq) {
  upd_w_part_body(Ut, ldu, N, Bc, part, status, seq);
}

__device__ __forceinline__ void upd_w_sum_body(double* __restrict__ w,
    const double* __restrict__ part, int64_t N, int32_t ngroups, const int32_t* __restrict__ status,
    int64_t seq) {
  if (seq_skip(status, seq)) return;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  double s = 0.0;
  for (int g = 0; g < ngroups; ++g) s += part[(int64_t)g * N + n];
  w[n] += s;
}

__global__ void __launch_bounds__(256) k_upd_w_sum(double* __restrict__ w,
    const double* __restrict__ part, int64_t N, int32_t ngroups, const int32_t* __restrict__ status,
    int64_t seq) {
  upd_w_sum_body(w, part, N, ngroups, status, seq);
}

// Touched row blocks of P: flags[c / SYRK_TILE] = 1 for every center c in
// the batch's regressor rows (flags cleared beforehand). The covariance
// product of the previous batch computes the tiles in these block rows and
// columns first, so the gather of this batch can start while it finishes
// the rest.
__global__ void __launch_bounds__(256) k_upd_flags(const int32_t* __restrict__ cols,
                                                   const int32_t* __restrict__ nnz, int32_t Bc,
                                                   int32_t Bp, int32_t* __restrict__ flags,
                                                   const int32_t* __restrict__ status,
                                                   int64_t seq) {
  if (seq_skip(status, seq)) return;
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= Bc) return;
  const int nz = nnz[b];
  for (int q = 0; q < nz; ++q) flags[cols[(int64_t)q * Bp + b] / SYRK_TILE] = 1;
}

rbf_status update_workspace(rbf_ctx* ctx, int64_t N, int32_t kmax, int64_t Bmax,
                            rbf_prec gemm_prec, UpdWs* ws) {
  const int32_t Bp = (int32_t)ceil_div(Bmax > 0 ? Bmax : 1, NB) * NB;
  const int32_t nblk_max = Bp / NB;
  const int64_t ldu = ceil_div(N + 1, 32) * 32;
  rbf_status st;
  char* ell = (char*)ws_get(ctx, WS_UPD_ELL, (size_t)Bp * kmax * 12 + (size_t)Bp * 4 + 256, &st);
  if (!ell) return st;
  ws->vals = (double*)ell;
  ws->cols = (int32_t*)(ell + (size_t)Bp * kmax * 8);
  ws->nnz = ws->cols + (size_t)Bp * kmax;
  ws->Ut = (double*)ws_get(ctx, WS_UPD_UT, sizeof(double) * (size_t)Bp * ldu, &st);
  if (!ws->Ut) return st;
  ws->Ut2 = (double*)ws_get(ctx, WS_UPD_UT2, sizeof(double) * (size_t)Bp * ldu, &st);
  if (!ws->Ut2) return st;
  ws->flags = (int32_t*)ws_get(ctx, WS_UPD_FLAGS,
                               sizeof(int32_t) * 2 * (size_t)ceil_div(N, SYRK_TILE), &st);
  if (!ws->flags) return st;
  ws->S = (double*)ws_get(ctx, WS_UPD_S, sizeof(double) * (size_t)Bp * Bp * 3, &st);
  if (!ws->S) return st;
  ws->Lb = ws->S + (size_t)Bp * Bp;
  ws->LiT = ws->Lb + (size_t)Bp * Bp;
  ws->Vt = (double*)ws_get(ctx, WS_UPD_VT, sizeof(double) * (size_t)Bp * ldu * 2, &st);
  if (!ws->Vt) return st;
  ws->Vt2 = ws->Vt + (size_t)Bp * ldu;
  ws->Linv = (double*)ws_get(ctx, WS_UPD_LINV, sizeof(double) * (size_t)nblk_max * NB * NB, &st);
  if (!ws->Linv) return st;
  ws->wpart = (double*)ws_get(ctx, WS_TMP3, sizeof(double) * (size_t)nblk_max * N, &st);
  if (!ws->wpart) return st;
  ws->Rcap = 0;
  ws->glist = nullptr;
  ws->gR = nullptr;
  ws->gH = nullptr;
  if (N <= GATHER_GROUP_NMAX) {
    const int64_t ng = Bp / 64;
    int64_t Rcap = std::min<int64_t>(N, (int64_t)64 * kmax);
    Rcap = (Rcap + 3) / 4 * 4 + 4;
    char* gw = (char*)ws_get(ctx, WS_UPD_GROUPS,
                             (size_t)ng * Rcap * (64 * sizeof(double) + sizeof(int32_t)) +
                                 (size_t)ng * sizeof(int32_t) + 256,
                             &st);
    if (!gw) return st;
    ws->Rcap = Rcap;
    ws->gH = (double*)gw;
    ws->glist = (int32_t*)(gw + (size_t)ng * Rcap * 64 * sizeof(double));
    ws->gR = ws->glist + (size_t)ng * Rcap;
  }
  if (gemm_prec == RBF_F32) {
    if (!ws_get(ctx, WS_UPD_VLO, sizeof(float) * (size_t)Bp * ldu, &st)) return st;
    if (ctx->joseph &&
        !ws_get(ctx, WS_JOSEPH,
                sizeof(double) * ((size_t)Bp * Bp + (size_t)Bp * ldu) +
                    sizeof(float) * 4 * (size_t)Bp * ldu,
                &st))
      return st;
  } else if (gemm_prec == RBF_BF16) {
    if (!ws_get(ctx, WS_UPD_VLO, 2 * 2 * (size_t)N * Bp, &st)) return st;
  }
  return RBF_OK;
}

rbf_status chol_blocked(rbf_ctx* ctx, double* S, int32_t n, double* Lb, double* Linv,
                        int64_t index, int64_t seq, double* LiT) {
  const int32_t nblk = n / NB;
  k_chol_first<<<1, 256, 0, ctx->stream>>>(S, n, Lb, Linv, LiT, ctx->d_status, index, seq);
  RBF_LAUNCHED(ctx, "k_chol_first");
  for (int32_t kb = 0; kb + 1 < nblk; ++kb) {
    const int m = nblk - kb - 1;
    const int extra = LiT ? kb + kb * (nblk - 1 - kb) : 0;
    k_chol_step<<<m + m * (m + 1) / 2 + extra, 256, 0, ctx->stream>>>(
        S, n, nblk, kb, Lb, Linv, LiT, ctx->d_status, index, seq);
    RBF_LAUNCHED(ctx, "k_chol_step");
  }
  if (LiT && nblk > 1) {
    k_linv_row<<<nblk - 1, 256, 0, ctx->stream>>>(n, nblk - 1, Lb, Linv, LiT, ctx->d_status,
                                                   seq);
    RBF_LAUNCHED(ctx, "k_linv_row");
  }
  return RBF_OK;
}

// Single right-hand side (x of nblk*64 entries, contiguous): one workgroup
// of 1024 threads with x in LDS walks the block rows in order. Block row i
// first forms r = x_i - sum_{j<i} L_ij x_j (TRANS: x_i - sum_{j>i} L_ji^T
// x_j), 16 partial sums per row combined in a fixed order, then
// x_i = Linv_ii r (TRANS: Linv_ii^T r). L is streamed once per solve.
template <bool TRANS>
__global__ void __launch_bounds__(1024) k_trsv1(double* __restrict__ x, int32_t nblk,
                                                const double* __restrict__ Lb, int64_t ldl,
                                                const double* __restrict__ Linv,
                                                const int32_t* __restrict__ status,
                                                int64_t seq) {
  if (seq_skip(status, seq)) return;
  extern __shared__ __attribute__((aligned(16))) double ys[];  // nblk*64 + 16*64 + 64
  const int n = nblk * NB;
  double* part = ys + n;       // [16][64] partial sums
  double* rv = part + 16 * NB; // r of the current block row
  const int tid = threadIdx.x;
  for (int e = tid; e < n; e += 1024) ys[e] = x[e];
  __syncthreads();
  for (int step = 0; step < nblk; ++step) {
    const int i = TRANS ? nblk - 1 - step : step;
    const int r0 = i * NB;
    if (!TRANS) {
      // thread (row r = tid / 16, lane cl = tid % 16): columns cl, cl+16, ... < r0
      const int r = tid >> 4, cl = tid & 15;
      const double* row = Lb + (int64_t)(r0 + r) * ldl;
      // four independent sums, unrolled: several loads in flight per lane
      double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
      int c = cl;
#pragma unroll 2
      for (; c + 48 < r0; c += 64) {
        t0 += row[c] * ys[c];
        t1 += row[c + 16] * ys[c + 16];
        t2 += row[c + 32] * ys[c + 32];
        t3 += row[c + 48] * ys[c + 48];
      }
      for (; c < r0; c += 16) t0 += row[c] * ys[c];
      double t = (t0 + t1) + (t2 + t3);
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) t += __shfl_xor(t, o, 16);
      if (cl == 0) rv[r] = ys[r0 + r] - t;
    } else {
      // thread (row r = tid % 64, lane cl = tid / 64): L rows c = r0+64+cl,
      // +16, ... of column r0 + r (64 consecutive columns per wave)
      const int r = tid & 63, cl = tid >> 6;
      const double* col = Lb + r0 + r;
      double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
      int c = r0 + NB + cl;
#pragma unroll 2
      for (; c + 48 < n; c += 64) {
        t0 += col[(int64_t)c * ldl] * ys[c];
        t1 += col[(int64_t)(c + 16) * ldl] * ys[c + 16];
        t2 += col[(int64_t)(c + 32) * ldl] * ys[c + 32];
        t3 += col[(int64_t)(c + 48) * ldl] * ys[c + 48];
      }
      for (; c < n; c += 16) t0 += col[(int64_t)c * ldl] * ys[c];
      part[cl * NB + r] = (t0 + t1) + (t2 + t3);
      __syncthreads();
      if (tid < NB) {
        double u = 0.0;
        for (int q = 0; q < 16; ++q) u += part[q * NB + tid];
        rv[tid] = ys[r0 + tid] - u;
      }
    }
    __syncthreads();
    // x_i = Linv_ii r (or its transpose): 16 lanes per output row
    {
      const int r = tid >> 4, cl = tid & 15;
      const double* Li = Linv + (int64_t)i * NB * NB;
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = cl + 16 * q;
        t += (TRANS ? Li[(int64_t)c * NB + r] : Li[(int64_t)r * NB + c]) * rv[c];
      }
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) t += __shfl_xor(t, o, 16);
      if (cl == 0) ys[r0 + r] = t;
    }
    __syncthreads();
  }
  for (int e = tid; e < n; e += 1024) x[e] = ys[e];
}

rbf_status trsm_blocks(rbf_ctx* ctx, double* X, int64_t ldx, int64_t ncols, int32_t nblk,
                       const double* Lb, int64_t ldl, const double* Linv, bool trans,
                       int64_t seq) {
  if (ncols <= 0 || nblk <= 0) return RBF_OK;
  const size_t lds1 = sizeof(double) * ((size_t)nblk * NB + 17 * NB);
  if (ncols == 1 && ldx == 1 && lds1 <= 64 * 1024) {
    if (trans)
      k_trsv1<true><<<1, 1024, lds1, ctx->stream>>>(X, nblk, Lb, ldl, Linv, ctx->d_status, seq);
    else
      k_trsv1<false><<<1, 1024, lds1, ctx->stream>>>(X, nblk, Lb, ldl, Linv, ctx->d_status, seq);
    RBF_LAUNCHED(ctx, "k_trsv1");
    return RBF_OK;
  }
  const unsigned grid = (unsigned)ceil_div(ncols, TW);
  if (trans)
    k_trsm_blocks<true><<<grid, 256, 0, ctx->stream>>>(X, ldx, ncols, nblk, Lb, ldl, Linv,
                                                       ctx->d_status, seq);
  else
    k_trsm_blocks<false><<<grid, 256, 0, ctx->stream>>>(X, ldx, ncols, nblk, Lb, ldl, Linv,
                                                        ctx->d_status, seq);
  RBF_LAUNCHED(ctx, "k_trsm_blocks");
  return RBF_OK;
}

rbf_status update_check(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g, const double* w,
                        const double* P, int64_t ldp, const double* xy, const double* z,
                        int64_t M, int64_t batch, rbf_prec gemm_prec) {
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
  return RBF_OK;
}

// Enqueue the recursive update of (w, P) (N x N, leading dimension ldp) by
// the M points in batches of B; regressor columns go through colmap when it
// is given (the active-rows form's compact problem). Only enqueues: the
// caller reads the status word (update_done).
rbf_status update_run(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                      const int32_t* colmap, int64_t N, double* w, double* P, int64_t ldp,
                      const double* xy, const double* z, int64_t M, int64_t B,
                      rbf_prec gemm_prec) {
  RBF_TRY(set_device(ctx));
  // The two-stream schedule is not captured: under stream capture (a
  // caller's graph) a context set to two streams returns an error instead
  // (a process crash was seen once while capturing it, with its cause not
  // established; the batched form's branches use one stream).
  hipStreamCaptureStatus cap_st = hipStreamCaptureStatusActive;
  if (hipStreamIsCapturing(ctx->stream, &cap_st) != hipSuccess) {
    (void)hipGetLastError();  // not left for the next launch check
    cap_st = hipStreamCaptureStatusActive;
  }
  if (!ctx->single_stream && cap_st != hipStreamCaptureStatusNone)
    return fail(ctx, RBF_E_INVALID_ARG,
                "rbf_update: the two-stream schedule cannot be captured (set streams = 1)");
  if (ctx->joseph && (gemm_prec != RBF_F32 || !ctx->single_stream))
    return fail(ctx, RBF_E_INVALID_ARG,
                "rbf_update: the Joseph form is available with FP32 products on one stream");
  const int32_t kmax = g->max_cand > 0 ? g->max_cand : 1;
  const int64_t ldu = ceil_div(N + 1, 32) * 32;
  UpdWs ws;
  RBF_TRY(update_workspace(ctx, N, kmax, B < M ? B : M, gemm_prec, &ws));
  double* vals = ws.vals;
  int32_t* cols = ws.cols;
  int32_t* nnz = ws.nnz;
  double* S = ws.S;
  double* Lb = ws.Lb;
  double* Linv = ws.Linv;
  double* wpart = ws.wpart;
  const RegKU rk = regku(p);
  const int64_t nb_total = ceil_div(M, B);
  // Launch group (sequence number) of batch bi: seq0 + bi. A failure in
  // batch bi stops the launches of batches >= bi only.
  const int64_t seq0 = ctx->seq;
  ctx->seq += nb_total;
  // Two streams when there is more than one batch: `ms` (the context's
  // stream) runs the covariance products, `as` the chain of the next batch
  // (regressor rows, U, S, Cholesky, V, w). Batch bi+1's gather reads only
  // the rows of P in its touched blocks, which part 1 of batch bi's product
  // finishes first; part 2 (all other tiles) overlaps the chain.
  const bool two = nb_total > 1 && !ctx->single_stream;
  if (two) RBF_TRY(ensure_aux(ctx));
  hipStream_t ms = ctx->stream;
  hipStream_t as = two ? ctx->aux : ctx->stream;
  const int64_t nfl = ceil_div(N, SYRK_TILE);
  double* UtB[2] = {ws.Ut, ws.Ut2};
  double* VtB[2] = {ws.Vt, ws.Vt2};
  int32_t* Fl[2] = {ws.flags, ws.flags + nfl};
  auto sizes = [&](int64_t bi, int32_t* Bc, int32_t* Bpc) {
    const int64_t s0 = bi * B;
    *Bc = (int32_t)((M - s0) < B ? (M - s0) : B);
    *Bpc = (int32_t)ceil_div(*Bc, NB) * NB;
  };
  // regressor rows, innovation y = z - H w and (two streams) touched blocks
  // of batch bi
  auto rows = [&](int64_t bi) -> rbf_status {
    int32_t Bc, Bpc;
    sizes(bi, &Bc, &Bpc);
    const int64_t s0 = bi * B;
    k_upd_rows<<<ceil_div(Bpc, 16), 256, 0, ctx->stream>>>(
        xy + 2 * s0, z + s0, Bc, Bpc, g->d_cxy, g->d_idx, colmap, g->d_start, geom(g), rk, kmax, w,
        vals, cols, nnz, UtB[bi & 1], ldu, N, ctx->d_status, ctx->index_base + bi, seq0 + bi);
    RBF_LAUNCHED(ctx, "k_upd_rows");
    if (!two) return RBF_OK;  // the touched blocks only steer the two-stream split
    RBF_TRY(fill_zero(ctx, Fl[bi & 1], sizeof(int32_t) * nfl));
    k_upd_flags<<<ceil_div(Bc, 256), 256, 0, ctx->stream>>>(cols, nnz, Bc, Bpc, Fl[bi & 1],
                                                             ctx->d_status, seq0 + bi);
    RBF_LAUNCHED(ctx, "k_upd_flags");
    return RBF_OK;
  };
  // U^T = H P, S = H U + R I, L L^T = S, V^T = L^{-1} U^T (with t), w += V t
  auto chain = [&](int64_t bi) -> rbf_status {
    int32_t Bc, Bpc;
    sizes(bi, &Bc, &Bpc);
    double* Ut = UtB[bi & 1];
    const int64_t sq = seq0 + bi;
    prof_begin(ctx, RBF_PROF_GATHER);
    if (ws.gH) {
      const int32_t words = gather_group_words(N);
      const size_t lds = gather_group_lds(words);
      k_gather_groups<<<Bpc / 64, GG_NT, lds, ctx->stream>>>(vals, cols, nnz, Bc, Bpc, kmax, words,
                                                           ws.Rcap, ws.glist, ws.gR, ws.gH,
                                                           ctx->d_status, sq);
      RBF_LAUNCHED(ctx, "k_gather_groups");
      dim3 gm((unsigned)ceil_div(N, 128), (unsigned)(Bpc / 64));
      k_gather_mfma<<<gm, 256, 0, ctx->stream>>>(P, ldp, N, ws.glist, ws.gR, ws.gH, ws.Rcap, Ut,
                                                  ldu, ctx->d_status, sq);
      RBF_LAUNCHED(ctx, "k_gather_mfma");
    }
    {  // all rows without the grouped data, else the groups it leaves
      dim3 gg((unsigned)ceil_div(N, 1024), (unsigned)ceil_div(Bpc, 8));
      k_upd_gather_u<<<gg, 256, 0, ctx->stream>>>(P, ldp, N, Bc, Bpc, vals, cols, nnz, Ut, ldu,
                                                   ws.gH ? ws.gR : nullptr, ctx->d_status, sq);
      RBF_LAUNCHED(ctx, "k_upd_gather_u");
    }
    prof_end(ctx, RBF_PROF_GATHER);
    if (ws.gH) {
      const int ng = Bpc / 64;
      k_upd_S_groups<<<ng * (ng + 1) / 2, 256, 0, ctx->stream>>>(
          ws.glist, ws.gR, ws.gH, ws.Rcap, Ut, ldu, Bc, Bpc, p->R, S, ctx->d_status, sq);
      RBF_LAUNCHED(ctx, "k_upd_S_groups");
    }
    {  // all rows without the grouped data, else the groups it leaves
      dim3 gs((unsigned)ceil_div(Bpc, 256), (unsigned)Bpc);
      k_upd_S<<<gs, 256, 0, ctx->stream>>>(vals, cols, nnz, Ut, ldu, Bc, Bpc, p->R, S,
                                           ws.gH ? ws.gR : nullptr, ctx->d_status, sq);
      RBF_LAUNCHED(ctx, "k_upd_S");
    }
    double* Vt = VtB[bi & 1];
    prof_begin(ctx, RBF_PROF_CHOL);
    RBF_TRY(fill_zero(ctx, ws.LiT, sizeof(double) * (size_t)Bpc * Bpc));
    RBF_TRY(chol_blocked(ctx, S, Bpc, Lb, Linv, ctx->index_base + bi, sq, ws.LiT));
    prof_end(ctx, RBF_PROF_CHOL);
    prof_begin(ctx, RBF_PROF_TRSM);
    RBF_TRY(linv_apply(ctx, ws.LiT, Bpc, Ut, ldu, N + 1, Vt, sq));
    prof_end(ctx, RBF_PROF_TRSM);
    dim3 gw((unsigned)ceil_div(N, 256), (unsigned)ceil_div(Bc, 64));
    k_upd_w_part<<<gw, 256, 0, ctx->stream>>>(Vt, ldu, N, Bc, wpart, ctx->d_status, sq);
    RBF_LAUNCHED(ctx, "k_upd_w_part");
    k_upd_w_sum<<<ceil_div(N, 256), 256, 0, ctx->stream>>>(w, wpart, N, (int32_t)gw.y,
                                                           ctx->d_status, sq);
    RBF_LAUNCHED(ctx, "k_upd_w_sum");
    return RBF_OK;
  };
  // whatever path leaves this function, `ms` ends up ordered after `as`
  struct Join {
    rbf_ctx* c;
    hipStream_t m, a;
    bool on;
    ~Join() {
      if (!on) return;
      (void)hipEventRecord(c->ev_back, a);
      (void)hipStreamWaitEvent(m, c->ev_back, 0);
    }
  } join{ctx, ms, as, two};
  if (!two) {
    for (int64_t bi = 0; bi < nb_total; ++bi) {
      int32_t Bc, Bpc;
      sizes(bi, &Bc, &Bpc);
      RBF_TRY(rows(bi));
      RBF_TRY(chain(bi));
      if (ctx->joseph)
        RBF_TRY(syrk_update_joseph(ctx, P, ldp, N, VtB[bi & 1], UtB[bi & 1], ws.LiT, ldu, Bc,
                                   Bpc, seq0 + bi));
      else
        RBF_TRY(syrk_update(ctx, P, ldp, N, VtB[bi & 1], ldu, Bc, gemm_prec, nullptr, 0,
                            seq0 + bi));
    }
  } else {
    RBF_HIP(ctx, hipEventRecord(ctx->ev_fwd, ms));
    RBF_HIP(ctx, hipStreamWaitEvent(as, ctx->ev_fwd, 0));
  }
  if (two) {
    StreamSwap sw(ctx, as);
    RBF_TRY(rows(0));
    RBF_TRY(chain(0));
    RBF_TRY(rows(1));
    RBF_HIP(ctx, hipEventRecord(ctx->ev_back, as));
  }
  for (int64_t bi = 0; two && bi < nb_total; ++bi) {
    int32_t Bc, Bpc;
    sizes(bi, &Bc, &Bpc);
    const bool more = bi + 1 < nb_total;
    RBF_HIP(ctx, hipStreamWaitEvent(ms, ctx->ev_back, 0));
    // part 1: tiles in the row/column blocks batch bi+1 touches (all tiles
    // for the last batch)
    RBF_TRY(syrk_update(ctx, P, ldp, N, VtB[bi & 1], ldu, Bc, gemm_prec,
                        more ? Fl[(bi + 1) & 1] : nullptr, more ? 1 : 0, seq0 + bi));
    if (!more) break;
    RBF_HIP(ctx, hipEventRecord(ctx->ev_fwd, ms));
    RBF_HIP(ctx, hipStreamWaitEvent(as, ctx->ev_fwd, 0));
    {
      StreamSwap sw(ctx, as);
      RBF_TRY(chain(bi + 1));
      if (bi + 2 < nb_total) RBF_TRY(rows(bi + 2));
      RBF_HIP(ctx, hipEventRecord(ctx->ev_back, as));
    }
    // part 2: the remaining tiles, concurrent with the chain above
    RBF_TRY(syrk_update(ctx, P, ldp, N, VtB[bi & 1], ldu, Bc, gemm_prec, Fl[(bi + 1) & 1], 2,
                        seq0 + bi));
  }
  return RBF_OK;
}

// After update_run: wait for the stream and report the points absorbed
// (all M, or the batches before the first failing one) and the status. An
// error recorded before this call's first launch group seq0 (a pending
// error of an earlier asynchronous call, or one outside any group) made
// every batch skip: nothing was absorbed, and that error is returned.
rbf_status update_done(rbf_ctx* ctx, int64_t M, int64_t B, int64_t seq0, int64_t* n_done) {
  int32_t h[6];
  RBF_HIP(ctx, hipMemcpyAsync(h, ctx->d_status, sizeof(h), hipMemcpyDeviceToHost,
                              ctx->stream));
  RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h[0] != 0) {
    int64_t idx;
    uint64_t key;
    memcpy(&idx, h + 2, sizeof(idx));
    memcpy(&key, h + 4, sizeof(key));
    const int64_t failed_seq = (int64_t)(SEQ_TOP - key);  // smallest failing group
    int64_t done = 0;
    if (failed_seq >= seq0) {
      done = (idx - ctx->index_base) * B;
      if (done < 0) done = 0;
    }
    *n_done = done < M ? done : M;
    return rbf_sync_status(ctx);
  }
  *n_done = M;
  return RBF_OK;
}

// ------------------------------------------------ grouped (many patches)
//
// One launch per stage over the round's jobs (blockIdx.z); a job's
// workgroups beyond its own grid return at once, the others run the body
// of the single-patch kernel with the job's arguments.

__global__ void __launch_bounds__(256) k_upd_rows_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];  // rows beyond Bp return inside the body
  upd_rows_body(J.xy, J.z, J.Bc, J.Bp, J.cxy, J.idx, nullptr, J.start, J.g, J.rk, J.kmax, J.w,
                J.vals, J.cols, J.nnz, J.Ut, J.ldu, J.N, J.status, J.index, J.seq);
}

__global__ void __launch_bounds__(GG_NT) k_gather_groups_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];
  if (!J.gH || (int32_t)blockIdx.x >= J.Bp / 64) return;
  gather_groups_body(J.vals, J.cols, J.nnz, J.Bc, J.Bp, J.kmax, J.words, J.Rcap, J.glist, J.gR,
                     J.gH, J.status, J.seq);
}

__global__ void __launch_bounds__(256) k_gather_mfma_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];
  if (!J.gH || (int64_t)blockIdx.x * 128 >= J.N || (int32_t)blockIdx.y >= J.Bp / 64) return;
  gather_mfma_body(J.P, J.ldp, J.N, J.glist, J.gR, J.gH, J.Rcap, J.Ut, J.ldu, J.status, J.seq);
}

__global__ void __launch_bounds__(256) k_upd_gather_u_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];
  if ((int64_t)blockIdx.x * 1024 >= J.N || (int32_t)blockIdx.y * 8 >= J.Bp) return;
  upd_gather_u_body(J.P, J.ldp, J.N, J.Bc, J.Bp, J.vals, J.cols, J.nnz, J.Ut, J.ldu,
                    J.gH ? J.gR : nullptr, J.status, J.seq);
}

__global__ void __launch_bounds__(256) k_upd_S_groups_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];
  const int32_t ng = J.Bp / 64;
  if (!J.gH || (int32_t)blockIdx.x >= ng * (ng + 1) / 2) return;
  upd_S_groups_body(J.glist, J.gR, J.gH, J.Rcap, J.Ut, J.ldu, J.Bc, J.Bp, J.R, J.S,
                    J.status, J.seq);
}

__global__ void __launch_bounds__(256) k_upd_S_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];
  if ((int32_t)blockIdx.x * 256 >= J.Bp || (int32_t)blockIdx.y >= J.Bp) return;
  upd_S_body(J.vals, J.cols, J.nnz, J.Ut, J.ldu, J.Bc, J.Bp, J.R, J.S, J.gH ? J.gR : nullptr,
             J.status, J.seq);
}

// L^{-1}^T starts at zero in every batch (its blocks accumulate partial sums).
__global__ void __launch_bounds__(256) k_zero_lit_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];
  const int64_t n = (int64_t)J.Bp * J.Bp;
  const int64_t e0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
  if (e0 >= n || seq_skip(J.status, J.seq)) return;
#pragma unroll
  for (int u = 0; u < 16; u += 2)
    *reinterpret_cast<double2*>(J.LiT + e0 + u) = make_double2(0.0, 0.0);
}

__global__ void __launch_bounds__(256) k_chol_first_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];
  chol_first_body(J.S, J.Bp, J.Lb, J.Linv, J.LiT, J.status, J.index, J.seq);
}

// Split form of Cholesky step kb, for launches over many factors (the
// batched form), which are bound by throughput rather than by the critical
// path of one factor. In chol_step_body every trailing tile forms L_ik and
// L_jk again from A and Linv_kk (three 64x64 products per tile, no waiting
// on the panel workgroups); here launch (a) forms each panel block L_ik
// once (into Lb), factors the next diagonal block and does the inverse's
// share of the step, and launch (b) updates the trailing tiles from the
// stored panel: one product per tile. Every element takes the same
// operations in the same order as in chol_step_body (the stored panel holds
// the same accumulator values the fused tile forms), so the factor is the
// same bit for bit.
__device__ __forceinline__ void chol_panel_body(double* __restrict__ S, int32_t Bp,
    int32_t nblk, int32_t kb, double* __restrict__ Lb, double* __restrict__ Linv,
    double* __restrict__ LiT, int32_t* __restrict__ status, int64_t batch, int64_t seq) {
  if (seq_skip(status, seq)) return;
  __shared__ double Ta[NB][LDT], Tb[NB][LDT];
  const int m = nblk - kb - 1;
  const int t = blockIdx.x;
  if (t > m) {  // the inverse's work of step kb
    linv_work(t - m - 1, kb, Bp, Lb, Linv, LiT, Ta, Tb);
    return;
  }
  const bool diag = t == m;
  const int i = diag ? kb + 1 : kb + 1 + t;
  double aii[3][4];
  if (diag) chol_diag_prefetch(S, Bp, i, aii);
  load_tile(Ta, Linv + (int64_t)kb * NB * NB, NB);
  load_tile(Tb, S + (int64_t)i * NB * Bp + (int64_t)kb * NB, Bp);
  __syncthreads();
  if (diag) {
    chol_step_diag(aii, Bp, i, Lb, Linv, LiT, Ta, Tb, status, batch, seq);
    return;
  }
  Acc64 A;
  mm_nt(Tb, Ta, A);  // L_ik = A_ik Linv_kk^T
  double* out = Lb + (int64_t)i * NB * Bp + (int64_t)kb * NB;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[(int64_t)acc_row(mi, v) * Bp + acc_col(ni)] = A.c[mi][ni][v];
}

// (b): A_ij -= L_ik L_jk^T for the trailing tiles kb < j <= i other than
// (kb + 1, kb + 1), which launch (a) factored.
__device__ __forceinline__ void chol_trail_body(double* __restrict__ S, int32_t Bp,
    int32_t nblk, int32_t kb, const double* __restrict__ Lb, const int32_t* __restrict__ status,
    int64_t seq) {
  if (seq_skip(status, seq)) return;
  __shared__ double Ta[NB][LDT], Tb[NB][LDT];
  const int u = blockIdx.x + 1;
  int ii = (int)((sqrt(8.0 * u + 1.0) - 1.0) * 0.5);
  while ((ii + 1) * (ii + 2) / 2 <= u) ++ii;
  while (ii * (ii + 1) / 2 > u) --ii;
  const int i = kb + 1 + ii;
  const int j = kb + 1 + (u - ii * (ii + 1) / 2);
  load_tile(Ta, Lb + (int64_t)i * NB * Bp + (int64_t)kb * NB, Bp);
  if (j != i) load_tile(Tb, Lb + (int64_t)j * NB * Bp + (int64_t)kb * NB, Bp);
  __syncthreads();
  Acc64 U;
  mm_nt(Ta, (j != i) ? Tb : Ta, U);  // L_ik L_jk^T
  double* Aij = S + (int64_t)i * NB * Bp + (int64_t)j * NB;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Aij[(int64_t)acc_row(mi, v) * Bp + acc_col(ni)] -= U.c[mi][ni][v];
}

// Workgroups of the split step's launches for a batch of Bp rows: (a) the
// panel tiles, the diagonal block and the inverse's share; (b) the trailing
// tiles but the first.
__host__ __device__ inline int32_t chol_panel_groups(int32_t Bp, int32_t kb) {
  const int32_t nblk = Bp / 64, m = nblk - kb - 1;
  return m <= 0 ? 0 : m + 1 + kb + kb * (nblk - 1 - kb);
}
__host__ __device__ inline int32_t chol_trail_groups(int32_t Bp, int32_t kb) {
  const int32_t nblk = Bp / 64, m = nblk - kb - 1;
  return m <= 0 ? 0 : m * (m + 1) / 2 - 1;
}

__global__ void __launch_bounds__(256, 2) k_chol_panel_g(const GJob* __restrict__ jobs,
                                                         int32_t kb) {
  const GJob& J = jobs[blockIdx.z];
  if ((int32_t)blockIdx.x >= chol_panel_groups(J.Bp, kb)) return;
  chol_panel_body(J.S, J.Bp, J.Bp / NB, kb, J.Lb, J.Linv, J.LiT, J.status, J.index, J.seq);
}

__global__ void __launch_bounds__(256, 2) k_chol_trail_g(const GJob* __restrict__ jobs,
                                                         int32_t kb) {
  const GJob& J = jobs[blockIdx.z];
  if ((int32_t)blockIdx.x >= chol_trail_groups(J.Bp, kb)) return;
  chol_trail_body(J.S, J.Bp, J.Bp / NB, kb, J.Lb, J.status, J.seq);
}

__global__ void __launch_bounds__(256, 2) k_chol_step_g(const GJob* __restrict__ jobs,
                                                        int32_t kb) {
  const GJob& J = jobs[blockIdx.z];
  if ((int32_t)blockIdx.x >= chol_step_groups(J.Bp, kb)) return;
  chol_step_body(J.S, J.Bp, J.Bp / NB, kb, J.Lb, J.Linv, J.LiT, J.status, J.index, J.seq);
}

__global__ void __launch_bounds__(256) k_linv_row_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];
  const int32_t nblk = J.Bp / NB;
  if ((int32_t)blockIdx.x >= nblk - 1) return;
  linv_row_body(J.Bp, nblk - 1, J.Lb, J.Linv, J.LiT, J.status, J.seq);
}

__global__ void __launch_bounds__(256) k_upd_w_part_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];
  if ((int32_t)blockIdx.y * 64 >= J.Bc) return;  // columns beyond N return in the body
  upd_w_part_body(J.Vt, J.ldu, J.N, J.Bc, J.wpart, J.status, J.seq);
}

__global__ void __launch_bounds__(256) k_upd_w_sum_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];
  upd_w_sum_body(J.w, J.wpart, J.N, (J.Bc + 63) / 64, J.status, J.seq);
}

rbf_status chol_grouped(rbf_ctx* ctx, const GRound& r) {
  if (r.n <= 0) return RBF_OK;
  const unsigned nz = (unsigned)r.n;
  hipStream_t s = ctx->stream;
  k_zero_lit_g<<<dim3(r.zero_x, 1, nz), 256, 0, s>>>(r.jobs);
  RBF_LAUNCHED(ctx, "k_zero_lit_g");
  k_chol_first_g<<<dim3(1, 1, nz), 256, 0, s>>>(r.jobs);
  RBF_LAUNCHED(ctx, "k_chol_first_g");
  for (int32_t kb = 0; kb < r.nsteps; ++kb) {
    // the fused step's workgroup count bounds both split launches' counts
    if (r.chol_split) {
      k_chol_panel_g<<<dim3(r.step_x[kb], 1, nz), 256, 0, s>>>(r.jobs, kb);
      RBF_LAUNCHED(ctx, "k_chol_panel_g");
      k_chol_trail_g<<<dim3(r.step_x[kb], 1, nz), 256, 0, s>>>(r.jobs, kb);
      RBF_LAUNCHED(ctx, "k_chol_trail_g");
    } else {
      k_chol_step_g<<<dim3(r.step_x[kb], 1, nz), 256, 0, s>>>(r.jobs, kb);
      RBF_LAUNCHED(ctx, "k_chol_step_g");
    }
  }
  if (r.lr_x > 0) {
    k_linv_row_g<<<dim3(r.lr_x, 1, nz), 256, 0, s>>>(r.jobs);
    RBF_LAUNCHED(ctx, "k_linv_row_g");
  }
  return RBF_OK;
}

rbf_status update_round_grouped(rbf_ctx* ctx, const GRound& r, rbf_prec prec) {
  if (r.n <= 0) return RBF_OK;
  const unsigned nz = (unsigned)r.n;
  hipStream_t s = ctx->stream;
  k_upd_rows_g<<<dim3(r.rows_x, 1, nz), 256, 0, s>>>(r.jobs);
  RBF_LAUNCHED(ctx, "k_upd_rows_g");
  if (r.gg_x > 0) {
    k_gather_groups_g<<<dim3(r.gg_x, 1, nz), GG_NT, r.gg_lds, s>>>(r.jobs);
    RBF_LAUNCHED(ctx, "k_gather_groups_g");
    k_gather_mfma_g<<<dim3(r.gm_x, r.gm_y, nz), 256, 0, s>>>(r.jobs);
    RBF_LAUNCHED(ctx, "k_gather_mfma_g");
  }
  k_upd_gather_u_g<<<dim3(r.gu_x, r.gu_y, nz), 256, 0, s>>>(r.jobs);
  RBF_LAUNCHED(ctx, "k_upd_gather_u_g");
  if (r.sg_x > 0) {
    k_upd_S_groups_g<<<dim3(r.sg_x, 1, nz), 256, 0, s>>>(r.jobs);
    RBF_LAUNCHED(ctx, "k_upd_S_groups_g");
  }
  k_upd_S_g<<<dim3(r.s_x, r.s_y, nz), 256, 0, s>>>(r.jobs);
  RBF_LAUNCHED(ctx, "k_upd_S_g");
  RBF_TRY(chol_grouped(ctx, r));
  RBF_TRY(linv_apply_grouped(ctx, r));
  k_upd_w_part_g<<<dim3(r.wp_x, r.wp_y, nz), 256, 0, s>>>(r.jobs);
  RBF_LAUNCHED(ctx, "k_upd_w_part_g");
  k_upd_w_sum_g<<<dim3(r.ws_x, 1, nz), 256, 0, s>>>(r.jobs);
  RBF_LAUNCHED(ctx, "k_upd_w_sum_g");
  return syrk_grouped(ctx, r, prec);
}

}  // namespace rbf

using namespace rbf;

extern "C" rbf_status rbf_update(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                                 double* w, double* P, int64_t ldp, const double* xy,
                                 const double* z, int64_t M, int64_t batch, rbf_prec gemm_prec,
                                 int64_t* n_done) {
  if (!ctx) return RBF_E_INVALID_ARG;
  if (n_done) *n_done = 0;
  RBF_TRY(update_check(ctx, p, g, w, P, ldp, xy, z, M, batch, gemm_prec));
  if (M == 0) return RBF_OK;
  const int64_t B = batch > 0 ? batch : UPDATE_DEFAULT_BATCH;
  const int64_t seq0 = ctx->seq;  // launch group of the first batch
  RBF_TRY(update_run(ctx, p, g, nullptr, g->N, w, P, ldp, xy, z, M, B, gemm_prec));
  if (!n_done) return RBF_OK;
  return update_done(ctx, M, B, seq0, n_done);
}
