// Regressor rows (ELL) and the ridge information matrix (CSR).
//
// m(x, c) = s_m exp(-d^2 / (2 sigma_t^2)) for d <= cutoff sigma_t, else 0,
// with sigma_t^2 = sigma^2 + sigma_eps^2 and s_m = sigma^2 / sigma_t^2
// (moment regressor of the ridge-regression subsection; eq. rbf_kernel is
// the matrix of these rows for one scan). calH = lambda I + sum_i m_i m_i^T
// and b = sum_i m_i z_i (eq. RBF_estimator with the ridge term).
//
// The support test d^2 <= rc^2 decides the sparsity pattern, so it is done
// with separately rounded products (no fused multiply-add) to be exactly the
// plain definition's decision.
#include <cmath>

#include "internal.hpp"

namespace rbf {

struct RegK {
  double rc2;    // (cutoff sigma_t)^2
  double den;    // 2 sigma_t^2, formed as (2 sigma_t) sigma_t
  double scale;  // s_m
};

static RegK reg_consts(const rbf_params* p) {
  RegK k;
  const double st = std::sqrt(p->sigma * p->sigma + p->sigma_eps * p->sigma_eps);
  const double rc = p->cutoff * st;
  k.rc2 = rc * rc;
  k.den = 2.0 * st * st;
  k.scale = (p->sigma * p->sigma) / (st * st);
  return k;
}

__device__ inline double sq_d(double px, double py, double cx, double cy) {
  const double dx = __dsub_rn(px, cx), dy = __dsub_rn(py, cy);
  return __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
}

__device__ inline double reg_val(double d2, const RegK& k) {
  return k.scale * exp(-d2 / k.den);
}

// ---------------------------------------------------------------- ELL rows

// Sixteen lanes per point: the lanes test the candidates of a bin row 16 at
// a time, and a ballot with a popcount prefix gives each hit its slot in
// candidate order (the order of a serial scan); the row's padding is then
// written 16 slots at a time. The 16 lanes of a point share its loop bounds,
// so they stay together through every ballot.
template <typename T>
__global__ void __launch_bounds__(256) k_assemble_phi(const double* __restrict__ xy, int64_t M,
                                                      const double* __restrict__ cxy,
                                                      const int32_t* __restrict__ idx,
                                                      const int32_t* __restrict__ start,
                                                      GridGeom g, RegK k, int32_t kmax,
                                                      T* __restrict__ vals,
                                                      int32_t* __restrict__ cols,
                                                      int32_t* __restrict__ nnz,
                                                      int32_t* __restrict__ status) {
  const int tid = threadIdx.x, l = tid & 15, gshift = tid & 48;
  const int64_t i = (int64_t)blockIdx.x * 16 + (tid >> 4);
  if (i >= M) return;  // whole groups of 16 lanes leave together
  const double x = xy[2 * i], y = xy[2 * i + 1];
  T* vrow = vals + i * kmax;
  int32_t* crow = cols + i * kmax;
  int n = 0;
  int bx0, bx1, by0, by1;
  if (bin_range(x, g.x0, g.inv_h, g.nbx, &bx0, &bx1) &&
      bin_range(y, g.y0, g.inv_h, g.nby, &by0, &by1)) {
    for (int by = by0; by <= by1; ++by) {
      const int row = by * g.nbx;
      const int s0 = start[row + bx0], s1 = start[row + bx1 + 1];
      for (int base = s0; base < s1; base += 16) {
        const int s = base + l;
        double d2 = 0.0;
        bool ok = false;
        if (s < s1) {
          d2 = sq_d(x, y, cxy[2 * s], cxy[2 * s + 1]);
          ok = d2 <= k.rc2;
        }
        const uint32_t gm = (uint32_t)(__ballot(ok) >> gshift) & 0xFFFFu;
        const int pos = n + __popc(gm & ((1u << l) - 1u));
        if (ok && pos < kmax) {
          vrow[pos] = (T)reg_val(d2, k);
          crow[pos] = idx[s];
        }
        n += __popc(gm);
      }
    }
  }
  if (l == 0 && n > kmax) set_status(status, RBF_E_CAPACITY, i);
  const int w = n < kmax ? n : kmax;
  for (int q = w + l; q < kmax; q += 16) {
    vrow[q] = (T)0;
    crow[q] = 0;
  }
  if (l == 0) nnz[i] = w;
}

// ---------------------------------------------------------- Gram pattern

// Row of center j: centers within 2 cutoff sigma_t, found in the 5x5 bins
// around j (bin side > cutoff sigma_t). count pass then fill pass.
__global__ void __launch_bounds__(256) k_gram_count(const double* __restrict__ cxy, int64_t N,
                                                    const int32_t* __restrict__ idx,
                                                    const int32_t* __restrict__ start, GridGeom g,
                                                    double r2, int64_t* __restrict__ rowcnt) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= N) return;
  const double x = cxy[2 * s], y = cxy[2 * s + 1];
  const int bx = bin_of(x, g.x0, g.inv_h, g.nbx), by = bin_of(y, g.y0, g.inv_h, g.nby);
  int64_t n = 0;
  for (int yy = (by > 1 ? by - 2 : 0); yy <= (by + 2 < g.nby ? by + 2 : g.nby - 1); ++yy) {
    const int row = yy * g.nbx;
    const int s0 = start[row + (bx > 1 ? bx - 2 : 0)];
    const int s1 = start[row + (bx + 2 < g.nbx ? bx + 2 : g.nbx - 1) + 1];
    for (int t = s0; t < s1; ++t) n += sq_d(x, y, cxy[2 * t], cxy[2 * t + 1]) <= r2;
  }
  rowcnt[idx[s]] = n;
}

__global__ void __launch_bounds__(256) k_gram_fill(const double* __restrict__ cxy, int64_t N,
                                                   const int32_t* __restrict__ idx,
                                                   const int32_t* __restrict__ start, GridGeom g,
                                                   double r2, const int64_t* __restrict__ rowptr,
                                                   int32_t* __restrict__ colidx, int64_t cap) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= N) return;
  const int64_t j = idx[s];
  const int64_t a = rowptr[j], e = rowptr[j + 1];
  if (e > cap) return;  // capacity error reported by the host
  const double x = cxy[2 * s], y = cxy[2 * s + 1];
  const int bx = bin_of(x, g.x0, g.inv_h, g.nbx), by = bin_of(y, g.y0, g.inv_h, g.nby);
  int64_t n = a;
  for (int yy = (by > 1 ? by - 2 : 0); yy <= (by + 2 < g.nby ? by + 2 : g.nby - 1); ++yy) {
    const int row = yy * g.nbx;
    const int s0 = start[row + (bx > 1 ? bx - 2 : 0)];
    const int s1 = start[row + (bx + 2 < g.nbx ? bx + 2 : g.nbx - 1) + 1];
    for (int t = s0; t < s1; ++t) {
      if (sq_d(x, y, cxy[2 * t], cxy[2 * t + 1]) <= r2 && n < e) {
        // insertion into the ascending run colidx[a, n)
        const int32_t c = idx[t];
        int64_t q = n;
        while (q > a && colidx[q - 1] > c) {
          colidx[q] = colidx[q - 1];
          --q;
        }
        colidx[q] = c;
        ++n;
      }
    }
  }
}

// ------------------------------------------------------------ Gram values

// One wavefront per row j. The points within the support of c_j are read as
// three contiguous runs of the bin-sorted point table (uniform across the
// wave); lane e handles row entry e (center c_k) and accumulates
// m(x_i, c_j) m(x_i, c_k) in point order, so the sums are deterministic.
__global__ void __launch_bounds__(256) k_gram_values(
    const double* __restrict__ cxy, const int32_t* __restrict__ rank, int64_t N,
    const int32_t* __restrict__ idx, const double* __restrict__ pxy,
    const double* __restrict__ pz, const int32_t* __restrict__ pstart, GridGeom g, RegK k,
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colidx, double lambda,
    double* __restrict__ vals, double* __restrict__ b) {
  const int lane = threadIdx.x & 63;
  const int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= N) return;
  const int64_t j = idx[s];
  const double cjx = cxy[2 * s], cjy = cxy[2 * s + 1];
  const int bx = bin_of(cjx, g.x0, g.inv_h, g.nbx), by = bin_of(cjy, g.y0, g.inv_h, g.nby);
  const int bx0 = bx > 0 ? bx - 1 : 0, bx1 = bx + 1 < g.nbx ? bx + 1 : g.nbx - 1;
  const int by0 = by > 0 ? by - 1 : 0, by1 = by + 1 < g.nby ? by + 1 : g.nby - 1;
  const int64_t a = rowptr[j], e = rowptr[j + 1];
  double bj = 0.0;
  for (int64_t base = a; base < e; base += 64) {
    const int64_t ent = base + lane;
    const bool act = ent < e;
    int32_t kk = act ? colidx[ent] : (int32_t)j;
    const int64_t sk = rank[kk];
    const double ckx = cxy[2 * sk], cky = cxy[2 * sk + 1];
    double acc = 0.0;
    for (int yy = by0; yy <= by1; ++yy) {
      const int row = yy * g.nbx;
      const int p0 = pstart[row + bx0], p1 = pstart[row + bx1 + 1];
      for (int p = p0; p < p1; ++p) {
        const double px = pxy[2 * p], py = pxy[2 * p + 1];
        const double dj = sq_d(px, py, cjx, cjy);
        if (dj <= k.rc2) {  // uniform across the wave
          const double mj = reg_val(dj, k);
          if (base == a) bj += mj * pz[p];
          const double dk = sq_d(px, py, ckx, cky);
          if (dk <= k.rc2) acc += mj * reg_val(dk, k);
        }
      }
    }
    if (act) {
      if (kk == j) acc += lambda;
      vals[ent] += acc;
    }
  }
  if (lane == 0) b[j] += bj;
}

}  // namespace rbf

using namespace rbf;

static rbf_status check_grid(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                             const char* who) {
  if (!p || !g) return fail(ctx, RBF_E_INVALID_ARG, "%s: null params or grid", who);
  if (g->device != ctx->device)
    return fail(ctx, RBF_E_INVALID_ARG, "%s: grid on another device", who);
  if (p->sigma != g->sigma || p->cutoff != g->cutoff || p->sigma_eps != g->sigma_eps)
    return fail(ctx, RBF_E_INVALID_ARG, "%s: params differ from the grid's", who);
  return RBF_OK;
}

extern "C" {

rbf_status rbf_assemble_phi(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                            const double* xy, int64_t M, rbf_prec prec, void* vals,
                            int32_t* cols, int32_t* nnz, int32_t kmax) {
  if (!ctx) return RBF_E_INVALID_ARG;
  RBF_TRY(check_grid(ctx, p, g, "rbf_assemble_phi"));
  if (M < 0 || kmax <= 0 || (M > 0 && (!xy || !vals || !cols || !nnz)))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_assemble_phi: bad pointer, M or kmax");
  if (prec != RBF_F64 && prec != RBF_F32)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_assemble_phi: prec must be F64 or F32");
  if (M == 0) return RBF_OK;
  RBF_TRY(set_device(ctx));
  RegK k = reg_consts(p);
  if (prec == RBF_F64)
    k_assemble_phi<double><<<ceil_div(M, 16), 256, 0, ctx->stream>>>(
        xy, M, g->d_cxy, g->d_idx, g->d_start, geom(g), k, kmax, (double*)vals, cols, nnz,
        ctx->d_status);
  else
    k_assemble_phi<float><<<ceil_div(M, 16), 256, 0, ctx->stream>>>(
        xy, M, g->d_cxy, g->d_idx, g->d_start, geom(g), k, kmax, (float*)vals, cols, nnz,
        ctx->d_status);
  RBF_LAUNCHED(ctx, "k_assemble_phi");
  return RBF_OK;
}

rbf_status rbf_gram_pattern(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                            int64_t* rowptr, int32_t* colidx, int64_t cap, int64_t* nnz_out) {
  if (!ctx) return RBF_E_INVALID_ARG;
  RBF_TRY(check_grid(ctx, p, g, "rbf_gram_pattern"));
  if (!rowptr || !nnz_out || cap < 0 || (cap > 0 && !colidx))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_gram_pattern: bad pointer or cap");
  RBF_TRY(set_device(ctx));
  const double st = std::sqrt(p->sigma * p->sigma + p->sigma_eps * p->sigma_eps);
  const double r = 2.0 * p->cutoff * st;
  const int64_t N = g->N;
  k_gram_count<<<ceil_div(N, 256), 256, 0, ctx->stream>>>(g->d_cxy, N, g->d_idx, g->d_start,
                                                          geom(g), r * r, rowptr);
  RBF_LAUNCHED(ctx, "k_gram_count");
  k_scan_excl_i64<<<1, 1024, 0, ctx->stream>>>(rowptr, N);
  RBF_LAUNCHED(ctx, "k_scan_excl_i64");
  if (cap > 0) {
    k_gram_fill<<<ceil_div(N, 256), 256, 0, ctx->stream>>>(g->d_cxy, N, g->d_idx, g->d_start,
                                                           geom(g), r * r, rowptr, colidx, cap);
    RBF_LAUNCHED(ctx, "k_gram_fill");
  }
  int64_t nnz = 0;
  RBF_HIP(ctx, hipMemcpyAsync(&nnz, rowptr + N, sizeof(int64_t), hipMemcpyDeviceToHost,
                              ctx->stream));
  RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *nnz_out = nnz;
  if (nnz > cap)
    return fail(ctx, RBF_E_CAPACITY, "rbf_gram_pattern: nnz %lld > cap %lld",
                (long long)nnz, (long long)cap);
  return RBF_OK;
}

rbf_status rbf_assemble_gram(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                             const double* xy, const double* z, int64_t M,
                             const int64_t* rowptr, const int32_t* colidx, double* vals,
                             double* b, int32_t add_lambda) {
  if (!ctx) return RBF_E_INVALID_ARG;
  RBF_TRY(check_grid(ctx, p, g, "rbf_assemble_gram"));
  if (M < 0 || M >= ((int64_t)1 << 31) || !rowptr || !colidx || !vals || !b ||
      (M > 0 && (!xy || !z)))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_assemble_gram: bad pointer or M");
  if (add_lambda && !(p->lambda >= 0))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_assemble_gram: lambda < 0");
  RBF_TRY(set_device(ctx));
  rbf_status st;
  const int64_t nbins = (int64_t)g->nbx * g->nby;
  const int64_t Mc = M > 0 ? M : 1;
  int32_t* keys = (int32_t*)ws_get(ctx, WS_SORT0, sizeof(int32_t) * Mc, &st);
  if (!keys) return st;
  int32_t* pstart = (int32_t*)ws_get(ctx, WS_SORT1, sizeof(int32_t) * (nbins + 1), &st);
  if (!pstart) return st;
  int32_t* perm = (int32_t*)ws_get(ctx, WS_TMP0, sizeof(int32_t) * Mc, &st);
  if (!perm) return st;
  double* pxy = (double*)ws_get(ctx, WS_TMP1, sizeof(double) * 2 * Mc, &st);
  if (!pxy) return st;
  double* pz = (double*)ws_get(ctx, WS_TMP3, sizeof(double) * Mc, &st);
  if (!pz) return st;
  RBF_TRY(rbf_sort_points(ctx, g, xy, z, M, pxy, pz, perm));
  if (M == 0) {
    // only the ridge term
    RBF_TRY(fill_zero(ctx, pstart, sizeof(int32_t) * (nbins + 1)));
  } else {
    // rbf_sort_points leaves the bin offsets of the sorted points in WS_SORT1
  }
  RegK k = reg_consts(p);
  const int64_t N = g->N;
  k_gram_values<<<ceil_div(N, 4), 256, 0, ctx->stream>>>(
      g->d_cxy, g->d_rank, N, g->d_idx, pxy, pz, pstart, geom(g), k, rowptr, colidx,
      add_lambda ? p->lambda : 0.0, vals, b);
  RBF_LAUNCHED(ctx, "k_gram_values");
  return RBF_OK;
}

rbf_status rbf_assemble(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g, const double* xy,
                        const double* z, int64_t M, int32_t what, rbf_prec prec, void* phi_val,
                        int32_t* phi_col, int32_t* phi_nnz, int32_t kmax, rbf_csr* H, double* b,
                        int32_t add_lambda) {
  if (!ctx) return RBF_E_INVALID_ARG;
  if (what == 0 || (what & ~(RBF_ASSEMBLE_PHI | RBF_ASSEMBLE_GRAM)) != 0)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_assemble: what must be PHI and/or GRAM");
  if ((what & RBF_ASSEMBLE_GRAM) != 0) {
    if (prec != RBF_F64)
      return fail(ctx, RBF_E_INVALID_ARG, "rbf_assemble: the Gram matrix is FP64 only");
    if (!H || !g || H->n != g->N)
      return fail(ctx, RBF_E_INVALID_ARG, "rbf_assemble: H missing or H->n != N");
  }
  if ((what & RBF_ASSEMBLE_PHI) != 0)
    RBF_TRY(rbf_assemble_phi(ctx, p, g, xy, M, prec, phi_val, phi_col, phi_nnz, kmax));
  if ((what & RBF_ASSEMBLE_GRAM) != 0)
    RBF_TRY(rbf_assemble_gram(ctx, p, g, xy, z, M, H->rowptr, H->colidx, H->vals, b,
                              add_lambda));
  return RBF_OK;
}

}  // extern "C"
