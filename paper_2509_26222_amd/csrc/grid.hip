// Neighbour-binned center table and spatial point sort.
//
// Centers are binned on a square grid whose side h slightly exceeds the
// largest kernel support radius (cutoff * sigma_t), so every center within
// the support of a point lies in the point's 3x3 neighbourhood of bins.
// Bins are row-major, so the three bins of one neighbourhood row are
// contiguous in the sorted center array: a lookup is three contiguous runs.
#include <cfloat>
#include <cmath>

#include "internal.hpp"

namespace rbf {

__global__ void __launch_bounds__(1024) k_bbox(const double* __restrict__ c, int64_t n,
                                               double* __restrict__ out) {
  __shared__ double s[4][1024];
  double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  bool bad = false;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    double x = c[2 * i], y = c[2 * i + 1];
    if (!isfinite(x) || !isfinite(y)) bad = true;
    mnx = fmin(mnx, x);
    mny = fmin(mny, y);
    mxx = fmax(mxx, x);
    mxy = fmax(mxy, y);
  }
  s[0][threadIdx.x] = bad ? NAN : mnx;
  s[1][threadIdx.x] = mny;
  s[2][threadIdx.x] = mxx;
  s[3][threadIdx.x] = mxy;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      double a = s[0][threadIdx.x], b = s[0][threadIdx.x + off];
      s[0][threadIdx.x] = (isnan(a) || isnan(b)) ? NAN : fmin(a, b);
      s[1][threadIdx.x] = fmin(s[1][threadIdx.x], s[1][threadIdx.x + off]);
      s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + off]);
      s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = s[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_bin_keys(const double* __restrict__ xy, int64_t n,
                                                  GridGeom g, int32_t* __restrict__ keys) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int bx = bin_of(xy[2 * i], g.x0, g.inv_h, g.nbx);
  int by = bin_of(xy[2 * i + 1], g.y0, g.inv_h, g.nby);
  keys[i] = by * g.nbx + bx;
}

__global__ void __launch_bounds__(256) k_egather(const double* __restrict__ c, int64_t n,
                                                 const int32_t* __restrict__ idx,
                                                 double* __restrict__ cxy) {
  int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  int64_t i = idx[s];
  cxy[2 * s] = c[2 * i];
  cxy[2 * s + 1] = c[2 * i + 1];
}

__global__ void __launch_bounds__(256) k_grid_gather(const double* __restrict__ c, int64_t n,
                                                     const int32_t* __restrict__ idx,
                                                     int32_t* __restrict__ rank,
                                                     double* __restrict__ cxy,
                                                     float* __restrict__ cxyf) {
  int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  int64_t i = idx[s];
  rank[i] = (int32_t)s;
  double x = c[2 * i], y = c[2 * i + 1];
  cxy[2 * s] = x;
  cxy[2 * s + 1] = y;
  cxyf[2 * s] = (float)x;
  cxyf[2 * s + 1] = (float)y;
}

// Largest number of centers in any 3x3 bin neighbourhood.
__global__ void __launch_bounds__(256) k_max_cand(const int32_t* __restrict__ start, GridGeom g,
                                                  int32_t* __restrict__ out) {
  int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= (int64_t)g.nbx * g.nby) return;
  int bx = (int)(b % g.nbx), by = (int)(b / g.nbx);
  int x0 = bx > 0 ? bx - 1 : 0, x1 = bx + 1 < g.nbx ? bx + 1 : g.nbx - 1;
  int y0 = by > 0 ? by - 1 : 0, y1 = by + 1 < g.nby ? by + 1 : g.nby - 1;
  int cnt = 0;
  for (int y = y0; y <= y1; ++y) cnt += start[y * g.nbx + x1 + 1] - start[y * g.nbx + x0];
  atomicMax(out, cnt);
}

__global__ void __launch_bounds__(256) k_permute_points(const double* __restrict__ xy,
                                                        const double* __restrict__ z,
                                                        int64_t n,
                                                        const int32_t* __restrict__ perm,
                                                        double* __restrict__ xy_out,
                                                        double* __restrict__ z_out) {
  int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  int64_t i = perm[s];
  xy_out[2 * s] = xy[2 * i];
  xy_out[2 * s + 1] = xy[2 * i + 1];
  if (z) z_out[s] = z[i];
}

// Node map of the mesh form: map[n] = -1 for every node of the padded
// array, then each center claims its node. flags bit 0: a center is off the
// mesh; bit 1: two centers share a node.
__global__ void __launch_bounds__(256) k_mesh_clear(int32_t* __restrict__ map, int64_t n) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s < n) map[s] = -1;
}

struct MeshDef {
  double x0, y0, res;
  int32_t ioff, joff, nx, ny, pw;  // node i -> column i + ioff; nx, ny nodes
};

// c: the centers in bin order, idx: their original indices.
__global__ void __launch_bounds__(256) k_mesh_map(const double* __restrict__ c,
                                                  const int32_t* __restrict__ idx, int64_t n,
                                                  MeshDef m, int32_t* __restrict__ map,
                                                  int32_t* __restrict__ flags) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  const double x = c[2 * s], y = c[2 * s + 1];
  const double fi = rint((x - m.x0) / m.res), fj = rint((y - m.y0) / m.res);
  // on the mesh: within a few rounding units of the node's coordinate
  const double nx = m.x0 + fi * m.res, ny = m.y0 + fj * m.res;
  const double tx = 16.0 * DBL_EPSILON * (fabs(x) + fabs(m.x0) + fabs(fi * m.res));
  const double ty = 16.0 * DBL_EPSILON * (fabs(y) + fabs(m.y0) + fabs(fj * m.res));
  const int64_t ci = (int64_t)fi + m.ioff, cj = (int64_t)fj + m.joff;
  if (!(fabs(x - nx) <= tx && fabs(y - ny) <= ty) || ci < m.ioff || cj < m.joff ||
      ci >= (int64_t)m.ioff + m.nx || cj >= (int64_t)m.joff + m.ny) {
    atomicOr(flags, 1);
    return;
  }
  if (atomicCAS(&map[cj * m.pw + ci], -1, idx[s]) != -1) atomicOr(flags, 2);
}

}  // namespace rbf

using namespace rbf;

extern "C" {

rbf_status rbf_grid_create(rbf_ctx* ctx, const rbf_params* p, const double* centers,
                           int64_t N, rbf_grid** out) {
  if (!ctx || !p || !out) return RBF_E_INVALID_ARG;
  *out = nullptr;
  if (!centers || N <= 0 || N > (int64_t)1 << 30)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_grid_create: bad centers or N=%lld",
                (long long)N);
  if (!(p->sigma > 0) || !(p->cutoff > 0) || !(p->sigma_eps >= 0) ||
      !std::isfinite(p->sigma) || !std::isfinite(p->cutoff) || !std::isfinite(p->sigma_eps))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_grid_create: bad sigma/cutoff/sigma_eps");
  RBF_TRY(set_device(ctx));
  rbf_status st;
  double* d_box = (double*)ws_get(ctx, WS_TMP0, 4 * sizeof(double), &st);
  if (!d_box) return st;
  k_bbox<<<1, 1024, 0, ctx->stream>>>(centers, N, d_box);
  RBF_LAUNCHED(ctx, "k_bbox");
  double box[4];
  RBF_HIP(ctx, hipMemcpyAsync(box, d_box, sizeof(box), hipMemcpyDeviceToHost, ctx->stream));
  RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (!std::isfinite(box[0]) || !std::isfinite(box[1]) || !std::isfinite(box[2]) ||
      !std::isfinite(box[3]))
    return fail(ctx, RBF_E_NONFINITE, "rbf_grid_create: non-finite center coordinate");

  const double sigma_t = std::sqrt(p->sigma * p->sigma + p->sigma_eps * p->sigma_eps);
  // bin side: support radius plus a relative margin that absorbs rounding of
  // the bin index (also of FP32 coordinates)
  const double h = p->cutoff * sigma_t * (1.0 + 1e-3);
  const double x0 = box[0] - h, y0 = box[1] - h;
  const double fx = std::floor((box[2] - x0) / h) + 2.0;
  const double fy = std::floor((box[3] - y0) / h) + 2.0;
  if (fx * fy > double(1 << 26))
    return fail(ctx, RBF_E_INVALID_ARG,
                "rbf_grid_create: %.0f x %.0f bins (centers too spread for sigma)", fx, fy);
  // evaluation bins over the same origin
  const double eh = p->cutoff * p->sigma * EVAL_BIN_MARGIN / EVAL_BINS_PER_RC;
  const double efx = std::floor((box[2] - x0) / eh) + 2.0;
  const double efy = std::floor((box[3] - y0) / eh) + 2.0;
  if (efx * efy > double(1 << 26) || efx > double(1 << 14) || efy > double(1 << 14))
    return fail(ctx, RBF_E_INVALID_ARG,
                "rbf_grid_create: %.0f x %.0f evaluation bins (at most 16384 per axis and "
                "2^26 in all; centers too spread for sigma)", efx, efy);
  rbf_grid* g = new (std::nothrow) rbf_grid;
  if (!g) return RBF_E_NOMEM;
  memset(g, 0, sizeof(*g));
  g->device = ctx->device;
  g->N = N;
  g->x0 = x0;
  g->y0 = y0;
  g->h = h;
  g->inv_h = 1.0 / h;
  g->nbx = (int32_t)fx;
  g->nby = (int32_t)fy;
  for (int q = 0; q < 4; ++q) g->box[q] = box[q];
  g->sigma = p->sigma;
  g->cutoff = p->cutoff;
  g->sigma_eps = p->sigma_eps;
  g->eh = eh;
  g->inv_eh = 1.0 / eh;
  g->enbx = (int32_t)efx;
  g->enby = (int32_t)efy;
  const int64_t nbins = (int64_t)g->nbx * g->nby;
  const int64_t enbins = (int64_t)g->enbx * g->enby;
  bool ok = hipMalloc(&g->d_start, sizeof(int32_t) * (nbins + 1)) == hipSuccess &&
            hipMalloc(&g->d_idx, sizeof(int32_t) * N) == hipSuccess &&
            hipMalloc(&g->d_rank, sizeof(int32_t) * N) == hipSuccess &&
            hipMalloc(&g->d_cxy, sizeof(double) * 2 * N) == hipSuccess &&
            hipMalloc(&g->d_cxyf, sizeof(float) * 2 * N) == hipSuccess &&
            hipMalloc(&g->d_estart, sizeof(int32_t) * (enbins + 1)) == hipSuccess &&
            hipMalloc(&g->d_eidx, sizeof(int32_t) * N) == hipSuccess &&
            hipMalloc(&g->d_ecxy, sizeof(double) * 2 * N) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    rbf_grid_destroy(g);
    return fail(ctx, RBF_E_NOMEM, "rbf_grid_create: allocation failed");
  }
  int32_t* keys = (int32_t*)ws_get(ctx, WS_SORT0, sizeof(int32_t) * N, &st);
  if (!keys) {
    rbf_grid_destroy(g);
    return st;
  }
  GridGeom gg = geom(g);
  k_bin_keys<<<ceil_div(N, 256), 256, 0, ctx->stream>>>(centers, N, gg, keys);
  st = check_launch(ctx, "k_bin_keys");
  if (st == RBF_OK) st = stable_key_sort(ctx, keys, N, (int32_t)nbins, g->d_idx, g->d_start);
  if (st == RBF_OK) {
    k_grid_gather<<<ceil_div(N, 256), 256, 0, ctx->stream>>>(centers, N, g->d_idx, g->d_rank,
                                                             g->d_cxy, g->d_cxyf);
    st = check_launch(ctx, "k_grid_gather");
  }
  // the same centers in evaluation-bin order
  if (st == RBF_OK) {
    GridGeom eg;
    eg.x0 = x0;
    eg.y0 = y0;
    eg.inv_h = g->inv_eh;
    eg.nbx = g->enbx;
    eg.nby = g->enby;
    k_bin_keys<<<ceil_div(N, 256), 256, 0, ctx->stream>>>(centers, N, eg, keys);
    st = check_launch(ctx, "k_bin_keys");
  }
  if (st == RBF_OK)
    st = stable_key_sort(ctx, keys, N, (int32_t)enbins, g->d_eidx, g->d_estart);
  if (st == RBF_OK) {
    k_egather<<<ceil_div(N, 256), 256, 0, ctx->stream>>>(centers, N, g->d_eidx, g->d_ecxy);
    st = check_launch(ctx, "k_egather");
  }
  int32_t* d_mc = nullptr;
  if (st == RBF_OK) {
    d_mc = (int32_t*)ws_get(ctx, WS_TMP1, sizeof(int32_t), &st);
    if (d_mc) st = fill_zero(ctx, d_mc, sizeof(int32_t));
  }
  if (st == RBF_OK) {
    k_max_cand<<<ceil_div(nbins, 256), 256, 0, ctx->stream>>>(g->d_start, gg, d_mc);
    st = check_launch(ctx, "k_max_cand");
  }
  if (st == RBF_OK) {
    if (hipMemcpyAsync(&g->max_cand, d_mc, sizeof(int32_t), hipMemcpyDeviceToHost,
                       ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      st = fail(ctx, RBF_E_HIP, "rbf_grid_create: readback failed");
  }
  if (st != RBF_OK) {
    rbf_grid_destroy(g);
    return st;
  }
  *out = g;
  return RBF_OK;
}

rbf_status rbf_bin_centers(rbf_ctx* ctx, const double* centers, int64_t N,
                           const rbf_params* p, rbf_grid** out) {
  return rbf_grid_create(ctx, p, centers, N, out);
}

rbf_status rbf_grid_set_mesh(rbf_ctx* ctx, rbf_grid* g, double x0, double y0, double res) {
  if (!ctx || !g) return RBF_E_INVALID_ARG;
  if (g->device != ctx->device)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_grid_set_mesh: grid on another device");
  if (g->plans > 0)
    return fail(ctx, RBF_E_INVALID_ARG,
                "rbf_grid_set_mesh: %d batched plan(s) evaluate on this grid (destroy them "
                "first)", (int)g->plans);
  RBF_TRY(set_device(ctx));
  if (res == 0.0) {  // back to the binned form
    RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (g->d_mesh_map) (void)hipFree(g->d_mesh_map);
    g->d_mesh_map = nullptr;
    g->mesh_w = 0;
    return RBF_OK;
  }
  if (!(res > 0) || !std::isfinite(res) || !std::isfinite(x0) || !std::isfinite(y0))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_grid_set_mesh: bad origin or res");
  // window: the integers in [u - R - pad, u + R + pad], R = cutoff sigma / res
  const double R = g->cutoff * g->sigma / res;
  const double wn = std::floor(2.0 * (R + MESH_PAD)) + 1.0;
  const int32_t mw = wn <= 4.0 ? 4 : wn <= 8.0 ? 8 : wn <= 12.0 ? 12 : 0;
  if (!mw)
    return fail(ctx, RBF_E_INVALID_ARG,
                "rbf_grid_set_mesh: the support spans %.0f nodes per axis (at most 12)", wn);
  const double fi0 = std::rint((g->box[0] - x0) / res), fi1 = std::rint((g->box[2] - x0) / res);
  const double fj0 = std::rint((g->box[1] - y0) / res), fj1 = std::rint((g->box[3] - y0) / res);
  const double nx = fi1 - fi0 + 1.0, ny = fj1 - fj0 + 1.0;
  if (!(std::fabs(fi0) < 1e9 && std::fabs(fj0) < 1e9) || nx > MESH_MAX_NODES_AXIS ||
      ny > MESH_MAX_NODES_AXIS || (nx + 2 * mw) * (ny + 2 * mw) > double(1 << 26))
    return fail(ctx, RBF_E_INVALID_ARG,
                "rbf_grid_set_mesh: %.0f x %.0f nodes (at most 16384 per axis and 2^26 in "
                "all with the margins)", nx, ny);
  MeshDef m;
  m.x0 = x0;
  m.y0 = y0;
  m.res = res;
  m.nx = (int32_t)nx;
  m.ny = (int32_t)ny;
  m.ioff = mw - (int32_t)fi0;
  m.joff = mw - (int32_t)fj0;
  m.pw = m.nx + 2 * mw;
  const int32_t ph = m.ny + 2 * mw;
  const int64_t nodes = (int64_t)m.pw * ph;
  int32_t* map = nullptr;
  if (hipMalloc(&map, sizeof(int32_t) * nodes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, RBF_E_NOMEM, "rbf_grid_set_mesh: allocation failed");
  }
  rbf_status st;
  int32_t* flags = (int32_t*)ws_get(ctx, WS_TMP0, sizeof(int32_t), &st);
  if (flags) st = fill_zero(ctx, flags, sizeof(int32_t));
  if (st == RBF_OK) {
    k_mesh_clear<<<ceil_div(nodes, 256), 256, 0, ctx->stream>>>(map, nodes);
    st = check_launch(ctx, "k_mesh_clear");
  }
  if (st == RBF_OK) {
    k_mesh_map<<<ceil_div(g->N, 256), 256, 0, ctx->stream>>>(g->d_cxy, g->d_idx, g->N, m,
                                                               map, flags);
    st = check_launch(ctx, "k_mesh_map");
  }
  int32_t hf = 0;
  if (st == RBF_OK &&
      (hipMemcpyAsync(&hf, flags, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream) !=
           hipSuccess ||
       hipStreamSynchronize(ctx->stream) != hipSuccess))
    st = fail(ctx, RBF_E_HIP, "rbf_grid_set_mesh: readback failed");
  if (st == RBF_OK && hf)
    st = fail(ctx, RBF_E_INVALID_ARG, "rbf_grid_set_mesh: %s",
              (hf & 1) ? "a center is not a node of the mesh"
                       : "two centers lie on the same node");
  if (st != RBF_OK) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(map);
    return st;
  }
  if (g->d_mesh_map) (void)hipFree(g->d_mesh_map);
  g->d_mesh_map = map;
  g->mesh_w = mw;
  g->mx0 = x0;
  g->my0 = y0;
  g->mres = res;
  g->imin = (int32_t)fi0;
  g->jmin = (int32_t)fj0;
  g->mnx = m.nx;
  g->mny = m.ny;
  g->mpw = m.pw;
  g->mph = ph;
  return RBF_OK;
}

rbf_status rbf_grid_destroy(rbf_grid* g) {
  if (!g || g->plans > 0) return RBF_E_INVALID_ARG;  // a batched plan still evaluates on it
  (void)hipSetDevice(g->device);
  if (g->d_mesh_map) (void)hipFree(g->d_mesh_map);
  if (g->d_start) (void)hipFree(g->d_start);
  if (g->d_idx) (void)hipFree(g->d_idx);
  if (g->d_rank) (void)hipFree(g->d_rank);
  if (g->d_cxy) (void)hipFree(g->d_cxy);
  if (g->d_cxyf) (void)hipFree(g->d_cxyf);
  if (g->d_estart) (void)hipFree(g->d_estart);
  if (g->d_eidx) (void)hipFree(g->d_eidx);
  if (g->d_ecxy) (void)hipFree(g->d_ecxy);
  delete g;
  return RBF_OK;
}

rbf_status rbf_grid_info(const rbf_grid* g, int64_t* N, int32_t* nbx, int32_t* nby,
                         int32_t* max_candidates) {
  if (!g) return RBF_E_INVALID_ARG;
  if (N) *N = g->N;
  if (nbx) *nbx = g->nbx;
  if (nby) *nby = g->nby;
  if (max_candidates) *max_candidates = g->max_cand;
  return RBF_OK;
}

rbf_status rbf_sort_points(rbf_ctx* ctx, const rbf_grid* g, const double* xy, const double* z,
                           int64_t M, double* xy_out, double* z_out, int32_t* perm) {
  if (!ctx || !g) return RBF_E_INVALID_ARG;
  if (M < 0 || M >= ((int64_t)1 << 31) || (M > 0 && (!xy || !xy_out || !perm)) ||
      (z && !z_out))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_sort_points: bad arguments");
  if (g->device != ctx->device)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_sort_points: grid on another device");
  if (M == 0) return RBF_OK;
  RBF_TRY(set_device(ctx));
  rbf_status st;
  int32_t* keys = (int32_t*)ws_get(ctx, WS_SORT0, sizeof(int32_t) * M, &st);
  if (!keys) return st;
  const int64_t nbins = (int64_t)g->nbx * g->nby;
  int32_t* start = (int32_t*)ws_get(ctx, WS_SORT1, sizeof(int32_t) * (nbins + 1), &st);
  if (!start) return st;
  GridGeom gg = geom(g);
  k_bin_keys<<<ceil_div(M, 256), 256, 0, ctx->stream>>>(xy, M, gg, keys);
  RBF_LAUNCHED(ctx, "k_bin_keys");
  RBF_TRY(stable_key_sort(ctx, keys, M, (int32_t)nbins, perm, start));
  k_permute_points<<<ceil_div(M, 256), 256, 0, ctx->stream>>>(xy, z, M, perm, xy_out, z_out);
  RBF_LAUNCHED(ctx, "k_permute_points");
  return RBF_OK;
}

}  // extern "C"
