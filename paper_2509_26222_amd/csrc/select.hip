// Adaptive center selection (subsection "The RBF Approximation Model"):
// candidate nodes on a mesh over the ROI are accepted when the number of
// terrain points supporting them exceeds a threshold.
//
// The paper counts points within r_kd with a k-d tree; here the points are
// binned on the candidate mesh itself (extended by the search reach) and each
// candidate scans the cells that can hold points within r_kd. Counts are
// integers, so the result equals the brute-force count exactly; every
// floating-point decision (node position, squared distance, voxel index) is
// computed with separately rounded operations in the same order as the plain
// definition.
#include <cmath>

#include "internal.hpp"

namespace rbf {

struct Mesh {
  double x0, y0, res;
  int32_t nx, ny;
};

__device__ inline double node_x(const Mesh& m, int i) {
  return __dadd_rn(m.x0, __dmul_rn((double)i + 0.5, m.res));
}
__device__ inline double node_y(const Mesh& m, int j) {
  return __dadd_rn(m.y0, __dmul_rn((double)j + 0.5, m.res));
}

// VOXEL: count points whose mesh cell floor((p - origin)/res) is (i, j).
__global__ void __launch_bounds__(256) k_voxel_count(const double* __restrict__ xy, int64_t M,
                                                     Mesh m, int32_t* __restrict__ cnt) {
  int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= M) return;
  double fx = floor(__ddiv_rn(__dsub_rn(xy[2 * p], m.x0), m.res));
  double fy = floor(__ddiv_rn(__dsub_rn(xy[2 * p + 1], m.y0), m.res));
  if (fx >= 0.0 && fx < (double)m.nx && fy >= 0.0 && fy < (double)m.ny)
    atomicAdd(&cnt[(int64_t)fy * m.nx + (int64_t)fx], 1);
}

// RADIUS, step 1: bin key of each point on the mesh extended by `ext` cells
// on every side; points beyond the extension cannot be within r_kd of a node.
__global__ void __launch_bounds__(256) k_radius_keys(const double* __restrict__ xy, int64_t M,
                                                     Mesh m, int32_t ext, int32_t* __restrict__ key,
                                                     int32_t* __restrict__ cnt) {
  int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= M) return;
  const int ex = m.nx + 2 * ext, ey = m.ny + 2 * ext;
  double fx = floor((xy[2 * p] - m.x0) / m.res) + ext;
  double fy = floor((xy[2 * p + 1] - m.y0) / m.res) + ext;
  int32_t k = -1;
  if (fx >= 0.0 && fx < (double)ex && fy >= 0.0 && fy < (double)ey)
    k = (int32_t)fy * ex + (int32_t)fx;
  key[p] = k;
  if (k >= 0) atomicAdd(&cnt[k], 1);
}

__global__ void __launch_bounds__(256) k_radius_scatter(const double* __restrict__ xy, int64_t M,
                                                        const int32_t* __restrict__ key,
                                                        int32_t* __restrict__ cursor,
                                                        double* __restrict__ sorted) {
  int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= M) return;
  int32_t k = key[p];
  if (k < 0) return;
  int32_t pos = atomicAdd(&cursor[k], 1);
  sorted[2 * (int64_t)pos] = xy[2 * p];
  sorted[2 * (int64_t)pos + 1] = xy[2 * p + 1];
}

// RADIUS, step 2: one thread per candidate counts points with
// (gx - px)^2 + (gy - py)^2 <= r_kd^2 over the cells within `reach`.
__global__ void __launch_bounds__(256) k_radius_count(const double* __restrict__ sorted,
                                                      const int32_t* __restrict__ start, Mesh m,
                                                      int32_t ext, int32_t reach, double r2,
                                                      int32_t* __restrict__ cnt) {
  int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= (int64_t)m.nx * m.ny) return;
  const int i = (int)(c % m.nx), j = (int)(c / m.nx);
  const double gx = node_x(m, i), gy = node_y(m, j);
  const int ex = m.nx + 2 * ext, ey = m.ny + 2 * ext;
  const int ci = i + ext, cj = j + ext;
  int x0 = ci - reach < 0 ? 0 : ci - reach, x1 = ci + reach >= ex ? ex - 1 : ci + reach;
  int y0 = cj - reach < 0 ? 0 : cj - reach, y1 = cj + reach >= ey ? ey - 1 : cj + reach;
  int32_t n = 0;
  for (int y = y0; y <= y1; ++y) {
    const int s0 = start[y * ex + x0], s1 = start[y * ex + x1 + 1];
    for (int s = s0; s < s1; ++s) {
      const double dx = __dsub_rn(gx, sorted[2 * s]);
      const double dy = __dsub_rn(gy, sorted[2 * s + 1]);
      const double d2 = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
      n += (d2 <= r2);
    }
  }
  cnt[c] = n;
}

__global__ void __launch_bounds__(256) k_accept_flags(const int32_t* __restrict__ cnt,
                                                      int64_t n, int32_t thr,
                                                      int64_t* __restrict__ flag) {
  int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  flag[c] = cnt[c] > thr ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_compact_nodes(const int32_t* __restrict__ cnt,
                                                       const int64_t* __restrict__ pos, Mesh m,
                                                       int32_t thr, double* __restrict__ out,
                                                       int64_t cap) {
  int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= (int64_t)m.nx * m.ny) return;
  if (cnt[c] <= thr) return;
  int64_t k = pos[c];
  if (k >= cap) return;
  out[2 * k] = node_x(m, (int)(c % m.nx));
  out[2 * k + 1] = node_y(m, (int)(c / m.nx));
}

// Growing selection: flag[c] = 1 iff this call's points take the running
// count of node c past thr (old <= thr < old + frame).
__global__ void __launch_bounds__(256) k_grow_flags(const int32_t* __restrict__ frame,
                                                    const int32_t* __restrict__ counts,
                                                    int64_t n, int32_t thr,
                                                    int64_t* __restrict__ flag) {
  int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  const int32_t old = counts[c];
  flag[c] = (old <= thr && old + frame[c] > thr) ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_grow_commit(const int32_t* __restrict__ frame,
                                                     int32_t* __restrict__ counts, int64_t n) {
  int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c < n) counts[c] += frame[c];
}

// Nodes flagged in the exclusive scan pos (pos[c + 1] > pos[c]) written in
// mesh order.
__global__ void __launch_bounds__(256) k_compact_flagged(const int64_t* __restrict__ pos, Mesh m,
                                                         double* __restrict__ out, int64_t cap) {
  int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= (int64_t)m.nx * m.ny || pos[c + 1] == pos[c]) return;
  const int64_t k = pos[c];
  if (k >= cap) return;
  out[2 * k] = node_x(m, (int)(c % m.nx));
  out[2 * k + 1] = node_y(m, (int)(c / m.nx));
}

// Argument checks of both selection entry points; the mesh on success.
static rbf_status select_check(rbf_ctx* ctx, const char* fn, const double* xy, int64_t M,
                               const double* roi, double res, double r_kd, int32_t mode,
                               double* centers_out, int64_t cap, int64_t* n_out, Mesh* m) {
  if (!roi || !n_out || M < 0 || M >= ((int64_t)1 << 31) || (M > 0 && !xy) || cap < 0 ||
      (cap > 0 && !centers_out))
    return fail(ctx, RBF_E_INVALID_ARG, "%s: bad pointer or size", fn);
  if (mode != RBF_SELECT_RADIUS && mode != RBF_SELECT_VOXEL)
    return fail(ctx, RBF_E_INVALID_ARG, "%s: unknown mode %d", fn, mode);
  for (int q = 0; q < 4; ++q)
    if (!std::isfinite(roi[q])) return fail(ctx, RBF_E_INVALID_ARG, "%s: roi", fn);
  if (!(res > 0) || !std::isfinite(res) || (mode == RBF_SELECT_RADIUS && !(r_kd >= 0)))
    return fail(ctx, RBF_E_INVALID_ARG, "%s: res/r_kd", fn);
  const double nxd = std::ceil((roi[2] - roi[0]) / res);
  const double nyd = std::ceil((roi[3] - roi[1]) / res);
  if (!(nxd >= 1) || !(nyd >= 1) || nxd * nyd > double(1 << 28))
    return fail(ctx, RBF_E_INVALID_ARG, "%s: empty or huge mesh", fn);
  if (mode == RBF_SELECT_RADIUS && r_kd / res > 64.0)
    return fail(ctx, RBF_E_INVALID_ARG, "%s: r_kd > 64 res", fn);
  *m = Mesh{roi[0], roi[1], res, (int32_t)nxd, (int32_t)nyd};
  return RBF_OK;
}

// Support counts of the mesh nodes from the M points (this call's points
// only) into cnt (nx * ny int32, workspace).
static rbf_status count_nodes(rbf_ctx* ctx, const double* xy, int64_t M, const Mesh& m,
                              double r_kd, int32_t mode, int32_t* cnt) {
  const int64_t nc = (int64_t)m.nx * m.ny;
  rbf_status st;
  if (mode == RBF_SELECT_VOXEL) {
    RBF_TRY(fill_zero(ctx, cnt, sizeof(int32_t) * nc));
    if (M > 0) {
      k_voxel_count<<<ceil_div(M, 256), 256, 0, ctx->stream>>>(xy, M, m, cnt);
      RBF_LAUNCHED(ctx, "k_voxel_count");
    }
    return RBF_OK;
  }
  const int32_t reach = (int32_t)std::ceil(r_kd / m.res) + 1;
  const int32_t ext = reach;
  const int64_t ne = (int64_t)(m.nx + 2 * ext) * (m.ny + 2 * ext);
  int32_t* key = (int32_t*)ws_get(ctx, WS_SORT0, sizeof(int32_t) * (M > 0 ? M : 1), &st);
  if (!key) return st;
  int32_t* start = (int32_t*)ws_get(ctx, WS_SORT1, sizeof(int32_t) * (ne + 1), &st);
  if (!start) return st;
  int32_t* cursor = (int32_t*)ws_get(ctx, WS_SORT2, sizeof(int32_t) * (ne + 1), &st);
  if (!cursor) return st;
  double* sorted = (double*)ws_get(ctx, WS_TMP1, sizeof(double) * 2 * (M > 0 ? M : 1), &st);
  if (!sorted) return st;
  RBF_TRY(fill_zero(ctx, start, sizeof(int32_t) * (ne + 1)));
  if (M > 0) {
    k_radius_keys<<<ceil_div(M, 256), 256, 0, ctx->stream>>>(xy, M, m, ext, key, start);
    RBF_LAUNCHED(ctx, "k_radius_keys");
  }
  k_scan_excl_i32<<<1, 1024, 0, ctx->stream>>>(start, ne);
  RBF_LAUNCHED(ctx, "k_scan_excl_i32");
  RBF_HIP(ctx, hipMemcpyAsync(cursor, start, sizeof(int32_t) * ne, hipMemcpyDeviceToDevice,
                              ctx->stream));
  if (M > 0) {
    k_radius_scatter<<<ceil_div(M, 256), 256, 0, ctx->stream>>>(xy, M, key, cursor, sorted);
    RBF_LAUNCHED(ctx, "k_radius_scatter");
  }
  k_radius_count<<<ceil_div(nc, 256), 256, 0, ctx->stream>>>(sorted, start, m, ext, reach,
                                                             r_kd * r_kd, cnt);
  RBF_LAUNCHED(ctx, "k_radius_count");
  return RBF_OK;
}

}  // namespace rbf

using namespace rbf;

extern "C" rbf_status rbf_select_centers(rbf_ctx* ctx, const double* xy, int64_t M,
                                         const double* roi, double res, double r_kd,
                                         int32_t thr, int32_t mode, double* centers_out,
                                         int64_t cap, int64_t* n_out) {
  if (!ctx) return RBF_E_INVALID_ARG;
  Mesh m;
  RBF_TRY(select_check(ctx, "rbf_select_centers", xy, M, roi, res, r_kd, mode, centers_out, cap,
                       n_out, &m));
  *n_out = 0;
  RBF_TRY(set_device(ctx));
  const int64_t nc = (int64_t)m.nx * m.ny;
  rbf_status st;
  int32_t* cnt = (int32_t*)ws_get(ctx, WS_TMP0, sizeof(int32_t) * nc, &st);
  if (!cnt) return st;
  RBF_TRY(count_nodes(ctx, xy, M, m, r_kd, mode, cnt));
  int64_t* pos = (int64_t*)ws_get(ctx, WS_TMP3, sizeof(int64_t) * (nc + 1), &st);
  if (!pos) return st;
  k_accept_flags<<<ceil_div(nc, 256), 256, 0, ctx->stream>>>(cnt, nc, thr, pos);
  RBF_LAUNCHED(ctx, "k_accept_flags");
  k_scan_excl_i64<<<1, 1024, 0, ctx->stream>>>(pos, nc);
  RBF_LAUNCHED(ctx, "k_scan_excl_i64");
  if (cap > 0) {
    k_compact_nodes<<<ceil_div(nc, 256), 256, 0, ctx->stream>>>(cnt, pos, m, thr, centers_out,
                                                                cap);
    RBF_LAUNCHED(ctx, "k_compact_nodes");
  }
  int64_t total = 0;
  RBF_HIP(ctx, hipMemcpyAsync(&total, pos + nc, sizeof(int64_t), hipMemcpyDeviceToHost,
                              ctx->stream));
  RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *n_out = total < cap ? total : cap;
  if (total > cap)
    return fail(ctx, RBF_E_CAPACITY, "rbf_select_centers: %lld nodes accepted, cap %lld",
                (long long)total, (long long)cap);
  return RBF_OK;
}

extern "C" rbf_status rbf_select_centers_grow(rbf_ctx* ctx, const double* xy, int64_t M,
                                              const double* roi, double res, double r_kd,
                                              int32_t thr, int32_t mode, int32_t* counts,
                                              double* centers_out, int64_t cap,
                                              int64_t* n_new) {
  if (!ctx) return RBF_E_INVALID_ARG;
  Mesh m;
  RBF_TRY(select_check(ctx, "rbf_select_centers_grow", xy, M, roi, res, r_kd, mode,
                       centers_out, cap, n_new, &m));
  if (!counts) return fail(ctx, RBF_E_INVALID_ARG, "rbf_select_centers_grow: null counts");
  *n_new = 0;
  RBF_TRY(set_device(ctx));
  const int64_t nc = (int64_t)m.nx * m.ny;
  rbf_status st;
  int32_t* cnt = (int32_t*)ws_get(ctx, WS_TMP0, sizeof(int32_t) * nc, &st);
  if (!cnt) return st;
  RBF_TRY(count_nodes(ctx, xy, M, m, r_kd, mode, cnt));
  int64_t* pos = (int64_t*)ws_get(ctx, WS_TMP3, sizeof(int64_t) * (nc + 1), &st);
  if (!pos) return st;
  k_grow_flags<<<ceil_div(nc, 256), 256, 0, ctx->stream>>>(cnt, counts, nc, thr, pos);
  RBF_LAUNCHED(ctx, "k_grow_flags");
  k_scan_excl_i64<<<1, 1024, 0, ctx->stream>>>(pos, nc);
  RBF_LAUNCHED(ctx, "k_scan_excl_i64");
  int64_t total = 0;
  RBF_HIP(ctx, hipMemcpyAsync(&total, pos + nc, sizeof(int64_t), hipMemcpyDeviceToHost,
                              ctx->stream));
  RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (total > cap)  // nothing committed: the running counts stay as they were
    return fail(ctx, RBF_E_CAPACITY, "rbf_select_centers_grow: %lld new nodes, cap %lld",
                (long long)total, (long long)cap);
  if (total > 0) {
    k_compact_flagged<<<ceil_div(nc, 256), 256, 0, ctx->stream>>>(pos, m, centers_out, cap);
    RBF_LAUNCHED(ctx, "k_compact_flagged");
  }
  k_grow_commit<<<ceil_div(nc, 256), 256, 0, ctx->stream>>>(cnt, counts, nc);
  RBF_LAUNCHED(ctx, "k_grow_commit");
  *n_new = total;
  return RBF_OK;
}
