// Evaluation of the terrain model and its adjoint.
//
// f(x) = sum_j w_j phi(x, c_j) (eq. RBF_fml), grad f = -sum_j w_j phi
// (x - c_j)/sigma^2 (eq. manidolf_grad_detail with the sign of d/dx exp
// restored), the manifold residual r = xi_z - z_off - f(xi_xy) at
// xi = R p + t (eq. residual_manifold_left_wheel) and its pose Jacobian
// J = [(p x R^T g)^T, g^T], g = (-f_x, -f_y, 1) (eqs. manifold_derivative,
// manifold_grad_2, right perturbation, body-frame point).
//
// Candidates. The grid keeps the centers sorted by evaluation bins of side
// eh ~ rc/3 (rc = cutoff sigma, row-major bins), so a point's support
// circle meets at most 7 bin rows, and in each row only the bins whose x
// range meets the circle are read: one contiguous run of the sorted table
// per row. About 42 candidates per point are tested against 28 in the
// support (a 3x3 neighbourhood of bins of side rc tests about 81).
//
// Four lanes per point: each forms two of the point's (at most 8) row runs
// and the quad shares them by DPP broadcasts; in every run lane j takes
// entries j, j + 4, ..., so the quad's loads cover consecutive entries (a
// wave's gather touches 16 cache lines, not 64), two loads per lane in
// flight. The partial sums meet in a quad butterfly. The packed table holds
// (x', y', w, index) with coordinates relative to the grid origin and
// scaled by ks, so that phi = exp(-d'^2) (FP64) or exp2(-d'^2) (FP32,
// v_exp_f32): per candidate two subtractions, the squared distance, the
// exponential, the support test and three accumulations.
#include <cmath>
#include <mutex>

#include "internal.hpp"

namespace rbf {

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  using type = float4;
};
template <>
struct Vec4<double> {
  using type = double4;
};
template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
  using type = float2;
};
template <>
struct Vec2<double> {
  using type = double2;
};

// Constants of one evaluation call (see the header of this file).
template <typename T>
struct EvalK {
  T x0, y0;  // grid origin
  T ks;      // coordinate scale: phi = exp(-(ks d)^2) or exp2(-(ks d)^2)
  T rc2s;    // (ks cutoff sigma)^2: support test on the scaled squared distance
  T gscale;  // -1/(ks sigma^2): grad f = gscale * sum w phi (x' - c')
  T inv_eh;  // 1/eh: bin coordinates
  T R[9];
  T t[3];
  T z_off;
};

// Linearisation pose (R0 row-major, t0) passed by value.
struct Pose0 {
  double v[12];
};

// Evaluation-bin geometry in bin units. Row range and half-widths carry a
// pad that absorbs the FP32 rounding of the bin coordinates (the grid
// limits both bin counts to 2^14, so |u|, |v| < 2^14 and their rounding
// stays below 2^-9) and of the support test.
struct EGeom {
  float rbp;  // rb + pad: rows within this distance
  float rb2;  // (rb (1 + 1e-5))^2, rb = support radius in bins
  float pad;
  int32_t nbx, nby;
};
constexpr float EVAL_PAD = 1.0f / 64.0f;

__device__ inline double kexp_eval(double a) { return exp(a); }
__device__ inline float kexp_eval(float a) { return __builtin_amdgcn_exp2f(a); }

__device__ inline float idx_bits(int32_t i, float) { return __int_as_float(i); }
__device__ inline double idx_bits(int32_t i, double) { return (double)i; }
__device__ inline int32_t bits_idx(float v) { return __float_as_int(v); }
__device__ inline int32_t bits_idx(double v) { return (int32_t)v; }

// tab[s] = ((x - x0) ks, (y - y0) ks, w, original index) in evaluation-bin
// order.
template <typename T>
__global__ void __launch_bounds__(256) k_pack_centers(const double* __restrict__ ecxy,
                                                      const int32_t* __restrict__ eidx,
                                                      const double* __restrict__ w, int64_t n,
                                                      double x0, double y0, double ks,
                                                      typename Vec4<T>::type* __restrict__ tab) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  const int32_t i = eidx[s];
  typename Vec4<T>::type v;
  v.x = (T)((ecxy[2 * s] - x0) * ks);
  v.y = (T)((ecxy[2 * s + 1] - y0) * ks);
  v.z = (T)w[i];
  v.w = idx_bits(i, T(0));
  tab[s] = v;
}

// Mesh form: wt[n] = weight of the center on dense node n, 0 where none.
template <typename T>
__global__ void __launch_bounds__(256) k_pack_mesh(const int32_t* __restrict__ map,
                                                   const double* __restrict__ w, int64_t n,
                                                   T* __restrict__ wt) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  const int32_t c = map[s];
  wt[s] = c >= 0 ? (T)w[c] : (T)0;
}

// Lanes per point: the four lanes of a quad share a point and read
// consecutive table entries (one 64-byte segment per load instruction), so a
// wave's gather touches 16 cache lines instead of 64.
constexpr int LPP = 4;

// Value of lane SRC (0..3) of this lane's quad (DPP quad_perm broadcast).
template <int SRC>
__device__ inline int quad_bcast(int v) {
  return __builtin_amdgcn_mov_dpp(v, SRC * 0x55, 0xf, 0xf, false);
}
// Value of the lane whose quad index differs in the bits of CTRL's pattern
// (quad_perm [1,0,3,2] = 0xb1: lane ^ 1; [2,3,0,1] = 0x4e: lane ^ 2).
template <int CTRL>
__device__ inline float quad_swap(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ inline double quad_swap(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
// Value of lane SRC of this lane's quad, for a float or a double.
template <int SRC>
__device__ inline float quad_bcast_v(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), SRC * 0x55, 0xf, 0xf, false));
}
template <int SRC>
__device__ inline double quad_bcast_v(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), SRC * 0x55, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), SRC * 0x55, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <typename T>
__device__ inline T quad_bcast_any(T v, int src) {  // src known at compile time
  return src == 0 ? quad_bcast_v<0>(v)
                  : src == 1 ? quad_bcast_v<1>(v) : src == 2 ? quad_bcast_v<2>(v)
                                                             : quad_bcast_v<3>(v);
}

// Sum over the quad (butterfly over lanes ^1 and ^2; every lane gets it).
template <typename T>
__device__ inline T quad_sum(T v) {
  v += quad_swap<0xb1>(v);
  v += quad_swap<0x4e>(v);
  return v;
}

// Candidate run of one bin row of the point at bin coordinates (u, v): the
// eval-sorted entries [s0, s1) of the row's bins that the support circle
// meets, from the bin holding u - hw to the one holding u + hw (hw: the
// circle's half-width over the row, taken at the row's nearest edge less
// the pad, plus the pad); empty if the row is out of range (by > by1).
__device__ inline void row_run(float u, float v, int by, int by1, const EGeom& g,
                               const int32_t* __restrict__ estart, int& s0, int& s1) {
  const float fb = (float)by;
  const float dy = fmaxf(fmaxf(fb - v, v - fb - 1.f) - g.pad, 0.f);
  const float hw = sqrtf(fmaxf(g.rb2 - dy * dy, 0.f)) + g.pad;
  const int bx0 = max((int)floorf(u - hw), 0);
  const int bx1 = min((int)floorf(u + hw), g.nbx - 1);
  const bool valid = by <= by1 && bx0 <= bx1;
  const int row = min(by, g.nby - 1) * g.nbx;  // in range whether or not valid
  s0 = estart[valid ? row + bx0 : 0];
  s1 = valid ? estart[row + bx1 + 1] : s0;
}

// The point's candidate runs, one per bin row within the support (at most
// EVAL_MAX_ROWS = 8): lane `part` of the quad forms rows part and part + 4,
// and every lane receives all eight by quad broadcasts.
__device__ inline void quad_runs(float u, float v, int part, const EGeom& g,
                                 const int32_t* __restrict__ estart, int (&s0)[EVAL_MAX_ROWS],
                                 int (&s1)[EVAL_MAX_ROWS]) {
  static_assert(EVAL_MAX_ROWS == 2 * LPP, "two rows per lane");
  const bool ok = fabsf(u) < 16777216.f && fabsf(v) < 16777216.f;  // also NaN
  const int by0 = ok ? max((int)floorf(v - g.rbp), 0) : 0;
  const int by1 = ok ? min((int)floorf(v + g.rbp), g.nby - 1) : -1;
  int a0, a1, b0, b1;
  row_run(u, v, by0 + part, by1, g, estart, a0, a1);
  row_run(u, v, by0 + part + LPP, by1, g, estart, b0, b1);
  s0[0] = quad_bcast<0>(a0);
  s1[0] = quad_bcast<0>(a1);
  s0[1] = quad_bcast<1>(a0);
  s1[1] = quad_bcast<1>(a1);
  s0[2] = quad_bcast<2>(a0);
  s1[2] = quad_bcast<2>(a1);
  s0[3] = quad_bcast<3>(a0);
  s1[3] = quad_bcast<3>(a1);
  s0[4] = quad_bcast<0>(b0);
  s1[4] = quad_bcast<0>(b1);
  s0[5] = quad_bcast<1>(b0);
  s1[5] = quad_bcast<1>(b1);
  s0[6] = quad_bcast<2>(b0);
  s1[6] = quad_bcast<2>(b1);
  s0[7] = quad_bcast<3>(b0);
  s1[7] = quad_bcast<3>(b1);
}

// The packed table read through a buffer resource: 32-bit offsets, one
// address add per step with the second load's offset in the instruction,
// and reads past the table return zeros (a slot past a run's end needs no
// clamp; it is masked out by its index).
template <typename T>
struct TabReader {
  __amdgpu_buffer_rsrc_t r;
  __device__ TabReader(const typename Vec4<T>::type* tab, int64_t n) {
    r = __builtin_amdgcn_make_buffer_rsrc((void*)tab, (short)0,
                                          (int)(n * (int64_t)sizeof(typename Vec4<T>::type)),
                                          0x00020000);
  }
  // (x', y', w) of entry a, and its original index if IDX
  template <bool IDX>
  __device__ typename Vec4<T>::type load(int a, int off) const;
};
// (One 16-byte load; the compiler narrows it to the components used.)
template <>
template <bool IDX>
__device__ inline float4 TabReader<float>::load(int a, int off) const {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, a * 16 + off, 0, 0));
}
template <>
template <bool IDX>
__device__ inline double4 TabReader<double>::load(int a, int off) const {
  const double2 xy =
      __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, a * 32 + off, 0, 0));
  double4 c;
  c.x = xy.x;
  c.y = xy.y;
  if (IDX) {
    const double2 wi = __builtin_bit_cast(
        double2, __builtin_amdgcn_raw_buffer_load_b128(r, a * 32 + off + 16, 0, 0));
    c.z = wi.x;
    c.w = wi.y;
  } else {
    c.z = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, a * 32 + off + 16,
                                                                        0, 0));
    c.w = 0.0;
  }
  return c;
}

// Candidates per lane and step: the table loads of EU candidates (4 apart,
// the quad covering 4 EU consecutive entries) are issued together; a slot
// past the run is masked out.
template <typename T>
constexpr int eval_unroll() { return 2; }

// This lane's share of the point's candidates: in every run, the entries
// s0 + part, s0 + part + 4, ...; op(c, dx', dy', e) with e = phi, or 0
// outside the support (and for masked slots). c.w holds the original index
// only if IDX.
template <typename T, bool IDX, typename Op>
__device__ inline void for_candidates(T xs, T ys, const TabReader<T>& tab,
                                      const int (&s0)[EVAL_MAX_ROWS],
                                      const int (&s1)[EVAL_MAX_ROWS], int part, T rc2s,
                                      Op op) {
  constexpr int EU = eval_unroll<T>();
  constexpr int STEP = (int)sizeof(typename Vec4<T>::type) * LPP;  // bytes between a lane's slots
#pragma unroll
  for (int k = 0; k < EVAL_MAX_ROWS; ++k) {
    const int e = s1[k];
    for (int a = s0[k] + part; a < e; a += EU * LPP) {
      typename Vec4<T>::type c[EU];
#pragma unroll
      for (int u = 0; u < EU; ++u) c[u] = tab.template load<IDX>(a, u * STEP);
#pragma unroll
      for (int u = 0; u < EU; ++u) {
        const T dx = xs - c[u].x, dy = ys - c[u].y;
        const T d2 = dx * dx + dy * dy;
        const T e0 = kexp_eval(-d2);
        const T ph = ((u == 0 || a + u * LPP < e) && d2 <= rc2s) ? e0 : (T)0;
        op(c[u], dx, dy, ph);
      }
    }
  }
}

// Point i: world coordinates relative to the grid origin (POSE: from the
// body point p, xi = R p + t).
template <typename T>
__device__ inline void pose_apply(const EvalK<T>& k, T px, T py, T pz, T& xr, T& yr, T& zw) {
  xr = (k.R[0] * px + k.R[1] * py + k.R[2] * pz + k.t[0]) - k.x0;
  yr = (k.R[3] * px + k.R[4] * py + k.R[5] * pz + k.t[1]) - k.y0;
  zw = k.R[6] * px + k.R[7] * py + k.R[8] * pz + k.t[2];
}
template <typename T, bool POSE>
__device__ inline void point_rel(const T* __restrict__ pts, int64_t i, const EvalK<T>& k, T& xr,
                                 T& yr, T& zw, T& px, T& py, T& pz) {
  if (POSE) {
    px = pts[3 * i];
    py = pts[3 * i + 1];
    pz = pts[3 * i + 2];
    pose_apply<T>(k, px, py, pz, xr, yr, zw);
  } else {
    const typename Vec2<T>::type p = reinterpret_cast<const typename Vec2<T>::type*>(pts)[i];
    xr = p.x - k.x0;
    yr = p.y - k.y0;
    zw = px = py = pz = (T)0;
  }
}

// The pose from device memory (R row-major, then t), when given there.
template <typename T>
__device__ inline void load_pose(EvalK<T>& k, const double* __restrict__ dpose) {
  if (!dpose) return;
#pragma unroll
  for (int q = 0; q < 9; ++q) k.R[q] = (T)dpose[q];
#pragma unroll
  for (int q = 0; q < 3; ++q) k.t[q] = (T)dpose[9 + q];
}

// f, sum w phi dx', sum w phi dy' at a point (coordinates relative to the
// grid origin), summed over the quad: every lane of the quad gets them.
template <typename T>
__device__ inline void sum_point(T xr, T yr, int part, const TabReader<T>& tab,
                                 const int32_t* __restrict__ estart, const EGeom& g,
                                 const EvalK<T>& k, T& f, T& sx, T& sy) {
  int s0[EVAL_MAX_ROWS], s1[EVAL_MAX_ROWS];
  quad_runs((float)(xr * k.inv_eh), (float)(yr * k.inv_eh), part, g, estart, s0, s1);
  T f_ = 0, sx_ = 0, sy_ = 0;
  for_candidates<T, false>(xr * k.ks, yr * k.ks, tab, s0, s1, part, k.rc2s,
                    [&](const typename Vec4<T>::type& c, T dx, T dy, T e) {
                      const T we = c.z * e;
                      f_ += we;
                      sx_ += we * dx;
                      sy_ += we * dy;
                    });
  f = quad_sum(f_);
  sx = quad_sum(sx_);
  sy = quad_sum(sy_);
}

// ---- mesh form (centers on the nodes of a square mesh)
//
// With every center a node (x0 + i res, y0 + j res) the Gaussian factors
// over the axes: phi = exp(-dx'^2) exp(-dy'^2). A point's support lies in a
// window of MW x MW nodes, whose weights are read from a dense node array
// (zero where no center, and in a margin of MW nodes around the mesh, so
// that no window needs a bounds test). Lane j of the quad takes the window
// columns j, j + 4, ...: per column one exponential, per row one; per node
// the support test, one product and two accumulations. Every quad does the
// same work, and the quad's loads cover consecutive nodes.

// Node geometry of one call.
template <typename T>
struct MGeom {
  T hs;       // node spacing in scaled coordinates (res ks)
  T inv_res;  // 1/res: node coordinates of a point relative to the mesh origin
  float rp;   // support radius in nodes plus MESH_PAD
  int32_t ilo, ihi, jlo, jhi;  // range of the window's first column / row
  int32_t ioff, joff;          // dense column / row of node 0
  int32_t pw;                  // dense row length (nodes)
};

// The dense node weights through a buffer resource (reads past the array
// return zeros; the clamped windows never reach them).
template <typename T>
struct MeshReader {
  __amdgpu_buffer_rsrc_t r;
  __device__ MeshReader(const T* wt, int64_t n) {
    r = __builtin_amdgcn_make_buffer_rsrc((void*)wt, (short)0, (int)(n * (int64_t)sizeof(T)),
                                          0x00020000);
  }
  __device__ T load(int voff, int soff) const;
};
template <>
__device__ inline float MeshReader<float>::load(int voff, int soff) const {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ inline double MeshReader<double>::load(int voff, int soff) const {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// f, sum w phi dx', sum w phi dy' at a point (coordinates relative to the
// mesh origin), summed over the quad.
template <typename T, int MW>
__device__ inline void sum_point_mesh(T xr, T yr, int part, const MeshReader<T>& wt,
                                      const MGeom<T>& m, const EvalK<T>& k, T& f, T& sx,
                                      T& sy) {
  constexpr int CPL = MW / LPP;  // columns per lane
  static_assert(CPL * LPP == MW, "window of whole quads");
  const float u = (float)(xr * m.inv_res), v = (float)(yr * m.inv_res);
  const bool ok = fabsf(u) < 16777216.f && fabsf(v) < 16777216.f;  // also NaN
  const int i0 = ok ? min(max((int)ceilf(u - m.rp), m.ilo), m.ihi) : m.ilo;
  const int j0 = ok ? min(max((int)ceilf(v - m.rp), m.jlo), m.jhi) : m.jlo;
  // a point with no finite node coordinates is moved far off the mesh (no
  // node in its support, every factor exp(-d'^2) zero): f = 0, as binned
  const T xs = ok ? xr * k.ks : (T)1e18, ys = ok ? yr * k.ks : (T)1e18;
  T dx[CPL], dx2[CPL], cs[CPL], cy[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    dx[q] = xs - (T)(i0 + part + LPP * q) * m.hs;
    dx2[q] = dx[q] * dx[q];
    cs[q] = 0;
    cy[q] = 0;
  }
  // row factors: lane j forms those of rows j, j + 4, ... and the quad
  // shares them by broadcasts
  T eown[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const T dyq = ys - (T)(j0 + part + LPP * q) * m.hs;
    eown[q] = kexp_eval(-(dyq * dyq));
  }
  constexpr int SZ = (int)sizeof(T);
  const int voff = ((j0 + m.joff) * m.pw + (i0 + m.ioff + part)) * SZ;
  const int rowb = m.pw * SZ;
#pragma unroll
  for (int r = 0; r < MW; ++r) {
    const T dy = ys - (T)(j0 + r) * m.hs;
    const T dy2 = dy * dy;
    const T ey = quad_bcast_any(eown[r / LPP], r % LPP);
    const T lim = k.rc2s - dy2;  // node in the support iff dx'^2 <= lim
    T w[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) w[q] = wt.load(voff + q * LPP * SZ, r * rowb);
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const T pq = w[q] * ey;
      const T pm = dx2[q] <= lim ? pq : (T)0;
      cs[q] += pm;
      cy[q] += pm * dy;
    }
  }
  T f_ = 0, sx_ = 0, sy_ = 0;
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const T ex = kexp_eval(-dx2[q]);
    const T a = ex * cs[q];
    f_ += a;
    sx_ += a * dx[q];
    sy_ += ex * cy[q];
  }
  f = quad_sum(f_);
  sx = quad_sum(sx_);
  sy = quad_sum(sy_);
}

// Neighbour structure of a call: the binned table (MW = 0) or the dense
// node weights of the mesh form (MW = window).
template <typename T>
struct Nbr {
  const void* tab;        // packed table (n entries) or node weights (n nodes)
  int64_t n;
  const int32_t* estart;  // binned form
  EGeom eg;               // binned form
  MGeom<T> mg;            // mesh form
};

template <typename T, int MW>
__device__ inline void sum_nbr(T xr, T yr, int part, const Nbr<T>& nb, const EvalK<T>& k, T& f,
                               T& sx, T& sy) {
  if constexpr (MW == 0) {
    const TabReader<T> tab((const typename Vec4<T>::type*)nb.tab, nb.n);
    sum_point<T>(xr, yr, part, tab, nb.estart, nb.eg, k, f, sx, sy);
  } else {
    const MeshReader<T> wt((const T*)nb.tab, nb.n);
    sum_point_mesh<T, MW>(xr, yr, part, wt, nb.mg, k, f, sx, sy);
  }
}

template <typename T, bool POSE, int MW>
__global__ void __launch_bounds__(256) k_eval(const T* __restrict__ pts, int64_t Q, Nbr<T> nb,
                                              EvalK<T> k0, const double* __restrict__ dpose,
                                              T* __restrict__ f_out, T* __restrict__ grad_out,
                                              T* __restrict__ r_out, T* __restrict__ jac_out) {
  using T2 = typename Vec2<T>::type;
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPP;
  const int part = threadIdx.x % LPP;
  if (i >= Q) return;  // the lanes of a quad leave together
  EvalK<T> k = k0;
  if (POSE) load_pose(k, dpose);
  T xr, yr, zw, px, py, pz;
  point_rel<T, POSE>(pts, i, k, xr, yr, zw, px, py, pz);
  T f, sx, sy;
  sum_nbr<T, MW>(xr, yr, part, nb, k, f, sx, sy);
  const T fx = sx * k.gscale, fy = sy * k.gscale;
  // the quad's lanes share the stores
  if (part == 0) f_out[i] = f;
  if (grad_out && part == 1) {
    T2 gv;
    gv.x = fx;
    gv.y = fy;
    reinterpret_cast<T2*>(grad_out)[i] = gv;
  }
  if (POSE) {
    if (r_out && part == 2) r_out[i] = zw - k.z_off - f;
    if (jac_out && part == 3) {
      // g = (-fx, -fy, 1); q = R^T g; J_rot = p x q
      const T g0 = -fx, g1 = -fy, g2 = (T)1;
      const T q0 = k.R[0] * g0 + k.R[3] * g1 + k.R[6] * g2;
      const T q1 = k.R[1] * g0 + k.R[4] * g1 + k.R[7] * g2;
      const T q2 = k.R[2] * g0 + k.R[5] * g1 + k.R[8] * g2;
      T2* J = reinterpret_cast<T2*>(jac_out + 6 * i);  // 6 i elements: T2-aligned
      T2 j01, j23, j45;
      j01.x = py * q2 - pz * q1;
      j01.y = pz * q0 - px * q2;
      j23.x = px * q1 - py * q0;
      j23.y = g0;
      j45.x = g1;
      j45.y = g2;
      J[0] = j01;
      J[1] = j23;
      J[2] = j45;
    }
  }
}

// ---- Gauss-Newton terms of the manifold residual (fused, J not written)

constexpr int GN_TERMS = 28;  // 21 upper entries of J^T J, 6 of J^T r, r^2
constexpr int64_t GN_MAX_BLOCKS = 1536;  // six waves per SIMD of 256 CUs

// Products of the 28 terms, the quad's lanes taking 7 each: lane j of a
// quad accumulates terms 7 j .. 7 j + 6 of the list (J0J0, J0J1, ..., J0J5,
// J1J1, ..., J5J5, J0 r, ..., J5 r, r r) into v[0..6]. Every lane of the
// quad holds the point's J and r, so the lanes' shares need no exchange.
__device__ inline void gn_share(int lp, const double (&J)[6], double r, double (&v)[7]) {
  switch (lp) {
    case 0:  // J0 J0..J5, J1 J1
      v[0] += J[0] * J[0]; v[1] += J[0] * J[1]; v[2] += J[0] * J[2]; v[3] += J[0] * J[3];
      v[4] += J[0] * J[4]; v[5] += J[0] * J[5]; v[6] += J[1] * J[1];
      break;
    case 1:  // J1 J2..J5, J2 J2..J4
      v[0] += J[1] * J[2]; v[1] += J[1] * J[3]; v[2] += J[1] * J[4]; v[3] += J[1] * J[5];
      v[4] += J[2] * J[2]; v[5] += J[2] * J[3]; v[6] += J[2] * J[4];
      break;
    case 2:  // J2 J5, J3 J3..J5, J4 J4, J4 J5, J5 J5
      v[0] += J[2] * J[5]; v[1] += J[3] * J[3]; v[2] += J[3] * J[4]; v[3] += J[3] * J[5];
      v[4] += J[4] * J[4]; v[5] += J[4] * J[5]; v[6] += J[5] * J[5];
      break;
    default:  // J0..J5 r, r r
      v[0] += J[0] * r; v[1] += J[1] * r; v[2] += J[2] * r; v[3] += J[3] * r;
      v[4] += J[4] * r; v[5] += J[5] * r; v[6] += r * r;
      break;
  }
}

// Each quad takes points i, i + stride, ... (grid-stride; the launch is a
// fixed function of Q) and its lanes accumulate their shares of the points'
// 28 products in FP64 registers (gn_share). The block's sums go through
// LDS: the 64 lane values of each term (16 quads x 4 waves) are added in
// eight runs of eight by 224 threads, then the eight run sums in order by 28
// threads, into part[term][block] (term-major, gridDim.x blocks).
template <typename T, int MW>
__global__ void __launch_bounds__(256) k_eval_gn(const T* __restrict__ pts, int64_t Q, Nbr<T> nb,
                                                 EvalK<T> k, double* __restrict__ part) {
  static_assert(GN_TERMS == 7 * LPP, "seven terms per lane of a quad");
  __shared__ double lv[256 * 7];           // [thread][7]
  __shared__ double runs[GN_TERMS * 8];    // [term][run]
  const int tid = threadIdx.x;
  const int lp = tid % LPP;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * (256 / LPP);
  for (int64_t i = ((int64_t)blockIdx.x * 256 + tid) / LPP; i < Q; i += stride) {
    T xr, yr, zw, px, py, pz;
    point_rel<T, true>(pts, i, k, xr, yr, zw, px, py, pz);
    T f, sx, sy;
    sum_nbr<T, MW>(xr, yr, lp, nb, k, f, sx, sy);
    const double fx = (double)sx * (double)k.gscale, fy = (double)sy * (double)k.gscale;
    const double r = (double)zw - (double)k.z_off - (double)f;
    const double g0 = -fx, g1 = -fy, g2 = 1.0;
    const double q0 = (double)k.R[0] * g0 + (double)k.R[3] * g1 + (double)k.R[6] * g2;
    const double q1 = (double)k.R[1] * g0 + (double)k.R[4] * g1 + (double)k.R[7] * g2;
    const double q2 = (double)k.R[2] * g0 + (double)k.R[5] * g1 + (double)k.R[8] * g2;
    const double J[6] = {(double)py * q2 - (double)pz * q1, (double)pz * q0 - (double)px * q2,
                         (double)px * q1 - (double)py * q0, g0, g1, g2};
    gn_share(lp, J, r, v);
  }
#pragma unroll
  for (int q = 0; q < 7; ++q) lv[tid * 7 + q] = v[q];
  __syncthreads();
  if (tid < GN_TERMS * 8) {
    // term 7 lp + q lives in the threads of lane lp of every quad
    const int term = tid >> 3, run = tid & 7;
    const int tl = term / 7, tq = term % 7;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += lv[((run * 8 + j) * LPP + tl) * 7 + tq];
    runs[tid] = s;
  }
  __syncthreads();
  if (tid < GN_TERMS) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += runs[tid * 8 + j];
    part[(int64_t)tid * gridDim.x + blockIdx.x] = s;
  }
}

// Sum the block partials in a fixed order, one workgroup per term:
// thread t adds the partials t, t + 256, ... of its term (every load issued
// before the first add), then the 256 sums meet in a fixed tree. Writes
// J^T J (6x6, both triangles), J^T r (6) and r^T r.
constexpr int GN_SUM_T = 256;
constexpr int GN_SUM_LOADS = (int)((GN_MAX_BLOCKS + GN_SUM_T - 1) / GN_SUM_T);
__global__ void __launch_bounds__(GN_SUM_T) k_eval_gn_sum(const double* __restrict__ part,
                                                          int64_t nblocks,
                                                          double* __restrict__ JtJ,
                                                          double* __restrict__ Jtr,
                                                          double* __restrict__ rtr) {
  __shared__ double red[GN_SUM_T];
  const int t = threadIdx.x, q = blockIdx.x;
  const double* __restrict__ p = part + (int64_t)q * nblocks;
  double v[GN_SUM_LOADS];
#pragma unroll
  for (int u = 0; u < GN_SUM_LOADS; ++u) {
    const int64_t e = t + (int64_t)u * GN_SUM_T;
    v[u] = e < nblocks ? p[e] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < GN_SUM_LOADS; ++u) s += v[u];
  red[t] = s;
  __syncthreads();
#pragma unroll
  for (int o = GN_SUM_T / 2; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t != 0) return;
  s = red[0];
  if (q < 21) {
    int a = 0, rem = q;
    while (rem >= 6 - a) {
      rem -= 6 - a;
      ++a;
    }
    const int b = a + rem;
    JtJ[a * 6 + b] = s;
    JtJ[b * 6 + a] = s;
  } else if (q < 27) {
    Jtr[q - 21] = s;
  } else if (rtr) {
    *rtr = s;
  }
}

// Adjoint: L = sum_i gf_i f_i + gr_i r_i. With a_i = gf_i - gr_i:
//   dL/dw_j   = sum_i a_i phi(xi_i, c_j)            (scattered, atomics)
//   dL/dxi_i  = (a_i f_x, a_i f_y, gr_i),  dL/dp_i = R^T dL/dxi_i
//   dL/dpose  = sum_i [p_i x (R^T dL/dxi_i), dL/dxi_i]  (block-reduced)
template <typename T, bool POSE>
__global__ void __launch_bounds__(256) k_eval_adjoint(
    const T* __restrict__ pts, int64_t Q, const typename Vec4<T>::type* __restrict__ tab0,
    int64_t N, const int32_t* __restrict__ estart, EGeom g, EvalK<T> k0,
    const double* __restrict__ dpose,
    const T* __restrict__ gbar_f, const T* __restrict__ gbar_r, T* __restrict__ d_pts,
    double* __restrict__ d_w, double* __restrict__ d_pose) {
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPP;
  const int part = threadIdx.x % LPP;
  EvalK<T> k = k0;
  if (POSE) load_pose(k, dpose);
  const TabReader<T> tab(tab0, N);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  if (i < Q) {  // the lanes of a quad share this branch
    T xr, yr, zw, px, py, pz;
    point_rel<T, POSE>(pts, i, k, xr, yr, zw, px, py, pz);
    const T gf = gbar_f ? gbar_f[i] : (T)0;
    const T gr = (POSE && gbar_r) ? gbar_r[i] : (T)0;
    const T a = gf - gr;
    int s0[EVAL_MAX_ROWS], s1[EVAL_MAX_ROWS];
    quad_runs((float)(xr * k.inv_eh), (float)(yr * k.inv_eh), part, g, estart, s0, s1);
    T sx = 0, sy = 0;
    const bool scatter = d_w && a != (T)0;
    for_candidates<T, true>(xr * k.ks, yr * k.ks, tab, s0, s1, part, k.rc2s,
                            [&](const typename Vec4<T>::type& c, T dx, T dy, T e) {
                        const T we = c.z * e;
                        sx += we * dx;
                        sy += we * dy;
                        if (scatter && e != (T)0)
                          atomicAdd(&d_w[bits_idx(c.w)], (double)(a * e));
                      });
    sx = quad_sum(sx);
    sy = quad_sum(sy);
    const T fx = sx * k.gscale, fy = sy * k.gscale;
    const T dx0 = a * fx, dx1 = a * fy, dx2 = gr;
    if (POSE) {
      const T q0 = k.R[0] * dx0 + k.R[3] * dx1 + k.R[6] * dx2;
      const T q1 = k.R[1] * dx0 + k.R[4] * dx1 + k.R[7] * dx2;
      const T q2 = k.R[2] * dx0 + k.R[5] * dx1 + k.R[8] * dx2;
      if (part == 0) {  // one lane of the quad writes and adds the point
        if (d_pts) {
          d_pts[3 * i] = q0;
          d_pts[3 * i + 1] = q1;
          d_pts[3 * i + 2] = q2;
        }
        acc[0] = (double)(py * q2 - pz * q1);
        acc[1] = (double)(pz * q0 - px * q2);
        acc[2] = (double)(px * q1 - py * q0);
        acc[3] = (double)dx0;
        acc[4] = (double)dx1;
        acc[5] = (double)dx2;
      }
    } else if (d_pts && part == 0) {
      d_pts[2 * i] = dx0;
      d_pts[2 * i + 1] = dx1;
    }
  }
  if (POSE && d_pose) {
    __shared__ double red[6][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      double v = acc[c];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) red[c][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
      double v = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] +
                 red[threadIdx.x][3];
      atomicAdd(&d_pose[threadIdx.x], v);
    }
  }
}

// ---- pose increments on SO(3) x R^3 (differentiation form)
//
// R = R0 Exp(dtheta), t = t0 + dt, and the right Jacobian J_r(dtheta)
// (Exp(v + e) = Exp(v) Exp(J_r(v) e) to first order), from the closed forms
// of the exponential map of SO(3) (Rodrigues' formula):
//   Exp(v) = I + a K + b K^2,   J_r(v) = I - b K + c K^2,
//   K = [v]_x, th = |v|, a = sin th / th, b = (1 - cos th) / th^2,
//   c = (th - sin th) / th^3,
// with 1 - cos th = 2 sin^2(th/2) and Taylor series of a, b, c for small th
// (no cancellation). Out: pose[12] (R row-major, t), jr[9] row-major.
__global__ void k_pose_exp(Pose0 p0, const double* __restrict__ delta, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const double v0 = delta[0], v1 = delta[1], v2 = delta[2];
  const double t2 = v0 * v0 + v1 * v1 + v2 * v2, th = sqrt(t2);
  double a, b, c;
  if (th < 1e-2) {
    a = 1.0 - t2 / 6.0 * (1.0 - t2 / 20.0 * (1.0 - t2 / 42.0));
    b = 0.5 * (1.0 - t2 / 12.0 * (1.0 - t2 / 30.0 * (1.0 - t2 / 56.0)));
  } else {
    const double sh = sin(0.5 * th);
    a = sin(th) / th;
    b = 2.0 * sh * sh / t2;
  }
  if (th < 1e-1)
    c = (1.0 - t2 / 20.0 * (1.0 - t2 / 42.0 * (1.0 - t2 / 72.0 * (1.0 - t2 / 110.0)))) / 6.0;
  else
    c = (th - sin(th)) / (t2 * th);
  const double K[9] = {0.0, -v2, v1, v2, 0.0, -v0, -v1, v0, 0.0};
  double K2[9];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q)
      K2[3 * r + q] = K[3 * r] * K[q] + K[3 * r + 1] * K[3 + q] + K[3 * r + 2] * K[6 + q];
  double E[9];
  for (int e = 0; e < 9; ++e) {
    const double id = (e % 4 == 0) ? 1.0 : 0.0;
    E[e] = id + a * K[e] + b * K2[e];
    out[12 + e] = id - b * K[e] + c * K2[e];
  }
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q)
      out[3 * r + q] =
          p0.v[3 * r] * E[q] + p0.v[3 * r + 1] * E[3 + q] + p0.v[3 * r + 2] * E[6 + q];
  for (int q = 0; q < 3; ++q) out[9 + q] = p0.v[9 + q] + delta[3 + q];
}

// d_delta[0:3] += J_r^T g[0:3] (g: the gradient w.r.t. the right
// perturbation of R), d_delta[3:6] += g[3:6].
__global__ void k_pose_back(const double* __restrict__ jr, const double* __restrict__ gpose,
                            double* __restrict__ d_delta) {
  const int q = threadIdx.x;
  if (q < 3)
    d_delta[q] += jr[q] * gpose[0] + jr[3 + q] * gpose[1] + jr[6 + q] * gpose[2];
  else if (q < 6)
    d_delta[q] += gpose[q];
}

// ---- host side

static double coord_scale(const rbf_params* p, bool fp32) {
  // exp(-d^2/(2 sigma^2)) = exp(-(ks d)^2) with ks = 1/(sqrt(2) sigma);
  // = exp2(-(ks d)^2) with ks = sqrt(log2(e)/2)/sigma
  const double l2e = 1.4426950408889634;
  return fp32 ? std::sqrt(0.5 * l2e) / p->sigma : std::sqrt(0.5) / p->sigma;
}

// Coordinates are taken relative to the grid origin (binned form) or to
// the mesh origin (mesh form).
template <typename T>
static EvalK<T> make_consts(const rbf_params* p, const rbf_grid* g, const double* pose,
                            double z_off, bool mesh = false) {
  EvalK<T> k;
  const double ks = coord_scale(p, sizeof(T) == 4);
  const double rcs = p->cutoff * p->sigma * ks;
  k.x0 = (T)(mesh ? g->mx0 : g->x0);
  k.y0 = (T)(mesh ? g->my0 : g->y0);
  k.ks = (T)ks;
  k.rc2s = (T)(rcs * rcs);
  k.gscale = (T)(-1.0 / (ks * p->sigma * p->sigma));
  k.inv_eh = (T)g->inv_eh;
  for (int q = 0; q < 9; ++q) k.R[q] = pose ? (T)pose[q] : (T)0;
  for (int q = 0; q < 3; ++q) k.t[q] = pose ? (T)pose[9 + q] : (T)0;
  k.z_off = (T)z_off;
  return k;
}

static EGeom egeom(const rbf_params* p, const rbf_grid* g) {
  EGeom e;
  const double rb = p->cutoff * p->sigma * g->inv_eh;
  e.pad = EVAL_PAD;
  e.rbp = (float)(rb + EVAL_PAD);
  const double rbe = rb * (1.0 + 1e-5);
  e.rb2 = (float)(rbe * rbe);
  e.nbx = g->enbx;
  e.nby = g->enby;
  return e;
}

template <typename T>
static MGeom<T> mgeom(const rbf_params* p, const rbf_grid* g) {
  MGeom<T> m;
  m.hs = (T)(g->mres * coord_scale(p, sizeof(T) == 4));
  m.inv_res = (T)(1.0 / g->mres);
  m.rp = (float)(p->cutoff * p->sigma / g->mres + MESH_PAD);
  m.ilo = g->imin - g->mesh_w;
  m.ihi = g->imin + g->mnx;
  m.jlo = g->jmin - g->mesh_w;
  m.jhi = g->jmin + g->mny;
  m.ioff = g->mesh_w - g->imin;
  m.joff = g->mesh_w - g->jmin;
  m.pw = g->mpw;
  return m;
}

// Bytes of the evaluation table of grid g in precision T: the packed
// center table, or the dense node weights of the mesh form.
template <typename T>
static size_t table_bytes(const rbf_grid* g, bool mesh) {
  return mesh ? sizeof(T) * (size_t)g->mpw * (size_t)g->mph
              : sizeof(typename Vec4<T>::type) * (size_t)(g->N > 0 ? g->N : 1);
}

static rbf_status check_eval_args(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                                  const double* w, const void* pts, int64_t Q, int32_t dim,
                                  const double* pose, rbf_prec prec, const char* who) {
  if (!p || !g || !w) return fail(ctx, RBF_E_INVALID_ARG, "%s: null params/grid/w", who);
  if (Q < 0 || (Q > 0 && !pts)) return fail(ctx, RBF_E_INVALID_ARG, "%s: bad pts/Q", who);
  if (dim != 2 && dim != 3) return fail(ctx, RBF_E_INVALID_ARG, "%s: dim must be 2 or 3", who);
  if ((dim == 3) != (pose != nullptr))
    return fail(ctx, RBF_E_INVALID_ARG, "%s: pose required iff dim == 3", who);
  if (prec != RBF_F64 && prec != RBF_F32)
    return fail(ctx, RBF_E_INVALID_ARG, "%s: prec must be F64 or F32", who);
  if (!(p->sigma > 0) || !(p->cutoff > 0) || p->sigma != g->sigma || p->cutoff != g->cutoff)
    return fail(ctx, RBF_E_INVALID_ARG,
                "%s: sigma/cutoff differ from the grid's (rebuild the grid)", who);
  if (g->device != ctx->device)
    return fail(ctx, RBF_E_INVALID_ARG, "%s: grid on another device", who);
  if (g->N > ((int64_t)1 << 26))  // table offsets are 32-bit byte offsets
    return fail(ctx, RBF_E_INVALID_ARG, "%s: more than 2^26 centers", who);
  const uintptr_t two = prec == RBF_F64 ? 16 : 8;  // two elements
  if (dim == 2 && ((uintptr_t)pts % two) != 0)
    return fail(ctx, RBF_E_INVALID_ARG, "%s: xy points must be aligned to two elements", who);
  if (pose)
    for (int q = 0; q < 12; ++q)
      if (!std::isfinite(pose[q])) return fail(ctx, RBF_E_NONFINITE, "%s: non-finite pose", who);
  return RBF_OK;
}

static rbf_status check_eval_out(rbf_ctx* ctx, rbf_prec prec, const void* grad, const void* jac,
                                 const char* who) {
  const uintptr_t two = prec == RBF_F64 ? 16 : 8;
  if (((uintptr_t)grad % two) != 0 || ((uintptr_t)jac % two) != 0)
    return fail(ctx, RBF_E_INVALID_ARG, "%s: grad and jac must be aligned to two elements",
                who);
  return RBF_OK;
}

// Pack the evaluation table of grid g with weights w into tab (N entries).
template <typename T>
static rbf_status pack_into(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                            const double* w, typename Vec4<T>::type* tab) {
  k_pack_centers<T><<<ceil_div(g->N, 256), 256, 0, ctx->stream>>>(
      g->d_ecxy, g->d_eidx, w, g->N, g->x0, g->y0, coord_scale(p, sizeof(T) == 4), tab);
  RBF_LAUNCHED(ctx, "k_pack_centers");
  return RBF_OK;
}

// The same in the context's workspace.
template <typename T>
static rbf_status pack(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g, const double* w,
                       typename Vec4<T>::type** tab_out) {
  rbf_status st;
  auto* tab = (typename Vec4<T>::type*)ws_get(ctx, WS_TMP2,
                                               sizeof(typename Vec4<T>::type) * g->N, &st);
  if (!tab) return st;
  RBF_TRY(pack_into<T>(ctx, p, g, w, tab));
  *tab_out = tab;
  return RBF_OK;
}

rbf_status eval_workspace(rbf_ctx* ctx, const rbf_grid* g) {
  rbf_status st;
  size_t bytes = table_bytes<double>(g, false);
  if (g->mesh_w && table_bytes<double>(g, true) > bytes) bytes = table_bytes<double>(g, true);
  if (!ws_get(ctx, WS_TMP2, bytes, &st)) return st;
  return RBF_OK;
}

// The table of one call in `tab`: the mesh form's node weights if mesh,
// else the packed (x', y', w, index) of the eval-sorted centers.
template <typename T>
static rbf_status pack_nbr(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                           const double* w, void* tab, bool mesh, Nbr<T>* nb) {
  nb->tab = tab;
  nb->estart = g->d_estart;
  if (mesh) {
    nb->n = (int64_t)g->mpw * g->mph;
    nb->mg = mgeom<T>(p, g);
    k_pack_mesh<T><<<ceil_div(nb->n, 256), 256, 0, ctx->stream>>>(g->d_mesh_map, w, nb->n,
                                                                  (T*)tab);
    RBF_LAUNCHED(ctx, "k_pack_mesh");
  } else {
    nb->n = g->N;
    nb->eg = egeom(p, g);
    RBF_TRY(pack_into<T>(ctx, p, g, w, (typename Vec4<T>::type*)tab));
  }
  return RBF_OK;
}

template <typename T, int MW>
static void launch_eval(rbf_ctx* ctx, unsigned blocks, int32_t dim, const void* pts, int64_t Q,
                        const Nbr<T>& nb, const EvalK<T>& k, const double* dpose, void* f,
                        void* grad, void* resid, void* jac) {
  if (dim == 3)
    k_eval<T, true, MW><<<blocks, 256, 0, ctx->stream>>>((const T*)pts, Q, nb, k, dpose, (T*)f,
                                                         (T*)grad, (T*)resid, (T*)jac);
  else
    k_eval<T, false, MW><<<blocks, 256, 0, ctx->stream>>>((const T*)pts, Q, nb, k, nullptr,
                                                          (T*)f, (T*)grad, nullptr, nullptr);
}

// Evaluation: the call's table in `tab` (table_bytes<T>(g, mesh) bytes),
// then one k_eval launch.
template <typename T>
static rbf_status eval_direct(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                              const double* w, const void* pts, int64_t Q, int32_t dim,
                              const double* pose, double z_off, void* f, void* grad,
                              void* resid, void* jac, void* tab, bool mesh,
                              const double* dpose = nullptr) {
  Nbr<T> nb;
  RBF_TRY(pack_nbr<T>(ctx, p, g, w, tab, mesh, &nb));
  const EvalK<T> k = make_consts<T>(p, g, pose, z_off, mesh);
  const unsigned blocks = (unsigned)ceil_div(Q * LPP, 256);
  prof_begin(ctx, RBF_PROF_EVAL);
  switch (mesh ? g->mesh_w : 0) {
    case 0: launch_eval<T, 0>(ctx, blocks, dim, pts, Q, nb, k, dpose, f, grad, resid, jac); break;
    case 4: launch_eval<T, 4>(ctx, blocks, dim, pts, Q, nb, k, dpose, f, grad, resid, jac); break;
    case 8: launch_eval<T, 8>(ctx, blocks, dim, pts, Q, nb, k, dpose, f, grad, resid, jac); break;
    default:
      launch_eval<T, 12>(ctx, blocks, dim, pts, Q, nb, k, dpose, f, grad, resid, jac);
      break;
  }
  RBF_LAUNCHED(ctx, "k_eval");
  prof_end(ctx, RBF_PROF_EVAL);
  return RBF_OK;
}

// The call's table in the context's workspace.
template <typename T>
static rbf_status eval_ws(rbf_ctx* ctx, const rbf_grid* g, bool mesh, void** tab) {
  rbf_status st;
  *tab = ws_get(ctx, WS_TMP2, table_bytes<T>(g, mesh), &st);
  return *tab ? RBF_OK : st;
}

template <typename T>
static rbf_status eval_t(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g, const double* w,
                         const void* pts, int64_t Q, int32_t dim, const double* pose,
                         double z_off, void* f, void* grad, void* resid, void* jac,
                         const double* dpose = nullptr) {
  const bool mesh = g->mesh_w != 0;
  void* tab;
  RBF_TRY(eval_ws<T>(ctx, g, mesh, &tab));
  return eval_direct<T>(ctx, p, g, w, pts, Q, dim, pose, z_off, f, grad, resid, jac, tab, mesh,
                        dpose);
}

template <typename T>
static rbf_status gn_t(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g, const double* w,
                       const void* pts, int64_t Q, const double* pose, double z_off,
                       double* JtJ, double* Jtr, double* rtr) {
  const bool mesh = g->mesh_w != 0;
  void* tab;
  RBF_TRY(eval_ws<T>(ctx, g, mesh, &tab));
  Nbr<T> nb;
  RBF_TRY(pack_nbr<T>(ctx, p, g, w, tab, mesh, &nb));
  const EvalK<T> k = make_consts<T>(p, g, pose, z_off, mesh);
  int64_t blocks = ceil_div(Q * LPP, 256);
  if (blocks > GN_MAX_BLOCKS) blocks = GN_MAX_BLOCKS;
  rbf_status st;
  double* part = (double*)ws_get(ctx, WS_TMP3, sizeof(double) * GN_TERMS * (size_t)blocks, &st);
  if (!part) return st;
  const dim3 gr((unsigned)blocks);
  switch (mesh ? g->mesh_w : 0) {
    case 0: k_eval_gn<T, 0><<<gr, 256, 0, ctx->stream>>>((const T*)pts, Q, nb, k, part); break;
    case 4: k_eval_gn<T, 4><<<gr, 256, 0, ctx->stream>>>((const T*)pts, Q, nb, k, part); break;
    case 8: k_eval_gn<T, 8><<<gr, 256, 0, ctx->stream>>>((const T*)pts, Q, nb, k, part); break;
    default: k_eval_gn<T, 12><<<gr, 256, 0, ctx->stream>>>((const T*)pts, Q, nb, k, part); break;
  }
  RBF_LAUNCHED(ctx, "k_eval_gn");
  k_eval_gn_sum<<<GN_TERMS, GN_SUM_T, 0, ctx->stream>>>(part, blocks, JtJ, Jtr, rtr);
  RBF_LAUNCHED(ctx, "k_eval_gn_sum");
  return RBF_OK;
}

template <typename T>
static rbf_status adjoint_t(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                            const double* w, const void* pts, int64_t Q, int32_t dim,
                            const double* pose, const void* gf, const void* gr, void* d_pts,
                            double* d_w, double* d_pose, const double* dpose = nullptr) {
  typename Vec4<T>::type* tab;
  RBF_TRY(pack<T>(ctx, p, g, w, &tab));
  const EvalK<T> k = make_consts<T>(p, g, pose, 0.0);
  const EGeom eg = egeom(p, g);
  const unsigned blocks = (unsigned)ceil_div(Q * LPP, 256);
  if (dim == 3)
    k_eval_adjoint<T, true><<<blocks, 256, 0, ctx->stream>>>(
        (const T*)pts, Q, tab, g->N, g->d_estart, eg, k, dpose, (const T*)gf, (const T*)gr,
        (T*)d_pts, d_w, d_pose);
  else
    k_eval_adjoint<T, false><<<blocks, 256, 0, ctx->stream>>>(
        (const T*)pts, Q, tab, g->N, g->d_estart, eg, k, nullptr, (const T*)gf, nullptr, (T*)d_pts,
        d_w, nullptr);
  RBF_LAUNCHED(ctx, "k_eval_adjoint");
  return RBF_OK;
}

// Pose (12) and right Jacobian (9) of the increment form in the context's
// workspace, followed by 6 doubles for the pose gradient.
static rbf_status pose_at(rbf_ctx* ctx, const double* pose0, const double* delta,
                          double** out) {
  rbf_status st;
  double* buf = (double*)ws_get(ctx, WS_POSE, sizeof(double) * 32, &st);
  if (!buf) return st;
  Pose0 p0;
  for (int q = 0; q < 12; ++q) p0.v[q] = pose0[q];
  k_pose_exp<<<1, 64, 0, ctx->stream>>>(p0, delta, buf);
  RBF_LAUNCHED(ctx, "k_pose_exp");
  *out = buf;
  return RBF_OK;
}

// ---- allocation-free evaluation (rbf_eval_noalloc)
//
// The packed center table of rbf_eval_noalloc lives in this device array
// instead of the context's workspace, so that entry point allocates
// nothing. Each GPU the library runs on holds its own copy at its own
// address until the process ends. In host code the array's name is only a
// host-side stand-in, never a device address: eval_scratch_init looks the
// device address up once per device (from rbf_ctx_create, with the device
// current) and kernels receive that pointer.
static __device__ __align__(256) double4 scratch[RBF_EVAL_NOALLOC_MAX_CENTERS];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

rbf_status eval_scratch_init(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return RBF_E_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return RBF_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return RBF_E_HIP;
  }
  g_scratch_ptr[device] = ptr;
  return RBF_OK;
}

static void* eval_scratch(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace rbf

using namespace rbf;

extern "C" {

rbf_status rbf_eval_noalloc(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                            const double* w, const void* pts, int64_t Q, int32_t dim,
                            const double* pose, double z_off, rbf_prec prec, void* f,
                            void* grad, void* resid, void* jac) {
  if (!ctx) return RBF_E_INVALID_ARG;
  RBF_TRY(check_eval_args(ctx, p, g, w, pts, Q, dim, pose, prec, "rbf_eval_noalloc"));
  RBF_TRY(check_eval_out(ctx, prec, grad, jac, "rbf_eval_noalloc"));
  if (Q > 0 && !f) return fail(ctx, RBF_E_INVALID_ARG, "rbf_eval_noalloc: f is required");
  if (dim == 2 && (resid || jac))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_eval_noalloc: resid/jac need dim == 3");
  // the mesh form when its node weights fit the scratch array (else the
  // binned form, which rbf_eval would not take)
  const size_t cap = sizeof(double4) * (size_t)RBF_EVAL_NOALLOC_MAX_CENTERS;
  const bool mesh = g->mesh_w != 0 && (prec == RBF_F64 ? table_bytes<double>(g, true)
                                                       : table_bytes<float>(g, true)) <= cap;
  if (g->mesh_w && !mesh)
    return fail(ctx, RBF_E_CAPACITY,
                "rbf_eval_noalloc: the mesh's %lld nodes exceed the scratch array (use "
                "rbf_eval)", (long long)g->mpw * g->mph);
  if (!mesh && g->N > RBF_EVAL_NOALLOC_MAX_CENTERS)
    return fail(ctx, RBF_E_CAPACITY,
                "rbf_eval_noalloc: %lld centers exceed the maximum of %d (use rbf_eval)",
                (long long)g->N, (int)RBF_EVAL_NOALLOC_MAX_CENTERS);
  if (Q == 0) return RBF_OK;
  RBF_TRY(set_device(ctx));
  void* tab = eval_scratch(ctx->device);
  if (!tab)
    return fail(ctx, RBF_E_HIP, "rbf_eval_noalloc: no device address of the scratch table");
  if (prec == RBF_F64)
    return eval_direct<double>(ctx, p, g, w, pts, Q, dim, pose, z_off, f, grad, resid, jac,
                               tab, mesh);
  return eval_direct<float>(ctx, p, g, w, pts, Q, dim, pose, z_off, f, grad, resid, jac, tab,
                            mesh);
}

rbf_status rbf_eval(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g, const double* w,
                    const void* pts, int64_t Q, int32_t dim, const double* pose, double z_off,
                    rbf_prec prec, void* f, void* grad, void* resid, void* jac) {
  if (!ctx) return RBF_E_INVALID_ARG;
  RBF_TRY(check_eval_args(ctx, p, g, w, pts, Q, dim, pose, prec, "rbf_eval"));
  RBF_TRY(check_eval_out(ctx, prec, grad, jac, "rbf_eval"));
  if (Q > 0 && !f) return fail(ctx, RBF_E_INVALID_ARG, "rbf_eval: f is required");
  if (dim == 2 && (resid || jac))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_eval: resid/jac need dim == 3");
  if (Q == 0) return RBF_OK;
  RBF_TRY(set_device(ctx));
  if (prec == RBF_F64) return eval_t<double>(ctx, p, g, w, pts, Q, dim, pose, z_off, f, grad,
                                             resid, jac);
  return eval_t<float>(ctx, p, g, w, pts, Q, dim, pose, z_off, f, grad, resid, jac);
}

rbf_status rbf_eval_at(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g, const double* w,
                       const void* pts, int64_t Q, const double* pose0, const double* delta,
                       double z_off, rbf_prec prec, void* f, void* grad, void* resid,
                       void* jac) {
  if (!ctx) return RBF_E_INVALID_ARG;
  RBF_TRY(check_eval_args(ctx, p, g, w, pts, Q, 3, pose0, prec, "rbf_eval_at"));
  RBF_TRY(check_eval_out(ctx, prec, grad, jac, "rbf_eval_at"));
  if (!delta) return fail(ctx, RBF_E_INVALID_ARG, "rbf_eval_at: delta is required");
  if (Q > 0 && !f) return fail(ctx, RBF_E_INVALID_ARG, "rbf_eval_at: f is required");
  if (Q == 0) return RBF_OK;
  RBF_TRY(set_device(ctx));
  double* buf;
  RBF_TRY(pose_at(ctx, pose0, delta, &buf));
  if (prec == RBF_F64)
    return eval_t<double>(ctx, p, g, w, pts, Q, 3, pose0, z_off, f, grad, resid, jac, buf);
  return eval_t<float>(ctx, p, g, w, pts, Q, 3, pose0, z_off, f, grad, resid, jac, buf);
}

rbf_status rbf_eval_adjoint_at(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                               const double* w, const void* pts, int64_t Q, const double* pose0,
                               const double* delta, rbf_prec prec, const void* gbar_f,
                               const void* gbar_r, void* d_pts, double* d_w, double* d_delta) {
  if (!ctx) return RBF_E_INVALID_ARG;
  RBF_TRY(check_eval_args(ctx, p, g, w, pts, Q, 3, pose0, prec, "rbf_eval_adjoint_at"));
  if (!delta) return fail(ctx, RBF_E_INVALID_ARG, "rbf_eval_adjoint_at: delta is required");
  if (Q == 0) return RBF_OK;
  RBF_TRY(set_device(ctx));
  double* buf;
  RBF_TRY(pose_at(ctx, pose0, delta, &buf));
  double* gpose = d_delta ? buf + 24 : nullptr;
  if (gpose) RBF_TRY(fill_zero(ctx, gpose, 6 * sizeof(double)));
  if (prec == RBF_F64)
    RBF_TRY(adjoint_t<double>(ctx, p, g, w, pts, Q, 3, pose0, gbar_f, gbar_r, d_pts, d_w, gpose,
                              buf));
  else
    RBF_TRY(adjoint_t<float>(ctx, p, g, w, pts, Q, 3, pose0, gbar_f, gbar_r, d_pts, d_w, gpose,
                             buf));
  if (gpose) {
    k_pose_back<<<1, 64, 0, ctx->stream>>>(buf + 12, gpose, d_delta);
    RBF_LAUNCHED(ctx, "k_pose_back");
  }
  return RBF_OK;
}

rbf_status rbf_eval_gn(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g, const double* w,
                       const void* pts, int64_t Q, const double* pose, double z_off,
                       rbf_prec prec, double* JtJ, double* Jtr, double* rtr) {
  if (!ctx) return RBF_E_INVALID_ARG;
  RBF_TRY(check_eval_args(ctx, p, g, w, pts, Q, 3, pose, prec, "rbf_eval_gn"));
  if (!JtJ || !Jtr) return fail(ctx, RBF_E_INVALID_ARG, "rbf_eval_gn: JtJ and Jtr required");
  RBF_TRY(set_device(ctx));
  if (Q == 0) {
    RBF_TRY(fill_zero(ctx, JtJ, 36 * sizeof(double)));
    RBF_TRY(fill_zero(ctx, Jtr, 6 * sizeof(double)));
    if (rtr) RBF_TRY(fill_zero(ctx, rtr, sizeof(double)));
    return RBF_OK;
  }
  if (prec == RBF_F64) return gn_t<double>(ctx, p, g, w, pts, Q, pose, z_off, JtJ, Jtr, rtr);
  return gn_t<float>(ctx, p, g, w, pts, Q, pose, z_off, JtJ, Jtr, rtr);
}

rbf_status rbf_eval_adjoint(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                            const double* w, const void* pts, int64_t Q, int32_t dim,
                            const double* pose, rbf_prec prec, const void* gbar_f,
                            const void* gbar_r, void* d_pts, double* d_w, double* d_pose) {
  if (!ctx) return RBF_E_INVALID_ARG;
  RBF_TRY(check_eval_args(ctx, p, g, w, pts, Q, dim, pose, prec, "rbf_eval_adjoint"));
  if (dim == 2 && (gbar_r || d_pose))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_eval_adjoint: gbar_r/d_pose need dim == 3");
  if (Q == 0) return RBF_OK;
  RBF_TRY(set_device(ctx));
  if (prec == RBF_F64)
    return adjoint_t<double>(ctx, p, g, w, pts, Q, dim, pose, gbar_f, gbar_r, d_pts, d_w,
                             d_pose);
  return adjoint_t<float>(ctx, p, g, w, pts, Q, dim, pose, gbar_f, gbar_r, d_pts, d_w, d_pose);
}

}  // extern "C"
