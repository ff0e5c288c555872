// Evaluation of the terrain model and its adjoint.
//
// f(x) = sum_j w_j phi(x, c_j) (eq. RBF_fml), grad f = -sum_j w_j phi
// (x - c_j)/sigma^2 (eq. manidolf_grad_detail with the sign of d/dx exp
// restored), the manifold residual r = xi_z - z_off - f(xi_xy) at
// xi = R p + t (eq. residual_manifold_left_wheel) and its pose Jacobian
// J = [(p x R^T g)^T, g^T], g = (-f_x, -f_y, 1) (eqs. manifold_derivative,
// manifold_grad_2, right perturbation, body-frame point).
//
// A point's candidates are the centers of its 3x3 bin neighbourhood: three
// contiguous runs of a packed, bin-sorted table (x, y, w) that stays
// resident in L2. The forward kernel gives each point four lanes that take
// every fourth candidate and combine their partial sums with lane shuffles;
// outputs are written in point order. A binned mode (per context, off by
// default) groups the points by bin with a counting sort and gives each bin
// a workgroup that stages the bin's candidates in LDS once; on points in
// arbitrary order its sort atomics and scattered output writes cost more
// than the table reads they save. The adjoint keeps one lane per point.
#include <cmath>

#include "internal.hpp"

#ifndef EVAL_EU32
#define EVAL_EU32 4
#endif
#ifndef EVAL_EU64
#define EVAL_EU64 1
#endif

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
struct EvalK {
  T rc2;     // (cutoff sigma)^2
  T kexp;    // f64: -1/(2 sigma^2); f32: -log2(e)/(2 sigma^2) for exp2
  T inv_s2;  // 1/sigma^2
  T R[9];
  T t[3];
  T z_off;
};

__device__ inline double kexp_eval(double a) { return exp(a); }
__device__ inline float kexp_eval(float a) { return __builtin_amdgcn_exp2f(a); }

template <typename T>
__global__ void __launch_bounds__(256) k_pack_centers(const T* __restrict__ cxy,
                                                      const int32_t* __restrict__ idx,
                                                      const double* __restrict__ w, int64_t n,
                                                      typename Vec4<T>::type* __restrict__ tab) {
  int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  typename Vec4<T>::type v;
  v.x = cxy[2 * s];
  v.y = cxy[2 * s + 1];
  v.z = (T)w[idx[s]];
  v.w = (T)0;
  tab[s] = v;
}

// Accumulate f, sum w phi dx, sum w phi dy over the 3x3 neighbourhood of
// (x, y), taking every LPP-th candidate starting at `part` (the lanes of one
// point split the candidates; their sums are combined by the caller).
constexpr int LPP = 4;  // lanes per point
// candidates per lane and pass: 4 in FP32 (29.4 -> 24.7 us for 200k points;
// 8 is no faster); FP64 lanes, with the software exp, gain nothing from
// more than one (the registers cost occupancy)
template <typename T>
constexpr int eval_unroll() { return sizeof(T) == 4 ? EVAL_EU32 : EVAL_EU64; }

template <typename T>
__device__ inline void accumulate(T x, T y, const typename Vec4<T>::type* __restrict__ tab,
                                  const int32_t* __restrict__ start, const GridGeom& g,
                                  const EvalK<T>& k, int part, T& f, T& sx, T& sy) {
  f = sx = sy = (T)0;
  int bx0, bx1, by0, by1;
  if (!bin_range((double)x, g.x0, g.inv_h, g.nbx, &bx0, &bx1)) return;
  if (!bin_range((double)y, g.y0, g.inv_h, g.nby, &by0, &by1)) return;
  for (int by = by0; by <= by1; ++by) {
    const int row = by * g.nbx;
    const int s0 = start[row + bx0], s1 = start[row + bx1 + 1];
    // EU candidates per pass with their table loads issued together (the
    // table is read from L2 in an order set by the points, so one load at a
    // time left each lane waiting on every one); a slot past the run reads
    // the run's last entry (s1 - 1 >= s0 whenever the pass runs) and is
    // masked out. Candidates are summed in the same order as one by one.
    constexpr int EU = eval_unroll<T>();
    for (int s = s0 + part; s < s1; s += EU * LPP) {
      typename Vec4<T>::type c[EU];
      bool in[EU];
#pragma unroll
      for (int u = 0; u < EU; ++u) {
        const int su = s + u * LPP;
        in[u] = su < s1;
        c[u] = tab[in[u] ? su : s1 - 1];
      }
#pragma unroll
      for (int u = 0; u < EU; ++u) {
        const T dx = x - c[u].x, dy = y - c[u].y;
        const T d2 = dx * dx + dy * dy;
        if (in[u] && d2 <= k.rc2) {
          const T we = c[u].z * kexp_eval(d2 * k.kexp);
          f += we;
          sx += we * dx;
          sy += we * dy;
        }
      }
    }
  }
}

// World coordinates of point i (POSE: xi = R p + t from the body point p).
template <typename T, bool POSE>
__device__ inline void world_of(const T* __restrict__ pts, int64_t i, const EvalK<T>& k, T& x,
                                T& y, T& zw, T& px, T& py, T& pz) {
  if (POSE) {
    px = pts[3 * i];
    py = pts[3 * i + 1];
    pz = pts[3 * i + 2];
    x = k.R[0] * px + k.R[1] * py + k.R[2] * pz + k.t[0];
    y = k.R[3] * px + k.R[4] * py + k.R[5] * pz + k.t[1];
    zw = k.R[6] * px + k.R[7] * py + k.R[8] * pz + k.t[2];
  } else {
    x = pts[2 * i];
    y = pts[2 * i + 1];
    zw = px = py = pz = (T)0;
  }
}

// Combine the LPP lanes' partial sums and write point i's outputs (the
// lanes of a point share the stores).
template <typename T, bool POSE>
__device__ inline void finish_point(int64_t i, int part, T f, T sx, T sy, T zw, T px, T py, T pz,
                                    const EvalK<T>& k, T* __restrict__ f_out,
                                    T* __restrict__ grad_out, T* __restrict__ r_out,
                                    T* __restrict__ jac_out) {
#pragma unroll
  for (int m = 1; m < LPP; m <<= 1) {
    f += __shfl_xor(f, m, 64);
    sx += __shfl_xor(sx, m, 64);
    sy += __shfl_xor(sy, m, 64);
  }
  const T fx = -sx * k.inv_s2, fy = -sy * k.inv_s2;
  if (part == 0) f_out[i] = f;
  if (grad_out && part == 1) {
    grad_out[2 * i] = fx;
    grad_out[2 * i + 1] = fy;
  }
  if (POSE) {
    if (r_out && part == 2) r_out[i] = zw - k.z_off - f;
    if (jac_out && part == 3) {
      // g = (-fx, -fy, 1); q = R^T g; J_rot = p x q
      const T g0 = -fx, g1 = -fy, g2 = (T)1;
      const T q0 = k.R[0] * g0 + k.R[3] * g1 + k.R[6] * g2;
      const T q1 = k.R[1] * g0 + k.R[4] * g1 + k.R[7] * g2;
      const T q2 = k.R[2] * g0 + k.R[5] * g1 + k.R[8] * g2;
      T* J = jac_out + 6 * i;
      J[0] = py * q2 - pz * q1;
      J[1] = pz * q0 - px * q2;
      J[2] = px * q1 - py * q0;
      J[3] = g0;
      J[4] = g1;
      J[5] = g2;
    }
  }
}

template <typename T, bool POSE>
__global__ void __launch_bounds__(256) k_eval(const T* __restrict__ pts, int64_t Q,
                                              const typename Vec4<T>::type* __restrict__ tab,
                                              const int32_t* __restrict__ start, GridGeom g,
                                              EvalK<T> k, T* __restrict__ f_out,
                                              T* __restrict__ grad_out, T* __restrict__ r_out,
                                              T* __restrict__ jac_out) {
  // LPP lanes per point: they share the point, split its candidates and
  // combine the partial sums with lane shuffles
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPP;
  const int part = threadIdx.x % LPP;
  if (i >= Q) return;  // the LPP lanes of a point exit together
  T x, y, zw, px, py, pz;
  world_of<T, POSE>(pts, i, k, x, y, zw, px, py, pz);
  T f, sx, sy;
  accumulate<T>(x, y, tab, start, g, k, part, f, sx, sy);
  finish_point<T, POSE>(i, part, f, sx, sy, zw, px, py, pz, k, f_out, grad_out, r_out, jac_out);
}

// ---- Gauss-Newton terms of the manifold residual (fused, J not written)

constexpr int GN_TERMS = 28;  // 21 upper entries of J^T J, 6 of J^T r, r^2

// Per point (pose form): r and J as in k_eval, in FP64 from here on; the
// block's sums of the 28 products go to part[block][28] (wave shuffles,
// then the four waves in order).
template <typename T>
__global__ void __launch_bounds__(256) k_eval_gn(const T* __restrict__ pts, int64_t Q,
                                                 const typename Vec4<T>::type* __restrict__ tab,
                                                 const int32_t* __restrict__ start, GridGeom g,
                                                 EvalK<T> k, double* __restrict__ part) {
  __shared__ double wsum[4][GN_TERMS];
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPP;
  const int lp = threadIdx.x % LPP, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double v[GN_TERMS];
#pragma unroll
  for (int q = 0; q < GN_TERMS; ++q) v[q] = 0.0;
  if (i < Q) {  // the LPP lanes of a point share this branch
    T x, y, zw, px, py, pz;
    world_of<T, true>(pts, i, k, x, y, zw, px, py, pz);
    T f, sx, sy;
    accumulate<T>(x, y, tab, start, g, k, lp, f, sx, sy);
#pragma unroll
    for (int m = 1; m < LPP; m <<= 1) {
      f += __shfl_xor(f, m, 64);
      sx += __shfl_xor(sx, m, 64);
      sy += __shfl_xor(sy, m, 64);
    }
    if (lp == 0) {
      const double fx = -(double)sx * (double)k.inv_s2, fy = -(double)sy * (double)k.inv_s2;
      const double r = (double)zw - (double)k.z_off - (double)f;
      const double g0 = -fx, g1 = -fy, g2 = 1.0;
      const double q0 = (double)k.R[0] * g0 + (double)k.R[3] * g1 + (double)k.R[6] * g2;
      const double q1 = (double)k.R[1] * g0 + (double)k.R[4] * g1 + (double)k.R[7] * g2;
      const double q2 = (double)k.R[2] * g0 + (double)k.R[5] * g1 + (double)k.R[8] * g2;
      const double J[6] = {(double)py * q2 - (double)pz * q1, (double)pz * q0 - (double)px * q2,
                           (double)px * q1 - (double)py * q0, g0, g1, g2};
      int q = 0;
#pragma unroll
      for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = a; b < 6; ++b) v[q++] = J[a] * J[b];
#pragma unroll
      for (int a = 0; a < 6; ++a) v[21 + a] = J[a] * r;
      v[27] = r * r;
    }
  }
#pragma unroll
  for (int q = 0; q < GN_TERMS; ++q) {
    double t = v[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) wsum[wave][q] = t;
  }
  __syncthreads();
  if (threadIdx.x < GN_TERMS) {
    const int q = threadIdx.x;
    part[(int64_t)blockIdx.x * GN_TERMS + q] =
        (wsum[0][q] + wsum[1][q]) + (wsum[2][q] + wsum[3][q]);
  }
}

// Sum the block partials in a fixed order (lane l of term q takes blocks
// l, l+32, ...; the 32 lane sums meet in a fixed shuffle tree); write
// J^T J (6x6, both triangles), J^T r (6) and r^T r.
__global__ void __launch_bounds__(1024) k_eval_gn_sum(const double* __restrict__ part,
                                                      int64_t nblocks, double* __restrict__ JtJ,
                                                      double* __restrict__ Jtr,
                                                      double* __restrict__ rtr) {
  const int q = threadIdx.x >> 5, l = threadIdx.x & 31;
  if (q >= GN_TERMS) return;  // whole groups of 32 leave together
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t b = l;
  for (; b + 96 < nblocks; b += 128) {
    s0 += part[b * GN_TERMS + q];
    s1 += part[(b + 32) * GN_TERMS + q];
    s2 += part[(b + 64) * GN_TERMS + q];
    s3 += part[(b + 96) * GN_TERMS + q];
  }
  for (; b < nblocks; b += 32) s0 += part[b * GN_TERMS + q];
  double s = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
  if (l != 0) return;
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

// ---- binned evaluation

// Bin key of each point (the far bucket nbins if its 3x3 neighbourhood
// misses the grid, non-finite coordinates included) and the bin counts.
// A point just outside the grid takes the clamped bin: that bin's
// neighbourhood contains the point's own (clipped) neighbourhood, and the
// extra centers lie beyond the bin side, which exceeds the cutoff.
template <typename T, bool POSE>
__global__ void __launch_bounds__(256) k_eval_keys(const T* __restrict__ pts, int64_t Q,
                                                   GridGeom g, EvalK<T> k, int32_t nbins,
                                                   int32_t* __restrict__ keys,
                                                   int32_t* __restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= Q) return;
  T x, y, zw, px, py, pz;
  world_of<T, POSE>(pts, i, k, x, y, zw, px, py, pz);
  int key = nbins, lo, hi;
  if (bin_range((double)x, g.x0, g.inv_h, g.nbx, &lo, &hi) &&
      bin_range((double)y, g.y0, g.inv_h, g.nby, &lo, &hi))
    key = bin_of((double)x, g.x0, g.inv_h, g.nbx) +
          g.nbx * bin_of((double)y, g.y0, g.inv_h, g.nby);
  keys[i] = key;
  atomicAdd(&counts[key], 1);
}

// perm[start[key] + rank] = i, rank taken from a per-bin cursor.
__global__ void __launch_bounds__(256) k_eval_scatter(const int32_t* __restrict__ keys,
                                                      int64_t Q,
                                                      const int32_t* __restrict__ start,
                                                      int32_t* __restrict__ cursor,
                                                      int32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= Q) return;
  const int key = keys[i];
  perm[start[key] + atomicAdd(&cursor[key], 1)] = (int32_t)i;
}

// One workgroup per bin (the last one for the far bucket): the bin's 3x3
// neighbourhood (at most maxc centers) is staged in LDS, then its points
// are evaluated LPP lanes each.
template <typename T, bool POSE>
__global__ void __launch_bounds__(256) k_eval_tiles(
    const T* __restrict__ pts, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ pstart, int32_t nbins,
    const typename Vec4<T>::type* __restrict__ tab, const int32_t* __restrict__ cstart,
    GridGeom g, EvalK<T> k, T* __restrict__ f_out, T* __restrict__ grad_out,
    T* __restrict__ r_out, T* __restrict__ jac_out) {
  using V = typename Vec4<T>::type;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  V* cand = reinterpret_cast<V*>(smem);
  const int b = blockIdx.x, tid = threadIdx.x;
  const int p0 = pstart[b], p1 = pstart[b + 1];
  if (p0 == p1) return;
  int nc = 0;
  if (b < nbins) {
    const int by = b / g.nbx, bx = b - by * g.nbx;
    const int bx0 = bx > 0 ? bx - 1 : 0, bx1 = bx + 1 < g.nbx ? bx + 1 : g.nbx - 1;
    const int by0 = by > 0 ? by - 1 : 0, by1 = by + 1 < g.nby ? by + 1 : g.nby - 1;
    for (int r = by0; r <= by1; ++r) {
      const int s0 = cstart[r * g.nbx + bx0], s1 = cstart[r * g.nbx + bx1 + 1];
      for (int s = s0 + tid; s < s1; s += 256) cand[nc + (s - s0)] = tab[s];
      nc += s1 - s0;
    }
  }
  __syncthreads();
  const int part = tid % LPP;
  for (int base = p0; base < p1; base += 256 / LPP) {
    const int pi = base + tid / LPP;
    if (pi >= p1) break;  // the LPP lanes of a point leave together
    const int64_t i = perm[pi];
    T x, y, zw, px, py, pz;
    world_of<T, POSE>(pts, i, k, x, y, zw, px, py, pz);
    T f = (T)0, sx = (T)0, sy = (T)0;
    for (int s = part; s < nc; s += LPP) {
      const V c = cand[s];
      const T dx = x - c.x, dy = y - c.y;
      const T d2 = dx * dx + dy * dy;
      if (d2 <= k.rc2) {
        const T we = c.z * kexp_eval(d2 * k.kexp);
        f += we;
        sx += we * dx;
        sy += we * dy;
      }
    }
    finish_point<T, POSE>(i, part, f, sx, sy, zw, px, py, pz, k, f_out, grad_out, r_out,
                          jac_out);
  }
}

// Adjoint: L = sum_i gf_i f_i + gr_i r_i. With a_i = gf_i - gr_i:
//   dL/dw_j   = sum_i a_i phi(xi_i, c_j)            (scattered, atomics)
//   dL/dxi_i  = (a_i f_x, a_i f_y, gr_i),  dL/dp_i = R^T dL/dxi_i
//   dL/dpose  = sum_i [p_i x (R^T dL/dxi_i), dL/dxi_i]  (block-reduced)
template <typename T, bool POSE>
__global__ void __launch_bounds__(256) k_eval_adjoint(
    const T* __restrict__ pts, int64_t Q, const typename Vec4<T>::type* __restrict__ tab,
    const int32_t* __restrict__ idx, const int32_t* __restrict__ start, GridGeom g,
    EvalK<T> k, const T* __restrict__ gbar_f, const T* __restrict__ gbar_r,
    T* __restrict__ d_pts, double* __restrict__ d_w, double* __restrict__ d_pose) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  if (i < Q) {
    T x, y, px = 0, py = 0, pz = 0;
    if (POSE) {
      px = pts[3 * i];
      py = pts[3 * i + 1];
      pz = pts[3 * i + 2];
      x = k.R[0] * px + k.R[1] * py + k.R[2] * pz + k.t[0];
      y = k.R[3] * px + k.R[4] * py + k.R[5] * pz + k.t[1];
    } else {
      x = pts[2 * i];
      y = pts[2 * i + 1];
    }
    const T gf = gbar_f ? gbar_f[i] : (T)0;
    const T gr = (POSE && gbar_r) ? gbar_r[i] : (T)0;
    const T a = gf - gr;
    T sx = 0, sy = 0;
    int bx0, bx1, by0, by1;
    if (bin_range((double)x, g.x0, g.inv_h, g.nbx, &bx0, &bx1) &&
        bin_range((double)y, g.y0, g.inv_h, g.nby, &by0, &by1)) {
      for (int by = by0; by <= by1; ++by) {
        const int row = by * g.nbx;
        const int s0 = start[row + bx0], s1 = start[row + bx1 + 1];
        for (int s = s0; s < s1; ++s) {
          const typename Vec4<T>::type c = tab[s];
          const T dx = x - c.x, dy = y - c.y;
          const T d2 = dx * dx + dy * dy;
          if (d2 <= k.rc2) {
            const T e = kexp_eval(d2 * k.kexp);
            const T we = c.z * e;
            sx += we * dx;
            sy += we * dy;
            if (d_w && a != (T)0) atomicAdd(&d_w[idx[s]], (double)(a * e));
          }
        }
      }
    }
    const T fx = -sx * k.inv_s2, fy = -sy * k.inv_s2;
    const T dx0 = a * fx, dx1 = a * fy, dx2 = gr;
    if (POSE) {
      const T q0 = k.R[0] * dx0 + k.R[3] * dx1 + k.R[6] * dx2;
      const T q1 = k.R[1] * dx0 + k.R[4] * dx1 + k.R[7] * dx2;
      const T q2 = k.R[2] * dx0 + k.R[5] * dx1 + k.R[8] * dx2;
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
    } else if (d_pts) {
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

template <typename T>
static EvalK<T> make_consts(const rbf_params* p, const double* pose, double z_off) {
  EvalK<T> k;
  const double rc = p->cutoff * p->sigma;
  k.rc2 = (T)(rc * rc);
  const double inv2s2 = 1.0 / (2.0 * p->sigma * p->sigma);
  if (sizeof(T) == 8)
    k.kexp = (T)(-inv2s2);
  else
    k.kexp = (T)(-inv2s2 * 1.4426950408889634);  // log2(e)
  k.inv_s2 = (T)(1.0 / (p->sigma * p->sigma));
  for (int q = 0; q < 9; ++q) k.R[q] = pose ? (T)pose[q] : (T)0;
  for (int q = 0; q < 3; ++q) k.t[q] = pose ? (T)pose[9 + q] : (T)0;
  k.z_off = (T)z_off;
  return k;
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
  if (pose)
    for (int q = 0; q < 12; ++q)
      if (!std::isfinite(pose[q])) return fail(ctx, RBF_E_NONFINITE, "%s: non-finite pose", who);
  return RBF_OK;
}

template <typename T>
static rbf_status pack(rbf_ctx* ctx, const rbf_grid* g, const double* w,
                       typename Vec4<T>::type** tab_out) {
  rbf_status st;
  auto* tab = (typename Vec4<T>::type*)ws_get(ctx, WS_TMP2,
                                               sizeof(typename Vec4<T>::type) * g->N, &st);
  if (!tab) return st;
  const T* cxy = sizeof(T) == 8 ? (const T*)g->d_cxy : (const T*)g->d_cxyf;
  k_pack_centers<T><<<ceil_div(g->N, 256), 256, 0, ctx->stream>>>(cxy, g->d_idx, w, g->N, tab);
  RBF_LAUNCHED(ctx, "k_pack_centers");
  *tab_out = tab;
  return RBF_OK;
}

rbf_status eval_workspace(rbf_ctx* ctx, const rbf_grid* g, int64_t Q, EvalWs* ws) {
  rbf_status st;
  const int64_t nb = (int64_t)g->nbx * g->nby + 2;
  ws->keys = (int32_t*)ws_get(ctx, WS_SORT0, sizeof(int32_t) * (size_t)(Q > 0 ? Q : 1), &st);
  if (!ws->keys) return st;
  ws->perm = (int32_t*)ws_get(ctx, WS_SORT1, sizeof(int32_t) * (size_t)(Q > 0 ? Q : 1), &st);
  if (!ws->perm) return st;
  ws->counts = (int32_t*)ws_get(ctx, WS_SORT2, sizeof(int32_t) * 2 * (size_t)nb, &st);
  if (!ws->counts) return st;
  ws->cursor = ws->counts + nb;
  if (!ws_get(ctx, WS_TMP2, sizeof(double4) * (size_t)(g->N > 0 ? g->N : 1), &st)) return st;
  return RBF_OK;
}

template <typename T>
static rbf_status eval_t(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g, const double* w,
                         const void* pts, int64_t Q, int32_t dim, const double* pose,
                         double z_off, void* f, void* grad, void* resid, void* jac) {
  typename Vec4<T>::type* tab;
  RBF_TRY(pack<T>(ctx, g, w, &tab));
  EvalK<T> k = make_consts<T>(p, pose, z_off);
  const size_t lds = sizeof(typename Vec4<T>::type) * (size_t)(g->max_cand > 0 ? g->max_cand : 1);
  if (ctx->eval_binned && Q >= EVAL_BINNED_MIN && lds <= EVAL_LDS_MAX && Q < INT32_MAX) {
    const int32_t nbins = g->nbx * g->nby;
    EvalWs ws;
    RBF_TRY(eval_workspace(ctx, g, Q, &ws));
    RBF_TRY(fill_zero(ctx, ws.counts, sizeof(int32_t) * 2 * (size_t)(nbins + 2)));
    const unsigned gq = (unsigned)ceil_div(Q, 256);
    prof_begin(ctx, RBF_PROF_EVAL);
    if (dim == 3)
      k_eval_keys<T, true><<<gq, 256, 0, ctx->stream>>>((const T*)pts, Q, geom(g), k, nbins,
                                                         ws.keys, ws.counts);
    else
      k_eval_keys<T, false><<<gq, 256, 0, ctx->stream>>>((const T*)pts, Q, geom(g), k, nbins,
                                                          ws.keys, ws.counts);
    RBF_LAUNCHED(ctx, "k_eval_keys");
    k_scan_excl_i32<<<1, 1024, 0, ctx->stream>>>(ws.counts, nbins + 1);
    RBF_LAUNCHED(ctx, "k_scan_excl_i32");
    k_eval_scatter<<<gq, 256, 0, ctx->stream>>>(ws.keys, Q, ws.counts, ws.cursor, ws.perm);
    RBF_LAUNCHED(ctx, "k_eval_scatter");
    if (dim == 3)
      k_eval_tiles<T, true><<<nbins + 1, 256, lds, ctx->stream>>>(
          (const T*)pts, ws.perm, ws.counts, nbins, tab, g->d_start, geom(g), k, (T*)f,
          (T*)grad, (T*)resid, (T*)jac);
    else
      k_eval_tiles<T, false><<<nbins + 1, 256, lds, ctx->stream>>>(
          (const T*)pts, ws.perm, ws.counts, nbins, tab, g->d_start, geom(g), k, (T*)f,
          (T*)grad, nullptr, nullptr);
    RBF_LAUNCHED(ctx, "k_eval_tiles");
    prof_end(ctx, RBF_PROF_EVAL);
    return RBF_OK;
  }
  const int64_t blocks = ceil_div(Q * LPP, 256);
  prof_begin(ctx, RBF_PROF_EVAL);
  if (dim == 3)
    k_eval<T, true><<<blocks, 256, 0, ctx->stream>>>((const T*)pts, Q, tab, g->d_start, geom(g),
                                                     k, (T*)f, (T*)grad, (T*)resid, (T*)jac);
  else
    k_eval<T, false><<<blocks, 256, 0, ctx->stream>>>((const T*)pts, Q, tab, g->d_start,
                                                      geom(g), k, (T*)f, (T*)grad, nullptr,
                                                      nullptr);
  RBF_LAUNCHED(ctx, "k_eval");
  prof_end(ctx, RBF_PROF_EVAL);
  return RBF_OK;
}

template <typename T>
static rbf_status gn_t(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g, const double* w,
                       const void* pts, int64_t Q, const double* pose, double z_off,
                       double* JtJ, double* Jtr, double* rtr) {
  typename Vec4<T>::type* tab;
  RBF_TRY(pack<T>(ctx, g, w, &tab));
  EvalK<T> k = make_consts<T>(p, pose, z_off);
  const int64_t blocks = ceil_div(Q * LPP, 256);
  rbf_status st;
  double* part = (double*)ws_get(ctx, WS_TMP3, sizeof(double) * GN_TERMS * (size_t)blocks, &st);
  if (!part) return st;
  k_eval_gn<T><<<(unsigned)blocks, 256, 0, ctx->stream>>>((const T*)pts, Q, tab, g->d_start,
                                                          geom(g), k, part);
  RBF_LAUNCHED(ctx, "k_eval_gn");
  k_eval_gn_sum<<<1, 1024, 0, ctx->stream>>>(part, blocks, JtJ, Jtr, rtr);
  RBF_LAUNCHED(ctx, "k_eval_gn_sum");
  return RBF_OK;
}

template <typename T>
static rbf_status adjoint_t(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g,
                            const double* w, const void* pts, int64_t Q, int32_t dim,
                            const double* pose, const void* gf, const void* gr, void* d_pts,
                            double* d_w, double* d_pose) {
  typename Vec4<T>::type* tab;
  RBF_TRY(pack<T>(ctx, g, w, &tab));
  EvalK<T> k = make_consts<T>(p, pose, 0.0);
  const int64_t blocks = ceil_div(Q, 256);
  if (dim == 3)
    k_eval_adjoint<T, true><<<blocks, 256, 0, ctx->stream>>>(
        (const T*)pts, Q, tab, g->d_idx, g->d_start, geom(g), k, (const T*)gf, (const T*)gr,
        (T*)d_pts, d_w, d_pose);
  else
    k_eval_adjoint<T, false><<<blocks, 256, 0, ctx->stream>>>(
        (const T*)pts, Q, tab, g->d_idx, g->d_start, geom(g), k, (const T*)gf, nullptr,
        (T*)d_pts, d_w, nullptr);
  RBF_LAUNCHED(ctx, "k_eval_adjoint");
  return RBF_OK;
}

}  // namespace rbf

using namespace rbf;

extern "C" {

rbf_status rbf_eval(rbf_ctx* ctx, const rbf_params* p, const rbf_grid* g, const double* w,
                    const void* pts, int64_t Q, int32_t dim, const double* pose, double z_off,
                    rbf_prec prec, void* f, void* grad, void* resid, void* jac) {
  if (!ctx) return RBF_E_INVALID_ARG;
  RBF_TRY(check_eval_args(ctx, p, g, w, pts, Q, dim, pose, prec, "rbf_eval"));
  if (Q > 0 && !f) return fail(ctx, RBF_E_INVALID_ARG, "rbf_eval: f is required");
  if (dim == 2 && (resid || jac))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_eval: resid/jac need dim == 3");
  if (Q == 0) return RBF_OK;
  RBF_TRY(set_device(ctx));
  if (prec == RBF_F64) return eval_t<double>(ctx, p, g, w, pts, Q, dim, pose, z_off, f, grad,
                                             resid, jac);
  return eval_t<float>(ctx, p, g, w, pts, Q, dim, pose, z_off, f, grad, resid, jac);
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
