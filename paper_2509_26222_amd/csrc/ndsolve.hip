// Sparse SPD solve calH X = B by nested dissection with dense frontal
// matrices (the "sparse kernel matrix inversion" of the GPU section,
// for repeated solves on one sparsity pattern).
//
// calH couples centers closer than 2 cutoff sigma_t: its graph is a
// geometric graph of bounded degree. Nested dissection cuts it recursively
// with small vertex separators, so that the Cholesky factor's dependent
// steps follow a tree of depth about log2(N / leaf) instead of the N / 64
// steps of a banded factor.
//
// Symbolic phase (host, once per pattern). A set of vertices is cut by a
// level of a breadth-first search from a pseudo-peripheral vertex: all
// edges join equal or adjacent levels, so the vertices of the middle level
// c that have a neighbour in level c + 1 separate the levels below from the
// levels above. Disconnected sets are split into their components instead.
// The tree is numbered in postorder (a node after its subtree); a node's
// front holds its own unknowns (k, padded to kp, a multiple of 64) and its
// boundary (m later unknowns coupled to its subtree).
//
// Numeric phase (device), front heights from the leaves up, all fronts of a
// height at once: the front is assembled from calH and the children's
// update matrices (extend-add), its leading block factored (the blocked
// FP64 Cholesky of the recursive update, L11 and L11^{-1}), the gain
// V^T = L11^{-1} F12 formed (FP64 MFMA) and the update matrix
// F22 - V V^T computed by the FP64 covariance product. The solves walk the
// tree up (y = L^{-1} b) and down
// (x = L^{-T} y); iterative refinement in FP64 repeats them on the residual
// b - calH x until rtol is met.
#include <algorithm>
#include <cmath>
#include <new>
#include <numeric>
#include <vector>

#include "internal.hpp"
#include "update.hpp"

namespace rbf {

// ------------------------------------------------------- symbolic (host)

struct NdNode {
  std::vector<int32_t> vars;  // the node's unknowns (original indices)
  std::vector<int32_t> bnd;   // boundary unknowns (original indices), in elimination order
  int32_t child[2] = {-1, -1};
  int32_t parent = -1;
  int32_t height = 0;
  int64_t first = 0;  // first position in the (padded) elimination order
  int32_t k = 0, kp = 0, m = 0, ldm = 0;
};

struct NdTree {
  int64_t N = 0, Np = 0;
  std::vector<NdNode> nodes;
  int32_t root = -1;
  std::vector<int32_t> new2old;  // Np entries, -1 for padding
  std::vector<int64_t> old2new;  // N entries
};

namespace {

class Dissector {
 public:
  Dissector(int64_t N, const int64_t* rp, const int32_t* ci, int32_t leaf, NdTree& t)
      : N_(N), rp_(rp), ci_(ci), leaf_(leaf), t_(t), mark_(N, -1), lev_(N, -1) {}

  int32_t run(std::vector<int32_t>& sub) {
    const int32_t id = (int32_t)t_.nodes.size();
    t_.nodes.emplace_back();
    if ((int64_t)sub.size() <= leaf_) {
      std::sort(sub.begin(), sub.end());
      t_.nodes[id].vars = sub;
      return id;
    }
    const int32_t cur = ++stamp_;
    for (int32_t v : sub) mark_[v] = cur;
    // a pseudo-peripheral vertex: the last vertex reached from the last
    // vertex reached from sub[0]
    std::vector<int32_t> order;
    bfs(sub[0], cur, order);
    if (order.size() < sub.size()) return split_components(id, sub, cur);
    bfs(order.back(), cur, order);
    const int32_t nlev = lev_[order.back()] + 1;
    if (nlev < 3) {  // no level separates: a dense leaf
      std::sort(sub.begin(), sub.end());
      t_.nodes[id].vars = sub;
      return id;
    }
    // the level holding the median vertex, kept inside [1, nlev - 2] (a
    // choice among the levels near it by separator size, tried, made the
    // tree deeper and its critical path longer)
    int32_t c = lev_[order[order.size() / 2]];
    c = std::max(1, std::min(c, nlev - 2));
    std::vector<int32_t> A, B, S;
    for (int32_t v : order) {
      const int32_t l = lev_[v];
      if (l < c) {
        A.push_back(v);
      } else if (l > c) {
        B.push_back(v);
      } else {
        bool up = false;
        for (int64_t e = rp_[v]; e < rp_[v + 1] && !up; ++e) {
          const int32_t u = ci_[e];
          up = mark_[u] == cur && lev_[u] == c + 1;
        }
        (up ? S : A).push_back(v);
      }
    }
    std::sort(S.begin(), S.end());
    t_.nodes[id].vars = S;
    int32_t slot = 0;
    for (std::vector<int32_t>* part : {&A, &B}) {
      if (part->empty()) continue;
      const int32_t ch = run(*part);
      t_.nodes[id].child[slot++] = ch;
      t_.nodes[ch].parent = id;
    }
    return id;
  }

 private:
  // Breadth-first search over the vertices marked cur; lev_ = level.
  void bfs(int32_t root, int32_t cur, std::vector<int32_t>& order) {
    order.clear();
    const int32_t seen = ++stamp_;  // visited vertices move to stamp `seen`
    order.push_back(root);
    mark_[root] = seen;
    lev_[root] = 0;
    for (size_t h = 0; h < order.size(); ++h) {
      const int32_t v = order[h];
      for (int64_t e = rp_[v]; e < rp_[v + 1]; ++e) {
        const int32_t u = ci_[e];
        if (mark_[u] != cur) continue;
        mark_[u] = seen;
        lev_[u] = lev_[v] + 1;
        order.push_back(u);
      }
    }
    for (int32_t v : order) mark_[v] = cur;  // restore the set's mark
  }

  // A disconnected set: a node without unknowns over two halves of its
  // components (by size), so the tree stays shallow.
  int32_t split_components(int32_t id, std::vector<int32_t>& sub, int32_t cur) {
    std::vector<std::vector<int32_t>> comps;
    std::vector<int32_t> order;
    for (int32_t v : sub) {
      if (mark_[v] != cur) continue;
      bfs(v, cur, order);
      for (int32_t u : order) mark_[u] = -1;  // out of the set once grouped
      comps.push_back(order);
    }
    std::sort(comps.begin(), comps.end(),
              [](const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
                return a.size() > b.size();
              });
    std::vector<int32_t> half[2];
    for (auto& cset : comps) {
      auto& h = half[0].size() <= half[1].size() ? half[0] : half[1];
      h.insert(h.end(), cset.begin(), cset.end());
    }
    int32_t slot = 0;
    for (auto& part : half) {
      if (part.empty()) continue;
      const int32_t ch = run(part);
      t_.nodes[id].child[slot++] = ch;
      t_.nodes[ch].parent = id;
    }
    return id;
  }

  int64_t N_;
  const int64_t* rp_;
  const int32_t* ci_;
  int32_t leaf_;
  NdTree& t_;
  std::vector<int32_t> mark_, lev_;
  int32_t stamp_ = 0;
};

}  // namespace

// Nested-dissection tree, elimination order and fronts of the pattern
// (rowptr, colidx on the host; the diagonal may be present or not).
static void nd_analyze(int64_t N, const int64_t* rp, const int32_t* ci, int32_t leaf,
                       NdTree& t) {
  t = NdTree{};
  t.N = N;
  std::vector<int32_t> all(N);
  std::iota(all.begin(), all.end(), 0);
  Dissector d(N, rp, ci, leaf, t);
  t.root = d.run(all);
  // postorder, heights and positions
  std::vector<int32_t> post;
  {
    std::vector<std::pair<int32_t, int>> st{{t.root, 0}};
    while (!st.empty()) {
      auto& [v, i] = st.back();
      if (i < 2 && t.nodes[v].child[i] >= 0) {
        const int32_t c = t.nodes[v].child[i++];
        st.push_back({c, 0});
        continue;
      }
      if (i < 2) {
        ++i;
        continue;
      }
      post.push_back(v);
      st.pop_back();
    }
  }
  t.old2new.assign(N, -1);
  int64_t pos = 0;
  for (int32_t v : post) {
    NdNode& n = t.nodes[v];
    for (int c = 0; c < 2; ++c)
      if (n.child[c] >= 0) n.height = std::max(n.height, t.nodes[n.child[c]].height + 1);
    n.k = (int32_t)n.vars.size();
    n.kp = (int32_t)((n.k + 63) / 64 * 64);
    n.first = pos;
    for (int32_t i = 0; i < n.k; ++i) t.old2new[n.vars[i]] = pos + i;
    pos += n.kp;
  }
  t.Np = pos;
  t.new2old.assign(t.Np, -1);
  for (int64_t v = 0; v < N; ++v) t.new2old[t.old2new[v]] = (int32_t)v;
  // boundaries, from the leaves up
  for (int32_t v : post) {
    NdNode& n = t.nodes[v];
    const int64_t lo = n.first, hi = n.first + n.kp;
    std::vector<int32_t> b;
    for (int32_t x : n.vars)
      for (int64_t e = rp[x]; e < rp[x + 1]; ++e)
        if (t.old2new[ci[e]] >= hi) b.push_back(ci[e]);
    for (int c = 0; c < 2; ++c) {
      if (n.child[c] < 0) continue;
      for (int32_t u : t.nodes[n.child[c]].bnd) {
        const int64_t q = t.old2new[u];
        if (q < lo || q >= hi) b.push_back(u);
      }
    }
    std::sort(b.begin(), b.end(),
              [&](int32_t a, int32_t c) { return t.old2new[a] < t.old2new[c]; });
    b.erase(std::unique(b.begin(), b.end()), b.end());
    n.bnd = std::move(b);
    n.m = (int32_t)n.bnd.size();
    n.ldm = (n.m + 31) / 32 * 32;
  }
}

// ------------------------------------------------------------- kernels

// One front on the device.
struct NdFront {
  double* F11;  // kp x kp (leading dimension kp)
  double* F12;  // kp x m (leading dimension ldm)
  double* F22;  // m x m (leading dimension ldm): the update matrix
  const double* LiT;  // L11^{-1} transposed (kp x kp)
  const double* Vt;   // V^T = L11^{-1} F12 (kp x m, leading dimension ldm)
  const int32_t* bnd_new;  // m positions of the boundary in the elimination order
  int64_t first, fvo;      // position of the node; row of its front vector
  int32_t k, kp, m, ldm;
};

// A child's update (matrix or vector) into its parent's front: cmap[a] is
// the parent's front row of the child's boundary entry a (< kp: the
// parent's own unknowns, else kp + boundary position).
struct NdEA {
  const double* U;  // child F22 (leading dimension ldc)
  const int32_t* cmap;
  int64_t cfvo;  // child's front-vector row (its update vector follows kp_c rows)
  int32_t mc, ldc, kpc;
  int32_t parent;  // index into the level's parent fronts
};

// arena[dst[i]] = vals[src[i]] (src < 0: 1, the padding's diagonal).
__global__ void __launch_bounds__(256) k_nd_assemble(const int64_t* __restrict__ src,
                                                     const int64_t* __restrict__ dst, int64_t n,
                                                     const double* __restrict__ vals,
                                                     double* __restrict__ arena) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t s = src[i];
  arena[dst[i]] = s >= 0 ? vals[s] : 1.0;
}

// Extend-add of child update matrices (one child per parent in a launch):
// entry (a, b) of U goes to F11, F12 or F22 of the parent by the maps
// (entries with a in the boundary and b in the own unknowns are the mirror
// images of stored ones and are skipped).
__global__ void __launch_bounds__(256) k_nd_extend_add(const NdEA* __restrict__ ea,
                                                       const NdFront* __restrict__ par) {
  const NdEA& E = ea[blockIdx.z];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t mc = E.mc;
  if (e >= mc * mc) return;
  const int32_t a = (int32_t)(e / mc), b = (int32_t)(e % mc);
  const NdFront& P = par[E.parent];
  const int32_t ra = E.cmap[a], rb = E.cmap[b];
  const double v = E.U[(int64_t)a * E.ldc + b];
  if (ra < P.kp) {
    if (rb < P.kp)
      P.F11[(int64_t)ra * P.kp + rb] += v;
    else
      P.F12[(int64_t)ra * P.ldm + (rb - P.kp)] += v;
  } else if (rb >= P.kp) {
    P.F22[(int64_t)(ra - P.kp) * P.ldm + (rb - P.kp)] += v;
  }
}

// Front vectors of a level: own rows from b (elimination order), boundary
// rows zero. fv and b hold nrhs columns (row-major); column r = blockIdx.y.
__global__ void __launch_bounds__(256) k_nd_fv_init(const NdFront* __restrict__ fr,
                                                    const double* __restrict__ bn,
                                                    double* __restrict__ fv, int64_t nrhs) {
  const NdFront& F = fr[blockIdx.z];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x, r = blockIdx.y;
  if (i >= F.kp + F.m) return;
  fv[(F.fvo + i) * nrhs + r] = i < F.kp ? bn[(F.first + i) * nrhs + r] : 0.0;
}

// Child update vectors into the parents' front vectors.
__global__ void __launch_bounds__(256) k_nd_fv_add(const NdEA* __restrict__ ea,
                                                   const NdFront* __restrict__ par,
                                                   double* __restrict__ fv, int64_t nrhs) {
  const NdEA& E = ea[blockIdx.z];
  const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x, r = blockIdx.y;
  if (a >= E.mc) return;
  const NdFront& P = par[E.parent];
  fv[(P.fvo + E.cmap[a]) * nrhs + r] += fv[(E.cfvo + E.kpc + a) * nrhs + r];
}

// out_i = sum_j A[j][i] x_j over rows j in [j0, j1(i)) of a row-major A:
// one workgroup of 1024 threads per 64 outputs, its 16 waves taking the
// rows j = j0 + wave, j0 + wave + 16, ... (coalesced row pieces) and the
// 16 partial sums meeting in LDS in a fixed order.
__device__ inline double colsum16(const double* __restrict__ A, int64_t lda, int32_t i, bool ok,
                                  int32_t j0, int32_t j1, const double* __restrict__ x,
                                  int64_t xs, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (ok) {
    int32_t j = j0 + wave;
    for (; j + 48 < j1; j += 64) {
      s0 += A[(int64_t)j * lda + i] * x[(int64_t)j * xs];
      s1 += A[(int64_t)(j + 16) * lda + i] * x[(int64_t)(j + 16) * xs];
      s2 += A[(int64_t)(j + 32) * lda + i] * x[(int64_t)(j + 32) * xs];
      s3 += A[(int64_t)(j + 48) * lda + i] * x[(int64_t)(j + 48) * xs];
    }
    for (; j < j1; j += 16) s0 += A[(int64_t)j * lda + i] * x[(int64_t)j * xs];
  }
  red[wave * 64 + lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  double t = 0.0;
  if (wave == 0)
    for (int w = 0; w < 16; ++w) t += red[w * 64 + lane];
  return t;
}

// Forward, own rows: y = L11^{-1} f (y_i = sum_{j <= i} LiT[j][i] f_j) into
// yn (elimination order).
__global__ void __launch_bounds__(1024) k_nd_fwd_l(const NdFront* __restrict__ fr,
                                                   const double* __restrict__ fv,
                                                   double* __restrict__ yn, int64_t nrhs) {
  __shared__ double red[1024];
  const NdFront& F = fr[blockIdx.z];
  const int32_t i = blockIdx.x * 64 + (threadIdx.x & 63);
  if ((int32_t)blockIdx.x * 64 >= F.kp) return;  // whole workgroup
  const int64_t r = blockIdx.y;
  const bool ok = i < F.kp;
  const double t = colsum16(F.LiT, F.kp, i, ok, 0, ok ? i + 1 : 0, fv + F.fvo * nrhs + r, nrhs,
                            red);
  if ((threadIdx.x >> 6) == 0 && ok) yn[(F.first + i) * nrhs + r] = t;
}

// Forward, boundary rows: u = f2 - V y (u_j = f2_j - sum_i Vt[i][j] y_i),
// left in the front vector's boundary rows (the node's update vector).
__global__ void __launch_bounds__(1024) k_nd_fwd_u(const NdFront* __restrict__ fr,
                                                   double* __restrict__ fv,
                                                   const double* __restrict__ yn, int64_t nrhs) {
  __shared__ double red[1024];
  const NdFront& F = fr[blockIdx.z];
  const int32_t j = blockIdx.x * 64 + (threadIdx.x & 63);
  if ((int32_t)blockIdx.x * 64 >= F.m) return;
  const int64_t r = blockIdx.y;
  const bool ok = j < F.m;
  const double t = colsum16(F.Vt, F.ldm, j, ok, 0, F.kp, yn + F.first * nrhs + r, nrhs, red);
  if ((threadIdx.x >> 6) == 0 && ok) fv[(F.fvo + F.kp + j) * nrhs + r] -= t;
}

// Backward: t_i = y_i - sum_j Vt[i][j] x(bnd_j), then x_i = sum_{j >= i}
// LiT[i][j] t_j. One wave per row, lanes across the row, a fixed shuffle
// tree; two launches (t needs every row before x).
__device__ inline double rowdot(const double* __restrict__ row, int32_t j0, int32_t j1,
                                const double* __restrict__ x, int64_t xs,
                                const int32_t* __restrict__ idx) {
  const int lane = threadIdx.x & 63;
  double s0 = 0.0, s1 = 0.0;
  int32_t j = j0 + lane;
  for (; j + 64 < j1; j += 128) {
    s0 += row[j] * x[(int64_t)(idx ? idx[j] : j) * xs];
    s1 += row[j + 64] * x[(int64_t)(idx ? idx[j + 64] : j + 64) * xs];
  }
  if (j < j1) s0 += row[j] * x[(int64_t)(idx ? idx[j] : j) * xs];
  double t = s0 + s1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  return t;
}

__global__ void __launch_bounds__(256) k_nd_bwd_t(const NdFront* __restrict__ fr,
                                                  const double* __restrict__ yn,
                                                  const double* __restrict__ xn,
                                                  double* __restrict__ tn, int64_t nrhs) {
  const NdFront& F = fr[blockIdx.z];
  const int32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= F.kp) return;  // whole waves
  const int64_t r = blockIdx.y;
  const double s = F.m > 0 ? rowdot(F.Vt + (int64_t)i * F.ldm, 0, F.m, xn + r, nrhs, F.bnd_new)
                           : 0.0;
  if ((threadIdx.x & 63) == 0) tn[(F.first + i) * nrhs + r] = yn[(F.first + i) * nrhs + r] - s;
}

__global__ void __launch_bounds__(256) k_nd_bwd_x(const NdFront* __restrict__ fr,
                                                  const double* __restrict__ tn,
                                                  double* __restrict__ xn, int64_t nrhs) {
  const NdFront& F = fr[blockIdx.z];
  const int32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= F.kp) return;
  const int64_t r = blockIdx.y;
  const double s =
      rowdot(F.LiT + (int64_t)i * F.kp, i, F.kp, tn + (F.first) * nrhs + r, nrhs, nullptr);
  if ((threadIdx.x & 63) == 0) xn[(F.first + i) * nrhs + r] = s;
}

// Right-hand side into the elimination order (padding rows zero), and the
// solution back: X (+)= x in the original order.
__global__ void __launch_bounds__(256) k_nd_perm_in(const int32_t* __restrict__ new2old,
                                                    int64_t Np, const double* __restrict__ R,
                                                    int64_t ldr, int64_t nrhs,
                                                    double* __restrict__ bn) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= Np * nrhs) return;
  const int64_t i = e / nrhs, r = e % nrhs;
  const int32_t o = new2old[i];
  bn[e] = o >= 0 ? R[(int64_t)o * ldr + r] : 0.0;
}

__global__ void __launch_bounds__(256) k_nd_perm_out(const int32_t* __restrict__ new2old,
                                                     int64_t Np, const double* __restrict__ xn,
                                                     int64_t nrhs, double* __restrict__ X,
                                                     int64_t ldx, int32_t first) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= Np * nrhs) return;
  const int64_t i = e / nrhs, r = e % nrhs;
  const int32_t o = new2old[i];
  if (o < 0) return;
  double* p = X + (int64_t)o * ldx + r;
  *p = first ? xn[e] : *p + xn[e];
}

}  // namespace rbf

using namespace rbf;

// ------------------------------------------------------------------ plan

struct rbf_solve_plan {
  rbf_ctx* ctx;
  NdTree tree;
  int64_t N, nnz;
  const int64_t* rowptr;  // device, the caller's
  const int32_t* colidx;
  std::vector<std::vector<int32_t>> levels;  // node ids by height
  // device memory
  double* arena;  // fronts and factors
  size_t arena_doubles;
  int32_t* imap;  // boundary positions, child maps, elimination order
  int64_t* asm_idx;  // assembly: src then dst per level
  NdFront* d_fronts;  // by level, level-major
  NdEA* d_ea;         // extend-add jobs by level and child slot
  GJob* d_jobs;       // factor jobs by level
  int64_t* d_pre;     // covariance-product prefixes by level
  // host tables
  std::vector<size_t> front_at, asm_at, asm_n;
  std::vector<size_t> ea_at[2];
  std::vector<int32_t> ea_n[2], ea_x[2];
  std::vector<GRound> rounds;
  std::vector<std::vector<int32_t>> step_x;
  std::vector<int32_t> lv_kp, lv_m;  // largest kp and m of a level (for grids)
  std::vector<int64_t> lvF0, lvF1;  // arena range of each level's F blocks
  int32_t* new2old_d;
  int64_t fv_rows;
  size_t asm_total;
  int32_t max_front;
  // graph replay: the factor reads a copy of the values, the sweeps work on
  // vectors of the plan's own, both captured on the plan's stream
  rbf_ctx* gctx;  // context over the plan's stream (launch checks, errors)
  hipEvent_t ev_a, ev_b;
  double* vals;   // nnz
  double* vec;    // bn, yn, tn, xn (Np x nrhs each), front vectors (fv_rows x nrhs)
  int64_t vec_cap;     // columns the vectors hold
  int64_t sweep_nrhs;  // columns of the captured sweeps
  hipGraphExec_t g_factor, g_sweeps;
};

namespace {

void plan_free(rbf_solve_plan* P) {
  if (!P) return;
  if (P->g_factor) (void)hipGraphExecDestroy(P->g_factor);
  if (P->g_sweeps) (void)hipGraphExecDestroy(P->g_sweeps);
  for (void* m : {(void*)P->arena, (void*)P->imap, (void*)P->asm_idx, (void*)P->d_fronts,
                  (void*)P->d_ea, (void*)P->d_jobs, (void*)P->d_pre, (void*)P->vals,
                  (void*)P->vec})
    if (m) (void)hipFree(m);
  if (P->ev_a) (void)hipEventDestroy(P->ev_a);
  if (P->ev_b) (void)hipEventDestroy(P->ev_b);
  if (P->gctx) rbf_ctx_destroy(P->gctx);
  delete P;
}

template <typename T>
rbf_status dev_copy(rbf_ctx* ctx, T** out, const std::vector<T>& h) {
  *out = nullptr;
  const size_t bytes = sizeof(T) * std::max<size_t>(h.size(), 1);
  if (hipMalloc(out, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, RBF_E_NOMEM, "rbf_solve_plan: %zu bytes", bytes);
  }
  if (!h.empty())
    RBF_HIP(ctx, hipMemcpy(*out, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
  return RBF_OK;
}

}  // namespace

extern "C" {

rbf_status rbf_solve_plan_create(rbf_ctx* ctx, int64_t N, const int64_t* rowptr,
                                 const int32_t* colidx, int32_t leaf,
                                 rbf_solve_plan** out) {
  if (!ctx || !out) return RBF_E_INVALID_ARG;
  *out = nullptr;
  if (N <= 0 || N >= ((int64_t)1 << 31) || !rowptr || !colidx || leaf < 0 || leaf > 16384)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_solve_plan_create: bad arguments");
  RBF_TRY(set_device(ctx));
  if (leaf == 0) leaf = 256;
  RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));  // the pattern may still be in flight
  std::vector<int64_t> rp(N + 1);
  RBF_HIP(ctx, hipMemcpy(rp.data(), rowptr, sizeof(int64_t) * (N + 1), hipMemcpyDeviceToHost));
  const int64_t nnz = rp[N];
  if (rp[0] != 0 || nnz < 0)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_solve_plan_create: bad rowptr");
  for (int64_t i = 0; i < N; ++i)
    if (rp[i + 1] < rp[i])
      return fail(ctx, RBF_E_INVALID_ARG, "rbf_solve_plan_create: rowptr not monotone");
  std::vector<int32_t> ci(std::max<int64_t>(nnz, 1));
  if (nnz > 0)
    RBF_HIP(ctx, hipMemcpy(ci.data(), colidx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
  for (int64_t e = 0; e < nnz; ++e)
    if (ci[e] < 0 || ci[e] >= N)
      return fail(ctx, RBF_E_INVALID_ARG, "rbf_solve_plan_create: column index out of range");
  rbf_solve_plan* P = new (std::nothrow) rbf_solve_plan();
  if (!P) return RBF_E_NOMEM;
  P->ctx = ctx;
  P->N = N;
  P->nnz = nnz;
  P->rowptr = rowptr;
  P->colidx = colidx;
  NdTree& t = P->tree;
  nd_analyze(N, rp.data(), ci.data(), leaf, t);
  const int32_t nn = (int32_t)t.nodes.size();
  int32_t H = 0;
  for (auto& n : t.nodes) H = std::max(H, n.height);
  P->levels.assign(H + 1, {});
  for (int32_t v = 0; v < nn; ++v) P->levels[t.nodes[v].height].push_back(v);
  // arena: per level, the fronts' F11, F12, F22 contiguous (cleared per
  // level), then per node Lb, LiT, Linv, Vt
  std::vector<int64_t> oF11(nn), oF12(nn), oF22(nn), oLb(nn), oLiT(nn), oLinv(nn), oVt(nn);
  std::vector<int64_t> lvF0(H + 1), lvF1(H + 1);
  int64_t o = 0;
  for (int32_t h = 0; h <= H; ++h) {
    lvF0[h] = o;
    for (int32_t v : P->levels[h]) {
      const NdNode& n = t.nodes[v];
      oF11[v] = o;
      o += (int64_t)n.kp * n.kp;
      oF12[v] = o;
      o += (int64_t)n.kp * n.ldm;
      oF22[v] = o;
      o += (int64_t)n.m * n.ldm;
      o = (o + 31) / 32 * 32;
    }
    lvF1[h] = o;
  }
  for (int32_t v = 0; v < nn; ++v) {
    const NdNode& n = t.nodes[v];
    oLb[v] = o;
    o += (int64_t)n.kp * n.kp;
    oLiT[v] = o;
    o += (int64_t)n.kp * n.kp;
    oLinv[v] = o;
    o += (int64_t)(n.kp / 64) * 4096;
    oVt[v] = o;
    o += (int64_t)n.kp * n.ldm;
    o = (o + 31) / 32 * 32;
    P->max_front = std::max(P->max_front, n.kp + n.m);
  }
  P->arena_doubles = (size_t)o;
  P->lvF0 = lvF0;
  P->lvF1 = lvF1;
  rbf_status st = RBF_OK;
  if (hipMalloc(&P->arena, sizeof(double) * std::max<size_t>(P->arena_doubles, 1)) !=
      hipSuccess) {
    (void)hipGetLastError();
    plan_free(P);
    return fail(ctx, RBF_E_NOMEM, "rbf_solve_plan_create: %zu bytes of fronts",
                sizeof(double) * (size_t)o);
  }
  // integer maps: boundary positions per node, child maps, elimination order
  std::vector<int32_t> im;
  std::vector<int64_t> oBnd(nn), oCmap(nn);
  for (int32_t v = 0; v < nn; ++v) {
    const NdNode& n = t.nodes[v];
    oBnd[v] = (int64_t)im.size();
    for (int32_t u : n.bnd) im.push_back((int32_t)t.old2new[u]);
  }
  for (int32_t v = 0; v < nn; ++v) {
    const NdNode& n = t.nodes[v];
    oCmap[v] = (int64_t)im.size();
    if (n.parent < 0) continue;
    const NdNode& p = t.nodes[n.parent];
    for (int32_t u : n.bnd) {
      const int64_t q = t.old2new[u];
      if (q >= p.first && q < p.first + p.kp) {
        im.push_back((int32_t)(q - p.first));
      } else {
        auto it = std::lower_bound(p.bnd.begin(), p.bnd.end(), u, [&](int32_t a, int32_t c) {
          return t.old2new[a] < t.old2new[c];
        });
        im.push_back(p.kp + (int32_t)(it - p.bnd.begin()));
      }
    }
  }
  const int64_t oPerm = (int64_t)im.size();
  im.insert(im.end(), t.new2old.begin(), t.new2old.end());
  st = dev_copy(ctx, &P->imap, im);
  P->new2old_d = st == RBF_OK ? P->imap + oPerm : nullptr;
  // assembly lists per level: CSR entries of each node's rows that land in
  // its front (own unknowns: F11, later ones: F12), and padding diagonals
  std::vector<int64_t> asrc, adst;
  for (int32_t h = 0; h <= H && st == RBF_OK; ++h) {
    P->asm_at.push_back(asrc.size());
    for (int32_t v : P->levels[h]) {
      const NdNode& n = t.nodes[v];
      for (int32_t i = 0; i < n.k; ++i) {
        const int32_t x = n.vars[i];
        for (int64_t e = rp[x]; e < rp[x + 1]; ++e) {
          const int64_t q = t.old2new[ci[e]];
          if (q >= n.first && q < n.first + n.kp) {
            asrc.push_back(e);
            adst.push_back(oF11[v] + (int64_t)i * n.kp + (q - n.first));
          } else if (q >= n.first + n.kp) {
            auto it = std::lower_bound(n.bnd.begin(), n.bnd.end(), ci[e],
                                       [&](int32_t a, int32_t c) {
                                         return t.old2new[a] < t.old2new[c];
                                       });
            asrc.push_back(e);
            adst.push_back(oF12[v] + (int64_t)i * n.ldm + (it - n.bnd.begin()));
          }
        }
      }
      for (int32_t i = n.k; i < n.kp; ++i) {
        asrc.push_back(-1);
        adst.push_back(oF11[v] + (int64_t)i * n.kp + i);
      }
    }
    P->asm_n.push_back(asrc.size() - P->asm_at.back());
  }
  const size_t atot = asrc.size();  // the dst lists follow the src lists
  {
    std::vector<int64_t> both(asrc);
    both.insert(both.end(), adst.begin(), adst.end());
    if (st == RBF_OK) st = dev_copy(ctx, &P->asm_idx, both);
  }
  // fronts, extend-add and factor jobs per level
  std::vector<NdFront> fronts;
  std::vector<NdEA> eas;
  std::vector<GJob> gjobs;
  std::vector<int64_t> pre;
  std::vector<size_t> job_at, pre_at;
  std::vector<int64_t> fvo(nn);
  std::vector<int32_t> lvidx(nn);  // index of a node among its level's fronts
  int64_t fvr = 0;
  for (int32_t h = 0; h <= H; ++h)
    for (size_t q = 0; q < P->levels[h].size(); ++q) {
      const int32_t v = P->levels[h][q];
      lvidx[v] = (int32_t)q;
      fvo[v] = fvr;
      fvr += t.nodes[v].kp + t.nodes[v].m;
    }
  P->fv_rows = fvr;
  P->rounds.assign(H + 1, GRound{});
  P->step_x.assign(H + 1, {});
  for (int32_t h = 0; h <= H; ++h) {
    P->front_at.push_back(fronts.size());
    int32_t xk = 0, xm = 0;
    for (int32_t v : P->levels[h]) {
      const NdNode& n = t.nodes[v];
      NdFront F{};
      F.F11 = P->arena + oF11[v];
      F.F12 = P->arena + oF12[v];
      F.F22 = P->arena + oF22[v];
      F.LiT = P->arena + oLiT[v];
      F.Vt = P->arena + oVt[v];
      F.bnd_new = st == RBF_OK ? P->imap + oBnd[v] : nullptr;
      F.first = n.first;
      F.fvo = fvo[v];
      F.k = n.k;
      F.kp = n.kp;
      F.m = n.m;
      F.ldm = n.ldm;
      fronts.push_back(F);
      xk = std::max(xk, n.kp);
      xm = std::max(xm, n.m);
    }
    P->lv_kp.push_back(xk);
    P->lv_m.push_back(xm);
    // extend-add jobs of this level's parents, by child slot
    for (int c = 0; c < 2; ++c) {
      P->ea_at[c].push_back(eas.size());
      int32_t mx = 0, cnt = 0;
      for (int32_t v : P->levels[h]) {
        const NdNode& n = t.nodes[v];
        const int32_t ch = n.child[c];
        if (ch < 0 || t.nodes[ch].m == 0) continue;
        const NdNode& cn = t.nodes[ch];
        NdEA E{};
        E.U = P->arena + oF22[ch];
        E.cmap = st == RBF_OK ? P->imap + oCmap[ch] : nullptr;
        E.cfvo = fvo[ch];
        E.mc = cn.m;
        E.ldc = cn.ldm;
        E.kpc = cn.kp;
        E.parent = lvidx[v];
        eas.push_back(E);
        mx = std::max(mx, cn.m);
        ++cnt;
      }
      P->ea_n[c].push_back(cnt);
      P->ea_x[c].push_back(mx);
    }
    // factor jobs (nodes with unknowns)
    job_at.push_back(gjobs.size());
    GRound& r = P->rounds[h];
    int32_t nsteps = 0;
    for (int32_t v : P->levels[h]) {
      const NdNode& n = t.nodes[v];
      if (n.k == 0) continue;
      GJob J{};
      J.S = P->arena + oF11[v];
      J.Bp = n.kp;
      J.Bc = n.k;
      J.Lb = P->arena + oLb[v];
      J.LiT = P->arena + oLiT[v];
      J.Linv = P->arena + oLinv[v];
      J.Ut = P->arena + oF12[v];
      J.Vt = P->arena + oVt[v];
      J.ldu = n.ldm;
      J.ncols = n.m;
      J.P = P->arena + oF22[v];
      J.ldp = n.ldm;
      J.N = n.m;
      J.status = ctx->d_status;
      J.index = v;
      syrk_tiles(n.m, ctx->cu_count, &J.T, &J.per_xcd, &J.main_per_xcd);
      gjobs.push_back(J);
      nsteps = std::max(nsteps, n.kp / 64 - 1);
      r.zero_x = std::max<int32_t>(r.zero_x, (int32_t)ceil_div((int64_t)n.kp * n.kp, 4096));
      r.lr_x = std::max(r.lr_x, n.kp / 64 - 1);
      r.la_x = std::max<int32_t>(
          r.la_x, (int32_t)(ceil_div(n.kp, SYRK_TILE) * ceil_div(n.m, SYRK_TILE)));
    }
    r.n = (int32_t)(gjobs.size() - job_at.back());
    r.nsteps = nsteps;
    P->step_x[h].assign(nsteps, 0);
    for (int32_t kb = 0; kb < nsteps; ++kb)
      for (size_t j = job_at.back(); j < gjobs.size(); ++j)
        P->step_x[h][kb] = std::max(P->step_x[h][kb], chol_step_groups(gjobs[j].Bp, kb));
    pre_at.push_back(pre.size());
    pre.push_back(0);
    for (size_t j = job_at.back(); j < gjobs.size(); ++j)
      pre.push_back(pre.back() + 8 * gjobs[j].main_per_xcd);
    r.n_main = pre.back();
    pre.push_back(0);
    for (size_t j = job_at.back(); j < gjobs.size(); ++j)
      pre.push_back(pre.back() +
                    8 * (gjobs[j].per_xcd - gjobs[j].main_per_xcd) * SYRK_SUB_PER_TILE);
    r.n_tail = pre.back();
  }
  if (st == RBF_OK) st = dev_copy(ctx, &P->d_fronts, fronts);
  if (st == RBF_OK) st = dev_copy(ctx, &P->d_ea, eas);
  if (st == RBF_OK) st = dev_copy(ctx, &P->d_pre, pre);
  if (st == RBF_OK) st = dev_copy(ctx, &P->d_jobs, gjobs);
  if (st == RBF_OK &&
      hipMalloc(&P->vals, sizeof(double) * std::max<int64_t>(nnz, 1)) != hipSuccess) {
    (void)hipGetLastError();
    st = fail(ctx, RBF_E_NOMEM, "rbf_solve_plan_create: values copy");
  }
  if (st == RBF_OK && (hipEventCreateWithFlags(&P->ev_a, hipEventDisableTiming) != hipSuccess ||
                       hipEventCreateWithFlags(&P->ev_b, hipEventDisableTiming) != hipSuccess))
    st = fail(ctx, RBF_E_HIP, "rbf_solve_plan_create: events");
  if (st == RBF_OK) {
    hipStream_t gs = nullptr;
    if (hipStreamCreateWithFlags(&gs, hipStreamNonBlocking) != hipSuccess) {
      st = fail(ctx, RBF_E_HIP, "rbf_solve_plan_create: stream");
    } else if (rbf_ctx_create(&P->gctx, ctx->device, gs) != RBF_OK) {
      (void)hipStreamDestroy(gs);
      st = fail(ctx, RBF_E_HIP, "rbf_solve_plan_create: stream context");
    } else {
      P->gctx->owns_stream = 1;
    }
  }
  if (st != RBF_OK) {
    plan_free(P);
    return st;
  }
  for (int32_t h = 0; h <= H; ++h) {
    GRound& r = P->rounds[h];
    r.jobs = P->d_jobs + job_at[h];
    r.pre_main = P->d_pre + pre_at[h];
    r.pre_tail = P->d_pre + pre_at[h] + r.n + 1;
    r.step_x = P->step_x[h].data();
  }
  P->asm_total = atot;
  ++ctx->plans;
  *out = P;
  return RBF_OK;
}

rbf_status rbf_solve_plan_info(const rbf_solve_plan* P, int32_t* nodes, int32_t* levels,
                               int64_t* front_bytes, int32_t* max_front) {
  if (!P) return RBF_E_INVALID_ARG;
  if (nodes) *nodes = (int32_t)P->tree.nodes.size();
  if (levels) *levels = (int32_t)P->levels.size();
  if (front_bytes) *front_bytes = (int64_t)(sizeof(double) * P->arena_doubles);
  if (max_front) *max_front = P->max_front;
  return RBF_OK;
}

rbf_status rbf_solve_plan_destroy(rbf_solve_plan* P) {
  if (!P) return RBF_E_INVALID_ARG;
  (void)hipSetDevice(P->ctx->device);
  (void)hipStreamSynchronize(P->ctx->stream);
  --P->ctx->plans;
  plan_free(P);
  return RBF_OK;
}

}  // extern "C"

namespace rbf {

// Numeric factorization of the plan's pattern with these values: per
// height, clear the level's fronts, scatter calH into them, add the
// children's update matrices, then factor, form V^T and the update matrix.
static rbf_status nd_factor(rbf_solve_plan* P, rbf_ctx* ctx) {
  const double* vals = P->vals;
  const int32_t H = (int32_t)P->levels.size() - 1;
  for (int32_t h = 0; h <= H; ++h) {
    const NdFront* fr = P->d_fronts + P->front_at[h];
    RBF_TRY(fill_zero(ctx, P->arena + P->lvF0[h],
                      sizeof(double) * (size_t)(P->lvF1[h] - P->lvF0[h])));
    const int64_t na = (int64_t)P->asm_n[h];
    if (na > 0) {
      const int64_t* src = P->asm_idx + P->asm_at[h];
      k_nd_assemble<<<(unsigned)ceil_div(na, 256), 256, 0, ctx->stream>>>(
          src, src + P->asm_total, na, vals, P->arena);
      RBF_LAUNCHED(ctx, "k_nd_assemble");
    }
    for (int c = 0; c < 2; ++c) {
      const int32_t n = P->ea_n[c][h];
      if (n == 0) continue;
      const int64_t mx = P->ea_x[c][h];
      k_nd_extend_add<<<dim3((unsigned)ceil_div(mx * mx, 256), 1, (unsigned)n), 256, 0,
                        ctx->stream>>>(P->d_ea + P->ea_at[c][h], fr);
      RBF_LAUNCHED(ctx, "k_nd_extend_add");
    }
    const GRound& r = P->rounds[h];
    if (r.n == 0) continue;
    RBF_TRY(chol_grouped(ctx, r));
    RBF_TRY(linv_apply_grouped(ctx, r));
    RBF_TRY(syrk_grouped(ctx, r, RBF_F64));
  }
  return RBF_OK;
}

// y = L^{-1} bn up the tree, then x = L^{-T} y down the tree (elimination
// order, nrhs columns); fv: front vectors, tn: scratch of Np x nrhs.
static rbf_status nd_sweeps(rbf_solve_plan* P, rbf_ctx* ctx, const double* bn, double* fv,
                            double* yn, double* tn, double* xn, int64_t nrhs) {
  const int32_t H = (int32_t)P->levels.size() - 1;
  const unsigned ny = (unsigned)nrhs;
  for (int32_t h = 0; h <= H; ++h) {
    const NdFront* fr = P->d_fronts + P->front_at[h];
    const unsigned nf = (unsigned)P->levels[h].size();
    const int32_t xk = P->lv_kp[h], xm = P->lv_m[h];
    if (xk + xm == 0) continue;  // fronts without unknowns or boundary (a root joining parts)
    k_nd_fv_init<<<dim3((unsigned)ceil_div(xk + xm, 256), ny, nf), 256, 0, ctx->stream>>>(
        fr, bn, fv, nrhs);
    RBF_LAUNCHED(ctx, "k_nd_fv_init");
    for (int c = 0; c < 2; ++c) {
      const int32_t n = P->ea_n[c][h];
      if (n == 0) continue;
      k_nd_fv_add<<<dim3((unsigned)ceil_div(P->ea_x[c][h], 256), ny, (unsigned)n), 256, 0,
                    ctx->stream>>>(P->d_ea + P->ea_at[c][h], fr, fv, nrhs);
      RBF_LAUNCHED(ctx, "k_nd_fv_add");
    }
    if (xk > 0) {
      k_nd_fwd_l<<<dim3((unsigned)ceil_div(xk, 64), ny, nf), 1024, 0, ctx->stream>>>(fr, fv, yn,
                                                                                   nrhs);
      RBF_LAUNCHED(ctx, "k_nd_fwd_l");
    }
    if (xm > 0) {
      k_nd_fwd_u<<<dim3((unsigned)ceil_div(xm, 64), ny, nf), 1024, 0, ctx->stream>>>(fr, fv, yn,
                                                                                   nrhs);
      RBF_LAUNCHED(ctx, "k_nd_fwd_u");
    }
  }
  for (int32_t h = H; h >= 0; --h) {
    const NdFront* fr = P->d_fronts + P->front_at[h];
    const unsigned nf = (unsigned)P->levels[h].size();
    const int32_t xk = P->lv_kp[h];
    if (xk == 0) continue;
    k_nd_bwd_t<<<dim3((unsigned)ceil_div(xk, 4), ny, nf), 256, 0, ctx->stream>>>(fr, yn, xn, tn,
                                                                               nrhs);
    RBF_LAUNCHED(ctx, "k_nd_bwd_t");
    k_nd_bwd_x<<<dim3((unsigned)ceil_div(xk, 4), ny, nf), 256, 0, ctx->stream>>>(fr, tn, xn,
                                                                               nrhs);
    RBF_LAUNCHED(ctx, "k_nd_bwd_x");
  }
  return RBF_OK;
}

// Capture `body` (launches on the plan's stream context) into *exec on the
// first use; every use then replays it on the plan's stream, ordered after
// the caller's stream and before its later work by events.
template <typename F>
static rbf_status plan_graph(rbf_solve_plan* P, hipGraphExec_t* exec, F body) {
  rbf_ctx* ctx = P->ctx;
  rbf_ctx* g = P->gctx;
  if (!*exec) {
    RBF_HIP(ctx, hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
    const rbf_status st = body(g);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(g->stream, &graph);
    if (st != RBF_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(ctx, st, "rbf_solve_plan_run: %s", g->err);
    }
    if (e != hipSuccess)
      return fail(ctx, RBF_E_HIP, "rbf_solve_plan_run: capture failed: %s",
                  hipGetErrorString(e));
    const hipError_t ie = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      *exec = nullptr;
      return fail(ctx, RBF_E_HIP, "rbf_solve_plan_run: instantiate: %s", hipGetErrorString(ie));
    }
  }
  RBF_HIP(ctx, hipEventRecord(P->ev_a, ctx->stream));
  RBF_HIP(ctx, hipStreamWaitEvent(g->stream, P->ev_a, 0));
  RBF_HIP(ctx, hipGraphLaunch(*exec, g->stream));
  RBF_HIP(ctx, hipEventRecord(P->ev_b, g->stream));
  RBF_HIP(ctx, hipStreamWaitEvent(ctx->stream, P->ev_b, 0));
  return RBF_OK;
}

}  // namespace rbf

extern "C" rbf_status rbf_solve_plan_run(rbf_solve_plan* P, const double* vals, const double* B,
                                         int64_t ldb, double* X, int64_t ldx, int64_t nrhs,
                                         double rtol, int32_t max_iter, rbf_prec inner,
                                         double* relres, int32_t* iters) {
  if (!P) return RBF_E_INVALID_ARG;
  rbf_ctx* ctx = P->ctx;
  if (iters) *iters = 0;
  const int64_t N = P->N, Np = P->tree.Np;
  if (!vals || !B || !X || nrhs <= 0 || nrhs > 65535 || ldb < nrhs || ldx < nrhs ||
      !(rtol > 0) || max_iter < 1)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_solve_plan_run: bad arguments");
  if (inner != RBF_F64)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_solve_plan_run: inner must be RBF_F64");
  RBF_TRY(set_device(ctx));
  RBF_TRY(rbf_sync_status(ctx));  // no pending error: this factor's failures are its own
  rbf_status st;
  // the plan's vectors for nrhs columns (grown when a call brings more); the
  // sweeps are captured for one column count and recaptured on a change
  if (P->g_sweeps && nrhs != P->sweep_nrhs) {
    (void)hipGraphExecDestroy(P->g_sweeps);
    P->g_sweeps = nullptr;
  }
  if (nrhs > P->vec_cap) {
    RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (P->vec) (void)hipFree(P->vec);
    P->vec = nullptr;
    P->vec_cap = 0;
    const size_t bytes = sizeof(double) * (4 * (size_t)Np + (size_t)P->fv_rows) * nrhs;
    if (hipMalloc(&P->vec, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, RBF_E_NOMEM, "rbf_solve_plan_run: %zu bytes of vectors", bytes);
    }
    P->vec_cap = nrhs;
  }
  const size_t vn = (size_t)Np * nrhs;
  double *bn = P->vec, *yn = P->vec + vn, *tn = P->vec + 2 * vn, *xn = P->vec + 3 * vn;
  double* fv = P->vec + 4 * vn;
  double* Rr = (double*)ws_get(ctx, WS_SOLVE1, sizeof(double) * (size_t)N * nrhs, &st);
  if (!Rr) return st;
  RBF_HIP(ctx, hipMemcpyAsync(P->vals, vals, sizeof(double) * (size_t)P->nnz,
                              hipMemcpyDeviceToDevice, ctx->stream));
  RBF_TRY(plan_graph(P, &P->g_factor, [&](rbf_ctx* g) { return nd_factor(P, g); }));
  {
    int32_t h[4];
    RBF_HIP(ctx, hipMemcpyAsync(h, ctx->d_status, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (h[0] != 0) return rbf_sync_status(ctx);
  }
  std::vector<double> bnorm, rn;
  RBF_TRY(solve_col_norms(ctx, B, ldb, N, nrhs, bnorm));
  const double* R = B;
  int64_t ldr = ldb;
  int32_t it = 0;
  bool conv = false;
  for (it = 0; it < max_iter && !conv; ++it) {
    k_nd_perm_in<<<(unsigned)ceil_div(Np * nrhs, 256), 256, 0, ctx->stream>>>(
        P->new2old_d, Np, R, ldr, nrhs, bn);
    RBF_LAUNCHED(ctx, "k_nd_perm_in");
    RBF_TRY(plan_graph(P, &P->g_sweeps,
                       [&](rbf_ctx* g) { return nd_sweeps(P, g, bn, fv, yn, tn, xn, nrhs); }));
    P->sweep_nrhs = nrhs;
    k_nd_perm_out<<<(unsigned)ceil_div(Np * nrhs, 256), 256, 0, ctx->stream>>>(
        P->new2old_d, Np, xn, nrhs, X, ldx, it == 0);
    RBF_LAUNCHED(ctx, "k_nd_perm_out");
    RBF_TRY(solve_residual(ctx, P->rowptr, P->colidx, vals, N, B, ldb, X, ldx, nrhs, Rr));
    R = Rr;
    ldr = nrhs;
    RBF_TRY(solve_col_norms(ctx, Rr, nrhs, N, nrhs, rn));
    conv = true;
    for (int64_t c = 0; c < nrhs; ++c) {
      const double rel = bnorm[c] > 0 ? rn[c] / bnorm[c] : rn[c];
      if (relres) relres[c] = rel;
      if (!(rel <= rtol)) conv = false;
    }
  }
  if (iters) *iters = it;
  RBF_TRY(rbf_sync_status(ctx));
  if (!conv)
    return fail(ctx, RBF_E_NO_CONVERGE, "rbf_solve_plan_run: relres above %g after %d sweeps",
                rtol, it);
  return RBF_OK;
}

// The symbolic phase alone, on host arrays (no device): the elimination
// order and the dissection tree, for checks of the ordering.
extern "C" rbf_status rbf_solve_order_host(int64_t N, const int64_t* rowptr,
                                           const int32_t* colidx, int32_t leaf,
                                           int32_t* new2old, int32_t* node_of,
                                           int32_t* parent, int32_t cap, int32_t* n_nodes) {
  if (N <= 0 || N >= ((int64_t)1 << 31) || !rowptr || !colidx || !new2old || !node_of ||
      !n_nodes || leaf < 0 || cap < 0 || (cap > 0 && !parent))
    return RBF_E_INVALID_ARG;
  for (int64_t i = 0; i < N; ++i)
    if (rowptr[i + 1] < rowptr[i]) return RBF_E_INVALID_ARG;
  for (int64_t e = 0; e < rowptr[N]; ++e)
    if (colidx[e] < 0 || colidx[e] >= N) return RBF_E_INVALID_ARG;
  NdTree t;
  nd_analyze(N, rowptr, colidx, leaf > 0 ? leaf : 256, t);
  *n_nodes = (int32_t)t.nodes.size();
  if ((int32_t)t.nodes.size() > cap) return RBF_E_CAPACITY;
  int64_t q = 0;  // the order without padding
  for (int64_t i = 0; i < t.Np; ++i)
    if (t.new2old[i] >= 0) new2old[q++] = t.new2old[i];
  for (size_t v = 0; v < t.nodes.size(); ++v) {
    parent[v] = t.nodes[v].parent;
    for (int32_t x : t.nodes[v].vars) node_of[x] = (int32_t)v;
  }
  return RBF_OK;
}
