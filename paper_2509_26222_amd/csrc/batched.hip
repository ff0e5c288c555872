// Many independent terrain patches updated and evaluated by ONE hipGraph
// launch, with the stages batched across patches.
//
// The recursion of every patch is cut into its Kalman batches and the
// patches advance in lockstep: round t absorbs batch t of each patch that
// has one. Every stage of a round (regressor rows, U = P H^T, S, each
// Cholesky step, V^T = L^{-1} U^T, w, the covariance product) is one launch
// over all of the round's jobs (update.hpp, GJob), so the latency-bound
// stages of small patches (the Cholesky of S takes the same 16 dependent
// steps whatever N_p is) run side by side instead of one patch after
// another, and the covariance products of all patches fill the GPU
// together. The patches are split into `chains` sets of about equal cost
// (longest processing time first on N_p^2 M_p), each advancing through its
// own rounds on its own stream, so that the latency-bound stages of one
// chain (the Cholesky steps, the gathers) run beside the covariance products
// of another. Each patch has its own workspace and status words, reserved
// at plan time; the first run captures the chains and the evaluations on the
// plan's streams, later runs relaunch the graph.
#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"
#include "update.hpp"

using namespace rbf;

struct rbf_batched {
  rbf_ctx* parent;
  rbf_ctx* cap;  // owns the capture / launch stream (never the legacy null stream)
  std::vector<rbf_ctx*> kids;  // chains 1.. (own stream and evaluation workspace)
  std::vector<hipEvent_t> joins;
  hipEvent_t fork;
  hipEvent_t ev_in, ev_out;
  rbf_params params;
  int32_t dim;
  rbf_prec eval_prec, gemm_prec;
  int64_t default_batch;
  double z_off;
  int32_t tile;
  int32_t nchains;
  std::vector<rbf_patch> patches;
  std::vector<std::vector<int32_t>> chain;  // patches of each chain
  std::vector<void*> mem;       // device allocations (per-patch workspaces, tables)
  int32_t* d_status;            // STATUS_WORDS per patch
  // rounds of each chain (device pointers filled once the tables are copied)
  std::vector<std::vector<GRound>> rounds;
  std::vector<std::vector<std::vector<int32_t>>> step_x;
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool captured;
};

static rbf_status batched_free(rbf_batched* b) {
  if (!b) return RBF_E_INVALID_ARG;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (void* m : b->mem)
    if (m) (void)hipFree(m);
  for (auto e : b->joins)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (auto k : b->kids)
    if (k) rbf_ctx_destroy(k);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->cap) rbf_ctx_destroy(b->cap);
  delete b;
  return RBF_OK;
}

namespace {

// Byte offsets of one patch's workspace (each part 256-byte aligned).
struct PatchLayout {
  size_t vals, cols, nnz, Ut, Vt, S, Lb, LiT, Linv, wpart, glist, gR, gH, vlo, total;
};

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

PatchLayout layout(int64_t N, int32_t kmax, int32_t Bp, bool groups, int64_t Rcap,
                   rbf_prec prec) {
  const int64_t ldu = ceil_div(N + 1, 32) * 32;
  const int64_t nblk = Bp / 64, ng = Bp / 64;
  PatchLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += up256(bytes);
    return at;
  };
  L.vals = take(sizeof(double) * (size_t)Bp * kmax);
  L.cols = take(sizeof(int32_t) * (size_t)Bp * kmax);
  L.nnz = take(sizeof(int32_t) * (size_t)Bp);
  L.Ut = take(sizeof(double) * (size_t)Bp * ldu);
  L.Vt = take(sizeof(double) * (size_t)Bp * ldu);
  L.S = take(sizeof(double) * (size_t)Bp * Bp);
  L.Lb = take(sizeof(double) * (size_t)Bp * Bp);
  L.LiT = take(sizeof(double) * (size_t)Bp * Bp);
  L.Linv = take(sizeof(double) * (size_t)nblk * 64 * 64);
  L.wpart = take(sizeof(double) * (size_t)nblk * N);
  L.glist = groups ? take(sizeof(int32_t) * (size_t)ng * Rcap) : 0;
  L.gR = groups ? take(sizeof(int32_t) * (size_t)ng) : 0;
  L.gH = groups ? take(sizeof(double) * (size_t)ng * Rcap * 64) : 0;
  if (prec == RBF_F32)
    L.vlo = take(sizeof(float) * (size_t)Bp * ldu);
  else if (prec == RBF_BF16)
    L.vlo = take(2 * 2 * (size_t)N * ceil_div(Bp, SYRK_BF16_KSTEP) * SYRK_BF16_KSTEP);
  L.total = o;
  return L;
}

}  // namespace

// Build the rounds: jobs, per-stage grids and covariance-product prefixes.
static rbf_status batched_build(rbf_batched* b, rbf_ctx* ctx) {
  const int32_t n = (int32_t)b->patches.size();
  std::vector<int64_t> B(n), nb(n);
  std::vector<char*> base(n, nullptr);
  std::vector<PatchLayout> lay(n);
  std::vector<int64_t> Rcap(n, 0);
  for (int32_t p = 0; p < n; ++p) {
    const rbf_patch& q = b->patches[p];
    B[p] = q.batch > 0 ? q.batch : b->default_batch;
    nb[p] = q.M > 0 ? ceil_div(q.M, B[p]) : 0;
    if (nb[p] == 0) continue;
    const int64_t N = q.grid->N;
    const int32_t kmax = q.grid->max_cand > 0 ? q.grid->max_cand : 1;
    const int32_t Bp = (int32_t)(ceil_div(std::min(B[p], q.M), 64) * 64);
    const bool groups = N <= GATHER_GROUP_NMAX;
    if (groups) {
      int64_t rc = std::min<int64_t>(N, (int64_t)64 * kmax);
      Rcap[p] = (rc + 3) / 4 * 4 + 4;
    }
    lay[p] = layout(N, kmax, Bp, groups, Rcap[p], b->gemm_prec);
    void* m = nullptr;
    if (hipMalloc(&m, lay[p].total) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, RBF_E_NOMEM, "rbf_batched_plan: workspace of patch %d (%zu bytes)", p,
                  lay[p].total);
    }
    b->mem.push_back(m);
    base[p] = (char*)m;
  }
  {
    void* m = nullptr;
    if (hipMalloc(&m, sizeof(int32_t) * STATUS_WORDS * (size_t)n) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, RBF_E_NOMEM, "rbf_batched_plan: status words");
    }
    b->mem.push_back(m);
    b->d_status = (int32_t*)m;
  }
  const RegKU rk = regku(&b->params);
  std::vector<GJob> jobs;
  std::vector<int64_t> pre;
  std::vector<std::vector<size_t>> job_at(b->nchains), pre_main_at(b->nchains),
      pre_tail_at(b->nchains);
  b->rounds.assign(b->nchains, {});
  b->step_x.assign(b->nchains, {});
  for (int32_t c = 0; c < b->nchains; ++c) {
    int64_t rounds = 0;
    for (int32_t p : b->chain[c]) rounds = std::max(rounds, nb[p]);
    b->rounds[c].assign(rounds, GRound{});
    b->step_x[c].assign(rounds, {});
    for (int64_t t = 0; t < rounds; ++t) {
      GRound& r = b->rounds[c][t];
      const size_t j0 = jobs.size();
      job_at[c].push_back(j0);
      for (int32_t p : b->chain[c]) {
        if (nb[p] <= t) continue;
        const rbf_patch& q = b->patches[p];
        const rbf_grid* g = q.grid;
        const PatchLayout& L = lay[p];
        char* m = base[p];
        GJob J{};
        J.P = (double*)q.P;
        J.ldp = q.ldp;
        J.N = g->N;
        J.w = (double*)q.w;
        const int64_t s0 = t * B[p];
        J.xy = (const double*)q.xy + 2 * s0;
        J.z = (const double*)q.z + s0;
        J.cxy = g->d_cxy;
        J.idx = g->d_idx;
        J.start = g->d_start;
        J.g = geom(g);
        J.rk = rk;
        J.R = b->params.R;
        J.kmax = g->max_cand > 0 ? g->max_cand : 1;
        J.Bc = (int32_t)std::min<int64_t>(B[p], q.M - s0);
        J.Bp = (int32_t)(ceil_div(J.Bc, 64) * 64);
        J.index = ((int64_t)p << 32) + t;
        J.seq = t + 1;
        J.status = b->d_status + (size_t)STATUS_WORDS * p;
        J.vals = (double*)(m + L.vals);
        J.cols = (int32_t*)(m + L.cols);
        J.nnz = (int32_t*)(m + L.nnz);
        J.Ut = (double*)(m + L.Ut);
        J.ldu = ceil_div(J.N + 1, 32) * 32;
        J.S = (double*)(m + L.S);
        J.Lb = (double*)(m + L.Lb);
        J.LiT = (double*)(m + L.LiT);
        J.Linv = (double*)(m + L.Linv);
        J.Vt = (double*)(m + L.Vt);
        J.wpart = (double*)(m + L.wpart);
        if (Rcap[p] > 0) {
          J.glist = (int32_t*)(m + L.glist);
          J.gR = (int32_t*)(m + L.gR);
          J.gH = (double*)(m + L.gH);
          J.Rcap = Rcap[p];
        }
        J.ncols = J.N + 1;
        J.words = gather_group_words(J.N);
        J.Kp = (int32_t)(ceil_div(J.Bc, SYRK_BF16_KSTEP) * SYRK_BF16_KSTEP);
        J.vlo = L.vlo ? (void*)(m + L.vlo) : nullptr;
        syrk_tiles(J.N, ctx->cu_count, &J.T, &J.per_xcd, &J.main_per_xcd);
        if (b->gemm_prec != RBF_F64 || b->tile == RBF_TILE_128)
          J.main_per_xcd = J.per_xcd;  // the FP32 / BF16 products have 128x128 tiles only
        else if (b->tile == RBF_TILE_SUB)
          J.main_per_xcd = 0;
        jobs.push_back(J);
      }
      r.n = (int32_t)(jobs.size() - j0);
      int32_t nsteps = 0;
      for (size_t j = j0; j < jobs.size(); ++j) {
        const GJob& J = jobs[j];
        const int32_t ng = J.Bp / 64, nblk = J.Bp / 64;
        auto mx = [](int32_t& a, int64_t v) { a = std::max<int32_t>(a, (int32_t)v); };
        mx(r.rows_x, ceil_div(J.Bp, 16));
        if (J.gH) {
          mx(r.gg_x, ng);
          r.gg_lds = std::max(r.gg_lds, gather_group_lds(J.words));
          mx(r.gm_x, ceil_div(J.N, 128));
          mx(r.gm_y, ng);
          mx(r.sg_x, (int64_t)ng * (ng + 1) / 2);
        }
        mx(r.gu_x, ceil_div(J.N, 1024));
        mx(r.gu_y, ceil_div(J.Bp, 8));
        mx(r.s_x, ceil_div(J.Bp, 256));
        mx(r.s_y, J.Bp);
        mx(r.zero_x, ceil_div((int64_t)J.Bp * J.Bp, 4096));
        nsteps = std::max(nsteps, nblk - 1);
        mx(r.lr_x, nblk - 1);
        mx(r.la_x, ceil_div(J.Bp, SYRK_TILE) * ceil_div(J.ncols, SYRK_TILE));
        mx(r.wp_x, ceil_div(J.N, 256));
        mx(r.wp_y, ceil_div(J.Bc, 64));
        mx(r.ws_x, ceil_div(J.N, 256));
        if (b->gemm_prec == RBF_F32) {
          mx(r.cvt_x, ceil_div((int64_t)J.Bc * J.ldu, 256));
          r.cvt_y = 1;
        } else if (b->gemm_prec == RBF_BF16) {
          mx(r.cvt_x, ceil_div(J.N, 64));
          mx(r.cvt_y, ceil_div(J.Kp, 64));
        }
      }
      r.nsteps = nsteps;
      r.chol_split = 1;  // many factors per launch: bound by throughput
      std::vector<int32_t>& sx = b->step_x[c][t];
      sx.assign(nsteps, 0);
      for (int32_t kb = 0; kb < nsteps; ++kb)
        for (size_t j = j0; j < jobs.size(); ++j)
          sx[kb] = std::max(sx[kb], chol_step_groups(jobs[j].Bp, kb));
      // covariance products: per-job workgroup counts (multiples of 8)
      pre_main_at[c].push_back(pre.size());
      pre.push_back(0);
      for (size_t j = j0; j < jobs.size(); ++j)
        pre.push_back(pre.back() + 8 * jobs[j].main_per_xcd);
      r.n_main = pre.back();
      pre_tail_at[c].push_back(pre.size());
      pre.push_back(0);
      for (size_t j = j0; j < jobs.size(); ++j)
        pre.push_back(pre.back() +
                      8 * (jobs[j].per_xcd - jobs[j].main_per_xcd) * SYRK_SUB_PER_TILE);
      r.n_tail = b->gemm_prec == RBF_F64 ? pre.back() : 0;
      if (r.n_main > INT32_MAX || r.n_tail > INT32_MAX)
        return fail(ctx, RBF_E_INVALID_ARG, "rbf_batched_plan: round %lld too large",
                    (long long)t);
    }
  }
  // device copies of the tables
  const size_t jb = sizeof(GJob) * std::max<size_t>(jobs.size(), 1);
  const size_t pb = sizeof(int64_t) * std::max<size_t>(pre.size(), 1);
  void* m = nullptr;
  if (hipMalloc(&m, up256(jb) + pb) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, RBF_E_NOMEM, "rbf_batched_plan: job tables");
  }
  b->mem.push_back(m);
  GJob* d_jobs = (GJob*)m;
  int64_t* d_pre = (int64_t*)((char*)m + up256(jb));
  if (!jobs.empty())
    RBF_HIP(ctx, hipMemcpy(d_jobs, jobs.data(), sizeof(GJob) * jobs.size(),
                           hipMemcpyHostToDevice));
  if (!pre.empty())
    RBF_HIP(ctx, hipMemcpy(d_pre, pre.data(), sizeof(int64_t) * pre.size(),
                           hipMemcpyHostToDevice));
  for (int32_t c = 0; c < b->nchains; ++c)
    for (size_t t = 0; t < b->rounds[c].size(); ++t) {
      GRound& r = b->rounds[c][t];
      r.jobs = d_jobs + job_at[c][t];
      r.pre_main = d_pre + pre_main_at[c][t];
      r.pre_tail = d_pre + pre_tail_at[c][t];
      r.step_x = b->step_x[c][t].data();
    }
  return RBF_OK;
}

// Chain c: its rounds, then the evaluation of its patches, on its context.
static rbf_status enqueue_chain(rbf_batched* b, int32_t c, rbf_ctx* ctx) {
  for (const GRound& r : b->rounds[c]) RBF_TRY(update_round_grouped(ctx, r, b->gemm_prec));
  for (int32_t pi : b->chain[c]) {
    const rbf_patch& p = b->patches[pi];
    if (p.Q == 0) continue;
    const rbf_status st =
        rbf_eval(ctx, &b->params, p.grid, p.w, p.pts, p.Q, b->dim,
                 b->dim == 3 ? p.pose : nullptr, b->z_off, b->eval_prec, p.f, p.grad, p.resid,
                 p.jac);
    if (st != RBF_OK) return fail(ctx, st, "batched: patch %d eval: %s", (int)pi, ctx->err);
  }
  return RBF_OK;
}

// Everything below is enqueued on the plan's own stream (captured): the
// status words cleared, the chains forked onto their streams and joined.
static rbf_status enqueue_all(rbf_batched* b) {
  rbf_ctx* ctx = b->cap;
  RBF_TRY(fill_zero(ctx, b->d_status, sizeof(int32_t) * STATUS_WORDS * b->patches.size()));
  RBF_HIP(ctx, hipEventRecord(b->fork, ctx->stream));
  rbf_status st = RBF_OK;
  for (size_t q = 0; q < b->kids.size(); ++q) {
    rbf_ctx* k = b->kids[q];
    RBF_HIP(ctx, hipStreamWaitEvent(k->stream, b->fork, 0));
    if (st == RBF_OK) {
      st = enqueue_chain(b, (int32_t)q + 1, k);
      if (st != RBF_OK) (void)fail(ctx, st, "%s", k->err);
    }
    // joined whatever happened, so that the capture can end
    RBF_HIP(ctx, hipEventRecord(b->joins[q], k->stream));
    RBF_HIP(ctx, hipStreamWaitEvent(ctx->stream, b->joins[q], 0));
  }
  RBF_TRY(st);
  RBF_TRY(enqueue_chain(b, 0, ctx));
  return RBF_OK;
}

extern "C" {

rbf_status rbf_batched_plan(rbf_ctx* ctx, const rbf_params* params, const rbf_patch* patches,
                            int32_t n, int32_t dim, rbf_prec eval_prec, rbf_prec gemm_prec,
                            int32_t tile, int32_t chains, int64_t default_batch,
                            double z_off, rbf_batched** out) {
  if (!ctx || !out) return RBF_E_INVALID_ARG;
  *out = nullptr;
  if (!params || !patches || n <= 0 || n > 65535 || (dim != 2 && dim != 3) ||
      (tile != RBF_TILE_AUTO && tile != RBF_TILE_128 && tile != RBF_TILE_SUB) || chains < 1 ||
      chains > 4 ||
      default_batch < 0 || default_batch > (1 << 16))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_batched_plan: bad arguments");
  if ((eval_prec != RBF_F64 && eval_prec != RBF_F32) ||
      (gemm_prec != RBF_F64 && gemm_prec != RBF_F32 && gemm_prec != RBF_BF16))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_batched_plan: bad precision");
  if (!(params->R > 0) || !std::isfinite(params->R))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_batched_plan: R must be > 0");
  for (int32_t i = 0; i < n; ++i) {
    const rbf_patch& p = patches[i];
    if (!p.grid || !p.w || !p.P || p.ldp < p.grid->N || p.M < 0 || (p.M > 0 && (!p.xy || !p.z)) ||
        p.Q < 0 || (p.Q > 0 && (!p.pts || !p.f)) || p.batch < 0 || p.batch > (1 << 16) ||
        p.grid->device != ctx->device)
      return fail(ctx, RBF_E_INVALID_ARG, "rbf_batched_plan: bad patch %d", i);
    if (params->sigma != p.grid->sigma || params->cutoff != p.grid->cutoff ||
        params->sigma_eps != p.grid->sigma_eps)
      return fail(ctx, RBF_E_INVALID_ARG, "rbf_batched_plan: patch %d grid params differ", i);
    if (dim == 2 && (p.resid || p.jac))
      return fail(ctx, RBF_E_INVALID_ARG, "rbf_batched_plan: resid/jac need dim == 3");
  }
  RBF_TRY(set_device(ctx));
  rbf_batched* b = new (std::nothrow) rbf_batched();
  if (!b) return RBF_E_NOMEM;
  b->parent = ctx;
  b->params = *params;
  b->dim = dim;
  b->eval_prec = eval_prec;
  b->gemm_prec = gemm_prec;
  b->default_batch = default_batch > 0 ? default_batch : UPDATE_DEFAULT_BATCH;
  b->z_off = z_off;
  b->tile = tile;
  b->patches.assign(patches, patches + n);
  // chains of about equal cost: longest processing time first
  b->nchains = std::min<int32_t>(chains, n);
  b->chain.assign(b->nchains, {});
  {
    std::vector<int32_t> order(n);
    for (int32_t i = 0; i < n; ++i) order[i] = i;
    auto cost = [&](int32_t i) {
      const double Np = (double)patches[i].grid->N;
      return Np * Np * (double)patches[i].M + 50.0 * Np * (double)patches[i].Q;
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t c) { return cost(a) > cost(c); });
    std::vector<double> load(b->nchains, 0.0);
    for (int32_t i : order) {
      const int32_t q = (int32_t)(std::min_element(load.begin(), load.end()) - load.begin());
      b->chain[q].push_back(i);
      load[q] += cost(i);
    }
    for (auto& c : b->chain) std::sort(c.begin(), c.end());
  }
  rbf_status st = RBF_OK;
  if (hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
    st = RBF_E_HIP;
  if (st == RBF_OK) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      st = RBF_E_HIP;
    } else if ((st = rbf_ctx_create(&b->cap, ctx->device, s)) != RBF_OK) {
      (void)hipStreamDestroy(s);
    } else {
      b->cap->owns_stream = 1;
    }
  }
  for (int32_t q = 1; q < b->nchains && st == RBF_OK; ++q) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      st = RBF_E_HIP;
      break;
    }
    rbf_ctx* k = nullptr;
    if ((st = rbf_ctx_create(&k, ctx->device, s)) != RBF_OK) {
      (void)hipStreamDestroy(s);
      break;
    }
    k->owns_stream = 1;
    b->kids.push_back(k);
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) st = RBF_E_HIP;
    b->joins.push_back(e);
  }
  if (st == RBF_OK) st = batched_build(b, ctx);
  for (int32_t c = 0; c < b->nchains && st == RBF_OK; ++c) {
    rbf_ctx* k = c == 0 ? b->cap : b->kids[c - 1];
    for (int32_t i : b->chain[c])
      if (st == RBF_OK && patches[i].Q > 0) st = eval_workspace(k, patches[i].grid);
  }
  if (st == RBF_OK && hipDeviceSynchronize() != hipSuccess) st = RBF_E_HIP;
  if (st != RBF_OK) {
    const std::string why = (b->cap && b->cap->err[0]) ? b->cap->err : ctx->err;
    batched_free(b);
    return fail(ctx, st, "rbf_batched_plan: setup failed: %s", why.c_str());
  }
  ++ctx->plans;
  for (const rbf_patch& q : b->patches) ++const_cast<rbf_grid*>(q.grid)->plans;
  *out = b;
  return RBF_OK;
}

rbf_status rbf_batched_run(rbf_batched* b) {
  if (!b) return RBF_E_INVALID_ARG;
  rbf_ctx* ctx = b->parent;
  rbf_ctx* cap = b->cap;
  RBF_TRY(set_device(ctx));
  if (!b->captured) {
    RBF_HIP(ctx, hipStreamBeginCapture(cap->stream, hipStreamCaptureModeThreadLocal));
    const rbf_status st = enqueue_all(b);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cap->stream, &g);
    if (st != RBF_OK) {
      if (g) (void)hipGraphDestroy(g);
      return fail(ctx, st, "rbf_batched_run: %s", cap->err);
    }
    if (e != hipSuccess)
      return fail(ctx, RBF_E_HIP, "rbf_batched_run: capture failed: %s", hipGetErrorString(e));
    b->graph = g;
    RBF_HIP(ctx, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->captured = true;
  }
  // ordered after earlier work on the caller's stream, and before later work
  RBF_HIP(ctx, hipEventRecord(b->ev_in, ctx->stream));
  RBF_HIP(ctx, hipStreamWaitEvent(cap->stream, b->ev_in, 0));
  RBF_HIP(ctx, hipGraphLaunch(b->exec, cap->stream));
  RBF_HIP(ctx, hipEventRecord(b->ev_out, cap->stream));
  RBF_HIP(ctx, hipStreamWaitEvent(ctx->stream, b->ev_out, 0));
  return RBF_OK;
}

rbf_status rbf_batched_sync(rbf_batched* b, int32_t* failed_patch) {
  if (!b) return RBF_E_INVALID_ARG;
  if (failed_patch) *failed_patch = -1;
  rbf_ctx* ctx = b->parent;
  RBF_TRY(set_device(ctx));
  if (b->cap) RBF_HIP(ctx, hipStreamSynchronize(b->cap->stream));
  RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const size_t n = b->patches.size();
  std::vector<int32_t> h(STATUS_WORDS * n);
  RBF_HIP(ctx, hipMemcpy(h.data(), b->d_status, sizeof(int32_t) * h.size(),
                         hipMemcpyDeviceToHost));
  for (size_t p = 0; p < n; ++p) {
    const int32_t code = h[STATUS_WORDS * p];
    if (code == 0) continue;
    // the first failing patch; every patch stops at its own failing batch
    if (failed_patch) *failed_patch = (int32_t)p;
    return fail(ctx, (rbf_status)code, "rbf_batched_sync: patch %d: device error %d (%s)",
                (int)p, (int)code, rbf_status_string((rbf_status)code));
  }
  for (rbf_ctx* k : b->kids) RBF_TRY(rbf_sync_status(k));
  return rbf_sync_status(b->cap);
}

rbf_status rbf_batched_destroy(rbf_batched* b) {
  if (!b) return RBF_E_INVALID_ARG;
  (void)hipSetDevice(b->parent->device);
  if (b->cap) (void)hipStreamSynchronize(b->cap->stream);
  (void)hipStreamSynchronize(b->parent->stream);
  --b->parent->plans;
  for (const rbf_patch& q : b->patches) --const_cast<rbf_grid*>(q.grid)->plans;
  return batched_free(b);
}

}  // extern "C"
