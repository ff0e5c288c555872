// Many independent terrain patches updated and evaluated by ONE hipGraph
// launch.
//
// The plan spreads the patches over K branches (longest processing time
// first on the cost N_p^2 M_p, the covariance product of one patch). Each
// branch is a child context with its own stream and workspace, reserved at
// plan time for the largest patch it will see, so the captured work
// allocates nothing and never synchronises. On the first run the parent
// stream is captured: a kernel clears the branch status words, an event
// forks the K branch streams off the parent, each branch enqueues
// rbf_update (asynchronous form) and rbf_eval for its patches in order, and
// the parent joins all branches. The instantiated graph is relaunched on
// later runs. Independent branches let the latency-bound steps of one patch
// (the Cholesky of S) overlap the MFMA steps of others.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "internal.hpp"
#include "update.hpp"

struct rbf_batched {
  rbf_ctx* parent;
  rbf_ctx* cap;  // owns the capture / launch stream (never the legacy null stream)
  hipEvent_t ev_in, ev_out;
  rbf_params params;
  int32_t dim;
  rbf_prec eval_prec, gemm_prec;
  int64_t default_batch;
  double z_off;
  std::vector<rbf_patch> patches;
  std::vector<rbf_ctx*> kids;
  std::vector<std::vector<int32_t>> assign;
  std::vector<hipEvent_t> joins;
  hipEvent_t fork;
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool captured;
};

using namespace rbf;

static rbf_status batched_free(rbf_batched* b) {
  if (!b) return RBF_E_INVALID_ARG;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto e : b->joins)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  for (auto k : b->kids)
    if (k) rbf_ctx_destroy(k);
  if (b->cap) rbf_ctx_destroy(b->cap);
  delete b;
  return RBF_OK;
}

// Everything below is enqueued on the plan's own stream (captured).
static rbf_status enqueue_all(rbf_batched* b) {
  rbf_ctx* ctx = b->cap;
  for (auto k : b->kids) RBF_TRY(fill_zero(ctx, k->d_status, STATUS_WORDS * sizeof(int32_t)));
  RBF_HIP(ctx, hipEventRecord(b->fork, ctx->stream));
  for (size_t q = 0; q < b->kids.size(); ++q) {
    rbf_ctx* k = b->kids[q];
    RBF_HIP(ctx, hipStreamWaitEvent(k->stream, b->fork, 0));
    for (int32_t pi : b->assign[q]) {
      const rbf_patch& p = b->patches[pi];
      const int64_t B = p.batch > 0 ? p.batch : b->default_batch;
      k->index_base = (int64_t)pi << 32;  // the status index names the patch
      rbf_status st = rbf_update(k, &b->params, p.grid, p.w, p.P, p.ldp, p.xy, p.z, p.M, B,
                                 b->gemm_prec, nullptr);
      k->index_base = 0;
      if (st != RBF_OK) return fail(ctx, st, "batched: patch %d update: %s", pi, k->err);
      st = rbf_eval(k, &b->params, p.grid, p.w, p.pts, p.Q, b->dim,
                    b->dim == 3 ? p.pose : nullptr, b->z_off, b->eval_prec, p.f, p.grad,
                    p.resid, p.jac);
      if (st != RBF_OK) return fail(ctx, st, "batched: patch %d eval: %s", pi, k->err);
    }
    RBF_HIP(ctx, hipEventRecord(b->joins[q], k->stream));
    RBF_HIP(ctx, hipStreamWaitEvent(ctx->stream, b->joins[q], 0));
  }
  return RBF_OK;
}

extern "C" {

rbf_status rbf_batched_plan(rbf_ctx* ctx, const rbf_params* params, const rbf_patch* patches,
                            int32_t n, int32_t dim, rbf_prec eval_prec, rbf_prec gemm_prec,
                            int32_t streams, int64_t default_batch, double z_off,
                            rbf_batched** out) {
  if (!ctx || !out) return RBF_E_INVALID_ARG;
  *out = nullptr;
  if (!params || !patches || n <= 0 || (dim != 2 && dim != 3) || streams < 1 || streams > 16 ||
      default_batch < 0 || default_batch > (1 << 16))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_batched_plan: bad arguments");
  if ((eval_prec != RBF_F64 && eval_prec != RBF_F32) ||
      (gemm_prec != RBF_F64 && gemm_prec != RBF_F32 && gemm_prec != RBF_BF16))
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_batched_plan: bad precision");
  for (int32_t i = 0; i < n; ++i) {
    const rbf_patch& p = patches[i];
    if (!p.grid || !p.w || !p.P || p.ldp < p.grid->N || p.M < 0 || (p.M > 0 && (!p.xy || !p.z)) ||
        p.Q < 0 || (p.Q > 0 && (!p.pts || !p.f)) || p.batch < 0 || p.grid->device != ctx->device)
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
  b->patches.assign(patches, patches + n);
  const int32_t K = std::min<int32_t>(streams, n);
  b->assign.resize(K);
  // longest processing time first
  std::vector<int32_t> order(n);
  for (int32_t i = 0; i < n; ++i) order[i] = i;
  auto cost = [&](int32_t i) {
    const double Np = (double)patches[i].grid->N;
    return Np * Np * (double)patches[i].M + 50.0 * Np * (double)patches[i].Q;
  };
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return cost(a) > cost(c); });
  std::vector<double> load(K, 0.0);
  for (int32_t i : order) {
    const int32_t q = (int32_t)(std::min_element(load.begin(), load.end()) - load.begin());
    b->assign[q].push_back(i);
    load[q] += cost(i);
  }
  for (int32_t q = 0; q < K; ++q) std::sort(b->assign[q].begin(), b->assign[q].end());
  rbf_status st = RBF_OK;
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess)
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
  for (int32_t q = 0; q < K && st == RBF_OK; ++q) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      st = RBF_E_HIP;
      break;
    }
    rbf_ctx* k = nullptr;
    st = rbf_ctx_create(&k, ctx->device, s);
    if (st != RBF_OK) {
      (void)hipStreamDestroy(s);
      break;
    }
    k->owns_stream = 1;
    k->single_stream = 1;
    b->kids.push_back(k);
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      st = RBF_E_HIP;
      break;
    }
    b->joins.push_back(e);
    // reserve the branch workspace for its largest patches
    for (int32_t pi : b->assign[q]) {
      const rbf_patch& p = patches[pi];
      const int64_t B = p.batch > 0 ? p.batch : b->default_batch;
      UpdWs ws;
      const int32_t kmax = p.grid->max_cand > 0 ? p.grid->max_cand : 1;
      st = update_workspace(k, p.grid->N, kmax, std::min<int64_t>(B, std::max<int64_t>(p.M, 1)),
                            gemm_prec, &ws);
      if (st != RBF_OK) break;
      if ((st = eval_workspace(k, p.grid)) != RBF_OK) break;
    }
  }
  if (st == RBF_OK && hipDeviceSynchronize() != hipSuccess) st = RBF_E_HIP;
  if (st != RBF_OK) {
    batched_free(b);
    return fail(ctx, st, "rbf_batched_plan: setup failed");
  }
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
    rbf_status st = enqueue_all(b);
    if (st != RBF_OK) {
      // rejoin every forked stream so that the capture can end
      for (size_t q = 0; q < b->kids.size(); ++q) {
        rbf_ctx* k = b->kids[q];
        if (k->aux) {
          (void)hipEventRecord(k->ev_back, k->aux);
          (void)hipStreamWaitEvent(k->stream, k->ev_back, 0);
        }
        (void)hipEventRecord(b->joins[q], k->stream);
        (void)hipStreamWaitEvent(cap->stream, b->joins[q], 0);
      }
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cap->stream, &g);
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
  rbf_status first = RBF_OK;
  int32_t worst = -1;
  for (size_t q = 0; q < b->kids.size(); ++q) {
    int32_t h[4];
    RBF_HIP(ctx, hipMemcpy(h, b->kids[q]->d_status, sizeof(h), hipMemcpyDeviceToHost));
    if (h[0] != 0) {
      // the recorded index is (patch << 32) + batch; the branch skipped its
      // later patches, which keep their previous state
      int64_t idx;
      memcpy(&idx, h + 2, sizeof(idx));
      const int32_t pi = (int32_t)(idx >> 32);
      if (first == RBF_OK || pi < worst) {
        first = (rbf_status)h[0];
        worst = pi;
      }
    }
  }
  if (failed_patch) *failed_patch = worst;
  if (first != RBF_OK)
    return fail(ctx, first, "rbf_batched_sync: device error %d (%s)", (int)first,
                rbf_status_string(first));
  return RBF_OK;
}

rbf_status rbf_batched_destroy(rbf_batched* b) {
  if (!b) return RBF_E_INVALID_ARG;
  (void)hipSetDevice(b->parent->device);
  if (b->cap) (void)hipStreamSynchronize(b->cap->stream);
  (void)hipStreamSynchronize(b->parent->stream);
  return batched_free(b);
}

}  // extern "C"
