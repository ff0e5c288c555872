// Context, status word, workspace and the small shared kernels (scans,
// stable key sort) of librbf.
#include "internal.hpp"

namespace rbf {

rbf_status fail(rbf_ctx* ctx, rbf_status s, const char* fmt, ...) {
  if (ctx) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
    va_end(ap);
  }
  return s;
}

rbf_status set_device(rbf_ctx* ctx) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess)
    return fail(ctx, RBF_E_HIP, "hipSetDevice(%d): %s", ctx->device,
                hipGetErrorString(e));
  return RBF_OK;
}

void* ws_get(rbf_ctx* ctx, int slot, size_t bytes, rbf_status* st) {
  *st = RBF_OK;
  if (bytes == 0) bytes = 256;
  if (ctx->ws_bytes[slot] >= bytes) return ctx->ws[slot];
  if (ctx->ws[slot]) {
    // the old buffer may still be read by queued kernels
    if ((ctx->aux && hipStreamSynchronize(ctx->aux) != hipSuccess) ||
        hipStreamSynchronize(ctx->stream) != hipSuccess ||
        hipFree(ctx->ws[slot]) != hipSuccess) {
      *st = fail(ctx, RBF_E_HIP, "workspace release failed");
      return nullptr;
    }
    ctx->ws[slot] = nullptr;
    ctx->ws_bytes[slot] = 0;
  }
  size_t want = bytes + bytes / 8;  // headroom for slightly larger calls
  want = (want + 4095) & ~size_t(4095);
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    *st = fail(ctx, RBF_E_NOMEM, "workspace slot %d: cannot allocate %zu bytes",
               slot, want);
    return nullptr;
  }
  ctx->ws[slot] = p;
  ctx->ws_bytes[slot] = want;
  return p;
}

rbf_status check_launch(rbf_ctx* ctx, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(ctx, RBF_E_HIP, "launch of %s failed: %s", what,
                hipGetErrorString(e));
  return RBF_OK;
}

// ---------------------------------------------------------------- scans

template <typename T>
__device__ void scan_excl_block(T* data, int64_t n) {
  // Each of the 1024 threads owns a contiguous chunk; chunk sums are
  // scanned in LDS, then each chunk is rewritten. data[n] = total.
  __shared__ T part[1024];
  const int tid = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t a = tid * per;
  const int64_t b = a + per < n ? a + per : n;
  T s = 0;
  for (int64_t i = a; i < b; ++i) s += data[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    T v = tid >= off ? part[tid - off] : T(0);
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  T run = tid ? part[tid - 1] : T(0);
  for (int64_t i = a; i < b; ++i) {
    T v = data[i];
    data[i] = run;
    run += v;
  }
  if (tid == 1023) data[n] = part[1023];
}

__global__ void __launch_bounds__(1024) k_scan_excl_i64(int64_t* data, int64_t n) {
  scan_excl_block<int64_t>(data, n);
}

__global__ void __launch_bounds__(1024) k_scan_excl_i32(int32_t* data, int64_t n) {
  scan_excl_block<int32_t>(data, n);
}

__global__ void __launch_bounds__(256) k_fill_zero_u32(uint32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * 256;
  for (; i < n; i += stride) p[i] = 0u;
}

__global__ void k_fill_zero_u8(uint8_t* p, int64_t n) {
  int64_t i = threadIdx.x;
  if (i < n) p[i] = 0;
}

rbf_status fill_zero(rbf_ctx* ctx, void* p, size_t bytes) {
  if (bytes == 0) return RBF_OK;
  const int64_t words = (int64_t)(bytes / 4);
  if (words > 0) {
    int64_t blocks = ceil_div(words, 256);
    if (blocks > 4096) blocks = 4096;
    k_fill_zero_u32<<<blocks, 256, 0, ctx->stream>>>((uint32_t*)p, words);
    RBF_LAUNCHED(ctx, "k_fill_zero_u32");
  }
  const int64_t tail = (int64_t)(bytes - 4 * (size_t)words);
  if (tail > 0) {
    k_fill_zero_u8<<<1, 64, 0, ctx->stream>>>((uint8_t*)p + 4 * words, tail);
    RBF_LAUNCHED(ctx, "k_fill_zero_u8");
  }
  return RBF_OK;
}

// --------------------------------------------------------- kernel timing

void prof_begin(rbf_ctx* ctx, int kind) {
  if (!ctx->prof_on || !ctx->prof_ev[kind]) return;
  const int n = ctx->prof_n[kind];
  if (n >= PROF_CAP) {
    ctx->prof_dropped[kind]++;
    return;
  }
  (void)hipEventRecord(ctx->prof_ev[kind][2 * n], ctx->stream);
}

void prof_end(rbf_ctx* ctx, int kind) {
  if (!ctx->prof_on || !ctx->prof_ev[kind]) return;
  const int n = ctx->prof_n[kind];
  if (n >= PROF_CAP) return;
  (void)hipEventRecord(ctx->prof_ev[kind][2 * n + 1], ctx->stream);
  ctx->prof_n[kind] = n + 1;
}

// ------------------------------------------------------ stable key sort
//
// Items are cut into chunks of SORT_CHUNK. counts[c * nkeys + k] counts key
// k in chunk c; an exclusive scan over (key, chunk) order gives the first
// output slot of each (key, chunk) run; inside a chunk an item's rank among
// equal keys is the number of equal keys before it (LDS compare loop).

constexpr int SORT_CHUNK = 1024;

__global__ void __launch_bounds__(256) k_sort_count(const int32_t* __restrict__ keys,
                                                    int64_t n, int32_t nkeys,
                                                    int32_t* __restrict__ counts) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int64_t c = i / SORT_CHUNK;
  atomicAdd(&counts[c * (int64_t)nkeys + keys[i]], 1);
}

// Exclusive scan of counts in (key-major, chunk-minor) order, in place, in
// three passes: each key's column over the chunks (one thread per key, reads
// coalesced across keys) leaving the key totals in start[k]; a scan of the
// totals; the key bases added back.
__global__ void __launch_bounds__(256) k_sort_colscan(int32_t* __restrict__ counts,
                                                      int64_t nchunks, int32_t nkeys,
                                                      int32_t* __restrict__ start) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= nkeys) return;
  int32_t run = 0;
  for (int64_t c = 0; c < nchunks; ++c) {
    const int32_t v = counts[c * nkeys + k];
    counts[c * nkeys + k] = run;
    run += v;
  }
  start[k] = run;
}

__global__ void __launch_bounds__(256) k_sort_addbase(int32_t* __restrict__ counts, int64_t n,
                                                      int32_t nkeys,
                                                      const int32_t* __restrict__ start) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  counts[e] += start[e % nkeys];
}

__global__ void __launch_bounds__(SORT_CHUNK) k_sort_scatter(const int32_t* __restrict__ keys,
                                                             int64_t n, int32_t nkeys,
                                                             const int32_t* __restrict__ offs,
                                                             int32_t* __restrict__ perm) {
  __shared__ int32_t lk[SORT_CHUNK];
  const int64_t c = blockIdx.x;
  const int64_t i = c * SORT_CHUNK + threadIdx.x;
  const int32_t k = i < n ? keys[i] : -1;
  lk[threadIdx.x] = k;
  __syncthreads();
  if (i >= n) return;
  int r = 0;
  for (int j = 0; j < (int)threadIdx.x; ++j) r += (lk[j] == k);
  perm[offs[c * nkeys + k] + r] = (int32_t)i;
}

// One stable counting sort (chunk counts, their scan, the scatter); the
// count table has nchunks x nkeys entries.
static rbf_status counting_sort(rbf_ctx* ctx, const int32_t* keys, int64_t n, int32_t nkeys,
                                int32_t* perm, int32_t* start) {
  const int64_t nchunks = n > 0 ? ceil_div(n, SORT_CHUNK) : 1;
  rbf_status st;
  int32_t* counts = (int32_t*)ws_get(ctx, WS_SORT2,
                                     sizeof(int32_t) * nchunks * (size_t)nkeys, &st);
  if (!counts) return st;
  RBF_TRY(fill_zero(ctx, counts, sizeof(int32_t) * nchunks * (size_t)nkeys));
  if (n > 0) {
    k_sort_count<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(keys, n, nkeys, counts);
    RBF_LAUNCHED(ctx, "k_sort_count");
  }
  k_sort_colscan<<<ceil_div(nkeys, 256), 256, 0, ctx->stream>>>(counts, nchunks, nkeys, start);
  RBF_LAUNCHED(ctx, "k_sort_colscan");
  k_scan_excl_i32<<<1, 1024, 0, ctx->stream>>>(start, nkeys);
  RBF_LAUNCHED(ctx, "k_scan_excl_i32");
  k_sort_addbase<<<ceil_div(nchunks * (int64_t)nkeys, 256), 256, 0, ctx->stream>>>(
      counts, nchunks * (int64_t)nkeys, nkeys, start);
  RBF_LAUNCHED(ctx, "k_sort_addbase");
  if (n > 0) {
    k_sort_scatter<<<nchunks, SORT_CHUNK, 0, ctx->stream>>>(keys, n, nkeys, counts, perm);
    RBF_LAUNCHED(ctx, "k_sort_scatter");
  }
  return RBF_OK;
}

// Radix passes of a large key space: digits of RADIX_BITS bits.
constexpr int RADIX_BITS = 13;
constexpr int64_t SORT_COUNTS_MAX = (int64_t)1 << 24;  // direct count table limit

__global__ void __launch_bounds__(256) k_sort_digit(const int32_t* __restrict__ keys,
                                                    const int32_t* __restrict__ order,
                                                    int64_t n, int shift,
                                                    int32_t* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  const int32_t k = keys[order ? order[s] : s];
  out[s] = (k >> shift) & ((1 << RADIX_BITS) - 1);
}

__global__ void __launch_bounds__(256) k_sort_compose(const int32_t* __restrict__ p1,
                                                      const int32_t* __restrict__ p2, int64_t n,
                                                      int32_t* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  out[s] = p1[p2[s]];
}

// start[k] = first sorted position whose key is >= k (k = 0..nkeys), by
// binary search over the sorted keys keys[perm[.]].
__global__ void __launch_bounds__(256) k_sort_starts(const int32_t* __restrict__ keys,
                                                     const int32_t* __restrict__ perm,
                                                     int64_t n, int32_t nkeys,
                                                     int32_t* __restrict__ start) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k > nkeys) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[perm[mid]] < k)
      lo = mid + 1;
    else
      hi = mid;
  }
  start[k] = (int32_t)lo;
}

rbf_status stable_key_sort(rbf_ctx* ctx, const int32_t* keys, int64_t n,
                           int32_t nkeys, int32_t* perm, int32_t* start) {
  const int64_t nchunks = n > 0 ? ceil_div(n, SORT_CHUNK) : 1;
  if (nchunks * (int64_t)nkeys <= SORT_COUNTS_MAX || n == 0)
    return counting_sort(ctx, keys, n, nkeys, perm, start);
  // Large key space: least-significant-digit radix sort, each pass a
  // stable counting sort on RADIX_BITS bits, so the result is the same
  // stable order; then the key offsets by binary search.
  if (nkeys > (1 << (2 * RADIX_BITS)))
    return fail(ctx, RBF_E_INVALID_ARG, "stable_key_sort: %d keys exceed the radix range",
                (int)nkeys);
  rbf_status st;
  const size_t nd = ((size_t)1 << RADIX_BITS) + 1;
  int32_t* tmp = (int32_t*)ws_get(ctx, WS_SORT3, sizeof(int32_t) * (3 * (size_t)n + nd), &st);
  if (!tmp) return st;
  int32_t* digit = tmp;
  int32_t* p1 = tmp + n;
  int32_t* p2 = tmp + 2 * n;
  int32_t* dstart = tmp + 3 * n;  // digit offsets of a pass (not needed after it)
  const unsigned gb = (unsigned)ceil_div(n, 256);
  k_sort_digit<<<gb, 256, 0, ctx->stream>>>(keys, nullptr, n, 0, digit);
  RBF_LAUNCHED(ctx, "k_sort_digit");
  RBF_TRY(counting_sort(ctx, digit, n, 1 << RADIX_BITS, p1, dstart));
  k_sort_digit<<<gb, 256, 0, ctx->stream>>>(keys, p1, n, RADIX_BITS, digit);
  RBF_LAUNCHED(ctx, "k_sort_digit");
  RBF_TRY(counting_sort(ctx, digit, n, 1 << RADIX_BITS, p2, dstart));
  k_sort_compose<<<gb, 256, 0, ctx->stream>>>(p1, p2, n, perm);
  RBF_LAUNCHED(ctx, "k_sort_compose");
  k_sort_starts<<<(unsigned)ceil_div((int64_t)nkeys + 1, 256), 256, 0, ctx->stream>>>(
      keys, perm, n, nkeys, start);
  RBF_LAUNCHED(ctx, "k_sort_starts");
  return RBF_OK;
}

rbf_status ensure_aux(rbf_ctx* ctx) {
  if (ctx->aux) return RBF_OK;
  RBF_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_fwd, hipEventDisableTiming));
  RBF_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_back, hipEventDisableTiming));
  RBF_HIP(ctx, hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
  return RBF_OK;
}

}  // namespace rbf

using namespace rbf;

extern "C" {

rbf_status rbf_ctx_create(rbf_ctx** out, int device, void* hip_stream) {
  if (!out) return RBF_E_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return RBF_E_INVALID_ARG;
  rbf_ctx* c = new (std::nothrow) rbf_ctx;
  if (!c) return RBF_E_NOMEM;
  memset(c, 0, sizeof(*c));
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->last_index = -1;
  c->tiles_key = -1;
  c->seq = 1;
  c->single_stream = 1;  // rbf_update on one stream unless asked for two
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return RBF_E_HIP;
  }
  if (eval_scratch_init(device) != RBF_OK) {
    delete c;
    return RBF_E_HIP;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess)
    c->cu_count = cus;
  else
    (void)hipGetLastError();
  if (hipMalloc(&c->d_status, STATUS_WORDS * sizeof(int32_t)) != hipSuccess) {
    delete c;
    return RBF_E_NOMEM;
  }
  if (hipMemset(c->d_status, 0, STATUS_WORDS * sizeof(int32_t)) != hipSuccess) {
    (void)hipFree(c->d_status);
    delete c;
    return RBF_E_HIP;
  }
  *out = c;
  return RBF_OK;
}

rbf_status rbf_ctx_destroy(rbf_ctx* ctx) {
  if (!ctx) return RBF_E_INVALID_ARG;
  // a plan keeps using its context's device and stream until it is
  // destroyed: the context must outlive it
  if (ctx->plans > 0)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_ctx_destroy: %d plan(s) made on this context "
                "are still alive (destroy them first)", (int)ctx->plans);
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->aux) (void)hipStreamSynchronize(ctx->aux);
  for (int i = 0; i < WS_COUNT; ++i)
    if (ctx->ws[i]) (void)hipFree(ctx->ws[i]);
  if (ctx->d_status) (void)hipFree(ctx->d_status);
  if (ctx->owns_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
  if (ctx->ev_fwd) (void)hipEventDestroy(ctx->ev_fwd);
  if (ctx->ev_back) (void)hipEventDestroy(ctx->ev_back);
  for (int k = 0; k < RBF_PROF_KINDS; ++k) {
    if (!ctx->prof_ev[k]) continue;
    for (int e = 0; e < 2 * PROF_CAP; ++e) (void)hipEventDestroy(ctx->prof_ev[k][e]);
    delete[] ctx->prof_ev[k];
  }
  delete ctx;
  return RBF_OK;
}

rbf_status rbf_ctx_set_update_streams(rbf_ctx* ctx, int32_t streams) {
  if (!ctx) return RBF_E_INVALID_ARG;
  if (streams != 1 && streams != 2)
    return fail(ctx, RBF_E_INVALID_ARG, "rbf_ctx_set_update_streams: streams must be 1 or 2");
  ctx->single_stream = streams == 1;
  return RBF_OK;
}

rbf_status rbf_ctx_set_update_joseph(rbf_ctx* ctx, int32_t on) {
  if (!ctx) return RBF_E_INVALID_ARG;
  ctx->joseph = on != 0;
  return RBF_OK;
}

rbf_status rbf_ctx_set_stream(rbf_ctx* ctx, void* hip_stream) {
  if (!ctx) return RBF_E_INVALID_ARG;
  ctx->stream = (hipStream_t)hip_stream;
  return RBF_OK;
}

rbf_status rbf_sync_status(rbf_ctx* ctx) {
  if (!ctx) return RBF_E_INVALID_ARG;
  RBF_TRY(set_device(ctx));
  int32_t h[4];
  RBF_HIP(ctx, hipMemcpyAsync(h, ctx->d_status, sizeof(h), hipMemcpyDeviceToHost,
                              ctx->stream));
  RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h[0] != 0) {
    int64_t idx;
    memcpy(&idx, h + 2, sizeof(idx));
    ctx->last_index = idx;
    RBF_TRY(fill_zero(ctx, ctx->d_status, STATUS_WORDS * sizeof(int32_t)));
    RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return fail(ctx, (rbf_status)h[0], "device error %d (%s) at index %lld", h[0],
                rbf_status_string((rbf_status)h[0]), (long long)idx);
  }
  ctx->last_index = -1;
  return RBF_OK;
}

rbf_status rbf_profile_enable(rbf_ctx* ctx, int32_t enable) {
  if (!ctx) return RBF_E_INVALID_ARG;
  RBF_TRY(set_device(ctx));
  if (enable) {
    for (int k = 0; k < RBF_PROF_KINDS; ++k) {
      if (!ctx->prof_ev[k]) {
        ctx->prof_ev[k] = new (std::nothrow) hipEvent_t[2 * PROF_CAP];
        if (!ctx->prof_ev[k]) return RBF_E_NOMEM;
        for (int e = 0; e < 2 * PROF_CAP; ++e)
          RBF_HIP(ctx, hipEventCreate(&ctx->prof_ev[k][e]));
      }
      ctx->prof_n[k] = 0;
      ctx->prof_dropped[k] = 0;
    }
  }
  ctx->prof_on = enable ? 1 : 0;
  return RBF_OK;
}

rbf_status rbf_profile_read(rbf_ctx* ctx, int32_t kind, double* total_ms, int64_t* launches) {
  if (!ctx || kind < 0 || kind >= RBF_PROF_KINDS || !total_ms || !launches)
    return RBF_E_INVALID_ARG;
  *total_ms = 0.0;
  *launches = 0;
  if (!ctx->prof_ev[kind]) return RBF_OK;
  RBF_TRY(set_device(ctx));
  RBF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  double tot = 0.0;
  for (int e = 0; e < ctx->prof_n[kind]; ++e) {
    float ms = 0.f;
    RBF_HIP(ctx, hipEventElapsedTime(&ms, ctx->prof_ev[kind][2 * e], ctx->prof_ev[kind][2 * e + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *launches = ctx->prof_n[kind];
  ctx->prof_n[kind] = 0;
  ctx->prof_dropped[kind] = 0;
  return RBF_OK;
}

int64_t rbf_last_error_index(const rbf_ctx* ctx) { return ctx ? ctx->last_index : -1; }

const char* rbf_last_error(const rbf_ctx* ctx) { return ctx ? ctx->err : "null context"; }

const char* rbf_status_string(rbf_status s) {
  switch (s) {
    case RBF_OK: return "ok";
    case RBF_E_INVALID_ARG: return "invalid argument";
    case RBF_E_NOMEM: return "out of device memory";
    case RBF_E_NOT_SPD: return "matrix not positive definite";
    case RBF_E_NONFINITE: return "non-finite value";
    case RBF_E_NO_CONVERGE: return "iterative refinement did not converge";
    case RBF_E_CAPACITY: return "output capacity exceeded";
    case RBF_E_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

}  // extern "C"
