// Internal declarations of librbf (gfx950). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "rbf.h"

namespace rbf {

// Workspace slots owned by a context (grow-only device buffers).
enum WsSlot {
  WS_TMP0 = 0,
  WS_TMP1,
  WS_TMP2,
  WS_TMP3,
  WS_SORT0,
  WS_SORT1,
  WS_SORT2,
  WS_SORT3,     // radix passes of stable_key_sort (digits, two permutations)
  WS_POSE,      // evaluation at a pose increment: pose, right Jacobian, gradient
  WS_JOSEPH,    // update, Joseph form: L^{-1}, K^T, FP32 operands
  WS_UPD_ELL,   // update: regressor rows of a batch
  WS_UPD_UT,    // update: U^T then V^T (B x ldu)
  WS_UPD_S,     // update: S then L (B x B)
  WS_UPD_LINV,  // update: inverses of the diagonal blocks of L
  WS_UPD_VLO,   // update: low-precision copy of V^T
  WS_UPD_TILES, // update: SYRK tile schedule
  WS_UPD_UT2,   // update: second U^T / V^T buffer (batches alternate)
  WS_UPD_FLAGS, // update: touched 128-row blocks of P, two batches
  WS_UPD_GROUPS,// update: per 64-row group, the distinct rows of P and dense H
  WS_UPD_VT,    // update: V^T = L^{-1} U^T, two buffers
  WS_ACT_IDX,   // active-rows update: flags / compact map, active list, w_A
  WS_ACT_P,     // active-rows update: compact block P_AA
  WS_SOLVE0,
  WS_SOLVE1,
  WS_SOLVE2,
  WS_SOLVE3,
  WS_SOLVE4,
  WS_SOLVE5,
  WS_SOLVE6,
  WS_SOLVE7,    // solve: L^{-1} of every diagonal block, transposed
  WS_SOLVE8,    // solve: one s x s block, and the second sweep vector
  WS_COUNT
};

}  // namespace rbf

struct rbf_ctx {
  int device;
  hipStream_t stream;
  // d_status (STATUS_WORDS int32): [0] first error code, [1] unused,
  // [2..3] int64 index attached to that error, [4..5] uint64 skip key
  // (see set_status / seq_skip).
  int32_t* d_status;
  // sequence number of the next sequenced launch group (a batch of
  // rbf_update, one rbf_solve); starts at 1
  int64_t seq;
  // second stream of rbf_update (created on first use, non-blocking,
  // default priority) and the two events that order it with `stream`
  hipStream_t aux;
  hipEvent_t ev_fwd, ev_back;
  // rbf_update keeps to one stream (set for the batched form's branches,
  // whose graph capture does not take the two-stream schedule)
  int32_t single_stream;
  // rbf_update applies the covariance update in the Joseph form (FP32
  // products only; rbf_ctx_set_update_joseph)
  int32_t joseph;
  void* ws[rbf::WS_COUNT];
  size_t ws_bytes[rbf::WS_COUNT];
  int64_t last_index;
  char err[512];
  int64_t tiles_key;  // cached SYRK schedule key (N, tile)
  int64_t tiles_count;
  // kernel timing (rbf_profile_*): event pairs per kind
  int32_t prof_on;
  hipEvent_t* prof_ev[RBF_PROF_KINDS];
  int32_t prof_n[RBF_PROF_KINDS];
  int32_t prof_dropped[RBF_PROF_KINDS];
  int32_t owns_stream;  // stream created by the library (batched branches)
  int32_t plans;        // live batched and solve plans made on this context
  int64_t index_base;   // added to the batch index rbf_update records
  int32_t cu_count;     // compute units of the device (0: unknown)
};

struct rbf_grid {
  int device;
  int64_t N;
  double x0, y0, h, inv_h;
  int32_t nbx, nby;
  int32_t max_cand;
  double sigma, cutoff, sigma_eps;
  int32_t* d_start;  // nbins + 1 offsets into the sorted arrays
  int32_t* d_idx;    // sorted position -> original center index
  int32_t* d_rank;   // original center index -> sorted position
  double* d_cxy;     // sorted centers, interleaved (x, y), f64
  float* d_cxyf;     // sorted centers, interleaved (x, y), f32
  // Evaluation bins: side eh of about a third of the evaluation support
  // cutoff*sigma, same origin (x0, y0), row-major; the centers sorted by
  // them give the evaluation kernels short candidate runs per bin row.
  double eh, inv_eh;
  int32_t enbx, enby;
  int32_t* d_estart;  // enbx*enby + 1 offsets into the eval-sorted order
  int32_t* d_eidx;    // eval-sorted position -> original center index
  double* d_ecxy;     // eval-sorted centers, interleaved (x, y), f64
  double box[4];      // center bounding box (min x, min y, max x, max y)
  // Mesh form of the evaluation (rbf_grid_set_mesh): every center is a node
  // (mx0 + i res, my0 + j res). mesh_w = 0: off; else the support window
  // in nodes per axis (4, 8 or 12). The dense node array covers nodes
  // imin - mesh_w .. imin + mnx - 1 + mesh_w (and the same in j), row-major
  // with rows of mpw = mnx + 2 mesh_w; d_mesh_map holds the center of each
  // node or -1.
  int32_t mesh_w;
  double mx0, my0, mres;
  int32_t imin, jmin, mnx, mny, mpw, mph;
  int32_t* d_mesh_map;
  // batched plans that evaluate on this grid (their captured launches keep
  // its tables' addresses and its form): while any is alive the grid's form
  // is fixed and the grid is not destroyed
  int32_t plans;
};

namespace rbf {
// Evaluation bin side in units of the support radius cutoff*sigma: a
// point's support spans at most 7 bin rows (2 * EVAL_BINS_PER_RC /
// (1 + margin) + a pad < 6 bin widths).
constexpr double EVAL_BINS_PER_RC = 3.0;
constexpr double EVAL_BIN_MARGIN = 1.01;
constexpr int EVAL_MAX_ROWS = 8;
// Mesh form: the window of a point is MESH_W nodes per axis from the first
// node within (support radius + MESH_PAD) nodes; the pad absorbs the FP32
// rounding of the node coordinates (at most 2^14 nodes per axis).
constexpr double MESH_PAD = 1.0 / 64.0;
constexpr int MESH_MAX_NODES_AXIS = 1 << 14;
}  // namespace rbf

namespace rbf {

rbf_status fail(rbf_ctx* ctx, rbf_status s, const char* fmt, ...);
void* ws_get(rbf_ctx* ctx, int slot, size_t bytes, rbf_status* st);
rbf_status check_launch(rbf_ctx* ctx, const char* what);
rbf_status set_device(rbf_ctx* ctx);

// Geometry of a grid, passed by value to kernels.
struct GridGeom {
  double x0, y0, inv_h;
  int32_t nbx, nby;
};

inline GridGeom geom(const rbf_grid* g) {
  GridGeom r;
  r.x0 = g->x0;
  r.y0 = g->y0;
  r.inv_h = g->inv_h;
  r.nbx = g->nbx;
  r.nby = g->nby;
  return r;
}

constexpr int STATUS_WORDS = 8;
constexpr uint64_t SEQ_TOP = 1ull << 62;

// Record a device-side error: the first error wins, its index is kept.
// `seq` is the sequence number of the failing launch group (0: an error
// outside any group). The skip key keeps the smallest failing sequence
// number, as SEQ_TOP - seq under an atomic max, so that seq_skip() lets
// the launches of earlier groups still in flight on another stream finish.
__device__ inline void set_status(int32_t* st, int code, int64_t index, int64_t seq = 0) {
  atomicMax(reinterpret_cast<unsigned long long*>(st + 4),
            (unsigned long long)(SEQ_TOP - (uint64_t)seq));
  if (atomicCAS(st, 0, code) == 0) {
    *reinterpret_cast<int64_t*>(st + 2) = index;
  }
}

// True if an error is pending from launch group `seq` or an earlier one
// (or from outside any group): the launches of group `seq` then do nothing.
__device__ inline bool seq_skip(const int32_t* st, int64_t seq) {
  const uint64_t key = *reinterpret_cast<const volatile unsigned long long*>(st + 4);
  return key != 0 && key >= SEQ_TOP - (uint64_t)seq;
}

// Bin range [lo, hi] of the 3x3 neighbourhood of coordinate v, clipped to
// [0, n-1]. Returns false if the neighbourhood misses the grid (or v is not
// finite), in which case no center can be within the kernel support.
__device__ inline bool bin_range(double v, double o, double inv_h, int n,
                                 int* lo, int* hi) {
  double f = (v - o) * inv_h;
  if (!(f >= -1.0 && f < (double)n + 1.0)) return false;
  int b = (int)floor(f);
  *lo = b - 1 < 0 ? 0 : b - 1;
  *hi = b + 1 > n - 1 ? n - 1 : b + 1;
  return *lo <= *hi;
}

// Bin of coordinate v clamped to [0, n-1] (non-finite -> 0).
__device__ inline int bin_of(double v, double o, double inv_h, int n) {
  double f = (v - o) * inv_h;
  if (!(f >= 0.0)) return 0;
  if (f >= (double)n) return n - 1;
  return (int)f;
}

// Single-workgroup exclusive scan (1024 threads) of n int64 counts in place;
// out[n] receives the total. Used for small scans (bins, rows).
__global__ void k_scan_excl_i64(int64_t* data, int64_t n);
__global__ void k_scan_excl_i32(int32_t* data, int64_t n);

// Kernel timing: record the opening / closing event of one timed launch.
constexpr int PROF_CAP = 4096;  // event pairs kept per kind between reads
void prof_begin(rbf_ctx* ctx, int kind);
void prof_end(rbf_ctx* ctx, int kind);

// Zero device memory with a kernel (no memset node, so the call is safe
// inside stream capture).
rbf_status fill_zero(rbf_ctx* ctx, void* p, size_t bytes);

// Workspace of an evaluation on grid g (the packed center table); the
// batched plan reserves it before capture.
rbf_status eval_workspace(rbf_ctx* ctx, const rbf_grid* g);

// Look up, once per device (that device current), the device address of
// the scratch table of rbf_eval_noalloc; called by rbf_ctx_create.
rbf_status eval_scratch_init(int device);

// Create the context's second stream and its two events if not yet done.
rbf_status ensure_aux(rbf_ctx* ctx);

// Enqueue on another stream of the context for the lifetime of the guard:
// every helper launches on ctx->stream, which the guard swaps and restores.
struct StreamSwap {
  rbf_ctx* ctx;
  hipStream_t saved;
  StreamSwap(rbf_ctx* c, hipStream_t s) : ctx(c), saved(c->stream) { c->stream = s; }
  ~StreamSwap() { ctx->stream = saved; }
  StreamSwap(const StreamSwap&) = delete;
  StreamSwap& operator=(const StreamSwap&) = delete;
};

// Stable sort by a precomputed key in [0, nkeys): writes perm (sorted
// position -> item) and start (nkeys + 1 offsets). One counting sort when
// its count table (one row of nkeys per 1024 items) is small, else two
// 13-bit radix passes (nkeys <= 2^26). start holds nkeys + 1 entries.
rbf_status stable_key_sort(rbf_ctx* ctx, const int32_t* keys, int64_t n,
                           int32_t nkeys, int32_t* perm, int32_t* start);

}  // namespace rbf

#define RBF_HIP(ctx, call)                                               \
  do {                                                                   \
    hipError_t e_ = (call);                                              \
    if (e_ != hipSuccess)                                                \
      return ::rbf::fail((ctx), RBF_E_HIP, "%s failed: %s", #call,       \
                         hipGetErrorString(e_));                         \
  } while (0)

#define RBF_TRY(expr)                 \
  do {                                \
    rbf_status s_ = (expr);           \
    if (s_ != RBF_OK) return s_;      \
  } while (0)

#define RBF_LAUNCHED(ctx, what) RBF_TRY(::rbf::check_launch((ctx), (what)))

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
