// Covariance product P -= V V^T on MFMA (the dominant step of the recursive
// update, eq. H_inverse_update in Kalman form).
//
// V^T (Bc x N) is read as two 128-column panels per 128x128 output tile;
// only tiles on or below the diagonal are computed and each result is
// written to both triangles, which keeps P exactly symmetric. Tiles are
// assigned so that each XCD works through a contiguous run of the tile
// list (neighbouring tiles share V^T panels in that XCD's L2).
//
// Lane layouts (v_mfma_f64_16x16x4_f64, checked on gfx950):
//   A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
//   D[i][j] in lane j + 16 (i % 4), item i / 4.
#include "update.hpp"

namespace rbf {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int ST = SYRK_TILE;  // output tile
constexpr int SKC = 16;     // rows of V^T per LDS stage
constexpr int SLD = ST + 8; // LDS pitch (doubles)

__device__ inline void tile_of(int64_t t, int* I, int* J) {
  int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(i + 1) * (i + 2) / 2 <= t) ++i;
  while ((int64_t)i * (i + 1) / 2 > t) --i;
  *I = i;
  *J = (int)(t - (int64_t)i * (i + 1) / 2);
}

// Lower tile t of an nt x nt tile grid in blocked order: bands of 8 tile
// rows, each band's full 8-column blocks left to right, then its diagonal
// triangle; tiles row by row inside a block. Consecutive tiles (those a
// round of workgroups of one XCD runs together) then share 16 panels of
// V^T instead of one row panel and 64 column panels.
__device__ inline void tile_of_blocked(int64_t t, int nt, int* I, int* J) {
  int b = (int)((sqrt(16.0 + 128.0 * (double)t) - 4.0) / 64.0);
  while (32 * (int64_t)(b + 1) * (b + 1) + 4 * (int64_t)(b + 1) <= t) ++b;
  while (32 * (int64_t)b * b + 4 * (int64_t)b > t) --b;
  const int r = (int)(t - (32 * (int64_t)b * b + 4 * (int64_t)b));
  const int h = min(8, nt - 8 * b);
  if (r < b * 8 * h) {
    const int bj = r / (8 * h), q = r % (8 * h);
    *I = 8 * b + q / 8;
    *J = 8 * bj + q % 8;
    return;
  }
  const int q = r - b * 8 * h;
  int i = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= q) ++i;
  while (i * (i + 1) / 2 > q) --i;
  *I = 8 * b + i;
  *J = 8 * b + (q - i * (i + 1) / 2);
}

// Tile filter of a split product: part 0 all tiles, part 1 the tiles in a
// flagged block row or column, part 2 the others.
__device__ inline bool tile_in_part(const int32_t* __restrict__ flags, int part, int I, int J) {
  if (part == 0) return true;
  const bool f = flags[I] != 0 || flags[J] != 0;
  return part == 1 ? f : !f;
}

// Workgroup bid (consecutive workgroups go to the 8 XCDs in turn) takes
// local tile bid >> 3 of the run of XCD bid & 7.
__device__ inline int64_t xcd_tile(int64_t bid, int64_t per_xcd) {
  return (bid & 7) * per_xcd + (bid >> 3);
}

// Stage loader of the FP64 product: the 16 x 128 panel slice (rows r0.. of
// V^T, columns c0..) as 4 double2 per thread; element pair i*256 + tid sits
// at row (i*256 + tid) / 64, column 2 ((i*256 + tid) % 64), so one wave
// reads one 1 KB row run and writes it to LDS with 16-byte stores that touch
// every bank once (zero outside [0, N) x [0, K)).
// W = 64: the 16 x 64 slice of a 64-column panel, the same way (one wave
// covers two rows).
template <int NT, int W = 128>
__device__ inline void load_stage(const double* __restrict__ Ut, int64_t ldu, int64_t N, int r0,
                                  int K, int64_t c0, double2 v[16 * W / 2 / NT]) {
  constexpr int H = W / 2;  // double2 per row
  const int tid = threadIdx.x;
  if (r0 + 16 <= K && c0 + W <= N) {  // whole slice inside: no per-load tests
#pragma unroll
    for (int i = 0; i < 16 * H / NT; ++i) {
      const int e = i * NT + tid;
      v[i] = *reinterpret_cast<const double2*>(Ut + (int64_t)(r0 + e / H) * ldu + c0 +
                                               2 * (e % H));
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 16 * H / NT; ++i) {
    const int e = i * NT + tid;
    const int r = r0 + e / H;
    const int64_t c = c0 + 2 * (e % H);
    v[i].x = (r < K && c < N) ? Ut[(int64_t)r * ldu + c] : 0.0;
    v[i].y = (r < K && c + 1 < N) ? Ut[(int64_t)r * ldu + c + 1] : 0.0;
  }
}

template <int NT, int LD, int W = 128>
__device__ inline void store_stage(double (*X)[LD], const double2 v[16 * W / 2 / NT]) {
  constexpr int H = W / 2;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 16 * H / NT; ++i) {
    const int e = i * NT + tid;
    *reinterpret_cast<double2*>(&X[e / H][2 * (e % H)]) = v[i];
  }
}

// 128x128 tile per workgroup of 8 waves (4 x 2, each 32 x 64 = 2 x 4 MFMA
// blocks), two workgroups per CU: four waves per SIMD hide the LDS and
// barrier latency of each 16-deep stage.
constexpr int SYRK_NT = 512;

__device__ __forceinline__ void syrk_f64_body(double* __restrict__ P, int64_t ldp, int64_t N,
    const double* __restrict__ Ut, int64_t ldu, int32_t K, int64_t T, int64_t per_xcd,
    const int32_t* __restrict__ flags, int part, const int32_t* __restrict__ status, int64_t seq,
    int64_t bid) {
  if (seq_skip(status, seq)) return;
  const int64_t t = xcd_tile(bid, per_xcd);
  if (t >= T) return;
  int I, J;
  tile_of_blocked(t, (int)((N + ST - 1) / ST), &I, &J);
  if (!tile_in_part(flags, part, I, J)) return;
  const int64_t I0 = (int64_t)I * ST, J0 = (int64_t)J * ST;
  __shared__ double As[2][SKC][SLD];
  __shared__ double Bs[2][SKC][SLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // rows wm*32.., columns wn*64..
  v4d acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  const int nch = (K + SKC - 1) / SKC;
  double2 ra[1024 / SYRK_NT], rb[1024 / SYRK_NT];
  load_stage<SYRK_NT>(Ut, ldu, N, 0, K, I0, ra);
  load_stage<SYRK_NT>(Ut, ldu, N, 0, K, J0, rb);
  store_stage<SYRK_NT, SLD>(As[0], ra);
  store_stage<SYRK_NT, SLD>(Bs[0], rb);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) {
      load_stage<SYRK_NT>(Ut, ldu, N, (ch + 1) * SKC, K, I0, ra);
      load_stage<SYRK_NT>(Ut, ldu, N, (ch + 1) * SKC, K, J0, rb);
    }
#pragma unroll
    for (int kk = 0; kk < SKC; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a[2], b[4];
#pragma unroll
      for (int q = 0; q < 2; ++q) a[q] = As[buf][kr][wm * 32 + q * 16 + (lane & 15)];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = Bs[buf][kr][wn * 64 + q * 16 + (lane & 15)];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
    if (ch + 1 < nch) {
      store_stage<SYRK_NT, SLD>(As[buf ^ 1], ra);
      store_stage<SYRK_NT, SLD>(Bs[buf ^ 1], rb);
    }
    __syncthreads();
  }
  // epilogue: P[gi][gj] -= C (lower tiles; diagonal tiles keep gi >= gj so
  // each element is written once), then the mirror P[gj][gi]. The mirror
  // goes through LDS (the stage buffer, free now) 32 columns at a time, so
  // each of its rows is written as one coalesced 1 KB run rather than in
  // 32-byte pieces of 16 rows per store instruction.
  const bool diag = (I == J);
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = I0 + wm * 32 + mi * 16 + 4 * v + (lane >> 4);
        const int64_t gj = J0 + wn * 64 + ni * 16 + (lane & 15);
        if (gi < N && gj < N && (!diag || gi >= gj)) {
          const double nv = P[gi * ldp + gj] - acc[mi][ni][v];
          P[gi * ldp + gj] = nv;
          acc[mi][ni][v] = nv;
        }
      }
  constexpr int MP = ST + 1;  // pitch of the transposed chunk (doubles)
  static_assert(32 * MP <= 2 * SKC * SLD, "a 32-column chunk fits the stage buffer");
  double (*Tm)[MP] = reinterpret_cast<double (*)[MP]>(&As[0][0][0]);
#pragma unroll
  for (int q = 0; q < ST / 32; ++q) {
    if (wn == q / 2) {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nn = 0; nn < 2; ++nn)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int ni = 2 * (q % 2) + nn;
            const int c = ni * 16 + (lane & 15) - 32 * (q % 2);  // column in the chunk
            const int r = wm * 32 + mi * 16 + 4 * v + (lane >> 4);
            Tm[c][r] = acc[mi][ni][v];
          }
    }
    __syncthreads();
    for (int e = tid; e < 32 * ST; e += SYRK_NT) {
      const int c = e / ST, r = e % ST;
      const int64_t gr = J0 + 32 * q + c, gc = I0 + r;  // mirror of (gc, gr)
      if (gr < N && gc < N && (!diag || gc > gr)) P[gr * ldp + gc] = Tm[c][r];
    }
    __syncthreads();  // the chunk is read before the next one is written
  }
}

__global__ void __launch_bounds__(SYRK_NT, 2) k_syrk_f64(double* __restrict__ P, int64_t ldp,
    int64_t N, const double* __restrict__ Ut, int64_t ldu, int32_t K, int64_t T, int64_t per_xcd,
    const int32_t* __restrict__ flags, int part, const int32_t* __restrict__ status, int64_t seq) {
  syrk_f64_body(P, ldp, N, Ut, ldu, K, T, per_xcd, flags, part, status, seq, blockIdx.x);
}

// Tail of the FP64 product. A launch of 128x128 tiles runs in rounds of
// (workgroups per CU x CUs per XCD) tiles per XCD; the tiles past the last
// full round would leave most CUs idle while they finish. They are computed
// instead as 32x64 sub-tiles by this kernel, eight per tile (six on the
// diagonal: the two above it are mirrors), each on 8 waves of 16 x 16 (one
// MFMA block): many short workgroups spread the leftover work over the
// chip and keep several waves per SIMD to hide the short stages' loads.
// Every element accumulates the same MFMAs over k in the same order as in
// the 128x128 kernel, so the result is bit for bit the same. Local tiles
// main_per_xcd .. per_xcd - 1 of each XCD.
constexpr int SUB_M = 32;
constexpr int SUB_N = 64;
constexpr int SUB_NT = 512;
constexpr int SUB_PER_TILE = (ST / SUB_M) * (ST / SUB_N);

__device__ __forceinline__ void syrk_f64_tail_body(double* __restrict__ P, int64_t ldp, int64_t N,
    const double* __restrict__ Ut, int64_t ldu, int32_t K, int64_t T, int64_t per_xcd,
    int64_t main_per_xcd, const int32_t* __restrict__ flags, int part,
    const int32_t* __restrict__ status, int64_t seq, int64_t bid) {
  if (seq_skip(status, seq)) return;
  const int64_t local = main_per_xcd + (bid >> 3) / SUB_PER_TILE;
  const int sub = (int)((bid >> 3) % SUB_PER_TILE);
  const int si = sub / (ST / SUB_N), sj = sub % (ST / SUB_N);
  if (local >= per_xcd) return;
  const int64_t t = (bid & 7) * per_xcd + local;
  if (t >= T) return;
  int I, J;
  tile_of_blocked(t, (int)((N + ST - 1) / ST), &I, &J);
  if (!tile_in_part(flags, part, I, J)) return;
  if (I == J && si * SUB_M + SUB_M - 1 < sj * SUB_N) return;  // above the diagonal
  const int64_t I0 = (int64_t)I * ST + si * SUB_M, J0 = (int64_t)J * ST + sj * SUB_N;
  if (I0 >= N || J0 >= N) return;
  __shared__ double As[2][SKC][SUB_M + 8];
  __shared__ double Bs[2][SKC][SUB_N + 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;  // rows wm*16.., columns wn*16..
  v4d acc = (v4d){0.0, 0.0, 0.0, 0.0};
  const int nch = (K + SKC - 1) / SKC;
  // a stage: the 16 x 32 slice of the row panel (threads 0-255, one double2
  // each) and the 16 x 64 slice of the column panel (all 512 threads)
  constexpr int NA = SUB_NT / 2;
  double2 ra[1], rb[1];
  if (tid < NA) load_stage<NA, SUB_M>(Ut, ldu, N, 0, K, I0, ra);
  load_stage<SUB_NT, SUB_N>(Ut, ldu, N, 0, K, J0, rb);
  if (tid < NA) store_stage<NA, SUB_M + 8, SUB_M>(As[0], ra);
  store_stage<SUB_NT, SUB_N + 8, SUB_N>(Bs[0], rb);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) {
      if (tid < NA) load_stage<NA, SUB_M>(Ut, ldu, N, (ch + 1) * SKC, K, I0, ra);
      load_stage<SUB_NT, SUB_N>(Ut, ldu, N, (ch + 1) * SKC, K, J0, rb);
    }
#pragma unroll
    for (int kk = 0; kk < SKC; kk += 4) {
      const int kr = kk + (lane >> 4);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(As[buf][kr][wm * 16 + (lane & 15)],
                                                 Bs[buf][kr][wn * 16 + (lane & 15)], acc, 0,
                                                 0, 0);
    }
    if (ch + 1 < nch) {
      if (tid < NA) store_stage<NA, SUB_M + 8, SUB_M>(As[buf ^ 1], ra);
      store_stage<SUB_NT, SUB_N + 8, SUB_N>(Bs[buf ^ 1], rb);
    }
    __syncthreads();
  }
  const bool diag = (I == J);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t gi = I0 + wm * 16 + 4 * v + (lane >> 4);
    const int64_t gj = J0 + wn * 16 + (lane & 15);
    if (gi < N && gj < N && (!diag || gi >= gj)) {
      const double nv = P[gi * ldp + gj] - acc[v];
      P[gi * ldp + gj] = nv;
      if (gi != gj) P[gj * ldp + gi] = nv;
    }
  }
}

__global__ void __launch_bounds__(SUB_NT) k_syrk_f64_tail(double* __restrict__ P, int64_t ldp,
    int64_t N, const double* __restrict__ Ut, int64_t ldu, int32_t K, int64_t T, int64_t per_xcd,
    int64_t main_per_xcd, const int32_t* __restrict__ flags, int part,
    const int32_t* __restrict__ status, int64_t seq) {
  syrk_f64_tail_body(P, ldp, N, Ut, ldu, K, T, per_xcd, main_per_xcd, flags, part, status, seq,
    blockIdx.x);
}

// Triangular solve of the update as one product: V^T = X U^T with
// X = L^{-1} (block lower triangular, held transposed in LiT[k][row],
// leading dimension n, zero above its diagonal blocks) and U^T (n x ncols,
// leading dimension ldu). Same 128x128 tile, stage loader and MFMA layout
// as k_syrk_f64; the k-range of row block I stops at its last row
// ((I + 1) * 128), where X is zero beyond. Heavier row blocks are issued
// first.
// UPPER: X upper triangular instead (the operand holds X transposed all
// the same), the k-range of row block I starting at its first row.
template <bool UPPER>
__device__ __forceinline__ void linv_apply_body(const double* __restrict__ LiT,
    int32_t n, const double* __restrict__ Ut, int64_t ldu, int64_t ncols, double* __restrict__ Vt,
    int32_t nJ, const int32_t* __restrict__ status, int64_t seq) {
  if (seq_skip(status, seq)) return;
  const int nI = (n + ST - 1) / ST;
  const int I = UPPER ? (int)(blockIdx.x / nJ) : nI - 1 - (int)(blockIdx.x / nJ);
  const int J = (int)(blockIdx.x % nJ);
  const int64_t I0 = (int64_t)I * ST, J0 = (int64_t)J * ST;
  const int kb = UPPER ? I * ST : 0;  // first k of the row block (a multiple of SKC)
  const int K = UPPER ? n : min(n, (I + 1) * ST);
  __shared__ double As[2][SKC][SLD];
  __shared__ double Bs[2][SKC][SLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  v4d acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  const int nch = (K - kb + SKC - 1) / SKC;
  double2 ra[1024 / SYRK_NT], rb[1024 / SYRK_NT];
  load_stage<SYRK_NT>(LiT, n, n, kb, K, I0, ra);
  load_stage<SYRK_NT>(Ut, ldu, ncols, kb, K, J0, rb);
  store_stage<SYRK_NT, SLD>(As[0], ra);
  store_stage<SYRK_NT, SLD>(Bs[0], rb);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) {
      load_stage<SYRK_NT>(LiT, n, n, kb + (ch + 1) * SKC, K, I0, ra);
      load_stage<SYRK_NT>(Ut, ldu, ncols, kb + (ch + 1) * SKC, K, J0, rb);
    }
#pragma unroll
    for (int kk = 0; kk < SKC; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a[2], b[4];
#pragma unroll
      for (int q = 0; q < 2; ++q) a[q] = As[buf][kr][wm * 32 + q * 16 + (lane & 15)];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = Bs[buf][kr][wn * 64 + q * 16 + (lane & 15)];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
    if (ch + 1 < nch) {
      store_stage<SYRK_NT, SLD>(As[buf ^ 1], ra);
      store_stage<SYRK_NT, SLD>(Bs[buf ^ 1], rb);
    }
    __syncthreads();
  }
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = I0 + wm * 32 + mi * 16 + 4 * v + (lane >> 4);
        const int64_t gj = J0 + wn * 64 + ni * 16 + (lane & 15);
        if (gi < n && gj < ncols) Vt[gi * ldu + gj] = acc[mi][ni][v];
      }
}

template <bool UPPER>
__global__ void __launch_bounds__(SYRK_NT, 2) k_linv_apply(const double* __restrict__ LiT,
    int32_t n, const double* __restrict__ Ut, int64_t ldu, int64_t ncols, double* __restrict__ Vt,
    int32_t nJ, const int32_t* __restrict__ status, int64_t seq) {
  linv_apply_body<UPPER>(LiT, n, Ut, ldu, ncols, Vt, nJ, status, seq);
}

// ------------------------------------------------ low-precision operands
//
// FP32: V^T is rounded to float (same k-major layout) and multiplied on
// v_mfma_f32_16x16x4_f32. BF16: V = V_hi + V_lo with V_hi = bf16(V) and
// V_lo = bf16(V - V_hi), stored i-major (N x Kp) so a lane reads its 8
// consecutive k values with one 16-byte load, and V V^T is formed as
// V_hi V_hi^T + V_hi V_lo^T + V_lo V_hi^T on v_mfma_f32_16x16x32_bf16. Both
// accumulate in FP32 and subtract from the FP64 P with the same mirrored
// write as the FP64 kernel.
// Lane layout of both FP32-accumulating instructions (checked on gfx950):
// D[i][j] in lane j + 16 (i / 4), item i % 4.

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void cvt_f32_body(const double* __restrict__ Ut, int64_t ldu, int32_t K,
    int64_t N, float* __restrict__ Uf, const int32_t* __restrict__ status, int64_t seq) {
  if (seq_skip(status, seq)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)K * ldu) return;
  const int64_t c = e % ldu;
  Uf[e] = c < N ? (float)Ut[e] : 0.0f;
}

__global__ void __launch_bounds__(256) k_cvt_f32(const double* __restrict__ Ut, int64_t ldu,
    int32_t K, int64_t N, float* __restrict__ Uf, const int32_t* __restrict__ status, int64_t seq) {
  cvt_f32_body(Ut, ldu, K, N, Uf, status, seq);
}

// Transposing split: Vhi[n][k], Vlo[n][k] (ld Kp) from U^T[k][n]; 64x64
// tiles through LDS; k >= K and n >= N are zero.
__device__ __forceinline__ void cvt_bf16x2_body(const double* __restrict__ Ut, int64_t ldu,
    int32_t K, int64_t N, int32_t Kp, __bf16* __restrict__ Vhi, __bf16* __restrict__ Vlo,
    const int32_t* __restrict__ status, int64_t seq) {
  if (seq_skip(status, seq)) return;
  __shared__ double t[64][65];
  const int64_t n0 = (int64_t)blockIdx.x * 64;
  const int k0 = blockIdx.y * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int kk = e >> 6, nn = e & 63;
    const int64_t gk = k0 + kk, gn = n0 + nn;
    t[kk][nn] = (gk < K && gn < N) ? Ut[gk * ldu + gn] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int nn = e >> 6, kk = e & 63;
    const int64_t gn = n0 + nn, gk = k0 + kk;
    if (gn < N && gk < Kp) {
      const double v = t[kk][nn];
      const __bf16 hi = (__bf16)v;
      const __bf16 lo = (__bf16)(v - (double)(float)hi);
      Vhi[gn * Kp + gk] = hi;
      Vlo[gn * Kp + gk] = lo;
    }
  }
}

__global__ void __launch_bounds__(256) k_cvt_bf16x2(const double* __restrict__ Ut, int64_t ldu,
    int32_t K, int64_t N, int32_t Kp, __bf16* __restrict__ Vhi, __bf16* __restrict__ Vlo,
    const int32_t* __restrict__ status, int64_t seq) {
  cvt_bf16x2_body(Ut, ldu, K, N, Kp, Vhi, Vlo, status, seq);
}

// P -= C (FP32 accumulators) for the 8-wave layout (wave: rows wm*32 +
// 2 x 16, columns wn*64 + 4 x 16), written to both triangles as in the FP64
// kernel.
//
// BATCH: per half, the P values are loaded, then all new values formed,
// then the stores. Element by element, a load that follows a store to P
// may alias it, so the compiler waits out a memory round trip per element;
// the loads (this thread's lower elements) and the stores (the same
// elements and their upper mirrors) never overlap, and each element's
// arithmetic is the same. It pays in the BF16x3 kernel (0.63 -> 0.54 ms per
// product at N = 10,000); the FP32 and FP64 kernels, MFMA-bound with
// registers to the limit, were slower with it and keep the element order.
template <bool BATCH>
__device__ inline void epilogue_f32acc_w8(double* __restrict__ P, int64_t ldp, int64_t N,
                                          int64_t I0, int64_t J0, bool diag,
                                          const v4f acc[2][4], double sgn = 1.0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  if (!BATCH) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 4; ++ni)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t gi = I0 + wm * 32 + mi * 16 + 4 * (lane >> 4) + v;
          const int64_t gj = J0 + wn * 64 + ni * 16 + (lane & 15);
          if (gi < N && gj < N && (!diag || gi >= gj)) {
            const double nv = P[gi * ldp + gj] - sgn * (double)acc[mi][ni][v];
            P[gi * ldp + gj] = nv;
            if (gi != gj) P[gj * ldp + gi] = nv;
          }
        }
    return;
  }
#pragma unroll
  for (int mi = 0; mi < 2; ++mi) {
    double pv[4][4];
#pragma unroll
    for (int ni = 0; ni < 4; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = I0 + wm * 32 + mi * 16 + 4 * (lane >> 4) + v;
        const int64_t gj = J0 + wn * 64 + ni * 16 + (lane & 15);
        pv[ni][v] = (gi < N && gj < N && (!diag || gi >= gj)) ? P[gi * ldp + gj] : 0.0;
      }
#pragma unroll
    for (int ni = 0; ni < 4; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        pv[ni][v] -= (double)acc[mi][ni][v];
        // keeps the subtraction from moving down into its store's branch
        asm volatile("" : "+v"(pv[ni][v]));
      }
#pragma unroll
    for (int ni = 0; ni < 4; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = I0 + wm * 32 + mi * 16 + 4 * (lane >> 4) + v;
        const int64_t gj = J0 + wn * 64 + ni * 16 + (lane & 15);
        if (gi < N && gj < N && (!diag || gi >= gj)) {
          P[gi * ldp + gj] = pv[ni][v];
          if (gi != gj) P[gj * ldp + gi] = pv[ni][v];
        }
      }
  }
}

constexpr int FKC = 32;      // rows of V^T per stage (FP32)
constexpr int FLD = ST + 4;  // LDS pitch (floats)

// Stage loader of the FP32 product: the 32 x 128 slice as 4 float4 per
// thread; float4 i*256 + tid sits at row (i*256 + tid) / 32, column
// 4 ((i*256 + tid) % 32), so half a wave reads one 512-byte row run and
// writes it with 16-byte stores (zero outside [0, N) x [0, K)).
template <int NT>
__device__ inline void load_stage_f32(const float* __restrict__ Uf, int64_t ldu, int64_t N,
                                      int r0, int K, int64_t c0, float4 v[1024 / NT]) {
  const int tid = threadIdx.x;
  if (r0 + FKC <= K && c0 + 128 <= N) {
#pragma unroll
    for (int i = 0; i < 1024 / NT; ++i) {
      const int e = i * NT + tid;
      v[i] = *reinterpret_cast<const float4*>(Uf + (int64_t)(r0 + (e >> 5)) * ldu + c0 +
                                              4 * (e & 31));
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 1024 / NT; ++i) {
    const int e = i * NT + tid;
    const int r = r0 + (e >> 5);
    const int64_t c = c0 + 4 * (e & 31);
    const float* src = Uf + (int64_t)r * ldu + c;
    v[i].x = (r < K && c < N) ? src[0] : 0.f;
    v[i].y = (r < K && c + 1 < N) ? src[1] : 0.f;
    v[i].z = (r < K && c + 2 < N) ? src[2] : 0.f;
    v[i].w = (r < K && c + 3 < N) ? src[3] : 0.f;
  }
}

template <int NT>
__device__ inline void store_stage_f32(float (*X)[FLD], const float4 v[1024 / NT]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 1024 / NT; ++i) {
    const int e = i * NT + tid;
    *reinterpret_cast<float4*>(&X[e >> 5][4 * (e & 31)]) = v[i];
  }
}

// P -= sgn X1 X2^T on the lower tiles, mirrored (X2 = X1 unless given:
// the product is symmetric in every use).
__device__ __forceinline__ void syrk_f32_body(double* __restrict__ P, int64_t ldp, int64_t N,
    const float* __restrict__ Uf, int64_t ldu, int32_t K, int64_t T, int64_t per_xcd,
    const int32_t* __restrict__ flags, int part, const int32_t* __restrict__ status, int64_t seq,
    const float* __restrict__ Uf2, double sgn, int64_t bid) {
  const float* __restrict__ Ub = Uf2 ? Uf2 : Uf;
  if (seq_skip(status, seq)) return;
  const int64_t t = xcd_tile(bid, per_xcd);
  if (t >= T) return;
  int I, J;
  tile_of_blocked(t, (int)((N + ST - 1) / ST), &I, &J);
  if (!tile_in_part(flags, part, I, J)) return;
  const int64_t I0 = (int64_t)I * ST, J0 = (int64_t)J * ST;
  __shared__ __attribute__((aligned(16))) float As[2][FKC][FLD];
  __shared__ __attribute__((aligned(16))) float Bs[2][FKC][FLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // rows wm*32.., columns wn*64..
  v4f acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
  const int nch = (K + FKC - 1) / FKC;
  float4 ra[1024 / SYRK_NT], rb[1024 / SYRK_NT];
  load_stage_f32<SYRK_NT>(Uf, ldu, N, 0, K, I0, ra);
  load_stage_f32<SYRK_NT>(Ub, ldu, N, 0, K, J0, rb);
  store_stage_f32<SYRK_NT>(As[0], ra);
  store_stage_f32<SYRK_NT>(Bs[0], rb);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) {
      load_stage_f32<SYRK_NT>(Uf, ldu, N, (ch + 1) * FKC, K, I0, ra);
      load_stage_f32<SYRK_NT>(Ub, ldu, N, (ch + 1) * FKC, K, J0, rb);
    }
#pragma unroll
    for (int kk = 0; kk < FKC; kk += 4) {
      const int kr = kk + (lane >> 4);
      float a[2], b[4];
#pragma unroll
      for (int q = 0; q < 2; ++q) a[q] = As[buf][kr][wm * 32 + q * 16 + (lane & 15)];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = Bs[buf][kr][wn * 64 + q * 16 + (lane & 15)];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
    if (ch + 1 < nch) {
      store_stage_f32<SYRK_NT>(As[buf ^ 1], ra);
      store_stage_f32<SYRK_NT>(Bs[buf ^ 1], rb);
    }
    __syncthreads();
  }
  epilogue_f32acc_w8<false>(P, ldp, N, I0, J0, I == J, acc, sgn);
}

__global__ void __launch_bounds__(SYRK_NT, 2) k_syrk_f32(double* __restrict__ P, int64_t ldp,
    int64_t N, const float* __restrict__ Uf, int64_t ldu, int32_t K, int64_t T, int64_t per_xcd,
    const int32_t* __restrict__ flags, int part, const int32_t* __restrict__ status, int64_t seq,
    const float* __restrict__ Uf2 = nullptr, double sgn = 1.0) {
  syrk_f32_body(P, ldp, N, Uf, ldu, K, T, per_xcd, flags, part, status, seq, Uf2, sgn, blockIdx.x);
}

constexpr int BKC = SYRK_BF16_KSTEP;  // k per stage (two 16x16x32 MFMA steps)
constexpr int BLD = BKC + 8; // LDS pitch in bf16 (144 bytes)

// One thread's share of a BF16 stage (8-wave layout: 4 threads per row of
// 64 k values, two 16-byte pieces each, at k0 and k0 + 32): row ga (I panel)
// and gb (J panel) of V_hi and V_lo. Rows beyond N read row N-1 (in bounds)
// and are zeroed by a mask, so no pointer is selected (a select between a
// global and a local address made the loads generic and put a zero on the
// stack).
struct Bf16Stage {
  uint4 ah[2], al[2], bh[2], bl[2];
};

__device__ __forceinline__ void mask4(uint4& v, uint32_t m) {
  v.x &= m; v.y &= m; v.z &= m; v.w &= m;
}

__device__ __forceinline__ void load_bf16_stage(const __bf16* __restrict__ Vhi,
                                                const __bf16* __restrict__ Vlo, int32_t Kp,
                                                int64_t N, int64_t ga, int64_t gb, int64_t k0,
                                                Bf16Stage& r) {
  const int64_t ra = ga < N ? ga : N - 1, rb = gb < N ? gb : N - 1;
  const uint32_t ma = ga < N ? 0xffffffffu : 0u, mb = gb < N ? 0xffffffffu : 0u;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t k = k0 + 32 * h;
    r.ah[h] = *reinterpret_cast<const uint4*>(Vhi + ra * Kp + k);
    r.al[h] = *reinterpret_cast<const uint4*>(Vlo + ra * Kp + k);
    r.bh[h] = *reinterpret_cast<const uint4*>(Vhi + rb * Kp + k);
    r.bl[h] = *reinterpret_cast<const uint4*>(Vlo + rb * Kp + k);
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    mask4(r.ah[h], ma); mask4(r.al[h], ma);
    mask4(r.bh[h], mb); mask4(r.bl[h], mb);
  }
}

__device__ __forceinline__ void syrk_bf16x3_body(double* __restrict__ P, int64_t ldp, int64_t N,
    const __bf16* __restrict__ Vhi, const __bf16* __restrict__ Vlo, int32_t Kp, int64_t T,
    int64_t per_xcd, const int32_t* __restrict__ flags, int part,
    const int32_t* __restrict__ status, int64_t seq, int64_t bid) {
  if (seq_skip(status, seq)) return;
  const int64_t t = xcd_tile(bid, per_xcd);
  if (t >= T) return;
  int I, J;
  tile_of_blocked(t, (int)((N + ST - 1) / ST), &I, &J);
  if (!tile_in_part(flags, part, I, J)) return;
  const int64_t I0 = (int64_t)I * ST, J0 = (int64_t)J * ST;
  __shared__ __attribute__((aligned(16))) __bf16 Ah[ST][BLD];
  __shared__ __attribute__((aligned(16))) __bf16 Al[ST][BLD];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[ST][BLD];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[ST][BLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // rows wm*32.., columns wn*64..
  const int lrow = tid >> 2, lq = (tid & 3) * 8;  // loader: row, first k of the piece
  v4f acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
  const int nch = Kp / BKC;
  Bf16Stage rs;
  load_bf16_stage(Vhi, Vlo, Kp, N, I0 + lrow, J0 + lrow, (int64_t)lq, rs);
  for (int ch = 0; ch < nch; ++ch) {
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      *reinterpret_cast<uint4*>(&Ah[lrow][lq + 32 * h]) = rs.ah[h];
      *reinterpret_cast<uint4*>(&Al[lrow][lq + 32 * h]) = rs.al[h];
      *reinterpret_cast<uint4*>(&Bh[lrow][lq + 32 * h]) = rs.bh[h];
      *reinterpret_cast<uint4*>(&Bl[lrow][lq + 32 * h]) = rs.bl[h];
    }
    __syncthreads();
    if (ch + 1 < nch)
      load_bf16_stage(Vhi, Vlo, Kp, N, I0 + lrow, J0 + lrow, (int64_t)(ch + 1) * BKC + lq, rs);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kq = 32 * h + 8 * (lane >> 4);
      v8bf ah[2], al[2], bh[4], bl[4];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int ra_ = wm * 32 + q * 16 + (lane & 15);
        ah[q] = *reinterpret_cast<const v8bf*>(&Ah[ra_][kq]);
        al[q] = *reinterpret_cast<const v8bf*>(&Al[ra_][kq]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rb_ = wn * 64 + q * 16 + (lane & 15);
        bh[q] = *reinterpret_cast<const v8bf*>(&Bh[rb_][kq]);
        bl[q] = *reinterpret_cast<const v8bf*>(&Bl[rb_][kq]);
      }
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
          acc[mi][ni] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mi], bh[ni], acc[mi][ni], 0, 0, 0);
          acc[mi][ni] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bl[ni], acc[mi][ni], 0, 0, 0);
          acc[mi][ni] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bh[ni], acc[mi][ni], 0, 0, 0);
        }
    }
  }
  epilogue_f32acc_w8<true>(P, ldp, N, I0, J0, I == J, acc);
}

__global__ void __launch_bounds__(SYRK_NT, 2) k_syrk_bf16x3(double* __restrict__ P, int64_t ldp,
    int64_t N, const __bf16* __restrict__ Vhi, const __bf16* __restrict__ Vlo, int32_t Kp,
    int64_t T, int64_t per_xcd, const int32_t* __restrict__ flags, int part,
    const int32_t* __restrict__ status, int64_t seq) {
  syrk_bf16x3_body(P, ldp, N, Vhi, Vlo, Kp, T, per_xcd, flags, part, status, seq, blockIdx.x);
}

static_assert(SUB_PER_TILE == SYRK_SUB_PER_TILE, "sub-tiles per tile");

void syrk_tiles(int64_t N, int32_t cu_count, int64_t* T, int64_t* per_xcd,
                int64_t* main_per_xcd) {
  const int64_t nt = ceil_div(N, ST);
  *T = nt * (nt + 1) / 2;
  *per_xcd = ceil_div(*T, 8);
  // whole rounds of 128x128 tiles per XCD, the rest as 32x64 sub-tiles
  const int64_t slots = cu_count > 0 ? (int64_t)cu_count / 8 * 2 : 64;
  *main_per_xcd = slots > 0 ? *per_xcd / slots * slots : *per_xcd;
}

rbf_status syrk_update(rbf_ctx* ctx, double* P, int64_t ldp, int64_t N, const double* Ut,
                       int64_t ldu, int32_t Bc, rbf_prec prec, const int32_t* flags,
                       int part, int64_t seq) {
  if (part != 0 && !flags) return fail(ctx, RBF_E_INVALID_ARG, "syrk_update: part without flags");
  int64_t T, per_xcd, main_per_xcd;
  syrk_tiles(N, ctx->cu_count, &T, &per_xcd, &main_per_xcd);
  const unsigned grid = (unsigned)(per_xcd * 8);
  rbf_status st;
  if (prec == RBF_F64) {
    prof_begin(ctx, RBF_PROF_SYRK);
    if (main_per_xcd > 0) {
      k_syrk_f64<<<(unsigned)(main_per_xcd * 8), SYRK_NT, 0, ctx->stream>>>(
          P, ldp, N, Ut, ldu, Bc, T, per_xcd, flags, part, ctx->d_status, seq);
      RBF_LAUNCHED(ctx, "k_syrk_f64");
    }
    if (main_per_xcd < per_xcd) {
      const unsigned gt = (unsigned)((per_xcd - main_per_xcd) * 8 * SUB_PER_TILE);
      k_syrk_f64_tail<<<gt, SUB_NT, 0, ctx->stream>>>(P, ldp, N, Ut, ldu, Bc, T, per_xcd,
                                                      main_per_xcd, flags, part, ctx->d_status,
                                                      seq);
      RBF_LAUNCHED(ctx, "k_syrk_f64_tail");
    }
    prof_end(ctx, RBF_PROF_SYRK);
    return RBF_OK;
  }
  if (prec == RBF_F32) {
    float* Uf = (float*)ws_get(ctx, WS_UPD_VLO, sizeof(float) * (size_t)Bc * ldu, &st);
    if (!Uf) return st;
    if (part != 2) {
      k_cvt_f32<<<ceil_div((int64_t)Bc * ldu, 256), 256, 0, ctx->stream>>>(Ut, ldu, Bc, N, Uf,
                                                                           ctx->d_status, seq);
      RBF_LAUNCHED(ctx, "k_cvt_f32");
    }
    prof_begin(ctx, RBF_PROF_SYRK);
    k_syrk_f32<<<grid, SYRK_NT, 0, ctx->stream>>>(P, ldp, N, Uf, ldu, Bc, T, per_xcd, flags, part,
                                              ctx->d_status, seq);
    RBF_LAUNCHED(ctx, "k_syrk_f32");
    prof_end(ctx, RBF_PROF_SYRK);
    return RBF_OK;
  }
  const int32_t Kp = (int32_t)ceil_div(Bc, BKC) * BKC;
  __bf16* V = (__bf16*)ws_get(ctx, WS_UPD_VLO, sizeof(__bf16) * 2 * (size_t)N * Kp, &st);
  if (!V) return st;
  __bf16* Vlo = V + (size_t)N * Kp;
  if (part != 2) {
    dim3 gc((unsigned)ceil_div(N, 64), (unsigned)ceil_div(Kp, 64));
    k_cvt_bf16x2<<<gc, 256, 0, ctx->stream>>>(Ut, ldu, Bc, N, Kp, V, Vlo, ctx->d_status, seq);
    RBF_LAUNCHED(ctx, "k_cvt_bf16x2");
  }
  prof_begin(ctx, RBF_PROF_SYRK);
  k_syrk_bf16x3<<<grid, SYRK_NT, 0, ctx->stream>>>(P, ldp, N, V, Vlo, Kp, T, per_xcd, flags, part,
                                               ctx->d_status, seq);
  RBF_LAUNCHED(ctx, "k_syrk_bf16x3");
  prof_end(ctx, RBF_PROF_SYRK);
  return RBF_OK;
}

// ------------------------------------------------ grouped (many patches)

// Covariance products of a round's jobs, each workgroup finding its job
// from the prefix of per-job workgroup counts (multiples of 8, so a job's
// local workgroup index keeps the XCD of the global one).
__global__ void __launch_bounds__(SYRK_NT, 2) k_syrk_f64_g(const GJob* __restrict__ jobs,
                                                           const int64_t* __restrict__ pre,
                                                           int32_t n) {
  const int64_t b = blockIdx.x;
  const int32_t j = job_of(pre, n, b);
  const GJob& J = jobs[j];
  syrk_f64_body(J.P, J.ldp, J.N, J.Vt, J.ldu, J.Bc, J.T, J.per_xcd, nullptr, 0, J.status,
                J.seq, b - pre[j]);
}

__global__ void __launch_bounds__(SUB_NT) k_syrk_f64_tail_g(const GJob* __restrict__ jobs,
                                                            const int64_t* __restrict__ pre,
                                                            int32_t n) {
  const int64_t b = blockIdx.x;
  const int32_t j = job_of(pre, n, b);
  const GJob& J = jobs[j];
  syrk_f64_tail_body(J.P, J.ldp, J.N, J.Vt, J.ldu, J.Bc, J.T, J.per_xcd, J.main_per_xcd,
                     nullptr, 0, J.status, J.seq, b - pre[j]);
}

__global__ void __launch_bounds__(256) k_cvt_f32_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];
  cvt_f32_body(J.Vt, J.ldu, J.Bc, J.N, (float*)J.vlo, J.status, J.seq);
}

__global__ void __launch_bounds__(SYRK_NT, 2) k_syrk_f32_g(const GJob* __restrict__ jobs,
                                                           const int64_t* __restrict__ pre,
                                                           int32_t n) {
  const int64_t b = blockIdx.x;
  const int32_t j = job_of(pre, n, b);
  const GJob& J = jobs[j];
  syrk_f32_body(J.P, J.ldp, J.N, (const float*)J.vlo, J.ldu, J.Bc, J.T, J.per_xcd, nullptr, 0,
                J.status, J.seq, nullptr, 1.0, b - pre[j]);
}

__global__ void __launch_bounds__(256) k_cvt_bf16x2_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];
  if ((int64_t)blockIdx.x * 64 >= J.N || (int)blockIdx.y * 64 >= J.Kp) return;
  __bf16* V = (__bf16*)J.vlo;
  cvt_bf16x2_body(J.Vt, J.ldu, J.Bc, J.N, J.Kp, V, V + (size_t)J.N * J.Kp, J.status, J.seq);
}

__global__ void __launch_bounds__(SYRK_NT, 2) k_syrk_bf16x3_g(const GJob* __restrict__ jobs,
                                                              const int64_t* __restrict__ pre,
                                                              int32_t n) {
  const int64_t b = blockIdx.x;
  const int32_t j = job_of(pre, n, b);
  const GJob& J = jobs[j];
  const __bf16* V = (const __bf16*)J.vlo;
  syrk_bf16x3_body(J.P, J.ldp, J.N, V, V + (size_t)J.N * J.Kp, J.Kp, J.T, J.per_xcd, nullptr,
                   0, J.status, J.seq, b - pre[j]);
}

rbf_status syrk_grouped(rbf_ctx* ctx, const GRound& r, rbf_prec prec) {
  if (r.n <= 0) return RBF_OK;
  if (prec == RBF_F64) {
    if (r.n_main > 0) {
      k_syrk_f64_g<<<(unsigned)r.n_main, SYRK_NT, 0, ctx->stream>>>(r.jobs, r.pre_main, r.n);
      RBF_LAUNCHED(ctx, "k_syrk_f64_g");
    }
    if (r.n_tail > 0) {
      k_syrk_f64_tail_g<<<(unsigned)r.n_tail, SUB_NT, 0, ctx->stream>>>(r.jobs, r.pre_tail,
                                                                        r.n);
      RBF_LAUNCHED(ctx, "k_syrk_f64_tail_g");
    }
    return RBF_OK;
  }
  if (r.n_main <= 0 || r.cvt_x <= 0) return RBF_OK;  // no tiles (no boundary rows)
  if (prec == RBF_F32) {
    k_cvt_f32_g<<<dim3((unsigned)r.cvt_x, 1, (unsigned)r.n), 256, 0, ctx->stream>>>(r.jobs);
    RBF_LAUNCHED(ctx, "k_cvt_f32_g");
    k_syrk_f32_g<<<(unsigned)r.n_main, SYRK_NT, 0, ctx->stream>>>(r.jobs, r.pre_main, r.n);
    RBF_LAUNCHED(ctx, "k_syrk_f32_g");
    return RBF_OK;
  }
  if (r.cvt_y <= 0) return RBF_OK;
  k_cvt_bf16x2_g<<<dim3((unsigned)r.cvt_x, (unsigned)r.cvt_y, (unsigned)r.n), 256, 0,
                   ctx->stream>>>(r.jobs);
  RBF_LAUNCHED(ctx, "k_cvt_bf16x2_g");
  k_syrk_bf16x3_g<<<(unsigned)r.n_main, SYRK_NT, 0, ctx->stream>>>(r.jobs, r.pre_main, r.n);
  RBF_LAUNCHED(ctx, "k_syrk_bf16x3_g");
  return RBF_OK;
}

// Grouped V^T = L^{-1} U^T (one launch over the round's jobs).
__global__ void __launch_bounds__(SYRK_NT, 2) k_linv_apply_g(const GJob* __restrict__ jobs) {
  const GJob& J = jobs[blockIdx.z];
  const int32_t nI = (J.Bp + ST - 1) / ST, nJ = (int32_t)((J.ncols + ST - 1) / ST);
  if ((int32_t)blockIdx.x >= nI * nJ) return;
  linv_apply_body<false>(J.LiT, J.Bp, J.Ut, J.ldu, J.ncols, J.Vt, nJ, J.status, J.seq);
}

rbf_status linv_apply_grouped(rbf_ctx* ctx, const GRound& r) {
  if (r.n <= 0 || r.la_x <= 0) return RBF_OK;
  k_linv_apply_g<<<dim3((unsigned)r.la_x, 1, (unsigned)r.n), SYRK_NT, 0, ctx->stream>>>(r.jobs);
  RBF_LAUNCHED(ctx, "k_linv_apply_g");
  return RBF_OK;
}

rbf_status linv_apply(rbf_ctx* ctx, const double* LiT, int32_t n, const double* Ut,
                      int64_t ldu, int64_t ncols, double* Vt, int64_t seq) {
  if (n <= 0 || ncols <= 0) return RBF_OK;
  const int64_t nI = ceil_div(n, ST), nJ = ceil_div(ncols, ST);
  k_linv_apply<false><<<(unsigned)(nI * nJ), SYRK_NT, 0, ctx->stream>>>(
      LiT, n, Ut, ldu, ncols, Vt, (int32_t)nJ, ctx->d_status, seq);
  RBF_LAUNCHED(ctx, "k_linv_apply");
  return RBF_OK;
}

__global__ void __launch_bounds__(256) k_transpose_f64(const double* __restrict__ A, int32_t n,
                                                       double* __restrict__ B,
                                                       const int32_t* __restrict__ status,
                                                       int64_t seq) {
  if (seq_skip(status, seq)) return;
  __shared__ double t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8)
    if (by + r < n && bx + tx < n) t[r][tx] = A[(int64_t)(by + r) * n + bx + tx];
  __syncthreads();
  for (int r = ty; r < 32; r += 8)
    if (bx + r < n && by + tx < n) B[(int64_t)(bx + r) * n + by + tx] = t[tx][r];
}

rbf_status syrk_update_joseph(rbf_ctx* ctx, double* P, int64_t ldp, int64_t N, const double* Vt,
                              const double* Ut, const double* LiT, int64_t ldu, int32_t Bc,
                              int32_t Bpc, int64_t seq) {
  rbf_status st;
  const size_t ku = (size_t)Bpc * ldu;
  char* wsb = (char*)ws_get(ctx, WS_JOSEPH,
                            sizeof(double) * ((size_t)Bpc * Bpc + ku) + sizeof(float) * 4 * ku,
                            &st);
  if (!wsb) return st;
  double* Lr = (double*)wsb;           // L^{-1} row-major
  double* Kt = Lr + (size_t)Bpc * Bpc;  // K^T = L^{-T} V^T (FP64)
  float* X = (float*)(Kt + ku);        // [K^T; U^T; K^T] (3 Bc rows), then V^T
  float* Vf = X + 3 * (size_t)Bc * ldu;
  const dim3 gt((unsigned)ceil_div(Bpc, 32), (unsigned)ceil_div(Bpc, 32));
  k_transpose_f64<<<gt, 256, 0, ctx->stream>>>(LiT, Bpc, Lr, ctx->d_status, seq);
  RBF_LAUNCHED(ctx, "k_transpose_f64");
  const int64_t nI = ceil_div(Bpc, ST), nJ = ceil_div(N, ST);
  k_linv_apply<true><<<(unsigned)(nI * nJ), SYRK_NT, 0, ctx->stream>>>(
      Lr, Bpc, Vt, ldu, N, Kt, (int32_t)nJ, ctx->d_status, seq);
  RBF_LAUNCHED(ctx, "k_linv_apply");
  const unsigned gc = (unsigned)ceil_div((int64_t)Bc * ldu, 256);
  k_cvt_f32<<<gc, 256, 0, ctx->stream>>>(Kt, ldu, Bc, N, X, ctx->d_status, seq);
  RBF_LAUNCHED(ctx, "k_cvt_f32");
  k_cvt_f32<<<gc, 256, 0, ctx->stream>>>(Ut, ldu, Bc, N, X + (size_t)Bc * ldu, ctx->d_status,
                                         seq);
  RBF_LAUNCHED(ctx, "k_cvt_f32");
  k_cvt_f32<<<gc, 256, 0, ctx->stream>>>(Kt, ldu, Bc, N, X + 2 * (size_t)Bc * ldu,
                                         ctx->d_status, seq);
  RBF_LAUNCHED(ctx, "k_cvt_f32");
  k_cvt_f32<<<gc, 256, 0, ctx->stream>>>(Vt, ldu, Bc, N, Vf, ctx->d_status, seq);
  RBF_LAUNCHED(ctx, "k_cvt_f32");
  const int64_t nt = ceil_div(N, ST);
  const int64_t T = nt * (nt + 1) / 2;
  const int64_t per_xcd = ceil_div(T, 8);
  const unsigned grid = (unsigned)(per_xcd * 8);
  prof_begin(ctx, RBF_PROF_SYRK);
  // P -= K U^T + U K^T: [K U] [U K]^T over 2 Bc terms
  k_syrk_f32<<<grid, SYRK_NT, 0, ctx->stream>>>(P, ldp, N, X, ldu, 2 * Bc, T, per_xcd, nullptr,
                                                0, ctx->d_status, seq, X + (size_t)Bc * ldu,
                                                1.0);
  RBF_LAUNCHED(ctx, "k_syrk_f32");
  // P += K S K^T = V V^T
  k_syrk_f32<<<grid, SYRK_NT, 0, ctx->stream>>>(P, ldp, N, Vf, ldu, Bc, T, per_xcd, nullptr, 0,
                                                ctx->d_status, seq, nullptr, -1.0);
  RBF_LAUNCHED(ctx, "k_syrk_f32");
  prof_end(ctx, RBF_PROF_SYRK);
  return RBF_OK;
}

}  // namespace rbf
