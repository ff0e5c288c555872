// Cholesky factor and inverse of one 64x64 SPD block held in LDS, for a
// 256-thread workgroup (included by update.hip inside namespace rbf, after
// its tile helpers).
//
// Right-looking over four 16-column panels. For panel c0:
//   A. wave 0 factors the 16x16 diagonal block in registers, one row per lane
//      (lane g, g = lane % 16, holds row g); step j takes the pivot from its
//      lane with a DPP row broadcast and updates the later columns with
//      FP64 FMAs whose column entry comes from its lane through the FMA's
//      own DPP source (no LDS, no barrier), scaling by the pivot's
//      reciprocal only; after the 16 steps lane j takes the square root of
//      pivot j and its reciprocal, and broadcasts the reciprocal. It writes
//      L and 1 / L_jj;
//   B. the panel rows below, L_p D^T = A_p, by forward substitution in
//      registers (waves 1-3, one row per lane; lane g also holds row g of
//      the diagonal factor D, whose entries reach the other lanes the same
//      way);
//   C. the trailing lower blocks: A_rs -= L_r L_s^T (FP64 MFMA).
// Then the four diagonal 16x16 inverses, one per wave, by forward
// substitution (lane c holds column c, lane g row g of D), and the
// off-diagonal 16x16 blocks
// of the inverse by block diagonals:
//   Linv_ij = -Linv_ii sum_{j<=k<i} L_ik Linv_kj,
// where the f64 MFMA output layout (lane j + 16 (i % 4), item i / 4) is the
// B-operand layout of the next product's k-steps, so the two products chain
// in registers. No panel waits for an inverse. A non-positive or non-finite
// pivot records RBF_E_NOT_SPD with `index` for launch group `seq` (the
// factor runs to its end; its output is then not used).
#pragma once

// Value of v in lane k of each row of 16 lanes: DPP row_newbcast (gfx90a
// and later), two 32-bit moves per double, no LDS and no scalar registers.
template <int K>
__device__ __forceinline__ double dpp_bcast16(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x150 + K, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x150 + K, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// k must fold to a constant (unrolled loops), which leaves one case.
__device__ __forceinline__ double row_bcast16(double v, int k) {
  switch (k) {
    case 0: return dpp_bcast16<0>(v);
    case 1: return dpp_bcast16<1>(v);
    case 2: return dpp_bcast16<2>(v);
    case 3: return dpp_bcast16<3>(v);
    case 4: return dpp_bcast16<4>(v);
    case 5: return dpp_bcast16<5>(v);
    case 6: return dpp_bcast16<6>(v);
    case 7: return dpp_bcast16<7>(v);
    case 8: return dpp_bcast16<8>(v);
    case 9: return dpp_bcast16<9>(v);
    case 10: return dpp_bcast16<10>(v);
    case 11: return dpp_bcast16<11>(v);
    case 12: return dpp_bcast16<12>(v);
    case 13: return dpp_bcast16<13>(v);
    case 14: return dpp_bcast16<14>(v);
    default: return dpp_bcast16<15>(v);
  }
}

// a += v(lane k of its row of 16) * m as one v_fmac_f64 with a DPP
// row_newbcast source (the only DPP control 64-bit operands take), instead
// of two 32-bit broadcasts and an FMA. Same fused operation, so the same
// result. A DPP read needs two wait states after the VALU write of its
// source; the compiler pads its own DPP reads after inline asm, but not
// the DPP read inside this asm, so every source given to it here is either
// loaded from LDS or written several dependent instructions earlier (a
// listing check over the compiled kernels confirms it).
template <int K>
__device__ __forceinline__ void fmac_bcast16_k(double& a, double v, double m) {
  asm volatile("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
               : "+v"(a)
               : "v"(v), "v"(m), "i"(K));
}
// a -= v(lane K of its row of 16) * m, the same instruction with the
// multiplier negated by the operand modifier.
template <int K>
__device__ __forceinline__ void fnmac_bcast16_k(double& a, double v, double m) {
  asm volatile("v_fmac_f64_dpp %0, %1, -%2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
               : "+v"(a)
               : "v"(v), "v"(m), "i"(K));
}
// k must fold to a constant (unrolled loops), which leaves one case.
#define RBF_BCAST16_CASES(F, ...)                                     \
  switch (k) {                                                        \
    case 0: F<0>(__VA_ARGS__); break;                                 \
    case 1: F<1>(__VA_ARGS__); break;                                 \
    case 2: F<2>(__VA_ARGS__); break;                                 \
    case 3: F<3>(__VA_ARGS__); break;                                 \
    case 4: F<4>(__VA_ARGS__); break;                                 \
    case 5: F<5>(__VA_ARGS__); break;                                 \
    case 6: F<6>(__VA_ARGS__); break;                                 \
    case 7: F<7>(__VA_ARGS__); break;                                 \
    case 8: F<8>(__VA_ARGS__); break;                                 \
    case 9: F<9>(__VA_ARGS__); break;                                 \
    case 10: F<10>(__VA_ARGS__); break;                               \
    case 11: F<11>(__VA_ARGS__); break;                               \
    case 12: F<12>(__VA_ARGS__); break;                               \
    case 13: F<13>(__VA_ARGS__); break;                               \
    case 14: F<14>(__VA_ARGS__); break;                               \
    default: F<15>(__VA_ARGS__); break;                               \
  }
__device__ __forceinline__ void fmac_bcast16(double& a, double v, double m, int k) {
  RBF_BCAST16_CASES(fmac_bcast16_k, a, v, m)
}
__device__ __forceinline__ void fnmac_bcast16(double& a, double v, double m, int k) {
  RBF_BCAST16_CASES(fnmac_bcast16_k, a, v, m)
}
#undef RBF_BCAST16_CASES

// 16x16 product tile on FP64 MFMA: acc += A[r0.., a0..] * B where B[k][j] is
// B_t[b0 + j][bk0 + k] (i.e. the operand is read transposed from LDS).
__device__ __forceinline__ v4d mma16_nt(const double (*A)[LDT], int r0, int a0, const double (*Bt)[LDT],
                               int b0, int bk0, v4d acc) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int ks = 0; ks < 16; ks += 4) {
    const int kk = ks + (lane >> 4);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[r0 + (lane & 15)][a0 + kk],
                                               Bt[b0 + (lane & 15)][bk0 + kk], acc, 0, 0, 0);
  }
  return acc;
}

// 1/p: the v_rcp_f64 estimate (about 24 correct bits) and one
// Newton-Raphson step r <- r + r (1 - p r), which doubles them: within 11
// ulp of 1/p (measured over random pivots), a relative error of the factor
// far below the rounding of its own sums. A second step (correctly rounded)
// costs two more dependent FMAs per pivot on the factor's critical path.
__device__ __forceinline__ double rcp_nr(double p) {
  double r = __builtin_amdgcn_rcp(p);
  r = fma(r, fma(-p, r, 1.0), r);
  return r;
}

// Phase A for the diagonal block at (c0, c0): T gets L (zero above the
// diagonal), dinv[c0 + j] = 1 / L_jj; returns false if a pivot was not
// positive and finite. Wave 0 only.
// Step j works on the unscaled column c (c_g = a[g][j], pivot p_j = c_j):
// a[g][k] -= c_g c_k / p_j for j < k, so the square roots are off the
// dependent chain; afterwards L[g][j] = c_g / sqrt(p_j).
__device__ __forceinline__ bool chol16_factor(double (*T)[LDT], double* dinv, int c0) {
  const int lane = threadIdx.x & 63;
  const int g = lane & 15;
  double a[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) a[k] = T[c0 + g][c0 + k];
  int nbad = 0;  // counted without branches: the 16 steps stay one block
  double mypiv = 1.0;  // lane g keeps pivot g
  // The pivot test stays off the dependent chain of the steps: a pivot that
  // is not positive and finite is counted (the batch is then discarded
  // through the status word) and the factor goes on with it. Each step
  // updates the next pivot column first and broadcasts the next pivot.
  double pj = row_bcast16(a[0], 0);
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    nbad += 1 - ((int)(pj > 0.0) & (int)(pj < INFINITY));
    mypiv = (g == j) ? pj : mypiv;
    const double negt = -(a[j] * rcp_nr(pj));
    // entries above the diagonal (lanes g < k) receive unused values
    if (j + 1 < 16) {
      fmac_bcast16(a[j + 1], a[j], negt, j + 1);
      pj = row_bcast16(a[j + 1], j + 1);
    }
#pragma unroll
    for (int k = j + 2; k < 16; ++k) fmac_bcast16(a[k], a[j], negt, k);
  }
  __builtin_amdgcn_sched_barrier(0);
  // each lane takes the root and reciprocal of its own pivot (one square
  // root and one division per lane rather than sixteen) and the others
  // receive the reciprocals by broadcast. The broadcasts are statements of
  // their own: inside an arm of the select below they would make it a
  // branch, with the source lane switched off while they read it.
  const double mine_d = sqrt(mypiv);
  const double mine = 1.0 / mine_d;
  double rinv[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) rinv[j] = row_bcast16(mine, j);
#pragma unroll
  for (int j = 0; j < 16; ++j) a[j] = (g == j) ? mine_d : a[j] * rinv[j];
  __builtin_amdgcn_sched_barrier(0);
  if (lane < 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) T[c0 + g][c0 + k] = (k <= g) ? a[k] : 0.0;
    dinv[c0 + g] = mine;
  }
  return nbad == 0;
}

// Phase B for panel c0: row r (one per lane of waves 1..3, g = lane % 16)
// solves l D^T = a for its 16 entries, D = the panel's diagonal factor.
// Lane g also holds row g of D and 1 / D_gg, so D_kj and 1 / D_jj reach
// every lane by DPP broadcast from lane k (resp. j) rather than as LDS
// reads; the DPP sources come from LDS loads, never from a VALU write.
__device__ __forceinline__ void panel_rows(double (*T)[LDT], const double* dinv, int c0, int r) {
  const int lane = threadIdx.x & 63;
  const int g = lane & 15;
  double x[16], d[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = T[r][c0 + k];
#pragma unroll
  for (int k = 0; k < 16; ++k) d[k] = T[c0 + g][c0 + k];
  const double dv = dinv[c0 + g];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    x[j] *= row_bcast16(dv, j);
#pragma unroll
    for (int k = j + 1; k < 16; ++k) fnmac_bcast16(x[k], d[j], x[j], k);  // x_k -= D_kj x_j
  }
  if (lane < 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) T[r][c0 + k] = x[k];
  }
}

// Inverse of the 16x16 diagonal factor block at (b0, b0) into Ti (lane c of
// the wave computes column c by forward substitution). Lane g holds row g
// of D and 1 / D_gg, broadcast by DPP as in panel_rows. The substitution is
// right-looking: once x_j is known, every later s_k takes its term at once,
// so the dependent chain is two operations per row (x_j, then s_{j+1})
// rather than a sum of up to 15 terms per row.
__device__ __forceinline__ void diag_inverse(const double (*T)[LDT], double (*Ti)[LDT],
                                             const double* dinv, int b0) {
  const int lane = threadIdx.x & 63;
  const int g = lane & 15;
  double x[16], d[16], s[16], dvb[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) d[k] = T[b0 + g][b0 + k];
  const double dv = dinv[b0 + g];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    s[k] = (g == k) ? 1.0 : 0.0;
    dvb[k] = row_bcast16(dv, k);
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    x[j] = s[j] * dvb[j];
#pragma unroll
    for (int k = j + 1; k < 16; ++k) fnmac_bcast16(s[k], d[j], x[j], k);  // s_k -= D_kj x_j
  }
  if (lane < 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) Ti[b0 + k][b0 + g] = (k >= g) ? x[k] : 0.0;
  }
}

__device__ __forceinline__ void chol64(double (*T)[LDT], double (*Ti)[LDT], int32_t* status,
                                    int64_t index, int64_t seq) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ int bad;
  __shared__ double dinv[NB];
  if (tid == 0) bad = 0;
  for (int c0 = 0; c0 < NB; c0 += 16) {
    // ---- A: 16x16 diagonal block (wave 0, registers)
    if (wave == 0) {
      const bool ok = chol16_factor(T, dinv, c0);
      if (lane == 0 && !ok) bad = 1;
    } else if (c0 == 0) {
      // meanwhile waves 1-3 clear the strictly upper 16x16 blocks of L and
      // of its inverse: no phase reads them, and the inverse's diagonal and
      // lower blocks are all written below
      for (int e = tid - 64; e < NB * NB; e += 192)
        if (((e & 63) >> 4) > (e >> 10)) {
          T[e >> 6][e & 63] = 0.0;
          Ti[e >> 6][e & 63] = 0.0;
        }
    }
    __syncthreads();
    const int nrb = (NB - c0 - 16) / 16;  // row blocks below the panel
    if (nrb == 0) break;
    // ---- B: panel rows below, L_p D^T = A_p
    if (wave >= 1 && wave <= nrb) panel_rows(T, dinv, c0, c0 + 16 * wave + (lane & 15));
    __syncthreads();
    // ---- C: trailing lower blocks A_rs -= L_r L_s^T
    const int nblocks = nrb * (nrb + 1) / 2;
    for (int bidx = wave; bidx < nblocks; bidx += 4) {
      int rb = 0;
      while ((rb + 1) * (rb + 2) / 2 <= bidx) ++rb;
      const int sb = bidx - rb * (rb + 1) / 2;
      const int r0 = c0 + 16 + 16 * rb, s0 = c0 + 16 + 16 * sb;
      v4d acc = (v4d){0.0, 0.0, 0.0, 0.0};
      acc = mma16_nt(T, r0, c0, T, s0, c0, acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) T[r0 + 4 * v + (lane >> 4)][s0 + (lane & 15)] -= acc[v];
    }
    __syncthreads();
  }
  // ---- the four diagonal inverses, one per wave
  diag_inverse(T, Ti, dinv, 16 * wave);
  __syncthreads();
  // ---- off-diagonal blocks of the inverse, by block diagonals d = i - j
  for (int d = 1; d < 4; ++d) {
    const int nb = 4 - d;
    if (wave < nb) {
      const int i = wave + d, j = wave;
      v4d t = (v4d){0.0, 0.0, 0.0, 0.0};
      for (int k = j; k < i; ++k) {
        // t += L_ik Linv_kj: B[kk][col] = Linv[16k + kk][16j + col]
#pragma unroll
        for (int ks = 0; ks < 16; ks += 4) {
          const int kk = ks + (lane >> 4);
          t = __builtin_amdgcn_mfma_f64_16x16x4f64(T[16 * i + (lane & 15)][16 * k + kk],
                                                   Ti[16 * k + kk][16 * j + (lane & 15)], t, 0,
                                                   0, 0);
        }
      }
      // result = -Linv_ii t; t (output layout) is the B operand, item = k-step
      v4d res = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = 4 * s + (lane >> 4);
        res = __builtin_amdgcn_mfma_f64_16x16x4f64(Ti[16 * i + (lane & 15)][16 * i + kk], t[s],
                                                   res, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Ti[16 * i + 4 * v + (lane >> 4)][16 * j + (lane & 15)] = -res[v];
    }
    __syncthreads();
  }
  if (tid == 0 && bad) set_status(status, RBF_E_NOT_SPD, index, seq);
}

