// Cholesky factor and inverse of one 64x64 SPD block held in LDS, for a
// 256-thread workgroup (included by update.hip inside namespace rbf, after
// its tile helpers).
//
// Right-looking over four 16-column panels. For panel c0:
//   A. wave 0 factors the 16x16 diagonal block and forms its inverse in the
//      same 16 steps: lane group g = lane / 4 (part p = lane % 4) holds entries
//      4k + p of row g of the block and of column g of its inverse; in step j
//      the groups g > j form L[g][j] (left-looking, partial dot products of
//      the four lanes meet through two shuffles, pivots from a running
//      remainder r_g = a_gg - sum L[g][q]^2) and the groups g <= j form
//      inverse row j;
//   B. the panel rows below: L_p = A_p D^{-T} (16x16x16 FP64 MFMA per wave);
//   C. the trailing lower blocks: A_rs -= L_r L_s^T (FP64 MFMA).
// Then the off-diagonal 16x16 blocks of the inverse by block diagonals:
//   Linv_ij = -Linv_ii sum_{j<=k<i} L_ik Linv_kj,
// where the f64 MFMA output layout (lane j + 16 (i % 4), item i / 4) is the
// B-operand layout of the next product's k-steps, so the two products chain
// in registers. A non-positive or non-finite pivot records RBF_E_NOT_SPD
// with `index` for launch group `seq` (the factor continues with pivot 1).
#pragma once

// 16x16 product tile on FP64 MFMA: acc += A[r0.., a0..] * B where B[k][j] is
// B_t[b0 + j][bk0 + k] (i.e. the operand is read transposed from LDS).
__device__ inline v4d mma16_nt(const double (*A)[LDT], int r0, int a0, const double (*Bt)[LDT],
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

__device__ __noinline__ void chol64(double (*T)[LDT], double (*Ti)[LDT], int32_t* status,
                                    int64_t index, int64_t seq) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ int bad;
  if (tid == 0) bad = 0;
  for (int e = tid; e < NB * NB; e += 256) Ti[e >> 6][e & 63] = 0.0;
  __syncthreads();
  const bool w0 = wave == 0;
  const int g = lane >> 2, p = lane & 3;
  for (int c0 = 0; c0 < NB; c0 += 16) {
    // ---- A: 16x16 diagonal block and its inverse (wave 0)
    double a[4], x[4], r = 0.0;
    if (w0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        a[k] = T[c0 + g][c0 + 4 * k + p];
        x[k] = 0.0;
      }
      r = T[c0 + g][c0 + g];
      if (g == 0 && p == 0) {
        const bool ok = r > 0.0 && isfinite(r);
        if (!ok) bad = 1;
        T[c0][c0] = ok ? sqrt(r) : 1.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (w0) {
        const double ljj = T[c0 + j][c0 + j];
        if (g > j) {
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int q = 4 * k + p;
            if (q < j) s += a[k] * T[c0 + j][c0 + q];
          }
          s += __shfl_xor(s, 1, 64);
          s += __shfl_xor(s, 2, 64);
          const double l = (T[c0 + g][c0 + j] - s) / ljj;
          if (p == (j & 3)) {
            a[j >> 2] = l;
            T[c0 + g][c0 + j] = l;
          }
          r -= l * l;
          if (g == j + 1 && p == 0) {
            const bool ok = r > 0.0 && isfinite(r);
            if (!ok) bad = 1;
            T[c0 + g][c0 + g] = ok ? sqrt(r) : 1.0;
          }
        } else {
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int q = 4 * k + p;
            if (q >= g && q < j) s += T[c0 + j][c0 + q] * x[k];
          }
          s += __shfl_xor(s, 1, 64);
          s += __shfl_xor(s, 2, 64);
          const double v = ((g == j ? 1.0 : 0.0) - s) / ljj;
          if (p == (j & 3)) x[j >> 2] = v;
        }
      }
      __syncthreads();
    }
    if (w0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int q = 4 * k + p;
        Ti[c0 + q][c0 + g] = (q >= g) ? x[k] : 0.0;
        if (q > g) T[c0 + g][c0 + q] = 0.0;
      }
    }
    __syncthreads();
    const int nrb = (NB - c0 - 16) / 16;  // row blocks below the panel
    if (nrb == 0) break;
    // ---- B: panel rows below: L_p = A_p D^{-T}
    if (wave < nrb) {
      const int r0 = c0 + 16 + 16 * wave;
      v4d acc = (v4d){0.0, 0.0, 0.0, 0.0};
      acc = mma16_nt(T, r0, c0, Ti, c0, c0, acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) T[r0 + 4 * v + (lane >> 4)][c0 + (lane & 15)] = acc[v];
    }
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
  // strictly upper 16x16 blocks of L are zero (the diagonal blocks were
  // cleared above); the loop below reads only lower blocks of T
  for (int e = tid; e < NB * NB; e += 256)
    if (((e & 63) >> 4) > (e >> 10)) T[e >> 6][e & 63] = 0.0;
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

