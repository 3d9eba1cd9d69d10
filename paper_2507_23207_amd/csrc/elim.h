// Inverse Cholesky factor of a small symmetric positive definite fp64
// matrix by one workgroup, for CholeskyQR (Algorithm 7, step 4; Algorithm 8,
// step 5; Algorithm 6, step 3).  R^{-1} comes from symmetric Gaussian
// elimination G = L D L^T applied to the rows of [I | G]: after the
// elimination the left part holds L^{-1} and the right part U = D L^T, and
// R^{-1} = L^{-T} D^{-1/2}; every thread owns a piece of a row, so a step is
// one rank-one row update and one workgroup barrier.
#pragma once
#include "device_common.h"

namespace krp {

constexpr int kElimThreads = 512;               // workgroup size the elimination assumes
constexpr int kElimMaxEll = 64;
constexpr int kElimPitch = kElimMaxEll + 1;     // pitch of G and R^{-1} in LDS
// Pivot rows of the elimination: 8 chunks of 16 columns, chunk stride 18
// (the chunks start on distinct LDS banks).
constexpr int kElimCPitch = 8 * 18;
__device__ __forceinline__ int elim_cpos(int c) { return (c >> 4) * 18 + (c & 15); }

struct ElimShared {
  __align__(16) double c[2 * kElimCPitch];  // pivot rows (by step parity)
  double diag_u[kElimMaxEll];               // U[i][i] of the elimination
  double diag_ref[kElimMaxEll];             // diagonal of G + shift I
};

// R^{-1} of G + shift I into g (LDS, pitch kElimPitch) by symmetric
// elimination of the rows of
// [I | G] (width 2 ell).  Every row takes the full update
//   row_i -= (U[k][i] / U[k][k]) row_k   for i > k
// at step k: the identity part of row k is zero beyond column k and the part
// of row i left of its diagonal is never read, so no column masks are needed.
// All eight waves take part (lane = 8 rows x 8 column chunks of 16 per
// wave): a lane owns one row x 16 columns in registers, and only the pivot
// row of the next step goes through LDS.  Columns past 2 ell carry values
// that are never used, so no step needs a per-column predicate.
// Called by all kElimThreads threads of the workgroup.  Returns false
// (uniformly) on a pivot breakdown, leaving g untouched.
constexpr int kElimMaxR = 1;   // rows per lane
constexpr int kElimMaxC = 16;  // columns per lane (8 chunks cover 2 ell <= 128)

__device__ inline bool chol_inv_elim(int ell, double shift, double* g, ElimShared& es) {
  const int tid = threadIdx.x;
  const int width = 2 * ell;
  constexpr int R = 1;
  constexpr int C = kElimMaxC;
  const bool part = tid < kElimThreads;
  const int grp = tid / 8, ch = tid % 8;
  const int r0 = grp * R, c0 = ch * C;
  double cv[kElimMaxR][kElimMaxC];
  __syncthreads();  // a previous elimination may still be reading es.c
  // combined row i: columns 0..ell-1 hold L^{-1}[i][.] (identity at first),
  // columns ell..2 ell - 1 hold the Schur complement row U[i][.]
#pragma unroll
  for (int r = 0; r < kElimMaxR; ++r) {
    const int i = r0 + r;
#pragma unroll
    for (int q = 0; q < kElimMaxC; ++q) {
      const int c = c0 + q;
      double v = 0.0;
      if (part && r < R && i < ell && c < width) {
        if (c < ell) v = (c == i) ? 1.0 : 0.0;
        else v = g[i * kElimPitch + c - ell] + ((c - ell == i) ? shift : 0.0);
        if (i == 0) es.c[elim_cpos(c)] = v;  // the first pivot row
      }
      cv[r][q] = v;
    }
  }
  if (tid < ell) es.diag_ref[tid] = g[tid * kElimPitch + tid] + shift;
  __syncthreads();
  // No early exit: a breakdown is recorded and tested after the loop (the
  // remaining steps then run on non-finite values that are discarded), and
  // the updates cover the whole register block unconditionally (multiplier 0
  // for rows not below the pivot; columns past the block's width are never
  // stored), which keeps every step free of divergent branches.
  bool ok = true;
  for (int k = 0; k < ell; ++k) {
    const double* ck = &es.c[(k & 1) * kElimCPitch];
    const double piv = ck[elim_cpos(ell + k)], ref = es.diag_ref[k];
    ok = ok && (piv > 1e-14 * ref) && isfinite(piv);
    if (part) {
      double rk[kElimMaxC], num[kElimMaxR];
#pragma unroll
      for (int q = 0; q < kElimMaxC; q += 2) {
        const double2 t = *reinterpret_cast<const double2*>(&ck[ch * 18 + q]);
        rk[q] = t.x;
        rk[q + 1] = t.y;
      }
#pragma unroll
      for (int r = 0; r < kElimMaxR; ++r) num[r] = ck[elim_cpos(ell + min(r0 + r, ell - 1))];
      const double rp = 1.0 / piv;
#pragma unroll
      for (int r = 0; r < kElimMaxR; ++r) {
        const double l = (r0 + r > k && r0 + r < ell) ? num[r] * rp : 0.0;
#pragma unroll
        for (int q = 0; q < kElimMaxC; ++q) cv[r][q] -= l * rk[q];
      }
      // the next pivot row is final now
      const int rn = k + 1 - r0;
      if (rn >= 0 && rn < R && k + 1 < ell) {
        double* cn = &es.c[((k + 1) & 1) * kElimCPitch + ch * 18];
#pragma unroll
        for (int q = 0; q < kElimMaxC; q += 2) {
          *reinterpret_cast<double2*>(&cn[q]) = make_double2(cv[0][q], cv[0][q + 1]);
        }
      }
    }
    if (tid == 0) es.diag_u[k] = piv;
    __syncthreads();
  }
  if (!ok) return false;
  // R^{-1}[m][i] = L^{-1}[i][m] / sqrt(U[i][i]) for m <= i, zero elsewhere
  // (including the padding up to the next multiple of 16)
  if (part) {
#pragma unroll
    for (int r = 0; r < kElimMaxR; ++r) {
      const int i = r0 + r;
      if (r < R && i < ell) {
        const double dinv = 1.0 / sqrt(es.diag_u[i]);
#pragma unroll
        for (int q = 0; q < kElimMaxC; ++q) {
          const int m = c0 + q;
          if (q < C && m <= i) g[m * kElimPitch + i] = cv[r][q] * dinv;
        }
      }
    }
  }
  const int lp = (ell + 15) / 16 * 16;
  for (int e = tid; e < lp * lp; e += kElimThreads) {
    const int m = e / lp, i = e % lp;
    if (m > i || i >= ell) g[m * kElimPitch + i] = 0.0;
  }
  __syncthreads();
  return true;
}

}  // namespace krp
