// Inverse Cholesky factor of a small symmetric positive definite fp64
// matrix by one workgroup, for CholeskyQR (Algorithm 7, step 4; Algorithm 8,
// step 5; Algorithm 6, step 3).  R^{-1} comes from symmetric Gaussian
// elimination G = L D L^T applied to the rows of [I | G]: after the
// elimination the left part holds L^{-1} and the right part U = D L^T, and
// R^{-1} = L^{-T} D^{-1/2}; every thread owns a piece of a row, so a step is
// one rank-one row update and one workgroup barrier.  A Gram matrix already
// close to the identity takes a closed form instead (chol_inv_near_identity).
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
constexpr int kElimPanel = 8;  // pivot rows per panel: the rows one wave owns

struct ElimShared {
  __align__(16) double c[2 * kElimPanel * kElimCPitch];  // a panel's pivot rows (by panel parity)
  double diag_u[kElimMaxEll];                            // U[i][i] of the elimination
  double diag_ref[kElimMaxEll];                          // diagonal of G + shift I
};

// LDS writes of a wave's lanes visible to the wave's other lanes.
__device__ __forceinline__ void elim_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// R^{-1} of G + shift I into g (LDS, pitch kElimPitch) by symmetric
// elimination of the rows of
// [I | G] (width 2 ell).  Every row takes the full update
//   row_i -= (U[k][i] / U[k][k]) row_k   for i > k
// at step k: the identity part of row k is zero beyond column k and the part
// of row i left of its diagonal is never read, so no column masks are needed.
// All eight waves take part (lane = 8 rows x 8 column chunks of 16 per
// wave): a lane owns one row x 16 columns in registers.  The steps go in
// panels of the eight rows one wave owns: that wave eliminates its rows
// among themselves, passing each pivot row to its own lanes through LDS
// (no workgroup barrier), then one barrier publishes the panel's pivot rows
// and every wave below applies the eight updates in step order.  Each row
// sees the same updates in the same order as in a step-by-step elimination,
// so the result is the same to the bit, with one barrier per panel instead
// of one per pivot.  Columns past 2 ell carry values that are never used, so
// no step needs a per-column predicate.
// Called by all kElimThreads threads of the workgroup.  Returns false
// (uniformly) on a pivot breakdown, leaving g untouched.
constexpr int kElimMaxR = 1;   // rows per lane
constexpr int kElimMaxC = 16;  // columns per lane (8 chunks cover 2 ell <= 128)

// (i, j), i <= j, of entry e of an upper triangle stored column by column
// (e = j (j + 1) / 2 + i).
__device__ __forceinline__ void tri_index(int e, int& i, int& j) {
  j = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
  while ((j + 1) * (j + 2) / 2 <= e) ++j;
  while (j * (j + 1) / 2 > e) --j;
  i = e - j * (j + 1) / 2;
}

// A Gram matrix within kNearIdentity (Frobenius norm) of the identity -- the
// second CholeskyQR pass, on a Q that the first pass has already made
// orthonormal to working accuracy -- has a Cholesky factor in closed form up
// to third-order terms.  With G = I + E and up(M) the upper triangle of a
// symmetric M with its diagonal halved (up(M) + up(M)^T = M):
//   R = I + F,  F = F1 + F2,  F1 = up(E),  F2 = up(-F1^T F1),
// so that R^T R = G + O(|E|^3), and R^{-1} = I - F + F^2 + O(|E|^3).  For
// |E|_F <= 1e-6 the neglected terms (about 1e-18) are below the rounding of
// the entries, so this is the factor the elimination would produce, without
// its one-barrier-per-pivot chain.  Called by all kElimThreads threads;
// returns false (uniformly) when G is not that close to I, leaving g as it
// was.  On success g holds R^{-1} as chol_inv_elim leaves it.
constexpr double kNearIdentity = 1e-6;

__device__ inline bool chol_inv_near_identity(int ell, double* g, ElimShared& es) {
  constexpr int P = kElimPitch;
  const int tid = threadIdx.x;
  const int nt = ell * (ell + 1) / 2;
  __syncthreads();  // g complete; a previous elimination may still be reading es.c
  double s = 0.0;
  for (int e = tid; e < nt; e += kElimThreads) {
    int i, j;
    tri_index(e, i, j);
    const double v = g[i * P + j] - (i == j ? 1.0 : 0.0);
    s += (i == j ? 1.0 : 2.0) * v * v;
  }
  s = wave_sum(s);
  if ((tid & 63) == 0) es.c[tid >> 6] = s;
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < kElimThreads / 64; ++w) tot += es.c[w];
  if (!(tot <= kNearIdentity * kNearIdentity)) return false;  // (also for NaN)
  // F1 in place: G's strict upper triangle, diagonal (G_ii - 1) / 2
  if (tid < ell) g[tid * P + tid] = 0.5 * (g[tid * P + tid] - 1.0);
  __syncthreads();
  // F = F1 - up(F1^T F1): strict upper part stored transposed in the lower
  // triangle (F[i][j] at g[j][i]), diagonal in diag_u; F1 is only read
  for (int e = tid; e < nt; e += kElimThreads) {
    int i, j;
    tri_index(e, i, j);
    // four terms per batch, their loads in flight together
    double p0 = 0.0, p1 = 0.0;
    int k = 0;
    for (; k + 3 <= i; k += 4) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = g[(k + u) * P + i];
        b[u] = g[(k + u) * P + j];
      }
      p0 = fma(a[0], b[0], p0);
      p1 = fma(a[1], b[1], p1);
      p0 = fma(a[2], b[2], p0);
      p1 = fma(a[3], b[3], p1);
    }
    for (; k <= i; ++k) p0 = fma(g[k * P + i], g[k * P + j], p0);
    const double p = p0 + p1;
    const double f1 = g[i * P + j];
    if (i == j)
      es.diag_u[i] = f1 - 0.5 * p;
    else
      g[j * P + i] = f1 - p;
  }
  __syncthreads();
  // R^{-1} = I - F + F^2 into the upper triangle (F is read from the lower
  // triangle and diag_u only)
  auto fv = [&](int a, int b) { return a == b ? es.diag_u[a] : g[b * P + a]; };  // F[a][b], a <= b
  for (int e = tid; e < nt; e += kElimThreads) {
    int i, j;
    tri_index(e, i, j);
    double q0 = 0.0, q1 = 0.0;
    int k = i;
    for (; k + 3 <= j; k += 4) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = fv(i, k + u);
        b[u] = fv(k + u, j);
      }
      q0 = fma(a[0], b[0], q0);
      q1 = fma(a[1], b[1], q1);
      q0 = fma(a[2], b[2], q0);
      q1 = fma(a[3], b[3], q1);
    }
    for (; k <= j; ++k) q0 = fma(fv(i, k), fv(k, j), q0);
    g[i * P + j] = ((i == j ? 1.0 : 0.0) - fv(i, j)) + (q0 + q1);
  }
  __syncthreads();
  const int lp = (ell + 15) / 16 * 16;
  for (int e = tid; e < lp * lp; e += kElimThreads) {
    const int m = e / lp, i = e % lp;
    if (m > i || i >= ell) g[m * P + i] = 0.0;
  }
  __syncthreads();
  return true;
}

__device__ inline bool chol_inv_elim(int ell, double shift, double* g, ElimShared& es) {
  if (shift == 0.0 && chol_inv_near_identity(ell, g, es)) return true;
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
  const int wave = tid >> 6;
  // step k with pivot row ck: row r0 -= (U[k][r0] / U[k][k]) row k below the pivot
  auto step = [&](int k, const double* ck) {
    const double piv = ck[elim_cpos(ell + k)];
    double rk[kElimMaxC];
#pragma unroll
    for (int q = 0; q < kElimMaxC; q += 2) {
      const double2 t = *reinterpret_cast<const double2*>(&ck[ch * 18 + q]);
      rk[q] = t.x;
      rk[q + 1] = t.y;
    }
    const double num = ck[elim_cpos(ell + min(r0, ell - 1))];
    const double rp = 1.0 / piv;
    const double l = (r0 > k && r0 < ell) ? num * rp : 0.0;
#pragma unroll
    for (int q = 0; q < kElimMaxC; ++q) cv[0][q] -= l * rk[q];
    return piv;
  };
  const int npanel = (ell + kElimPanel - 1) / kElimPanel;
  for (int pn = 0; pn < npanel; ++pn) {
    const int k0 = pn * kElimPanel, k1 = min(ell, k0 + kElimPanel);
    double* buf = &es.c[(pn & 1) * kElimPanel * kElimCPitch];
    if (wave == pn) {
      for (int k = k0; k < k1; ++k) {
        double* ck = &buf[(k - k0) * kElimCPitch];
        if (r0 == k) {  // row k has all its updates: it is the pivot row
#pragma unroll
          for (int q = 0; q < kElimMaxC; q += 2)
            *reinterpret_cast<double2*>(&ck[ch * 18 + q]) = make_double2(cv[0][q], cv[0][q + 1]);
        }
        elim_wave_sync();
        const double piv = step(k, ck);
        if ((tid & 63) == 0) es.diag_u[k] = piv;
      }
    }
    __syncthreads();
    if (wave > pn) {
      // the panel's multipliers first (their divisions in flight together),
      // then the updates in step order; steps past the panel's end (its last
      // pivot row re-read) take multiplier 0
      double l[kElimPanel];
#pragma unroll
      for (int u = 0; u < kElimPanel; ++u) {
        const int k = min(k0 + u, k1 - 1);
        const double* ck = &buf[(k - k0) * kElimCPitch];
        const double piv = ck[elim_cpos(ell + k)];
        const double num = ck[elim_cpos(ell + min(r0, ell - 1))];
        const double rp = 1.0 / piv;
        l[u] = (k0 + u < k1 && r0 > k && r0 < ell) ? num * rp : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kElimPanel; ++u) {
        const double* ck = &buf[(min(k0 + u, k1 - 1) - k0) * kElimCPitch];
#pragma unroll
        for (int q = 0; q < kElimMaxC; q += 2) {
          const double2 t = *reinterpret_cast<const double2*>(&ck[ch * 18 + q]);
          cv[0][q] -= l[u] * t.x;
          cv[0][q + 1] -= l[u] * t.y;
        }
      }
    }
  }
  // a breakdown (non-positive, tiny or non-finite pivot), the same in every wave
  bool bad = false;
  for (int k = tid & 63; k < ell; k += 64) {
    const double piv = es.diag_u[k];
    bad = bad || !((piv > 1e-14 * es.diag_ref[k]) && isfinite(piv));
  }
  const bool ok = !__any(bad);
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
