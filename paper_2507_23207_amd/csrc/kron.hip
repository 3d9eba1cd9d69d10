// Algorithm 6 on general block-structured matrices M = sum_j B_j kron C_j
// (Section 4.1, eq. (4.2); Section 4.3) and the Nystrom variant for SPSD M.
// The contractions with the stacked blocks and the tall-times-small products
// run on the TTM kernels (B_j Omega1 and C_j Omega2 for all j at once, Z K^T,
// Q U_W); this file holds what is specific: the tall A^T B products (Psi^T Q
// and the Gram matrices) split over row chunks, the Khatri-Rao combination of the per-term products
// (Y = sum_j (B_j Omega1) kr (C_j Omega2)), explicit KRP rows, the small
// dense steps (pseudo-inverse by the Cholesky factor of G^T G, the Nystrom
// Cholesky factor), the Nystrom shift, and the sign convention.
#include "device_common.h"
#include "driver.h"
#include "elim.h"
#include "kron.h"

#include <algorithm>

namespace krp {

namespace {

// out[(a n2 + b) + rows c] = sum_j x1[a s1a + c s1c + j s1j] x2[b s2b + c s2c + j s2j]
// for a < n1, b < n2, c < ell (rows = n1 n2); one thread per entry, b fastest.
__global__ __launch_bounds__(256) void kron_combine_kernel(KronCombineArgs a) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t rows = a.n1 * a.n2;
  if (e >= rows * a.ell) return;
  const int64_t c = e / rows;
  const int64_t row = e - c * rows;
  const int64_t ia = row / a.n2, ib = row - ia * a.n2;
  const double* x1 = a.x1 + ia * a.s1a + c * a.s1c;
  const double* x2 = a.x2 + ib * a.s2b + c * a.s2c;
  double s0 = 0.0, s1 = 0.0;
  int64_t j = 0;
  for (; j + 1 < a.t; j += 2) {
    s0 += x1[j * a.s1j] * x2[j * a.s2j];
    s1 += x1[(j + 1) * a.s1j] * x2[(j + 1) * a.s2j];
  }
  if (j < a.t) s0 += x1[j * a.s1j] * x2[j * a.s2j];
  a.out[e] = s0 + s1;
}

// Explicit KRP (F1 kr F2)[(a n2 + b), c] = F1[a, c] F2[b, c] (column-major).
__global__ __launch_bounds__(256) void kron_krp_kernel(const double* __restrict__ f1, const double* __restrict__ f2,
                                                       int64_t n1, int64_t n2, int ell, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t rows = n1 * n2;
  if (e >= rows * ell) return;
  const int64_t c = e / rows;
  const int64_t row = e - c * rows;
  const int64_t ia = row / n2, ib = row - ia * n2;
  out[e] = f1[ia + n1 * c] * f2[ib + n2 * c];
}

// Small dense steps on one workgroup of kElimThreads threads.
//   kPinv:    in G (l1 x l2), out K^T = G (G^T G)^{-1}  (l1 x l2), the
//             transpose of the pseudo-inverse of a full-column-rank G;
//   kCholInv: in B (l2 x l2, symmetrised), out R^{-1} (l2 x l2), B = R^T R.
// A Cholesky breakdown raises kStatCholFail and writes zeros.
__global__ __launch_bounds__(kElimThreads) void kron_small_kernel(KronSmallArgs a) {
  __shared__ __align__(16) double g[kElimMaxEll * kElimPitch];
  __shared__ double gs[kElimMaxEll * kElimMaxEll];  // G (l1 x l2), then G R^{-1}
  __shared__ ElimShared es;
  const int tid = threadIdx.x;
  const int l1 = a.l1, l2 = a.l2;
  if (a.mode == kKronPinv) {
    for (int e = tid; e < l1 * l2; e += kElimThreads) gs[e] = a.in[e];
    __syncthreads();
    for (int e = tid; e < l2 * l2; e += kElimThreads) {
      const int i = e / l2, j = e % l2;
      double s = 0.0;
      for (int k = 0; k < l1; ++k) s += gs[k + l1 * i] * gs[k + l1 * j];
      g[i * kElimPitch + j] = s;
    }
  } else {
    for (int e = tid; e < l2 * l2; e += kElimThreads) {
      const int i = e / l2, j = e % l2;
      g[i * kElimPitch + j] = 0.5 * (a.in[i + l2 * j] + a.in[j + l2 * i]);
    }
  }
  // chol_inv_elim synchronises before it reads g
  const bool ok = chol_inv_elim(l2, 0.0, g, es);
  if (!ok) {
    if (tid == 0) raise_status(a.status, kStatCholFail);
    const int n = a.mode == kKronPinv ? l1 * l2 : l2 * l2;
    for (int e = tid; e < n; e += kElimThreads) a.out[e] = 0.0;
    return;
  }
  // g[m * pitch + i] = R^{-1}[m][i], upper triangular
  if (a.mode == kKronCholInv) {
    for (int e = tid; e < l2 * l2; e += kElimThreads) {
      const int m = e % l2, i = e / l2;
      a.out[e] = g[m * kElimPitch + i];  // column-major R^{-1}
    }
    return;
  }
  // T = G R^{-1} (l1 x l2) into gs, then K^T = T R^{-T}
  double tv[(kElimMaxEll * kElimMaxEll + kElimThreads - 1) / kElimThreads];
  int nt = 0;
  for (int e = tid; e < l1 * l2; e += kElimThreads, ++nt) {
    const int k = e % l1, j = e / l1;
    double s = 0.0;
    for (int i = 0; i <= j; ++i) s += gs[k + l1 * i] * g[i * kElimPitch + j];
    tv[nt] = s;
  }
  __syncthreads();
  nt = 0;
  for (int e = tid; e < l1 * l2; e += kElimThreads, ++nt) gs[e] = tv[nt];
  __syncthreads();
  for (int e = tid; e < l1 * l2; e += kElimThreads) {
    const int k = e % l1, j = e / l1;
    double s = 0.0;
    for (int i = j; i < l2; ++i) s += gs[k + l1 * i] * g[j * kElimPitch + i];  // R^{-T}[i][j] = R^{-1}[j][i]
    a.out[e] = s;
  }
}

// Leading eigenpairs -> scaled vectors: sigma_k = sqrt(max(ev_k, 0)),
// d[:, k] = w[:, k] / sigma_k (0 when sigma_k = 0); vals[k] = sigma_k
// (singular values) or max(ev_k - shift, 0) (Nystrom eigenvalues, shift read
// from *shift_dev).
__global__ __launch_bounds__(256) void kron_scale_kernel(const double* __restrict__ w, const double* __restrict__ ev,
                                                         int ell, int r, const double* shift_dev,
                                                         double* __restrict__ d, double* __restrict__ vals) {
  for (int e = threadIdx.x; e < ell * r; e += 256) {
    const int k = e / ell;
    const double s = sqrt(fmax(ev[k], 0.0));
    d[e] = s > 0.0 ? w[e] / s : 0.0;
  }
  for (int k = threadIdx.x; k < r; k += 256)
    vals[k] = shift_dev ? fmax(ev[k] - *shift_dev, 0.0) : sqrt(fmax(ev[k], 0.0));
}

// Nystrom shift nu = sqrt(N) u ||Y||_F (u = 2^-52, ||Y||_F^2 in *sumsq), and
// Y <- Y + nu Omega.
__global__ __launch_bounds__(256) void kron_shift_kernel(double* __restrict__ y, const double* __restrict__ omega,
                                                         int64_t count, double sqrt_n, const double* sumsq,
                                                         double* nu_out) {
  const double nu = sqrt_n * 0x1.0p-52 * sqrt(*sumsq);
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e == 0) *nu_out = nu;
  if (e < count) y[e] += nu * omega[e];
}

// Column k of U (rows x r, fp64): the entry of largest magnitude (lowest row
// on ties) made positive; the same sign goes to column k of V (if any).  One
// workgroup per column.
__global__ __launch_bounds__(256) void kron_sign_kernel(double* __restrict__ u, int64_t rows, double* __restrict__ v,
                                                        int64_t vrows) {
  __shared__ double sv[4];
  __shared__ int64_t sj[4];
  const int k = blockIdx.x;
  double* uc = u + rows * k;
  double best = -1.0;
  int64_t bj = rows;
  for (int64_t i = threadIdx.x; i < rows; i += 256) {
    const double x = fabs(uc[i]);
    if (x > best) {
      best = x;
      bj = i;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(best, off);
    const int64_t oj = __shfl_xor(bj, off);
    if (ov > best || (ov == best && oj < bj)) {
      best = ov;
      bj = oj;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    sv[threadIdx.x >> 6] = best;
    sj[threadIdx.x >> 6] = bj;
  }
  __syncthreads();
  best = sv[0];
  bj = sj[0];
  for (int w = 1; w < 4; ++w)
    if (sv[w] > best || (sv[w] == best && sj[w] < bj)) {
      best = sv[w];
      bj = sj[w];
    }
  const double sgn = (bj < rows && uc[bj] < 0.0) ? -1.0 : 1.0;
  __syncthreads();  // every thread has read uc[bj] before any flip
  if (sgn < 0.0) {
    for (int64_t i = threadIdx.x; i < rows; i += 256) uc[i] = -uc[i];
    if (v)
      for (int64_t i = threadIdx.x; i < vrows; i += 256) v[vrows * k + i] = -v[vrows * k + i];
  }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Partial A^T B over a chunk of kAtbRows rows: A (rows x la), B (rows x lb)
// fp64 column-major; partial block z holds out[i][j] (j fastest), the layout
// of the fixed-order reduction kernels.  The chunk of both matrices is staged
// in LDS; each thread owns la lb / 256 outputs.
__global__ __launch_bounds__(256) void kron_atb_kernel(const double* __restrict__ A, const double* __restrict__ B,
                                                       int64_t rows, int la, int lb, double* __restrict__ part) {
  __shared__ double as[kAtbRows * (kElimMaxEll + 1)];
  __shared__ double bs[kAtbRows * (kElimMaxEll + 1)];
  const int64_t r0 = (int64_t)blockIdx.x * kAtbRows;
  const int nr = (int)min<int64_t>(kAtbRows, rows - r0);
  constexpr int P = kElimMaxEll + 1;  // odd pitch: row k of the chunk at k * P
  for (int e = threadIdx.x; e < kAtbRows * la; e += 256) {
    const int k = e % kAtbRows, i = e / kAtbRows;
    as[k * P + i] = k < nr ? A[r0 + k + rows * i] : 0.0;
  }
  for (int e = threadIdx.x; e < kAtbRows * lb; e += 256) {
    const int k = e % kAtbRows, j = e / kAtbRows;
    bs[k * P + j] = k < nr ? B[r0 + k + rows * j] : 0.0;
  }
  __syncthreads();
  double* out = part + (int64_t)blockIdx.x * la * lb;
  for (int e = threadIdx.x; e < la * lb; e += 256) {
    const int i = e / lb, j = e % lb;
    double s0 = 0.0, s1 = 0.0;
    for (int k = 0; k < kAtbRows; k += 2) {
      s0 += as[k * P + i] * bs[k * P + j];
      s1 += as[(k + 1) * P + i] * bs[(k + 1) * P + j];
    }
    out[e] = s0 + s1;
  }
}

}  // namespace

hipError_t launch_kron_combine(const KronCombineArgs& a, hipStream_t st) {
  const int64_t n = a.n1 * a.n2 * a.ell;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(kron_combine_kernel, dim3(blocks_for(n)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_kron_krp(const double* f1, const double* f2, int64_t n1, int64_t n2, int ell, double* out,
                           hipStream_t st) {
  hipLaunchKernelGGL(kron_krp_kernel, dim3(blocks_for(n1 * n2 * ell)), dim3(256), 0, st, f1, f2, n1, n2, ell, out);
  return hipGetLastError();
}

hipError_t launch_kron_small(const KronSmallArgs& a, hipStream_t st) {
  if (a.l2 < 1 || a.l2 > kElimMaxEll || a.l1 < 1 || a.l1 > kElimMaxEll) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kron_small_kernel, dim3(1), dim3(kElimThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_kron_scale(const double* w, const double* ev, int ell, int r, const double* shift_dev, double* d,
                             double* vals, hipStream_t st) {
  hipLaunchKernelGGL(kron_scale_kernel, dim3(1), dim3(256), 0, st, w, ev, ell, r, shift_dev, d, vals);
  return hipGetLastError();
}

hipError_t launch_kron_shift(double* y, const double* omega, int64_t count, double sqrt_n, const double* sumsq,
                             double* nu_out, hipStream_t st) {
  hipLaunchKernelGGL(kron_shift_kernel, dim3(blocks_for(std::max<int64_t>(count, 1))), dim3(256), 0, st, y, omega,
                     count, sqrt_n, sumsq, nu_out);
  return hipGetLastError();
}

size_t kron_atb_bytes(int64_t rows, int la, int lb) {
  const int64_t parts = (rows + kAtbRows - 1) / kAtbRows;
  return align_up((size_t)parts * la * lb * sizeof(double)) + align_up(partial_reduce_lvl_bytes((int)parts, la, lb, 1));
}

hipError_t launch_kron_atb(const double* A, const double* B, int64_t rows, int la, int lb, double* out, void* ws,
                           hipStream_t st) {
  if (la < 1 || lb < 1 || la > kElimMaxEll || lb > kElimMaxEll) return hipErrorInvalidValue;
  const int64_t parts = (rows + kAtbRows - 1) / kAtbRows;
  double* part = reinterpret_cast<double*>(ws);
  char* lvl = reinterpret_cast<char*>(ws) + align_up((size_t)parts * la * lb * sizeof(double));
  hipLaunchKernelGGL(kron_atb_kernel, dim3((unsigned)parts), dim3(256), 0, st, A, B, rows, la, lb, part);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_partial_reduce(part, true, (int)parts, la, lb, lb, 1, lvl, out, nullptr, 1, st);
}

hipError_t launch_kron_sign(double* u, int64_t rows, int r, double* v, int64_t vrows, hipStream_t st) {
  hipLaunchKernelGGL(kron_sign_kernel, dim3(r), dim3(256), 0, st, u, rows, v, vrows);
  return hipGetLastError();
}

}  // namespace krp
