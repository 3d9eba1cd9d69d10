// Thin QR of tall-skinny sketches (Algorithm 7, step 4; Algorithm 8, step 5;
// Algorithm 6, step 3) by CholeskyQR2 in fp64, one workgroup per matrix:
//   G = Y^T Y,  R = chol(G) (upper, positive diagonal),  Q = Y R^{-1},
// repeated once on Q.  A pivot that is non-positive, non-finite or below
// 1e-14 of its column's squared norm marks Y as too ill-conditioned for the
// Gram route; that pass is then redone on G + s I with
// s = 11 (n l + l (l + 1)) 2^-53 ||Y||_F^2 (shifted CholeskyQR, Fukaya et al.
// 2020) and followed by two unshifted passes (shifted CholeskyQR3).  Since
// diag(R) > 0 the result equals the Householder Q with positive-diagonal R.
#include "device_common.h"
#include "kernels.h"

namespace krp {

namespace {

constexpr int kQrMaxEll = 64;
constexpr int kQrThreads = 512;
constexpr int kQrChunk = 32;  // rows staged in LDS at a time

struct QrShared {
  double g[kQrMaxEll * kQrMaxEll];       // Gram, then R in its upper triangle and R^{-1} (transposed) below
  double rinv_diag[kQrMaxEll];
  double chunk[kQrChunk * kQrMaxEll];    // row chunk, column-major [col][row]
  double trace;
  int fail;
};

// Gram matrix of src (n x ell column-major) into sh.g (upper triangle + mirror).
__device__ void qr_gram(const double* src, int64_t n, int ell, QrShared& sh) {
  const int tid = threadIdx.x;
  const int npairs = ell * (ell + 1) / 2;
  double acc[(kQrMaxEll * (kQrMaxEll + 1) / 2 + kQrThreads - 1) / kQrThreads];
  constexpr int kU = (kQrMaxEll * (kQrMaxEll + 1) / 2 + kQrThreads - 1) / kQrThreads;
  int pi[kU], pj[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    acc[u] = 0.0;
    int p = tid + u * kQrThreads;
    int i = 0;
    // pair p -> (i, j), i <= j, enumerated column by column of the upper triangle
    int j = 0;
    if (p < npairs) {
      // j such that j(j+1)/2 <= p < (j+1)(j+2)/2
      j = (int)((__builtin_sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
      while ((j + 1) * (j + 2) / 2 <= p) ++j;
      while (j * (j + 1) / 2 > p) --j;
      i = p - j * (j + 1) / 2;
    }
    pi[u] = i;
    pj[u] = j;
  }
  for (int64_t r0 = 0; r0 < n; r0 += kQrChunk) {
    const int rc = (int)min<int64_t>(kQrChunk, n - r0);
    __syncthreads();
    for (int e = tid; e < kQrChunk * ell; e += kQrThreads) {
      const int c = e / kQrChunk, r = e - c * kQrChunk;
      sh.chunk[c * kQrChunk + r] = (r < rc) ? src[r0 + r + n * c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (tid + u * kQrThreads < npairs) {
        const double* ci = sh.chunk + pi[u] * kQrChunk;
        const double* cj = sh.chunk + pj[u] * kQrChunk;
        double s = acc[u];
#pragma unroll 8
        for (int r = 0; r < kQrChunk; ++r) s += ci[r] * cj[r];
        acc[u] = s;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    if (tid + u * kQrThreads < npairs) {
      sh.g[pi[u] * kQrMaxEll + pj[u]] = acc[u];
      sh.g[pj[u] * kQrMaxEll + pi[u]] = acc[u];
    }
  }
  __syncthreads();
}

// In-place upper Cholesky of sh.g (+ shift on the diagonal).  Returns true on
// success; R overwrites the upper triangle.
__device__ bool qr_chol(int ell, double shift, QrShared& sh) {
  const int tid = threadIdx.x;
  if (tid < ell) sh.rinv_diag[tid] = sh.g[tid * kQrMaxEll + tid];  // original diagonal
  if (tid == 0) sh.fail = 0;
  __syncthreads();
  if (shift != 0.0) {
    if (tid < ell) sh.g[tid * kQrMaxEll + tid] += shift;
    __syncthreads();
  }
  for (int k = 0; k < ell; ++k) {
    if (tid == 0) {
      const double dk = sh.g[k * kQrMaxEll + k];
      const double ref = sh.rinv_diag[k] + shift;
      if (!(dk > 1e-14 * ref) || !isfinite(dk)) {
        sh.fail = 1;
      } else {
        sh.g[k * kQrMaxEll + k] = __builtin_sqrt(dk);
      }
    }
    __syncthreads();
    if (sh.fail) return false;
    const double rkk = sh.g[k * kQrMaxEll + k];
    for (int j = k + 1 + tid; j < ell; j += kQrThreads) sh.g[k * kQrMaxEll + j] /= rkk;
    __syncthreads();
    const int m = ell - k - 1;
    for (int e = tid; e < m * m; e += kQrThreads) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      if (i <= j) sh.g[i * kQrMaxEll + j] -= sh.g[k * kQrMaxEll + i] * sh.g[k * kQrMaxEll + j];
    }
    __syncthreads();
  }
  return true;
}

// R^{-1} (upper) stored transposed in the strict lower triangle of sh.g plus
// its diagonal in sh.rinv_diag; one thread per column, back substitution.
__device__ void qr_rinv(int ell, QrShared& sh) {
  const int j = threadIdx.x;
  if (j < ell) {
    const double djj = 1.0 / sh.g[j * kQrMaxEll + j];
    sh.rinv_diag[j] = djj;
    // x_i = -(sum_{k=i+1..j} R[i][k] x_k) / R[i][i], x_j = 1 / R[j][j]
    for (int i = j - 1; i >= 0; --i) {
      double s = sh.g[i * kQrMaxEll + j] * djj;
      for (int k = i + 1; k < j; ++k) s += sh.g[i * kQrMaxEll + k] * sh.g[j * kQrMaxEll + k];
      sh.g[j * kQrMaxEll + i] = -s / sh.g[i * kQrMaxEll + i];
    }
  }
  __syncthreads();
}

// dst = src R^{-1} (rows staged in LDS, so dst may alias src).
template <bool FINAL>
__device__ void qr_apply(const double* src, double* dst, int64_t n, int ell, void* q_out,
                         int out_double, QrShared& sh) {
  const int tid = threadIdx.x;
  for (int64_t r0 = 0; r0 < n; r0 += kQrChunk) {
    const int rc = (int)min<int64_t>(kQrChunk, n - r0);
    __syncthreads();
    for (int e = tid; e < kQrChunk * ell; e += kQrThreads) {
      const int c = e / kQrChunk, r = e - c * kQrChunk;
      sh.chunk[c * kQrChunk + r] = (r < rc) ? src[r0 + r + n * c] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < kQrChunk * ell; e += kQrThreads) {
      const int j = e / kQrChunk, r = e - j * kQrChunk;
      if (r < rc) {
        double s = sh.chunk[j * kQrChunk + r] * sh.rinv_diag[j];
        for (int k = 0; k < j; ++k) s += sh.chunk[k * kQrChunk + r] * sh.g[j * kQrMaxEll + k];
        const int64_t o = r0 + r + n * j;
        dst[o] = s;
        if (FINAL && q_out) {
          if (out_double)
            reinterpret_cast<double*>(q_out)[o] = s;
          else
            reinterpret_cast<float*>(q_out)[o] = (float)s;
        }
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kQrThreads) void cholqr_kernel(int64_t n_default, int ell,
                                                            const double* y, double* q,
                                                            void* q_out, int out_double,
                                                            const int64_t* offsets,
                                                            const int64_t* nrows, int* status) {
  __shared__ QrShared sh;
  const int b = blockIdx.x;
  const int64_t off = offsets ? offsets[b] : 0;
  const int64_t n = nrows ? nrows[b] : n_default;
  const double* src = y + off;
  double* dst = q + off;
  char* qo = nullptr;
  if (q_out) qo = reinterpret_cast<char*>(q_out) + off * (out_double ? 8 : 4);

  int clean = 0;  // consecutive unshifted passes
  bool shifted_once = false;
  for (int pass = 0; pass < 6; ++pass) {
    qr_gram(src, n, ell, sh);
    if (threadIdx.x == 0) {
      double tr = 0.0;
      for (int k = 0; k < ell; ++k) tr += sh.g[k * kQrMaxEll + k];
      sh.trace = tr;
    }
    __syncthreads();
    const double tr = sh.trace;
    if (!isfinite(tr)) {
      if (threadIdx.x == 0) raise_status(status, kStatNonFinite);
      // propagate NaN into Q
      for (int64_t e = threadIdx.x; e < n * ell; e += kQrThreads) {
        dst[e] = __builtin_nan("");
        if (qo) {
          if (out_double)
            reinterpret_cast<double*>(qo)[e] = __builtin_nan("");
          else
            reinterpret_cast<float*>(qo)[e] = __builtin_nanf("");
        }
      }
      return;
    }
    bool ok = qr_chol(ell, 0.0, sh);
    if (ok) {
      ++clean;
    } else {
      if (threadIdx.x == 0) raise_status(status, kStatCholShift);
      shifted_once = true;
      qr_gram(src, n, ell, sh);
      const double shift = 11.0 * ((double)n * ell + (double)ell * (ell + 1)) * 0x1.0p-53 * tr;
      if (!qr_chol(ell, shift, sh)) {
        if (threadIdx.x == 0) raise_status(status, kStatCholFail);
        return;
      }
      clean = 0;
    }
    qr_rinv(ell, sh);
    const bool last = (clean == 2);
    if (last)
      qr_apply<true>(src, dst, n, ell, qo, out_double, sh);
    else
      qr_apply<false>(src, dst, n, ell, nullptr, out_double, sh);
    src = dst;
    if (last) return;
  }
  (void)shifted_once;
  if (threadIdx.x == 0) raise_status(status, kStatCholFail);
}

}  // namespace

hipError_t launch_cholqr(int batch, int64_t n, int ell, const double* y64, double* q64, void* q_out,
                         int out_is_double, const int64_t* offsets, const int64_t* nrows, int* status,
                         hipStream_t st) {
  if (ell > kQrMaxEll || ell < 1) return hipErrorInvalidValue;
  if (batch == 0) return hipSuccess;
  hipLaunchKernelGGL(cholqr_kernel, dim3(batch), dim3(kQrThreads), 0, st, n, ell, y64, q64, q_out,
                     out_is_double, offsets, nrows, status);
  return hipGetLastError();
}

}  // namespace krp
