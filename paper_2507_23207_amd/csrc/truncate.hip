// FP64 truncation of the ell-sized core: for each mode i (in the sweep
// order) the r_i leading left singular vectors W_i of the current core's
// mode-i unfolding are the leading eigenvectors of its Gram matrix; the core
// is projected (G <- G x_i W_i^T) before the next mode, and the factors
// become Q_i W_i.  Eigenvectors come from a cyclic (round-robin parallel)
// Jacobi method in one workgroup.
#include "device_common.h"
#include "kernels.h"
#include "truncate.h"

#include <algorithm>

namespace krp {

namespace {

constexpr int kEigThreads = 256;
constexpr int kEigMax = 64;

// Gram matrix of mode `mode` of a fp64 tensor viewed as [P][l][Q]:
// gram[a + l b] = sum_{p,q} g[p, a, q] g[p, b, q].  One block per pair a <= b.
__global__ void mode_gram_kernel(const double* __restrict__ g, int64_t P, int l, int64_t Q,
                                 double* __restrict__ gram) {
  __shared__ double red[kEigThreads / 64];
  int pair = blockIdx.x;
  int b = 0;
  while ((b + 1) * (b + 2) / 2 <= pair) ++b;
  const int a = pair - b * (b + 1) / 2;
  double s = 0.0;
  const int64_t total = P * Q;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int64_t p = e % P, q = e / P;
    s += g[p + P * (a + (int64_t)l * q)] * g[p + P * (b + (int64_t)l * q)];
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    gram[a + (int64_t)l * b] = t;
    gram[b + (int64_t)l * a] = t;
  }
}

__global__ __launch_bounds__(kEigThreads) void jacobi_eig_kernel(int ell, int r, const double* a_in,
                                                                 int64_t a_stride, double* w,
                                                                 int64_t w_stride, double* evals,
                                                                 int64_t ev_stride) {
  __shared__ double A[kEigMax * kEigMax];
  __shared__ double V[kEigMax * kEigMax];
  __shared__ double cs[kEigMax / 2], sn[kEigMax / 2];
  __shared__ int pp[kEigMax / 2], qq[kEigMax / 2];
  __shared__ double red[kEigThreads / 64];
  __shared__ int order_idx[kEigMax];
  __shared__ int done;

  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int np = ell + (ell & 1);
  const double* ain = a_in + b * a_stride;
  for (int e = tid; e < np * np; e += kEigThreads) {
    const int i = e % np, j = e / np;
    double v = 0.0;
    if (i < ell && j < ell) v = ain[i + (int64_t)ell * j];
    else if (i == j) v = -1.0;  // padding index: decoupled, sorts last (the input is PSD)
    A[i + np * j] = v;
    V[i + np * j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int half = np / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    // convergence: sum of squared off-diagonal entries against the diagonal
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < np * np; e += kEigThreads) {
      const int i = e % np, j = e / np;
      const double v = A[e];
      if (i != j) off += v * v;
      else dia += v * v;
    }
    off = wave_sum(off);
    dia = wave_sum(dia);
    if ((tid & 63) == 0) red[tid >> 6] = off;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int k = 0; k < kEigThreads / 64; ++k) t += red[k];
      red[0] = t;
    }
    __syncthreads();
    const double off_all = red[0];
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = dia;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int k = 0; k < kEigThreads / 64; ++k) t += red[k];
      done = (off_all <= 1e-30 * t) ? 1 : 0;
    }
    __syncthreads();
    if (done) break;
    for (int round = 0; round < np - 1; ++round) {
      if (tid < half) {
        int p, q;
        if (tid == 0) {
          p = np - 1;
          q = round;
        } else {
          p = (round + tid) % (np - 1);
          q = (round - tid + np - 1) % (np - 1);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        const double apq = A[p + np * q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          const double app = A[p + np * p], aqq = A[q + np * q];
          const double theta = (aqq - app) / (2.0 * apq);
          const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
        }
        pp[tid] = p;
        qq[tid] = q;
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      // A <- A J (columns p, q of every row)
      for (int e = tid; e < np * half; e += kEigThreads) {
        const int i = e % np, k = e / np;
        const int p = pp[k], q = qq[k];
        const double c = cs[k], s = sn[k];
        const double aip = A[i + np * p], aiq = A[i + np * q];
        A[i + np * p] = c * aip - s * aiq;
        A[i + np * q] = s * aip + c * aiq;
      }
      __syncthreads();
      // A <- J^T A (rows p, q of every column) and V <- V J
      for (int e = tid; e < np * half; e += kEigThreads) {
        const int i = e % np, k = e / np;
        const int p = pp[k], q = qq[k];
        const double c = cs[k], s = sn[k];
        const double api = A[p + np * i], aqi = A[q + np * i];
        A[p + np * i] = c * api - s * aqi;
        A[q + np * i] = s * api + c * aqi;
        const double vip = V[i + np * p], viq = V[i + np * q];
        V[i + np * p] = c * vip - s * viq;
        V[i + np * q] = s * vip + c * viq;
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    // descending eigenvalues (stable: ties keep the lower index first)
    for (int i = 0; i < np; ++i) order_idx[i] = i;
    for (int i = 0; i < np; ++i) {
      int best = i;
      for (int j = i + 1; j < np; ++j)
        if (A[order_idx[j] * (np + 1)] > A[order_idx[best] * (np + 1)]) best = j;
      const int t = order_idx[i];
      order_idx[i] = order_idx[best];
      order_idx[best] = t;
    }
  }
  __syncthreads();
  double* wout = w + b * w_stride;
  for (int j = tid; j < r; j += kEigThreads) {
    const int c = order_idx[j];
    int imax = 0;
    double vmax = -1.0;
    for (int i = 0; i < ell; ++i) {
      const double v = fabs(V[i + np * c]);
      if (v > vmax) {
        vmax = v;
        imax = i;
      }
    }
    const double sgn = V[imax + np * c] < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < ell; ++i) wout[i + (int64_t)ell * j] = sgn * V[i + np * c];
    if (evals) evals[b * ev_stride + j] = A[c * (np + 1)];
  }
}

// out = q (n x l) * w (l x r), fp64; also in the storage type if out_s.
__global__ void small_gemm_kernel(const double* __restrict__ q, int64_t n, int l,
                                  const double* __restrict__ w, int r, double* out64, void* out_s,
                                  int out_double) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * r) return;
  const int64_t i = idx % n;
  const int j = (int)(idx / n);
  double s = 0.0;
  for (int k = 0; k < l; ++k) s += q[i + n * k] * w[k + (int64_t)l * j];
  if (out64) out64[idx] = s;
  if (out_s) {
    if (out_double)
      reinterpret_cast<double*>(out_s)[idx] = s;
    else
      reinterpret_cast<float*>(out_s)[idx] = (float)s;
  }
}

}  // namespace

TruncPlan plan_truncate(int d, const int* ell, const int* rank, const int64_t* dims, const int* order) {
  TruncPlan p;
  p.d = d;
  int64_t elems = 1;
  for (int k = 0; k < d; ++k) {
    p.ell[k] = ell[k];
    p.rank[k] = rank[k];
    p.order[k] = order[k];
    p.dims[k] = dims[k];
    elems *= ell[k];
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) / 256 * 256;
    return o;
  };
  p.off_g[0] = take(elems * sizeof(double));
  p.off_g[1] = take(elems * sizeof(double));
  p.off_gram = take((size_t)kEigMax * kEigMax * sizeof(double));
  for (int k = 0; k < d; ++k) p.off_w[k] = take((size_t)ell[k] * rank[k] * sizeof(double));
  for (int k = 0; k < d; ++k) p.off_qt[k] = take((size_t)dims[k] * rank[k] * sizeof(double));
  p.ws_bytes = off;
  return p;
}

double* truncated_q64(const TruncPlan& p, char* ws, int k) {
  return reinterpret_cast<double*>(ws + p.off_qt[k]);
}

hipError_t launch_sym_eig(int batch, int ell, int r, const double* a, int64_t a_stride, double* w,
                          int64_t w_stride, double* evals, int64_t ev_stride, hipStream_t st) {
  if (ell < 1 || ell > kEigMax || r < 1 || r > ell) return hipErrorInvalidValue;
  if (batch == 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_eig_kernel, dim3(batch), dim3(kEigThreads), 0, st, ell, r, a, a_stride, w,
                     w_stride, evals, ev_stride);
  return hipGetLastError();
}

hipError_t launch_truncate(const TruncPlan& p, const void* core, int core_double, double* const* q64,
                           void* core_out, void* const* q_out, int out_double, char* ws,
                           hipStream_t st) {
  const int d = p.d;
  int64_t cur[kMaxDims];
  int64_t elems = 1;
  for (int k = 0; k < d; ++k) {
    cur[k] = p.ell[k];
    elems *= cur[k];
  }
  double* g[2] = {reinterpret_cast<double*>(ws + p.off_g[0]), reinterpret_cast<double*>(ws + p.off_g[1])};
  hipError_t e = launch_cast(core, core_double, g[0], 1, elems, st);
  if (e != hipSuccess) return e;
  double* gram = reinterpret_cast<double*>(ws + p.off_gram);
  for (int s = 0; s < d; ++s) {
    const int i = p.order[s];
    int64_t P = 1, Q = 1;
    for (int k = 0; k < i; ++k) P *= cur[k];
    for (int k = i + 1; k < d; ++k) Q *= cur[k];
    const int l = (int)cur[i];
    const int npairs = l * (l + 1) / 2;
    hipLaunchKernelGGL(mode_gram_kernel, dim3(npairs), dim3(kEigThreads), 0, st, g[s & 1], P, l, Q, gram);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    double* wi = reinterpret_cast<double*>(ws + p.off_w[i]);
    e = launch_sym_eig(1, l, p.rank[i], gram, 0, wi, 0, nullptr, 0, st);
    if (e != hipSuccess) return e;
    TtmProblem tp;
    tp.g = g[s & 1];
    tp.g_is_double = 1;
    tp.d = d;
    for (int k = 0; k < d; ++k) tp.dims[k] = cur[k];
    tp.mode = i;
    tp.ell = p.rank[i];
    tp.prec = kFP64;
    tp.q64 = wi;
    tp.out = g[(s + 1) & 1];
    tp.out_is_double = 1;
    e = launch_ttm(tp, nullptr, st);
    if (e != hipSuccess) return e;
    cur[i] = p.rank[i];
  }
  for (int k = 0; k < d; ++k) {
    const int64_t n = p.dims[k];
    const int64_t cnt = n * p.rank[k];
    const unsigned grid = (unsigned)((cnt + 255) / 256);
    hipLaunchKernelGGL(small_gemm_kernel, dim3(grid), dim3(256), 0, st, q64[k], n, p.ell[k],
                       reinterpret_cast<const double*>(ws + p.off_w[k]), p.rank[k],
                       reinterpret_cast<double*>(ws + p.off_qt[k]), q_out[k], out_double);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  int64_t relems = 1;
  for (int k = 0; k < d; ++k) relems *= p.rank[k];
  return launch_cast(g[d & 1], 1, core_out, out_double, relems, st);
}

}  // namespace krp
