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
constexpr int kGramThreads = 256;
constexpr int kEigMax = 64;

// Gram matrix of mode `mode` of a fp64 tensor viewed as [P][l][Q]:
// gram[a + l b] = sum_{p,q} g[p, a, q] g[p, b, q].  One block per pair a <= b.
__global__ void mode_gram_kernel(const double* __restrict__ g, int64_t P, int l, int64_t Q,
                                 double* __restrict__ gram) {
  __shared__ double red[kGramThreads / 64];
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

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cyclic Jacobi with the round-robin ("chess tournament") ordering: in every
// round the np/2 disjoint pairs (p, q) are rotated at once.  A round reads
// A_cur and writes A_next = J^T A_cur J block by block (every 2x2 block
// {p1, q1} x {p2, q2} of A_next depends only on the same block of A_cur and
// the two rotations).  Every wave computes the round's rotations itself (so
// a round needs one workgroup barrier); pair indices are recomputed from the
// round number; each thread owns one row pair k1 (and one pair of V's
// columns) and loads every input of its tasks before it stores any result.
// Sweeps stop when the off-diagonal Frobenius norm is below 1e-13 of the
// diagonal's.
constexpr int kJBlocks = 4;  // block tasks per thread: ceil(32 / (256 / 32))
constexpr int kJVtasks = 8;  // V tasks per thread: ceil(64 / (256 / 32))

// Pair k of round `round` in the round-robin schedule over np indices.
__device__ __forceinline__ void jacobi_pair(int round, int k, int np, int& p, int& q) {
  const int m = np - 1;
  if (k == 0) {
    p = m;
    q = round;
  } else {
    p = round + k;
    if (p >= m) p -= m;
    q = round - k;
    if (q < 0) q += m;
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

__global__ __launch_bounds__(kEigThreads) void jacobi_eig_kernel(int ell, int r, const double* a_in,
                                                                 int64_t a_stride, double* w,
                                                                 int64_t w_stride, double* evals,
                                                                 int64_t ev_stride) {
  constexpr int P = kEigMax + 1;
  constexpr int NW = kEigThreads / 64;
  __shared__ double A[2][kEigMax * P];
  __shared__ double V[kEigMax * P];
  __shared__ double2 rcs[NW][kEigMax / 2];
  __shared__ double red[2][NW];
  __shared__ int order_idx[kEigMax];

  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int np = ell + (ell & 1);
  const int half = np / 2;
  const int cpp = kEigThreads / half;  // thread columns per pass (>= 8)
  const bool active = tid < half * cpp;
  const int k1 = tid % half, kb = tid / half;
  const double* ain = a_in + b * a_stride;
  for (int e = tid; e < np * np; e += kEigThreads) {
    const int i = e % np, j = e / np;
    double v = 0.0;
    if (i < ell && j < ell) v = ain[i + (int64_t)ell * j];
    else if (i == j) v = -1.0;  // padding index: decoupled, sorts last (the input is PSD)
    A[0][i * P + j] = v;
    V[i * P + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  int cur = 0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < np * np; e += kEigThreads) {
      const int i = e % np, j = e / np;
      const double v = A[cur][i * P + j];
      if (i != j) off += v * v;
      else dia += v * v;
    }
    off = wave_sum(off);
    dia = wave_sum(dia);
    if (lane == 0) {
      red[0][wave] = off;
      red[1][wave] = dia;
    }
    __syncthreads();
    double to = 0.0, td = 0.0;
    for (int k = 0; k < NW; ++k) {
      to += red[0][k];
      td += red[1][k];
    }
    __syncthreads();
    if (to <= 1e-26 * td) break;
    for (int round = 0; round < np - 1; ++round) {
      const double* Ac = A[cur];
      double* An = A[cur ^ 1];
      if (lane < half) {
        int p, q;
        jacobi_pair(round, lane, np, p, q);
        const double apq = Ac[p * P + q];
        const double app = Ac[p * P + p], aqq = Ac[q * P + q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          const double theta = (aqq - app) / (2.0 * apq);
          const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
        }
        rcs[wave][lane] = make_double2(c, s);
      }
      wave_sync();
      if (active) {
        int p1, q1;
        jacobi_pair(round, k1, np, p1, q1);
        const double2 r1 = rcs[wave][k1];
        int p2[kJBlocks], q2[kJBlocks], pv[kJVtasks];
        double2 r2[kJBlocks];
        double bb[kJBlocks][4], v0[kJVtasks], v1[kJVtasks];
        // loads
#pragma unroll
        for (int u = 0; u < kJBlocks; ++u) {
          const int k2 = kb + u * cpp;
          if (k2 < half) {
            jacobi_pair(round, k2, np, p2[u], q2[u]);
            r2[u] = rcs[wave][k2];
            bb[u][0] = Ac[p1 * P + p2[u]];
            bb[u][1] = Ac[p1 * P + q2[u]];
            bb[u][2] = Ac[q1 * P + p2[u]];
            bb[u][3] = Ac[q1 * P + q2[u]];
          }
        }
#pragma unroll
        for (int u = 0; u < kJVtasks; ++u) {
          const int i = kb + u * cpp;
          if (i < np) {
            pv[u] = i * P;
            v0[u] = V[pv[u] + p1];
            v1[u] = V[pv[u] + q1];
          }
        }
        // rotations and stores
#pragma unroll
        for (int u = 0; u < kJBlocks; ++u) {
          const int k2 = kb + u * cpp;
          if (k2 < half) {
            const double c2 = r2[u].x, s2 = r2[u].y, c1 = r1.x, s1 = r1.y;
            const double t00 = c2 * bb[u][0] - s2 * bb[u][1], t01 = s2 * bb[u][0] + c2 * bb[u][1];
            const double t10 = c2 * bb[u][2] - s2 * bb[u][3], t11 = s2 * bb[u][2] + c2 * bb[u][3];
            double n00 = c1 * t00 - s1 * t10, n01 = c1 * t01 - s1 * t11;
            double n10 = s1 * t00 + c1 * t10, n11 = s1 * t01 + c1 * t11;
            if (k2 == k1) {
              n01 = 0.0;
              n10 = 0.0;
            }
            An[p1 * P + p2[u]] = n00;
            An[p1 * P + q2[u]] = n01;
            An[q1 * P + p2[u]] = n10;
            An[q1 * P + q2[u]] = n11;
          }
        }
#pragma unroll
        for (int u = 0; u < kJVtasks; ++u) {
          const int i = kb + u * cpp;
          if (i < np) {
            V[pv[u] + p1] = r1.x * v0[u] - r1.y * v1[u];
            V[pv[u] + q1] = r1.y * v0[u] + r1.x * v1[u];
          }
        }
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  // descending eigenvalues by ranking (ties keep the lower index first)
  if (tid < np) order_idx[tid] = tid;
  __syncthreads();
  if (tid < np) {
    const double li = A[cur][tid * (P + 1)];
    int rank = 0;
    for (int j = 0; j < np; ++j) {
      const double lj = A[cur][j * (P + 1)];
      rank += (lj > li || (lj == li && j < tid)) ? 1 : 0;
    }
    order_idx[rank] = tid;
  }
  __syncthreads();
  double* wout = w + b * w_stride;
  for (int j = tid; j < r; j += kEigThreads) {
    const int c = order_idx[j];
    int imax = 0;
    double vmax = -1.0;
    for (int i = 0; i < ell; ++i) {
      const double v = fabs(V[i * P + c]);
      if (v > vmax) {
        vmax = v;
        imax = i;
      }
    }
    const double sgn = V[imax * P + c] < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < ell; ++i) wout[i + (int64_t)ell * j] = sgn * V[i * P + c];
    if (evals) evals[b * ev_stride + j] = A[cur][c * (P + 1)];
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
    hipLaunchKernelGGL(mode_gram_kernel, dim3(npairs), dim3(kGramThreads), 0, st, g[s & 1], P, l, Q, gram);
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
