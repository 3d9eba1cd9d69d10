// Sensor placement (Section 6): sensor indices from a column-pivoted QR of
// Q_i^T, interpolation factors A_i = Q_i (P_i^T Q_i)^{-1}, measurement of a
// field on the sensor grid and the transposed factors the reconstruction
// multiplies with (T_hat x_1 A_1 ... x_d A_d runs on the TTM kernels).
//
// The pivoted QR is greedy (Businger-Golub) column pivoting carried out with
// modified Gram-Schmidt on the columns of Q_i^T: one workgroup per mode keeps
// the residual of every column (an fp64 copy of Q_i, column j of Q_i^T being
// row j of Q_i, so a residual component is read coalesced across threads),
// takes the column of largest residual norm (lowest index on ties), projects
// its direction out of all columns not yet taken and recomputes their norms
// in the same pass.  Q_i has at most 64 columns; the rows are unbounded.
#include "device_common.h"
#include "sensor.h"

#include <algorithm>
#include <cmath>

namespace krp {

namespace {

constexpr int kPivThreads = 512;
constexpr int kPivWaves = kPivThreads / 64;
// A pivot whose residual norm is at most 64 unit roundoffs of the largest
// row norm of Q counts as zero (Q has fewer than ell independent columns).
constexpr double kSingularRel = 64.0 * 1.1102230246251565e-16;

template <typename T>
__device__ __forceinline__ T ld(const void* p, int64_t i) {
  return reinterpret_cast<const T*>(p)[i];
}

// (value, index) maximum over the workgroup; ties go to the lower index.
// Returns the winner in every thread.
__device__ __forceinline__ void block_argmax(double& v, int64_t& j, double* sv, int64_t* sj) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int64_t oj = __shfl_xor(j, off);
    if (ov > v || (ov == v && oj < j)) {
      v = ov;
      j = oj;
    }
  }
  if (lane == 0) {
    sv[wave] = v;
    sj[wave] = j;
  }
  __syncthreads();
  v = sv[0];
  j = sj[0];
#pragma unroll
  for (int w = 1; w < kPivWaves; ++w) {
    if (sv[w] > v || (sv[w] == v && sj[w] < j)) {
      v = sv[w];
      j = sj[w];
    }
  }
  __syncthreads();  // sv/sj are reused by the next call
}

template <typename Tq>
__global__ __launch_bounds__(kPivThreads) void sensor_pivot_kernel(SensorSelectArgs a) {
  extern __shared__ __align__(16) double aug[];  // ell x (2 ell + 1): [M | I] of the inversion
  __shared__ double u[64];
  __shared__ double sv[kPivWaves];
  __shared__ int64_t sj[kPivWaves];
  __shared__ int64_t sel[64];
  __shared__ double fac[64];
  __shared__ int s_fail;
  __shared__ int s_piv;

  const SensorMode& m = a.mode[blockIdx.x];
  const int64_t n = m.n;
  const int ell = m.ell;
  const int tid = threadIdx.x;
  double* W = m.w;
  if (tid == 0) s_fail = 0;
  __syncthreads();

  // residual <- Q (fp64), column norms of Q^T, finiteness
  double bv = -1.0;
  int64_t bj = n;
  bool bad = false;
  for (int64_t j = tid; j < n; j += kPivThreads) {
    double nv = 0.0;
    for (int k = 0; k < ell; ++k) {
      const double x = (double)ld<Tq>(m.q, j + n * k);
      bad |= !isfinite(x);
      W[j + n * k] = x;
      nv += x * x;
    }
    m.taken[j] = 0;
    if (nv > bv) {
      bv = nv;
      bj = j;
    }
  }
  if (bad) {
    s_fail = kStatNonFinite;  // benign race: every writer stores the same value
    raise_status(a.status, kStatNonFinite);
  }
  __syncthreads();

  int fail = s_fail;
  int steps = 0;
  double floor2 = 0.0;  // squared residual norm below which Q^T counts as rank-deficient
  for (int s = 0; s < ell && !fail; ++s) {
    block_argmax(bv, bj, sv, sj);
    // bv: squared residual norm of the pivot (uniform across the workgroup);
    // the first pivot has the largest row norm of Q
    if (s == 0) floor2 = bv * kSingularRel * kSingularRel;
    if (!(bv > floor2) || bj >= n) {
      fail = kStatSingular;
      break;
    }
    const int64_t p = bj;
    const double rinv = 1.0 / sqrt(bv);
    if (tid < ell) u[tid] = W[p + n * tid] * rinv;
    if (tid == 0) {
      sel[s] = p;
      m.taken[p] = 1;
    }
    __syncthreads();
    steps = s + 1;
    if (s + 1 == ell) break;
    // project u out of every column not taken; the new norms give the next pivot
    bv = -1.0;
    bj = n;
    for (int64_t j = tid; j < n; j += kPivThreads) {
      if (m.taken[j]) continue;
      double c = 0.0;
      for (int k = 0; k < ell; ++k) c += u[k] * W[j + n * k];
      double nv = 0.0;
      for (int k = 0; k < ell; ++k) {
        const double x = W[j + n * k] - c * u[k];
        W[j + n * k] = x;
        nv += x * x;
      }
      if (nv > bv) {
        bv = nv;
        bj = j;
      }
    }
    __syncthreads();
  }
  if (fail == kStatSingular && tid == 0) raise_status(a.status, kStatSingular);

  // (P^T Q)^{-1} by Gauss-Jordan elimination with partial pivoting on [M | I]
  const int pitch = 2 * ell + 1;
  if (!fail) {
    for (int e = tid; e < ell * 2 * ell; e += kPivThreads) {
      const int r = e / (2 * ell), c = e % (2 * ell);
      aug[r * pitch + c] = c < ell ? (double)ld<Tq>(m.q, sel[r] + n * c) : (c - ell == r ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int k = 0; k < ell; ++k) {
      if (tid < 64) {
        // pivot row: largest |a_rk|, r >= k (lowest index on ties)
        double v = -1.0;
        int64_t j = ell;
        for (int r = k + tid; r < ell; r += 64) {
          const double x = fabs(aug[r * pitch + k]);
          if (x > v) {
            v = x;
            j = r;
          }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          const double ov = __shfl_xor(v, off);
          const int64_t oj = __shfl_xor(j, off);
          if (ov > v || (ov == v && oj < j)) {
            v = ov;
            j = oj;
          }
        }
        if (tid == 0) {
          s_piv = (int)j;
          if (!(v > 0.0)) s_fail = kStatSingular;
        }
      }
      __syncthreads();
      if (s_fail) break;
      const int pr = s_piv;
      if (pr != k)
        for (int c = tid; c < 2 * ell; c += kPivThreads) {
          const double t = aug[k * pitch + c];
          aug[k * pitch + c] = aug[pr * pitch + c];
          aug[pr * pitch + c] = t;
        }
      __syncthreads();
      const double pinv = 1.0 / aug[k * pitch + k];
      if (tid < ell) fac[tid] = aug[tid * pitch + k];
      __syncthreads();
      for (int c = tid; c < 2 * ell; c += kPivThreads) aug[k * pitch + c] *= pinv;
      __syncthreads();
      for (int e = tid; e < ell * 2 * ell; e += kPivThreads) {
        const int r = e / (2 * ell), c = e % (2 * ell);
        if (r != k) aug[r * pitch + c] -= fac[r] * aug[k * pitch + c];
      }
      __syncthreads();
    }
    fail = s_fail;
    if (fail && tid == 0) raise_status(a.status, kStatSingular);
  }
  // M^{-1} (column-major) and the sensor indices in pivot order; after a
  // failure the indices are -1 and M^{-1} (so the factor A) is zero
  for (int e = tid; e < ell * ell; e += kPivThreads) {
    const int r = e % ell, c = e / ell;
    m.minv[e] = fail ? 0.0 : aug[r * pitch + ell + c];
  }
  for (int k = tid; k < ell; k += kPivThreads) m.idx[k] = fail || k >= steps ? -1 : (int32_t)sel[k];
}

// A[j, c] = sum_k Q[j, k] Minv[k, c]; one thread per entry, j fastest.
template <typename Tq>
__global__ __launch_bounds__(256) void sensor_apply_kernel(SensorSelectArgs a) {
  __shared__ double mi[64 * 64];
  const SensorMode& m = a.mode[blockIdx.y];
  const int ell = m.ell;
  for (int e = threadIdx.x; e < ell * ell; e += 256) mi[e] = m.minv[e];
  __syncthreads();
  const int64_t n = m.n;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * ell) return;
  const int64_t j = e % n;
  const int c = (int)(e / n);
  double acc = 0.0;
  for (int k = 0; k < ell; ++k) acc += (double)ld<Tq>(m.q, j + n * k) * mi[k + ell * c];
  reinterpret_cast<Tq*>(m.a)[e] = (Tq)acc;
}

// T_hat[j_1, .., j_d, b] = T[idx_1[j_1], .., idx_d[j_d], b]; an index outside
// its mode gives NaN (never an access outside T).
template <typename T>
__global__ __launch_bounds__(256) void sensor_measure_kernel(SensorMeasureArgs a) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= a.total) return;
  int64_t rem = e, src = 0, stride = 1;
  bool bad = false;
  for (int i = 0; i < a.d; ++i) {
    const int64_t ji = rem % a.ell[i];
    rem /= a.ell[i];
    const int64_t v = a.idx[i][ji];
    const bool ok = v >= 0 && v < a.dims[i];
    bad |= !ok;
    src += (ok ? v : 0) * stride;
    stride *= a.dims[i];
  }
  src += rem * stride;  // snapshot index
  const T x = reinterpret_cast<const T*>(a.t)[src];
  reinterpret_cast<T*>(a.out)[e] = bad ? (T)__builtin_nan("") : x;
}

// At[k + ell j] = A[j + n k] in fp64 (the TTM operand of the reconstruction).
template <typename T>
__global__ __launch_bounds__(256) void sensor_transpose_kernel(const void* A, int64_t n, int ell, double* At) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * ell) return;
  const int k = (int)(e % ell);
  const int64_t j = e / ell;
  At[e] = (double)reinterpret_cast<const T*>(A)[j + n * k];
}

// Expansion T x_i A of one mode (a reduction of length ell <= LMAX, an output
// mode of N >= ell): out[p, c, q] = sum_a A[c, a] g[p, a, q] for g viewed as
// P x ell x Q and out as P x N x Q.  Output-bound: the products run on the
// vector ALUs in the storage precision.
//
// P > 1: a wave owns 64 consecutive p of one q and holds g[p, :, q] in
// registers (zero past ell); the block's chunk of A rows sits in LDS as
// [c][a] and every lane reads the same entry (broadcast); loads of g and
// stores of out are coalesced along p.
template <typename T, int LMAX>
__global__ __launch_bounds__(256) void sensor_expand_cols_kernel(SensorExpandArgs e) {
  __shared__ T As[kExpandLds / sizeof(T)];
  const int c0 = blockIdx.y * e.cc;
  const int cn = (int)min<int64_t>(e.cc, e.n - c0);
  const T* A = reinterpret_cast<const T*>(e.a);
  for (int i = threadIdx.x; i < cn * LMAX; i += 256) {
    const int c = i / LMAX, a = i % LMAX;
    As[i] = a < e.ell ? A[(c0 + c) + e.n * a] : (T)0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= e.items) return;
  const int64_t q = item / e.p_tiles;
  const int64_t p = (item % e.p_tiles) * 64 + lane;
  if (p >= e.p) return;
  const T* g = reinterpret_cast<const T*>(e.g) + p + e.p * e.ell * q;
  T gv[LMAX];
#pragma unroll
  for (int a = 0; a < LMAX; ++a) gv[a] = a < e.ell ? g[e.p * a] : (T)0;
  T* out = reinterpret_cast<T*>(e.out) + p + e.p * (c0 + e.n * q);
  // four output rows at a time: independent sums keep the LDS reads in flight
  int c = 0;
  for (; c + 3 < cn; c += 4) {
    T acc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < LMAX; ++a)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += As[(c + u) * LMAX + a] * gv[a];
#pragma unroll
    for (int u = 0; u < 4; ++u) out[e.p * (c + u)] = acc[u];
  }
  for (; c < cn; ++c) {
    T acc = 0;
#pragma unroll
    for (int a = 0; a < LMAX; ++a) acc += As[c * LMAX + a] * gv[a];
    out[e.p * c] = acc;
  }
}

// P == 1 (mode 1 of the tensor): out[c + N q] = sum_a A[c, a] g[a + ell q].
// A workgroup owns 256 consecutive c (rows of A in registers) and a block of
// kExpandRowsQ values of q, whose columns of g it stages in LDS with
// coalesced loads; every lane then reads the same LDS entry (broadcast) and
// the stores are coalesced along c.
template <typename T, int LMAX>
__global__ __launch_bounds__(256) void sensor_expand_rows_kernel(SensorExpandArgs e) {
  constexpr int QB = kExpandRowsQ;
  __shared__ T gs[QB * LMAX];
  const int64_t q0 = (int64_t)blockIdx.x * QB;
  const int qn = (int)min<int64_t>(QB, e.q - q0);
  const T* g = reinterpret_cast<const T*>(e.g) + e.ell * q0;
  for (int i = threadIdx.x; i < QB * LMAX; i += blockDim.x) {
    const int qq = i / LMAX, a = i % LMAX;
    gs[i] = (qq < qn && a < e.ell) ? g[a + e.ell * qq] : (T)0;
  }
  const int64_t c = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  const bool cv = c < e.n;
  const T* A = reinterpret_cast<const T*>(e.a);
  T ar[LMAX];
#pragma unroll
  for (int a = 0; a < LMAX; ++a) ar[a] = (cv && a < e.ell) ? A[c + e.n * a] : (T)0;
  __syncthreads();
  if (!cv) return;
  T* out = reinterpret_cast<T*>(e.out) + c + e.n * q0;
  for (int qq = 0; qq < qn; ++qq) {
    T acc = 0;
#pragma unroll
    for (int a = 0; a < LMAX; ++a) acc += ar[a] * gs[qq * LMAX + a];
    out[e.n * qq] = acc;
  }
}

template <typename T, int LMAX>
hipError_t expand_go(SensorExpandArgs e, hipStream_t st) {
  if (e.p > 1) {
    e.cc = (int)std::min<int64_t>(e.n, kExpandLds / (LMAX * sizeof(T)));
    e.p_tiles = (e.p + 63) / 64;
    e.items = e.p_tiles * e.q;
    const dim3 grid((unsigned)((e.items + 3) / 4), (unsigned)((e.n + e.cc - 1) / e.cc));
    hipLaunchKernelGGL((sensor_expand_cols_kernel<T, LMAX>), grid, dim3(256), 0, st, e);
  } else {
    const dim3 grid((unsigned)((e.q + kExpandRowsQ - 1) / kExpandRowsQ), (unsigned)((e.n + 255) / 256));
    hipLaunchKernelGGL((sensor_expand_rows_kernel<T, LMAX>), grid, dim3(256), 0, st, e);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t expand_dispatch(const SensorExpandArgs& e, hipStream_t st) {
  if (e.ell <= 8) return expand_go<T, 8>(e, st);
  if (e.ell <= 16) return expand_go<T, 16>(e, st);
  if (e.ell <= 32) return expand_go<T, 32>(e, st);
  return expand_go<T, 64>(e, st);
}

}  // namespace

hipError_t launch_sensor_expand(const SensorExpandArgs& e, int is_double, hipStream_t st) {
  if (e.ell < 1 || e.ell > kExpandMaxEll || e.n < 1) return hipErrorInvalidValue;
  if (e.p * e.q == 0) return hipSuccess;
  return is_double ? expand_dispatch<double>(e, st) : expand_dispatch<float>(e, st);
}

size_t sensor_pivot_lds(int ell_max) { return (size_t)ell_max * (2 * ell_max + 1) * sizeof(double); }

hipError_t launch_sensor_select(const SensorSelectArgs& a, int q_is_double, hipStream_t st) {
  int ell_max = 1;
  int64_t work_max = 1;
  for (int i = 0; i < a.nmodes; ++i) {
    ell_max = std::max(ell_max, a.mode[i].ell);
    work_max = std::max(work_max, a.mode[i].n * a.mode[i].ell);
  }
  const size_t lds = sensor_pivot_lds(ell_max);
  auto piv = q_is_double ? sensor_pivot_kernel<double> : sensor_pivot_kernel<float>;
  hipError_t e = hipFuncSetAttribute((const void*)piv, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)sensor_pivot_lds(64));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(piv, dim3(a.nmodes), dim3(kPivThreads), lds, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)((work_max + 255) / 256), (unsigned)a.nmodes);
  if (q_is_double)
    hipLaunchKernelGGL(sensor_apply_kernel<double>, grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(sensor_apply_kernel<float>, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_sensor_measure(const SensorMeasureArgs& a, int is_double, hipStream_t st) {
  if (a.total == 0) return hipSuccess;
  const unsigned grid = (unsigned)((a.total + 255) / 256);
  if (is_double)
    hipLaunchKernelGGL(sensor_measure_kernel<double>, dim3(grid), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(sensor_measure_kernel<float>, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_sensor_transpose(const void* A, int is_double, int64_t n, int ell, double* At, hipStream_t st) {
  const unsigned grid = (unsigned)((n * ell + 255) / 256);
  if (is_double)
    hipLaunchKernelGGL(sensor_transpose_kernel<double>, dim3(grid), dim3(256), 0, st, A, n, ell, At);
  else
    hipLaunchKernelGGL(sensor_transpose_kernel<float>, dim3(grid), dim3(256), 0, st, A, n, ell, At);
  return hipGetLastError();
}

}  // namespace krp
