// Small helper kernels: storage-type casts, fp64 sums of squares and integer
// fills (used instead of hipMemsetAsync so that every launch sequence can be
// captured in a HIP graph).
#include "device_common.h"
#include "kernels.h"

namespace krp {

namespace {

template <typename Ti, typename To>
__global__ void cast_kernel(const Ti* __restrict__ in, To* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (To)in[i];
}

// Per-block fp64 partial sums of squares; the last stage sums the partials in
// a fixed order, so the result does not depend on scheduling.
template <typename T>
__global__ void sumsq_partial_kernel(const T* __restrict__ x, int64_t n, double* __restrict__ part) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = (double)x[i];
    s += v * v;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

__global__ void sum_final_kernel(const double* __restrict__ part, int n, double* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    *out = t;
  }
}

__global__ void fill_int_kernel(int* p, int v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

unsigned grid_for(int64_t n, int t) {
  int64_t b = (n + t - 1) / t;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

template <typename T>
__global__ void compact_rows_kernel(const T* __restrict__ src, int64_t src_ld, T* __restrict__ dst, int64_t rows,
                                    int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t c = e / rows, r = e - c * rows;
  dst[e] = src[r + src_ld * c];
}

hipError_t launch_compact_rows(const void* src, int64_t src_ld, void* dst, int64_t rows, int64_t cols, int is_double,
                               hipStream_t st) {
  const int64_t n = rows * cols;
  if (n == 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (is_double)
    hipLaunchKernelGGL(compact_rows_kernel<double>, dim3(grid), dim3(256), 0, st,
                       reinterpret_cast<const double*>(src), src_ld, reinterpret_cast<double*>(dst), rows, n);
  else
    hipLaunchKernelGGL(compact_rows_kernel<float>, dim3(grid), dim3(256), 0, st,
                       reinterpret_cast<const float*>(src), src_ld, reinterpret_cast<float*>(dst), rows, n);
  return hipGetLastError();
}

hipError_t launch_cast(const void* in, int in_is_double, void* out, int out_is_double, int64_t count,
                       hipStream_t st) {
  if (count == 0) return hipSuccess;
  const int t = 256;
  const unsigned g = grid_for(count, t);
  if (in_is_double && out_is_double)
    hipLaunchKernelGGL((cast_kernel<double, double>), dim3(g), dim3(t), 0, st, (const double*)in, (double*)out, count);
  else if (in_is_double)
    hipLaunchKernelGGL((cast_kernel<double, float>), dim3(g), dim3(t), 0, st, (const double*)in, (float*)out, count);
  else if (out_is_double)
    hipLaunchKernelGGL((cast_kernel<float, double>), dim3(g), dim3(t), 0, st, (const float*)in, (double*)out, count);
  else
    hipLaunchKernelGGL((cast_kernel<float, float>), dim3(g), dim3(t), 0, st, (const float*)in, (float*)out, count);
  return hipGetLastError();
}

hipError_t launch_sumsq(const void* x, int is_double, int64_t count, double* acc, double* scratch,
                        int scratch_len, hipStream_t st) {
  const int t = 1024;
  int64_t b = (count + t - 1) / t;
  if (b > scratch_len) b = scratch_len;
  if (b < 1) b = 1;
  if (is_double)
    hipLaunchKernelGGL(sumsq_partial_kernel<double>, dim3((unsigned)b), dim3(t), 0, st, (const double*)x, count, scratch);
  else
    hipLaunchKernelGGL(sumsq_partial_kernel<float>, dim3((unsigned)b), dim3(t), 0, st, (const float*)x, count, scratch);
  hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(1024), 0, st, scratch, (int)b, acc);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int value, int64_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_int_kernel, dim3(grid_for(count, 256)), dim3(256), 0, st, p, value, count);
  return hipGetLastError();
}

}  // namespace krp
