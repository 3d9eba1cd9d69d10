// Sensor placement (Section 6): launch interfaces.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kernels.h"

namespace krp {

// One mode of the training phase.
struct SensorMode {
  const void* q;     // N x ell factor (storage type, column-major)
  void* a;           // N x ell interpolation factor (storage type)
  double* w;         // N x ell fp64 residual of the pivoted QR (workspace)
  unsigned char* taken;  // N flags (workspace)
  double* minv;      // ell x ell (P^T Q)^{-1} (workspace)
  int32_t* idx;      // ell sensor indices in pivot order
  int64_t n;
  int ell;
};

struct SensorSelectArgs {
  SensorMode mode[kMaxDims];
  int nmodes;
  int* status;
};

struct SensorMeasureArgs {
  const void* t;
  void* out;
  int d;
  int64_t dims[kMaxDims];
  int64_t ell[kMaxDims];
  const int32_t* idx[kMaxDims];
  int64_t total;  // prod(ell) * snapshots
};

// One mode of the reconstruction: out (P x N x Q) = g (P x ell x Q) x_2 A,
// A N x ell column-major; storage type for g, A and out.
constexpr int kExpandMaxEll = 64;
constexpr int kExpandLds = 32768;   // bytes of A rows staged per workgroup (P > 1)
constexpr int kExpandRowsQ = 32;    // values of q per workgroup (P == 1)
struct SensorExpandArgs {
  const void* g;
  const void* a;
  void* out;
  int64_t p, n, q;
  int ell;
  // set by the launcher
  int cc;
  int64_t p_tiles, items;
};
hipError_t launch_sensor_expand(const SensorExpandArgs& e, int is_double, hipStream_t st);

size_t sensor_pivot_lds(int ell_max);
hipError_t launch_sensor_select(const SensorSelectArgs& a, int q_is_double, hipStream_t st);
hipError_t launch_sensor_measure(const SensorMeasureArgs& a, int is_double, hipStream_t st);
hipError_t launch_sensor_transpose(const void* A, int is_double, int64_t n, int ell, double* At, hipStream_t st);

}  // namespace krp
