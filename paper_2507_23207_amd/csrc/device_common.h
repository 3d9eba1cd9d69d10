// Device-side building blocks shared by the gfx950 kernels of libkrp:
// MFMA fragment types, the arithmetic "precision policies" used by the sketch
// and TTM kernels, bf16 splitting and status reporting.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace krp {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float floatx4;
typedef __attribute__((ext_vector_type(4))) double doublex4;

// Arithmetic precisions of the bulk contractions (matches krp_prec in krp.h).
enum Prec : int { kFP64 = 0, kFP32 = 1, kBF16 = 2, kBF16X3 = 3 };

// Status bits OR-ed into the device status word.
enum StatusBits : int {
  kStatCholShift = 1,    // shifted CholeskyQR fallback was taken
  kStatCholFail = 2,     // Cholesky broke down even with the shift
  kStatNonFinite = 4,    // a non-finite value reached an orthonormalisation
  kStatSingular = 8,     // a sensor matrix P^T Q is singular (rank-deficient Q)
};

__device__ __forceinline__ void raise_status(int* status, int bits) {
  if (status) atomicOr(status, bits);
}

// ---------------------------------------------------------------------------
// 16x16 MFMA tiles on a 64-lane wavefront.
// A fragment: lane l holds row (l % 16) of A and 8 reduction slots j = 0..7
// that belong to lane group g = l / 16.  B fragment: lane l holds column
// (l % 16) of B and the same 8 slots of group g.  Any mapping of
// (g, j) -> reduction index k is valid provided A and B use the same one.
// C/D: lane l holds four rows of column l % 16 (register r is row
// 4 (l / 16) + r for fp32/bf16 and row 4 r + l / 16 for fp64; see out_row).
// fp32 and fp64 MFMAs (K = 4 per instruction) consume slot j in instruction
// j; the bf16 MFMA (K = 32) consumes all 8 slots at once.
// ---------------------------------------------------------------------------

template <int P>
struct Policy;

template <>
struct Policy<kFP64> {
  using T = double;       // compute type of operands
  using Acc = doublex4;   // accumulator fragment
  using AccT = double;
  struct Frag {
    double v[8];
  };
  __device__ static Frag make(const double (&x)[8]) {
    Frag f;
#pragma unroll
    for (int j = 0; j < 8; ++j) f.v[j] = x[j];
    return f;
  }
  __device__ static void mma(Acc& acc, const Frag& a, const Frag& b) {
#pragma unroll
    for (int j = 0; j < 8; ++j) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[j], b.v[j], acc, 0, 0, 0);
  }
  __device__ static Acc zero() { return Acc{0.0, 0.0, 0.0, 0.0}; }
  // fp64 16x16x4: lane l, register r holds D[4 r + l / 16][l % 16].
  __device__ static int out_row(int g, int r) { return 4 * r + g; }
};

template <>
struct Policy<kFP32> {
  using T = float;
  using Acc = floatx4;
  using AccT = float;
  struct Frag {
    float v[8];
  };
  __device__ static Frag make(const float (&x)[8]) {
    Frag f;
#pragma unroll
    for (int j = 0; j < 8; ++j) f.v[j] = x[j];
    return f;
  }
  __device__ static void mma(Acc& acc, const Frag& a, const Frag& b) {
#pragma unroll
    for (int j = 0; j < 8; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[j], b.v[j], acc, 0, 0, 0);
  }
  __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  // fp32/bf16 16x16 tiles: lane l, register r holds D[4 (l / 16) + r][l % 16].
  __device__ static int out_row(int g, int r) { return 4 * g + r; }
};

__device__ __forceinline__ float bf16_to_float(__bf16 h) { return (float)h; }

template <>
struct Policy<kBF16> {
  using T = float;
  using Acc = floatx4;
  using AccT = float;
  struct Frag {
    bf16x8 v;
  };
  __device__ static Frag make(const float (&x)[8]) {
    Frag f;
#pragma unroll
    for (int j = 0; j < 8; ++j) f.v[j] = (__bf16)x[j];
    return f;
  }
  __device__ static void mma(Acc& acc, const Frag& a, const Frag& b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc, 0, 0, 0);
  }
  __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  // fp32/bf16 16x16 tiles: lane l, register r holds D[4 (l / 16) + r][l % 16].
  __device__ static int out_row(int g, int r) { return 4 * g + r; }
};

// Split-precision products: x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (x - hi is exact in fp32); a*b is approximated by
// hi_a hi_b + hi_a lo_b + lo_a hi_b, each an MFMA with fp32 accumulation.
template <>
struct Policy<kBF16X3> {
  using T = float;
  using Acc = floatx4;
  using AccT = float;
  struct Frag {
    bf16x8 hi, lo;
  };
  __device__ static Frag make(const float (&x)[8]) {
    Frag f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const __bf16 h = (__bf16)x[j];
      f.hi[j] = h;
      f.lo[j] = (__bf16)(x[j] - (float)h);
    }
    return f;
  }
  __device__ static void mma(Acc& acc, const Frag& a, const Frag& b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, acc, 0, 0, 0);
  }
  __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  // fp32/bf16 16x16 tiles: lane l, register r holds D[4 (l / 16) + r][l % 16].
  __device__ static int out_row(int g, int r) { return 4 * g + r; }
};

// Rounds an fp64 Gaussian to the factor precision of policy P (the fp32
// value for every non-fp64 policy; bf16 rounding happens when fragments of
// the Khatri-Rao products are built).
template <int P>
__device__ __forceinline__ typename Policy<P>::T factor_value(double g) {
  return (typename Policy<P>::T)g;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace krp
