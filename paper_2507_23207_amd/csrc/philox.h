// Counter-based Gaussian factors for Khatri-Rao random projections.
//
// The paper asks for factor matrices with independent mean-zero, unit-variance
// sub-Gaussian entries (Definition 2.1), Gaussian in its experiments.  Every
// entry here is a pure function of (seed, row, column, counter word 2,
// instance), so any workgroup can draw exactly the factor rows its tile needs,
// in registers, and nothing is ever stored in HBM.
//
// Generator: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// Counter of the entries (a, 4j .. 4j+3) of factor f for sketch k under draw
// `draw`:  (a, j, draw << 32 | k << 16 | f, instance), key (seed, 0).
// Output words (w0, w1) and (w2, w3) are two Box-Muller pairs (wu, wv):
//   u1 = ((wu >> 11) + 1) 2^-53 in (0, 1],  k2 = wv >> 11,  r = sqrt(-2 ln u1),
//   entry 4j + 2p     = r cos(2 pi k2 2^-53),
//   entry 4j + 2p + 1 = r sin(2 pi k2 2^-53) = r cos(2 pi (k2 - 2^51) 2^-53),
// for pair p = 0 (w0, w1) and p = 1 (w2, w3).  The cosine and sine outputs of
// one pair are independent standard normals.
// ln and cos are evaluated by the fixed sequences below with separately
// rounded IEEE-754 operations (contraction into FMA is disabled), so every
// entry is fully specified by the operation order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace krp {

struct u64x4 {
  uint64_t v0, v1, v2, v3;
};

// Full 64 x 64 -> 128-bit product by a constant from four 32 x 32 -> 64
// partial products (the low and high halves share them).
template <uint64_t K>
__device__ __forceinline__ void mul128(uint64_t x, uint64_t& lo, uint64_t& hi) {
  constexpr uint32_t kl = (uint32_t)K, kh = (uint32_t)(K >> 32);
  const uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32);
  const uint64_t p00 = (uint64_t)xl * kl;
  const uint64_t p01 = (uint64_t)xl * kh;
  const uint64_t p10 = (uint64_t)xh * kl;
  const uint64_t p11 = (uint64_t)xh * kh;
  const uint64_t mid = (p00 >> 32) + (uint32_t)p01 + (uint32_t)p10;
  lo = (mid << 32) | (uint32_t)p00;
  hi = p11 + (p01 >> 32) + (p10 >> 32) + (mid >> 32);
}

__device__ __forceinline__ u64x4 philox4x64_10(u64x4 c, uint64_t k0, uint64_t k1) {
  constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t kMul1 = 0xCA5A826395121157ull;
  constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t lo0, hi0, lo1, hi1;
    mul128<kMul0>(c.v0, lo0, hi0);
    mul128<kMul1>(c.v2, lo1, hi1);
    u64x4 n;
    n.v0 = hi1 ^ c.v1 ^ k0;
    n.v1 = lo1;
    n.v2 = hi0 ^ c.v3 ^ k1;
    n.v3 = lo0;
    c = n;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  return c;
}

// ln(u) for u in (0, 1].  u = m 2^e exactly (m in [1, 2)); m is halved when it
// exceeds sqrt(2) so that s = (m - 1) / (m + 1) satisfies |s| <= 0.1716, then
// ln m = 2 s sum_{j=0}^{11} s^{2j} / (2j + 1) and
// ln u = e ln2_hi + (e ln2_lo + ln m), where ln2_hi is ln 2 rounded to nearest
// and cut to 32 significant bits (e ln2_hi is exact) and ln2_lo the rounded
// remainder.
__device__ __forceinline__ double log_unit(double u) {
#pragma clang fp contract(off)
  constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
  constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
  constexpr double kSqrt2 = 0x1.6a09e667f3bcdp+0;
  constexpr double kC[12] = {1.0,        1.0 / 3.0,  1.0 / 5.0,  1.0 / 7.0,
                             1.0 / 9.0,  1.0 / 11.0, 1.0 / 13.0, 1.0 / 15.0,
                             1.0 / 17.0, 1.0 / 19.0, 1.0 / 21.0, 1.0 / 23.0};
  const uint64_t bits = (uint64_t)__double_as_longlong(u);
  int e = (int)((bits >> 52) & 0x7FF) - 1023;
  double m = __longlong_as_double(
      (long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
  if (m > kSqrt2) {
    m = m * 0.5;
    e = e + 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double p = kC[11];
#pragma unroll
  for (int j = 10; j >= 0; --j) {
    p = p * z;
    p = p + kC[j];
  }
  const double ln_m = (s + s) * p;
  const double ef = (double)e;
  const double t = ef * kLn2Lo;
  const double t2 = t + ln_m;
  const double h = ef * kLn2Hi;
  return h + t2;
}

// cos(2 pi k2 2^-53) for 0 <= k2 < 2^53.  The nearest quarter turn q is taken
// in integers, so f = (k2 - q 2^51) 2^-53 in [-1/8, 1/8] is exact;
// theta = 2 pi f and the Taylor sums of cos (11 terms) and sin (10 terms) on
// |theta| <= pi/4 are combined by the quadrant q mod 4.
__device__ __forceinline__ double cos_two_pi(uint64_t k2) {
#pragma clang fp contract(off)
  constexpr double kTwoPi = 0x1.921fb54442d18p+2;
  constexpr double kCos[11] = {1.0,
                               -1.0 / 2.0,
                               1.0 / 24.0,
                               -1.0 / 720.0,
                               1.0 / 40320.0,
                               -1.0 / 3628800.0,
                               1.0 / 479001600.0,
                               -1.0 / 87178291200.0,
                               1.0 / 20922789888000.0,
                               -1.0 / 6402373705728000.0,
                               1.0 / 2432902008176640000.0};
  constexpr double kSin[10] = {1.0,
                               -1.0 / 6.0,
                               1.0 / 120.0,
                               -1.0 / 5040.0,
                               1.0 / 362880.0,
                               -1.0 / 39916800.0,
                               1.0 / 6227020800.0,
                               -1.0 / 1307674368000.0,
                               1.0 / 355687428096000.0,
                               -1.0 / 121645100408832000.0};
  const uint64_t q = (k2 + (1ull << 50)) >> 51;
  const int64_t rem = (int64_t)k2 - (int64_t)(q << 51);
  const double f = (double)rem * 0x1.0p-53;
  const double th = kTwoPi * f;
  const double z = th * th;
  // One Horner chain per entry: the cosine sum (quadrants 0, 2) or the sine
  // sum (1, 3).  The sine chain starts from 0, whose first step gives
  // kSin[9] exactly, so both produce the same operations as separate sums.
  const bool odd = (q & 1) != 0;
  double p = odd ? 0.0 : kCos[10];
#pragma unroll
  for (int j = 9; j >= 0; --j) {
    p = p * z;
    p = p + (odd ? kSin[j] : kCos[j]);
  }
  const double v = odd ? th * p : p;
  // quadrant 0: cos, 1: -sin, 2: -cos, 3: sin
  return ((q + 1) & 2) ? -v : v;
}

// cos and sin of 2 pi k2 2^-53 from one reduction: the sine is the cosine a
// quarter turn earlier, i.e. the same reduced angle in quadrant q - 1, so both
// values equal what cos_two_pi gives for k2 and for (k2 - 2^51) mod 2^53.
__device__ __forceinline__ void sincos_two_pi(uint64_t k2, double& c_out, double& s_out) {
#pragma clang fp contract(off)
  constexpr double kTwoPi = 0x1.921fb54442d18p+2;
  constexpr double kCos[11] = {1.0,
                               -1.0 / 2.0,
                               1.0 / 24.0,
                               -1.0 / 720.0,
                               1.0 / 40320.0,
                               -1.0 / 3628800.0,
                               1.0 / 479001600.0,
                               -1.0 / 87178291200.0,
                               1.0 / 20922789888000.0,
                               -1.0 / 6402373705728000.0,
                               1.0 / 2432902008176640000.0};
  constexpr double kSin[10] = {1.0,
                               -1.0 / 6.0,
                               1.0 / 120.0,
                               -1.0 / 5040.0,
                               1.0 / 362880.0,
                               -1.0 / 39916800.0,
                               1.0 / 6227020800.0,
                               -1.0 / 1307674368000.0,
                               1.0 / 355687428096000.0,
                               -1.0 / 121645100408832000.0};
  const uint64_t q = (k2 + (1ull << 50)) >> 51;
  const int64_t rem = (int64_t)k2 - (int64_t)(q << 51);
  const double f = (double)rem * 0x1.0p-53;
  const double th = kTwoPi * f;
  const double z = th * th;
  double pc = kCos[10];
#pragma unroll
  for (int j = 9; j >= 0; --j) {
    pc = pc * z;
    pc = pc + kCos[j];
  }
  double ps = kSin[9];
#pragma unroll
  for (int j = 8; j >= 0; --j) {
    ps = ps * z;
    ps = ps + kSin[j];
  }
  const double sv = th * ps;
  const bool odd = (q & 1) != 0;
  // cosine: quadrant 0: C, 1: -S, 2: -C, 3: S;  sine (quadrant q - 1): 0: S, 1: C, 2: -S, 3: -C
  const double vc = odd ? sv : pc;
  const double vs = odd ? pc : sv;
  c_out = ((q + 1) & 2) ? -vc : vc;
  s_out = (q & 2) ? -vs : vs;
}

__device__ __forceinline__ double box_muller_radius(uint64_t wu) {
#pragma clang fp contract(off)
  const double u1 = (double)((wu >> 11) + 1ull) * 0x1.0p-53;
  return __builtin_sqrt(-2.0 * log_unit(u1));
}

__host__ __device__ __forceinline__ uint64_t counter_word2(uint32_t draw, uint32_t sketch,
                                                           uint32_t f) {
  return ((uint64_t)draw << 32) | ((uint64_t)(sketch & 0xFFFFu) << 16) | (uint64_t)(f & 0xFFFFu);
}

// Entries (row, 4j), (row, 4j+1), (row, 4j+2), (row, 4j+3) of the factor
// identified by (seed, w2, instance): one generator call.
__device__ __forceinline__ void gauss_quad(uint64_t seed, uint64_t w2, uint64_t instance,
                                           uint64_t row, uint64_t j, double (&g)[4]) {
#pragma clang fp contract(off)
  u64x4 c{row, j, w2, instance};
  const u64x4 w = philox4x64_10(c, seed, 0ull);
  double c0, s0, c1, s1;
  sincos_two_pi(w.v1 >> 11, c0, s0);
  sincos_two_pi(w.v3 >> 11, c1, s1);
  const double r0 = box_muller_radius(w.v0);
  const double r1 = box_muller_radius(w.v2);
  g[0] = r0 * c0;
  g[1] = r0 * s0;
  g[2] = r1 * c1;
  g[3] = r1 * s1;
}

// Entry (row, col) alone: one generator call, one radius, one of cos / sin.
__device__ __forceinline__ double gauss_entry(uint64_t seed, uint64_t w2, uint64_t instance,
                                              uint64_t row, uint64_t col) {
#pragma clang fp contract(off)
  u64x4 c{row, col >> 2, w2, instance};
  const u64x4 w = philox4x64_10(c, seed, 0ull);
  const bool second = (col & 2) != 0;
  const uint64_t wu = second ? w.v2 : w.v0;
  const uint64_t wv = second ? w.v3 : w.v1;
  const uint64_t k2 = wv >> 11;
  const uint64_t k2s = (col & 1) ? ((k2 - (1ull << 51)) & ((1ull << 53) - 1)) : k2;
  return box_muller_radius(wu) * cos_two_pi(k2s);
}

}  // namespace krp
