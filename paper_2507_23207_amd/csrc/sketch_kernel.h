// The KRP sketch kernel of one mode unfolding (see sketch.hip for the
// method) as a template over the input type, the arithmetic policy, the load
// mode and the tile counts, plus its launch dispatch.  Each arithmetic policy
// is instantiated in a translation unit of its own (sketch_p*.hip).
#pragma once
#include "device_common.h"
#include "kernels.h"
#include "philox.h"

namespace krp {
namespace skdetail {

struct SketchArgs {
  const void* x;
  void* partial;
  int64_t n_rows, s_row, n_f, s_f;
  int64_t o_size[kMaxDims], o_stride[kMaxDims], o_period[kMaxDims];
  int o_fid[kMaxDims];
  int n_out;
  int64_t o_total, o_per_wg;
  int f_blocks, ell, nparts, wm, wo, rows_per_wg, fid_f, lds_rows;
  uint64_t seed, w2_base;
};

// Load modes of the X slab:
//   kLoadScalar  one element per lane and slot (any strides);
//   kLoadVecF    16-byte loads along the 32-wide f block (f contiguous);
//   kLoadVecF2   the same with 2-element (8-byte) fp32 loads, for an even n_f
//                that is not a multiple of 4;
//   kLoadRowVec  mode 0 (rows contiguous): each lane loads MT consecutive rows
//                of one f index as one vector and hands row MT n + m to the
//                m-th row tile, i.e. the MT tiles of a wave interleave their
//                rows, so the A fragments come straight from the loads.
enum LoadMode : int { kLoadScalar = 0, kLoadVecF = 1, kLoadRowVec = 2, kLoadVecF2 = 3 };

// Elements per load along f of the vector modes.
template <typename Tin, int LM>
constexpr int vecf_width() {
  return LM == kLoadVecF ? (int)(16 / sizeof(Tin)) : 2;
}

// Reduction slot -> k offset inside the 32-wide block.  With vector loads
// along f (the block is contiguous in memory) lane group g reads 16-byte
// pieces so that the four groups of a row cover 64 contiguous bytes per
// instruction.
template <typename Tin, int LM>
__device__ __forceinline__ int kmap(int g, int j) {
  if constexpr (LM == kLoadVecF || LM == kLoadVecF2) {
    constexpr int V = vecf_width<Tin, LM>();
    return V * g + 4 * V * (j / V) + (j % V);
  } else {
    return 8 * g + j;
  }
}

// MT consecutive elements starting at p (aligned to MT elements).
template <typename Tin, int MT>
__device__ __forceinline__ void load_rows(const Tin* p, Tin (&q)[MT]) {
  if constexpr (sizeof(Tin) * MT == 16) {
    if constexpr (sizeof(Tin) == 4) {
      const float4 t = *reinterpret_cast<const float4*>(p);
      q[0] = t.x;
      q[1] = t.y;
      q[2] = t.z;
      q[3] = t.w;
    } else {
      const double2 t = *reinterpret_cast<const double2*>(p);
      q[0] = t.x;
      q[1] = t.y;
    }
  } else if constexpr (sizeof(Tin) * MT == 8 && sizeof(Tin) == 4) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    q[0] = t.x;
    q[1] = t.y;
  } else {
#pragma unroll
    for (int m = 0; m < MT; ++m) q[m] = p[m];
  }
}

template <typename Tin, int P, int LM, int MT, int NT>
__global__ __launch_bounds__(512) void sketch_kernel(SketchArgs a) {
  using Pol = Policy<P>;
  using T = typename Pol::T;
  using AccT = typename Pol::AccT;
  constexpr int CP = 16 * NT;
  static_assert(CP % 4 == 0, "column chunks start at multiples of four generator columns");
  static_assert(LM != kLoadRowVec || sizeof(Tin) * MT <= 16, "one vector load per lane and slot");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tab = reinterpret_cast<T*>(smem_raw);

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int w_m = wave % a.wm;
  const int w_o = wave / a.wm;
  const int kg = blockIdx.x;
  const int fb = kg % a.f_blocks;
  const int64_t orange = kg / a.f_blocks;
  const int64_t f0 = (int64_t)fb * 32;
  const int64_t a0 = (int64_t)blockIdx.y * a.rows_per_wg + (int64_t)w_m * 16 * MT;
  const int col0 = blockIdx.z * CP;
  const int64_t o_begin = orange * a.o_per_wg;
  const int64_t o_end = min(o_begin + a.o_per_wg, a.o_total);
  const int n = lane & 15, g = lane >> 4;

  // Rows of each outer-mode factor that this workgroup's o range touches.
  int lo[kMaxDims];
  int toff[kMaxDims];
  int rows_total = 32;
#pragma unroll
  for (int k = 0; k < kMaxDims; ++k) {
    lo[k] = 0;
    toff[k] = 0;
    if (k < a.n_out) {
      // The o range visits digits lo, lo+1, ... (cyclically, mod o_size) of
      // this mode: at most q1 - q0 + 1 distinct values.
      const int64_t q0 = o_begin / a.o_period[k], q1 = (o_end - 1) / a.o_period[k];
      const int64_t cnt = min(a.o_size[k], q1 - q0 + 1);
      lo[k] = cnt == a.o_size[k] ? 0 : (int)(q0 % a.o_size[k]);
      toff[k] = rows_total;
      rows_total += (int)cnt;
    }
  }

  // Output row of accumulator tile m, fragment row rr.
  auto out_row = [&](int m, int rr) -> int64_t {
    if constexpr (LM == kLoadRowVec)
      return a0 + (int64_t)MT * rr + m;
    else
      return a0 + 16 * m + rr;
  };
  // One partial per workgroup (its waves are summed first); partial sums hold
  // only the chunk's real columns (row stride ncz); chunks keep slots of CP
  // columns.
  const int ncz = min(CP, a.ell - col0);
  AccT* part = reinterpret_cast<AccT*>(a.partial) + (int64_t)blockIdx.z * a.nparts * a.n_rows * CP +
               (int64_t)kg * a.n_rows * ncz;
  // The host sized the LDS for lds_rows table rows.  A plan that undercounts
  // would be a planner bug: the workgroup then poisons its partial sums with
  // NaN (reported as non-finite by the QR) instead of overrunning the LDS.
  if (rows_total > a.lds_rows) {
    if (w_o == 0) {
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = out_row(m, Pol::out_row(g, r));
          if (row < a.n_rows) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
              if (16 * t + n < ncz) part[row * ncz + 16 * t + n] = (AccT)__builtin_nan("");
          }
        }
    }
    return;
  }

  typename Pol::Acc acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = Pol::zero();

  const Tin* X = reinterpret_cast<const Tin*>(a.x);
  // Outer index o as an odometer (digits, element offset, table rows): the
  // wave starts at o_begin + w_o and advances by wo.  All uniform (SGPRs).
  struct Odo {
    int64_t o, off;
    int dig[kMaxDims];  // every mode size is below 2^31
  };
  auto odo_init = [&](int64_t o) {
    Odo z;
    z.o = o;
    z.off = 0;
    int64_t rem = o;
#pragma unroll
    for (int k = 0; k < kMaxDims; ++k) {
      z.dig[k] = 0;
      if (k < a.n_out) {
        z.dig[k] = (int)(rem % a.o_size[k]);
        rem /= a.o_size[k];
        z.off += z.dig[k] * a.o_stride[k];
      }
    }
    return z;
  };
  auto odo_step = [&](Odo& z, int by) {
    z.o += by;
    int64_t carry = by;
#pragma unroll
    for (int k = 0; k < kMaxDims; ++k) {
      if (k < a.n_out && carry != 0) {
        int64_t dnew = z.dig[k] + carry;
        carry = 0;
        while (dnew >= a.o_size[k]) {
          dnew -= a.o_size[k];
          ++carry;
        }
        z.off += (dnew - z.dig[k]) * a.o_stride[k];
        z.dig[k] = (int)dnew;
      }
    }
  };
  // A fragments of the outer step at element offset `off` (raw input values,
  // converted at use).  The loads carry no conditions, so that the compiler
  // keeps the next step's loads in flight while the current one is
  // multiplied: rows past n_rows are clamped to the last row (their
  // accumulator rows are never stored) and f indices past n_f to the last one
  // (the factor table holds zeros there, so they add nothing).
  auto load_a = [&](Tin (&buf)[MT][8], int64_t off) {
    if constexpr (LM == kLoadRowVec) {
      // lane (n, g): rows a0 + MT n .. a0 + MT n + MT - 1 of f index f0 + 8 g + j
      const int64_t row = min(a0 + (int64_t)MT * n, a.n_rows - MT);  // n_rows is a multiple of MT
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t kk = min(f0 + 8 * g + j, a.n_f - 1);
        Tin q[MT];
        load_rows<Tin, MT>(X + off + row + kk * a.s_f, q);
#pragma unroll
        for (int m = 0; m < MT; ++m) buf[m][j] = q[m];
      }
      return;
    }
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int64_t row = min(a0 + 16 * m + n, a.n_rows - 1);
      const int64_t base = off + row * a.s_row;
      if constexpr (LM == kLoadVecF || LM == kLoadVecF2) {
        constexpr int V = vecf_width<Tin, LM>();  // n_f is a multiple of V
#pragma unroll
        for (int h = 0; h < 8 / V; ++h) {
          const int64_t kk = min(f0 + V * g + 4 * V * h, a.n_f - V);
          Tin q[V];
          load_rows<Tin, V>(X + base + kk, q);
#pragma unroll
          for (int v = 0; v < V; ++v) buf[m][V * h + v] = q[v];
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int64_t kk = min(f0 + 8 * g + j, a.n_f - 1);
          buf[m][j] = X[base + kk * a.s_f];
        }
      }
    }
  };
  // Multiply the buffered slice of step z into the accumulators.
  auto compute = [&](const Tin (&buf)[MT][8], const Odo& z) {
    T w[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) w[t] = (T)1;
#pragma unroll
    for (int k = 0; k < kMaxDims; ++k) {
      if (k < a.n_out) {
        // digit and first digit both lie in [0, o_size): one wrap at most
        int dd = z.dig[k] - lo[k];
        dd = dd < 0 ? dd + (int)a.o_size[k] : dd;
        const int rr = toff[k] + dd;
#pragma unroll
        for (int t = 0; t < NT; ++t) w[t] = w[t] * tab[rr * CP + 16 * t + n];
      }
    }
    typename Pol::Frag bf[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      T v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = tab[kmap<Tin, LM>(g, j) * CP + 16 * t + n] * w[t];
      bf[t] = Pol::make(v);
    }
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      T v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = (T)buf[m][j];
      const typename Pol::Frag af = Pol::make(v);
#pragma unroll
      for (int t = 0; t < NT; ++t) Pol::mma(acc[m][t], af, bf[t]);
    }
  };

  // Software pipeline: the loads of step o + wo are in flight while step o is
  // multiplied (two register buffers, alternating).
  Tin bufA[MT][8], bufB[MT][8];
  Odo cur = odo_init(o_begin + w_o);
  load_a(bufA, cur.o < o_end ? cur.off : 0);
  // The factor table is drawn while the first slab loads are in flight.
  // Draw the factor rows (fp64 Gaussians rounded to the working precision),
  // four columns per generator call (the chunk start is a multiple of four),
  // the factor and row chosen without branches; zeros in the padding.
  const int ncol = min(CP, a.ell - col0);
  const int nq = (ncol + 3) >> 2;
  for (int e = threadIdx.x; e < rows_total * nq; e += blockDim.x) {
    const int r = e / nq, jq = e - (e / nq) * nq;
    int k = 0;
#pragma unroll
    for (int kk = 1; kk < kMaxDims; ++kk)
      if (kk < a.n_out && r >= toff[kk]) k = kk;
    const bool fr = r < 32;
    int dd = lo[k] + (r - toff[k]);
    dd = dd >= (int)a.o_size[k] ? dd - (int)a.o_size[k] : dd;
    const int64_t row = fr ? f0 + r : (int64_t)dd;
    const uint64_t fid = fr ? (uint64_t)a.fid_f : (uint64_t)a.o_fid[k];
    const bool live = !fr || row < a.n_f;
    double gq[4];
    gauss_quad(a.seed, a.w2_base | fid, 0, row, (uint64_t)((col0 >> 2) + jq), gq);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = 4 * jq + u;
      tab[r * CP + c] = (live && c < ncol) ? factor_value<P>(gq[u]) : (T)0;
    }
  }
  for (int e = threadIdx.x; e < rows_total * (CP - 4 * nq); e += blockDim.x) {
    const int r = e / (CP - 4 * nq), c = 4 * nq + e % (CP - 4 * nq);
    tab[r * CP + c] = (T)0;
  }
  // LDS-only barrier: the first slab loads stay in flight across it.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  // (past the end of the range the prefetch re-reads the current step)
  while (cur.o < o_end) {
    Odo nxt = cur;
    odo_step(nxt, a.wo);
    load_a(bufB, nxt.o < o_end ? nxt.off : cur.off);
    compute(bufA, cur);
    cur = nxt;
    if (cur.o >= o_end) break;
    odo_step(nxt, a.wo);
    load_a(bufA, nxt.o < o_end ? nxt.off : cur.off);
    compute(bufB, cur);
    cur = nxt;
  }

  if (a.wo > 1) {
    // The waves that share rows (same w_m) are summed in fp64 in wave order
    // through LDS (the factor table is no longer needed), and wave w_o = 0
    // writes the workgroup's partial.
    double* red = reinterpret_cast<double*>(smem_raw) + (int64_t)w_m * (MT * NT * 4 * 64);
    __syncthreads();
    for (int w = 0; w < a.wo; ++w) {
      if (w_o == w) {
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              double* s = &red[((m * NT + t) * 4 + r) * 64 + lane];
              *s = (w == 0 ? 0.0 : *s) + (double)acc[m][t][r];
            }
      }
      __syncthreads();
    }
    if (w_o != 0) return;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[m][t][r] = (AccT)red[((m * NT + t) * 4 + r) * 64 + lane];
  }
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = out_row(m, Pol::out_row(g, r));
      if (row < a.n_rows) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (16 * t + n < ncz) part[row * ncz + 16 * t + n] = acc[m][t][r];
      }
    }
}

// Bytes of LDS the end-of-kernel wave reduction needs (fp64, wm row groups).
inline size_t wave_reduce_lds(int wm, int wo, int mt, int nt) {
  return wo > 1 ? (size_t)wm * mt * nt * 4 * 64 * sizeof(double) : 0;
}

template <typename Tin, int P, int LM, int MT, int NT>
hipError_t launch_inst(const SketchArgs& args, dim3 grid, int threads, size_t lds, hipStream_t st) {
  auto kern = sketch_kernel<Tin, P, LM, MT, NT>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, grid, dim3(threads), lds, st, args);
  return hipGetLastError();
}

template <typename Tin, int P, int LM, int MT>
hipError_t dispatch_nt(int nt, const SketchArgs& args, dim3 grid, int threads, size_t lds, hipStream_t st) {
  switch (nt) {
    case 1: return launch_inst<Tin, P, LM, MT, 1>(args, grid, threads, lds, st);
    case 2: return launch_inst<Tin, P, LM, MT, 2>(args, grid, threads, lds, st);
    case 3: return launch_inst<Tin, P, LM, MT, 3>(args, grid, threads, lds, st);
    default: return launch_inst<Tin, P, LM, MT, 4>(args, grid, threads, lds, st);
  }
}

template <typename Tin, int P, int LM>
hipError_t dispatch_mt(int mt, int nt, const SketchArgs& args, dim3 grid, int threads, size_t lds,
                       hipStream_t st) {
  switch (mt) {
    case 1: return dispatch_nt<Tin, P, LM, 1>(nt, args, grid, threads, lds, st);
    case 2: return dispatch_nt<Tin, P, LM, 2>(nt, args, grid, threads, lds, st);
    default:
      if constexpr (LM == kLoadRowVec && sizeof(Tin) == 8) {
        return hipErrorInvalidValue;  // a row vector of four doubles is not one load
      } else {
        return dispatch_nt<Tin, P, LM, 4>(nt, args, grid, threads, lds, st);
      }
  }
}

template <typename Tin, int P>
hipError_t dispatch_lm(int lm, int mt, int nt, const SketchArgs& args, dim3 grid, int threads,
                       size_t lds, hipStream_t st) {
  if (lm == kLoadVecF) return dispatch_mt<Tin, P, kLoadVecF>(mt, nt, args, grid, threads, lds, st);
  if constexpr (sizeof(Tin) == 4) {
    if (lm == kLoadVecF2) return dispatch_mt<Tin, P, kLoadVecF2>(mt, nt, args, grid, threads, lds, st);
  }
  if (lm == kLoadRowVec) return dispatch_mt<Tin, P, kLoadRowVec>(mt, nt, args, grid, threads, lds, st);
  return dispatch_mt<Tin, P, kLoadScalar>(mt, nt, args, grid, threads, lds, st);
}

// Per-policy entry points (one translation unit each).
hipError_t dispatch_fp64(bool x_double, int lm, int mt, int nt, const SketchArgs& args, dim3 grid,
                         int threads, size_t lds, hipStream_t st);
hipError_t dispatch_fp32(int lm, int mt, int nt, const SketchArgs& args, dim3 grid, int threads,
                         size_t lds, hipStream_t st);
hipError_t dispatch_bf16(int lm, int mt, int nt, const SketchArgs& args, dim3 grid, int threads,
                         size_t lds, hipStream_t st);
hipError_t dispatch_bf16x3(int lm, int mt, int nt, const SketchArgs& args, dim3 grid, int threads,
                           size_t lds, hipStream_t st);

}  // namespace skdetail
}  // namespace krp
