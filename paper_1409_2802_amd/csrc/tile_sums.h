// Kernel values and kernel sums on the 64 x 64 tile engine, shared by the
// evaluation kernels (sibling cover, treecode, FMM-style lists) and the direct
// sum: u_i = sum_j K(y_i, x_j) q_j (Section 1, eq. e:sum) accumulated per
// thread over source chunks, then reduced across the 16 threads of a row in a
// fixed order, so results are deterministic.
#pragma once

#include "ffc_internal.h"
#include "tile_engine.h"

#include <type_traits>

namespace ffc {
namespace tile {

// The Laplace kernel r^(2-d) of r2 = r^2 > 0. Up to d = 7 it is a small power
// of y = 1/r (odd d: y^(d-2)) or of z = 1/r^2 (even d: z^((d-2)/2)), each from
// the hardware estimate refined by two Newton steps (y <- y + y (1 - r2 y^2) / 2,
// z <- z + z (1 - r2 z)), a few times cheaper than the general power, which
// serves larger d and r2 below 2^-900 (where the estimate's range ends).
// The general power, out of line: the kernels call it only for d > 7 or tiny
// distances, so it is kept out of their unrolled loops.
__device__ __attribute__((noinline)) double laplace_pow(double r2, double expo) { return pow(r2, expo); }

__device__ inline double laplace_of_r2(double r2, const KParams& kp) {
  if (kp.lap_small && r2 > 0x1p-900) {
    double b;
    if (kp.lap_odd) {
      b = __builtin_amdgcn_rsq(r2);
      b = fma(0.5 * b, fma(-r2, b * b, 1.0), b);
      b = fma(0.5 * b, fma(-r2, b * b, 1.0), b);
    } else {
      b = __builtin_amdgcn_rcp(r2);
      b = fma(b, fma(-r2, b, 1.0), b);
      b = fma(b, fma(-r2, b, 1.0), b);
    }
    double v = b;
    for (int i = 1; i < kp.lap_m; ++i) v *= b;
    return v;
  }
  return laplace_pow(r2, kp.lap_expo);
}

// Kernel-function code of the Laplace kernel in d = 3 (1/r): its own kernel
// instances, whose values need no run-time choice of power.
constexpr int KF_LAPLACE_R1 = 3;

// 1/r of r2 for the d = 3 Laplace kernel: the arithmetic of laplace_of_r2
// (odd d, power 1), with r2 = 0 selected to 0 and only the rare range
// (0, 2^-900] branching to the general power.
__device__ inline double laplace_r1(double r2, const KParams& kp) {
  double b = __builtin_amdgcn_rsq(r2);
  b = fma(0.5 * b, fma(-r2, b * b, 1.0), b);
  b = fma(0.5 * b, fma(-r2, b * b, 1.0), b);
  double v = r2 > 0x1p-900 ? b : 0.0;
  if (r2 > 0.0 && !(r2 > 0x1p-900)) v = laplace_pow(r2, kp.lap_expo);
  return v;
}

// Kernel function of an accumulated distance^2 (or inner product for the
// polynomial kernel); KF is the ffc_kernel_kind (or KF_LAPLACE_R1), fixed at
// compile time so each kernel instance holds only its own function.
template <int KF>
__device__ inline double kfun(double acc, const KParams& kp) {
  if constexpr (KF == FFC_POLYNOMIAL) {
    const double base = fma(acc, kp.inv_h, kp.c);
    double r = 1.0;
    for (int i = 0; i < kp.p; ++i) r *= base;
    return r;
  } else if constexpr (KF == FFC_GAUSSIAN) {
    return exp(acc * kp.neg_inv_2h2);
  } else if constexpr (KF == KF_LAPLACE_R1) {
    return laplace_r1(acc, kp);
  } else {
    return acc > 0.0 ? laplace_of_r2(acc, kp) : 0.0;
  }
}

template <int KF>
__device__ inline double kfun(float acc, const KParams& kp) {
  if constexpr (KF == FFC_POLYNOMIAL) {
    const float base = fmaf(acc, (float)kp.inv_h, (float)kp.c);
    float r = 1.0f;
    for (int i = 0; i < kp.p; ++i) r *= base;
    return (double)r;
  } else if constexpr (KF == FFC_GAUSSIAN) {
    return (double)expf(acc * (float)kp.neg_inv_2h2);
  } else {
    return acc > 0.0f ? laplace_of_r2((double)acc, kp) : 0.0;   // the power in FP64 (range)
  }
}

__device__ inline void flag_nonfinite(unsigned int* flag) { atomicOr(flag, 1u); }

// ---------------------------------------------------------------------------
// Kernel sums: accumulate sum_j K(y_i, x_j) q_j over one source set into
// per-thread partial sums part[i] (rows tr + 16 i of the tile).
// ---------------------------------------------------------------------------
template <typename T, int KF>
__device__ inline void sum_over_sources(const double* __restrict__ Y, IdxMap rows, int nrows,
                                        const double* __restrict__ X, IdxMap cols, int ncols,
                                        const double* __restrict__ q, int d, const KParams& kp, TileSmem<T>& sm,
                                        double (&part)[4], bool& bad) {
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  for (int c0 = 0; c0 < ncols; c0 += BN) {
    IdxMap cm{cols.idx ? cols.idx + c0 : nullptr, cols.base + c0};
    T acc[4][4];
    tile_accumulate<T, KF == FFC_POLYNOMIAL>(Y, rows, nrows, X, cm, ncols - c0, d, sm, acc);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + tc + 16 * j;
      if (c < ncols) {
        const double qj = q[c];
#pragma unroll
        for (int i = 0; i < 4; ++i) part[i] = fma(kfun<KF>(acc[i][j], kp), qj, part[i]);
      }
    }
  }
  // A kernel value that is not finite leaves its partial sum not finite
  // (q = 0 gives NaN), so one test per row after the loop finds it.
#pragma unroll
  for (int i = 0; i < 4; ++i) bad |= !isfinite(part[i]);
}

// ---------------------------------------------------------------------------
// Kernel sums for d <= DM (DM = 4 or 32 <= KC), where one chunk holds every
// dimension. The 64 target rows of a workgroup never change, so stage_rows puts
// them in LDS once; the sums then stage only source chunks, fetching the next
// chunk's coordinates into registers (64·DM / 256 per thread) while the current
// one is computed. The arithmetic per pair is that of sum_over_sources (same
// order), so the results are the same bits. DM = 0 selects sum_over_sources.
// ---------------------------------------------------------------------------
// LDS of the evaluation kernels: DM dimensions per chunk when DM > 0.
template <typename T, int DM>
using EvalSmem = TileSmem<T, (DM > 0 ? DM : KC)>;

template <typename T, int DM>
__device__ inline void stage_rows(const double* __restrict__ Y, IdxMap rows, int nrows, int d,
                                  EvalSmem<T, DM>& sm) {
  const int tid = threadIdx.x;
  const int sh = 32 - __clz(d - 1);
#pragma unroll
  for (int it = 0; it < BM * DM / NT; ++it) {
    const int e = tid + it * NT;
    if (e < (BM << sh)) {
      const int r = e >> sh, kk = e & ((1 << sh) - 1);
      if (kk < d) sm.ys[kk][r] = r < nrows ? (T)Y[rows(r) * d + kk] : T(0);
    }
  }
}

template <typename T, int KF, int DM>
__device__ inline void sum_staged_rows(const double* __restrict__ X, IdxMap cols, int ncols,
                                       const double* __restrict__ q, int d, const KParams& kp, EvalSmem<T, DM>& sm,
                                       double (&part)[4], bool& bad) {
  constexpr int IT = BM * DM / NT;
  constexpr bool DOT = KF == FFC_POLYNOMIAL;
  const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;
  const int sh = 32 - __clz(d - 1);
  T pre[IT];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = tid + it * NT;
      const int r = e >> sh, kk = e & ((1 << sh) - 1);
      pre[it] = (e < (BM << sh) && kk < d && r < ncols - c0) ? (T)X[cols(c0 + r) * d + kk] : T(0);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = tid + it * NT;
      const int r = e >> sh, kk = e & ((1 << sh) - 1);
      if (e < (BM << sh) && kk < d) sm.xs[kk][r] = pre[it];
    }
  };
  if (ncols <= 0) return;
  fetch(0);
  store();
  __syncthreads();
  for (int c0 = 0; c0 < ncols; c0 += BN) {
    const bool more = c0 + BN < ncols;
    if (more) fetch(c0 + BN);   // in flight while this chunk is computed
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = T(0);
#pragma unroll (DM < 8 ? DM : 8)
    for (int kk = 0; kk < d; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sm.ys[kk][tr + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sm.xs[kk][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (DOT) {
            acc[i][j] = fma(a[i], b[j], acc[i][j]);
          } else {
            const T df = a[i] - b[j];
            acc[i][j] = fma(df, df, acc[i][j]);
          }
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + tc + 16 * j;
      if (c < ncols) {
        const double qj = q[c];
#pragma unroll
        for (int i = 0; i < 4; ++i) part[i] = fma(kfun<KF>(acc[i][j], kp), qj, part[i]);
      }
    }
    __syncthreads();   // every thread is done with this chunk's sources
    if (more) {
      store();
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) bad |= !isfinite(part[i]);
}

// Sum over one source set with the tile's rows: the staged-rows form when DM > 0
// (stage_rows must have run in this workgroup), the general form otherwise.
template <typename T, int KF, int DM>
__device__ inline void sum_sources(const double* __restrict__ Y, IdxMap rows, int nrows, const double* __restrict__ X,
                                   IdxMap cols, int ncols, const double* __restrict__ q, int d, const KParams& kp,
                                   EvalSmem<T, DM>& sm, double (&part)[4], bool& bad) {
  if constexpr (DM > 0) sum_staged_rows<T, KF, DM>(X, cols, ncols, q, d, kp, sm, part, bad);
  else sum_over_sources<T, KF>(Y, rows, nrows, X, cols, ncols, q, d, kp, sm, part, bad);
}

// Host side: the kernel function (ffc_kernel_kind, or KF_LAPLACE_R1 for the
// Laplace kernel in d = 3) as a compile-time constant.
template <typename F>
inline auto with_kind(const KParams& kp, F&& f) {
  if (kp.kind == FFC_GAUSSIAN) return f(std::integral_constant<int, FFC_GAUSSIAN>());
  if (kp.kind == FFC_LAPLACE && kp.lap_small && kp.lap_odd && kp.lap_m == 1)
    return f(std::integral_constant<int, KF_LAPLACE_R1>());
  if (kp.kind == FFC_LAPLACE) return f(std::integral_constant<int, FFC_LAPLACE>());
  return f(std::integral_constant<int, FFC_POLYNOMIAL>());
}

// Host side: the dimension class of the evaluation kernels (4, 32, or 0 for the
// general path) as a compile-time constant passed to f.
template <typename F>
inline auto with_dims(int d, F&& f) {
  if (d <= 4) return f(std::integral_constant<int, 4>());
  if (d <= KC) return f(std::integral_constant<int, KC>());
  return f(std::integral_constant<int, 0>());
}

// Fixed-order reduction of part[] across the 16 column threads of each row.
__device__ inline void reduce_rows(double (&part)[4], double* red /* 16 x 64 */, double* rowsum /* 64 */) {
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) red[tc * BM + tr + 16 * i] = part[i];
  __syncthreads();
  if (threadIdx.x < BM) {
    double s = 0.0;
    for (int c = 0; c < 16; ++c) s += red[c * BM + threadIdx.x];
    rowsum[threadIdx.x] = s;
  }
  __syncthreads();
}

}  // namespace tile
}  // namespace ffc
