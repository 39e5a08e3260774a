// Last stage of the learned proposal's features: per-target partial results
// over the column subsample (the 4 smallest distances / rho and their sum,
// from `parts` partial sets) are merged in a fixed order, the distance to the
// centroid and the anchor projections are formed in FP64, and the 16 features
// are written.
#pragma once

#include "ffc_internal.h"

namespace ffc {
namespace feat {

constexpr int kNF = 16;      // features per target
constexpr int kNAnch = 7;    // anchor directions
constexpr int kSub = 256;    // column subsample size

__device__ inline void insert4(double (&b)[4], double v) {   // keep the 4 smallest, ascending
  if (!(v < b[3])) return;
  b[3] = v;
#pragma unroll
  for (int a = 3; a > 0; --a)
    if (b[a] < b[a - 1]) {
      const double t = b[a];
      b[a] = b[a - 1];
      b[a - 1] = t;
    }
}

// red: [parts][64 rows][5] (4 smallest, then the sum), complete before the
// call; dots: scratch of 64 x (1 + kNAnch) doubles. Called by all 256 threads
// of the workgroup (it synchronizes once).
__device__ inline void finish_rows(const double* __restrict__ Xt, int d, const GeomArgs& ga, int b,
                                   const int32_t* __restrict__ tg, int t0, int nt, int ns, double rho,
                                   const double* red, int parts, double* dots, float* __restrict__ feat,
                                   int64_t feat_stride) {
  const int tid = threadIdx.x;
  // The centroid distance and the anchor projections of every row: 64 rows x
  // (1 + kNAnch) dot products over d, spread over all threads (each one a
  // sequential sum, so the values do not depend on the spreading).
  const double* c = ga.cen + (int64_t)b * d;
  const double* U = ga.U + (int64_t)b * kNAnch * d;
  for (int task = tid; task < 64 * (1 + kNAnch); task += 256) {
    const int row = task / (1 + kNAnch), a = task % (1 + kNAnch);
    if (t0 + row >= nt) continue;
    const double* y = Xt + (int64_t)tg[row] * d;
    double p = 0.0;
    // (Unrolled so that many coordinates' loads are in flight at once; the
    // sums stay sequential.)
    if (a == 0) {
#pragma unroll 32
      for (int k = 0; k < d; ++k) {
        const double df = y[k] - c[k];
        p = fma(df, df, p);
      }
    } else {
      const double* u = U + (int64_t)(a - 1) * d;
#pragma unroll 32
      for (int k = 0; k < d; ++k) p = fma(y[k] - c[k], u[k], p);
    }
    dots[row * (1 + kNAnch) + a] = p;
  }
  __syncthreads();
  if (tid >= 64) return;
  const int row = tid;
  if (t0 + row >= nt) return;
  double b4[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
  double tot = 0.0;
  for (int q = 0; q < parts; ++q) {
    const double* r = red + ((int64_t)q * 64 + row) * 5;
#pragma unroll
    for (int u = 0; u < 4; ++u) insert4(b4, r[u]);
    tot += r[4];
  }
  const double dc = sqrt(dots[row * (1 + kNAnch)]) / rho;
  float* f = feat + (int64_t)b * feat_stride + (int64_t)(t0 + row) * kNF;
  f[0] = (float)dc;
  f[1] = (float)log(dc + 1e-12);
  for (int q = 0; q < 4; ++q) f[2 + q] = (float)(q < ns ? b4[q] : b4[max(ns - 1, 0)]);
  f[6] = (float)(ns > 0 ? tot / ns : 0.0);
  f[7] = (float)log(b4[0] + 1e-12);
  for (int a = 0; a < kNAnch; ++a) f[8 + a] = (float)(dots[row * (1 + kNAnch) + 1 + a] / rho);
  f[15] = 1.0f;
}

}  // namespace feat
}  // namespace ffc
