// The 64 x 64 point-pair tile engine shared by the kernel tiles (sampled
// blocks, evaluation, direct sums).
//
// A 256-thread workgroup computes a 64 x 64 tile of squared distances (or, with
// DOT, inner products) between a row set and a column set of points stored
// point-major (N x d, float64). Coordinates are staged through LDS in chunks
// of 32 dimensions, transposed so that each thread reads 4 row values and 4
// column values per dimension and owns a 4 x 4 block of the tile: rows
// r0 + tr + 16 i and columns c0 + tc + 16 j with tr = thread % 16, tc =
// thread / 16. Squared distances are formed from explicit coordinate
// differences, so they carry no cancellation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ffc {
namespace tile {

constexpr int BM = 64, BN = 64, KC = 32, NT = 256;
constexpr int LDSP = BM + 1;   // padded LDS row (bank spread)

// K dimensions per chunk (KC for the general path; the evaluation kernels for
// small d stage only DM of them and size their LDS to match).
template <typename T, int K = KC>
struct TileSmem {
  T ys[K][LDSP];
  T xs[K][LDSP];
};

// Row / column index maps: an explicit index list or a contiguous range.
struct IdxMap {
  const int32_t* idx;
  int64_t base;
  __device__ inline int64_t operator()(int i) const { return idx ? (int64_t)idx[i] : base + i; }
};

// acc[i][j] for rows r0 + tr + 16 i and columns c0 + tc + 16 j.
template <typename T, bool DOT>
__device__ inline void tile_accumulate(const double* __restrict__ Y, IdxMap rows, int nrows, const double* __restrict__ X,
                                       IdxMap cols, int ncols, int d, TileSmem<T>& sm, T (&acc)[4][4]) {
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = T(0);
  for (int k0 = 0; k0 < d; k0 += KC) {
    const int kc = min(KC, d - k0);   // dimensions present in this chunk
    // Stage 64 rows x kc dimensions: element e is row e >> sh, dimension
    // e & (2^sh - 1) with 2^sh the power of two >= kc, so a chunk of few
    // dimensions takes few passes and consecutive lanes still read consecutive
    // coordinates of a row. Dimensions >= kc are never read below.
    const int sh = 32 - __clz(kc - 1);
#pragma unroll
    for (int it = 0; it < BM * KC / NT; ++it) {
      const int e = tid + it * NT;
      if (e < (BM << sh)) {
        const int r = e >> sh, kk = e & ((1 << sh) - 1);
        if (kk < kc) {
          const int k = k0 + kk;
          T yv = T(0), xv = T(0);
          if (r < nrows) yv = (T)Y[rows(r) * d + k];
          if (r < ncols) xv = (T)X[cols(r) * d + k];
          sm.ys[kk][r] = yv;
          sm.xs[kk][r] = xv;
        }
      }
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kc; ++kk) {
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
    __syncthreads();
  }
}

}  // namespace tile
}  // namespace ffc
