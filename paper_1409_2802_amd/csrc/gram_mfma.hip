// Mixed-precision kernel tiles on matrix cores (FFC_MIXED_BF16X3).
//
// Distances in high dimension are Gram contractions: ||y - x||^2 =
// ||y||^2 + ||x||^2 - 2 y.x. Each coordinate z is split into bfloat16 parts
// hi = bf16(z), lo = bf16(z - hi), which carry z to about 2^-17 relative. The
// Gram product is hi.hi + hi.lo + lo.hi (the lo.lo term is below that error) on
// v_mfma_f32_16x16x32_bf16 with float32 accumulation. The kernel function
// (Gaussian exp of the distance, or the polynomial power of the inner product)
// runs in float32 in the epilogue; sampled blocks are stored in float64 for
// the QR.
//
// The split only carries 16 bits, so coordinates are centred first: on the
// node's centroid for a sampled block and on the target leaf's centroid for
// the evaluation (distances do not depend on the centre, and a nearby one keeps
// the coordinates and norms small; the polynomial kernel needs the raw inner
// product and centres on the origin). Left uncentred, points far from the
// origin lose the distance of near pairs to cancellation. The tree's points
// are stored once in float32 less the root centroid (tree order, rows padded
// with zeros to a multiple of 32 dimensions), with the nodes' centroids in the
// same frame; a tile loads 16-byte groups of them, subtracts its centre,
// splits and forms the squared norms while staging, and prefetches the next
// 32-dimension chunk while the matrix cores work. The direct sum, on arbitrary
// point sets, converts from float64 while staging and centres both sets on its
// first target.
//
// A 256-thread workgroup computes a 64 x 64 tile; operands go through LDS 32
// dimensions at a time. The MFMA A operand holds the column points and B the
// row points, so each output lane owns one sampled row of a column and the
// column-major stores coalesce. Operand layout of the instruction (lane l,
// element i): A[l % 16][(l / 16) * 8 + i], B[(l / 16) * 8 + i][l % 16],
// D[(l / 16) * 4 + i][l % 16].
#include <vector>

#include "ffc_internal.h"

namespace ffc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // (selects on it are per element)

constexpr int TM = 64, TN = 64, KCH = 32, NTH = 256;
constexpr int LROW = KCH + 8;   // bf16 per LDS row (16-byte aligned, spread over banks)

struct __attribute__((aligned(16))) MixSmem {
  __bf16 xh[TN][LROW], xl[TN][LROW];   // column points (A operand)
  __bf16 yh[TM][LROW], yl[TM][LROW];   // row points (B operand)
  float xn[TN], yn[TM];                // squared norms of the centred points
};

struct Idx {
  const int32_t* idx;
  int64_t base;
  __device__ inline int64_t operator()(int i) const { return idx ? (int64_t)idx[i] : base + i; }
};

// acc[bi][bj][e] = Gram entry (column point cb + bi*16 + (l/16)*4 + e, row point rb + bj*16 + l%16)
// with cb = (wave >> 1) * 32 and rb = (wave & 1) * 32 inside the tile. When CENTRED, norms of the
// centred points are left in sm.xn / sm.yn.
template <bool CENTRED>
__device__ void mixed_tile(const double* __restrict__ Y, Idx rows, int nrows, const double* __restrict__ X, Idx cols,
                           int ncols, int d, const double* __restrict__ center, MixSmem& sm, f32x4 (&acc)[2][2]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
  // Staging map: thread t handles dimension kk = t % 32 of points t / 32 + 8 j, j < 8.
  const int kk = tid & 31, p0 = tid >> 5;
  float yacc[8], xacc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) yacc[j] = xacc[j] = 0.f;
  int64_t yrow[8], xrow[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int p = p0 + 8 * j;
    yrow[j] = p < nrows ? rows(p) : -1;
    xrow[j] = p < ncols ? cols(p) : -1;
  }
  for (int k0 = 0; k0 < d; k0 += KCH) {
    const int k = k0 + kk;
    const double c = (CENTRED && k < d) ? center[k] : 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int p = p0 + 8 * j;
      const double yv = (yrow[j] >= 0 && k < d) ? Y[yrow[j] * d + k] - c : 0.0;
      const double xv = (xrow[j] >= 0 && k < d) ? X[xrow[j] * d + k] - c : 0.0;
      const __bf16 yh = (__bf16)(float)yv, xh = (__bf16)(float)xv;
      sm.yh[p][kk] = yh;
      sm.yl[p][kk] = (__bf16)(float)(yv - (double)(float)yh);
      sm.xh[p][kk] = xh;
      sm.xl[p][kk] = (__bf16)(float)(xv - (double)(float)xh);
      const float yf = (float)yv, xf = (float)xv;
      yacc[j] = fmaf(yf, yf, yacc[j]);
      xacc[j] = fmaf(xf, xf, xacc[j]);
    }
    __syncthreads();
    const int kofs = (lane >> 4) * 8;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int xr = (w >> 1) * 32 + bi * 16 + (lane & 15);
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&sm.xh[xr][kofs]);
      const bf16x8 al = *reinterpret_cast<const bf16x8*>(&sm.xl[xr][kofs]);
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int yr = (w & 1) * 32 + bj * 16 + (lane & 15);
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&sm.yh[yr][kofs]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&sm.yl[yr][kofs]);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[bi][bj], 0, 0, 0);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[bi][bj], 0, 0, 0);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[bi][bj], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (CENTRED) {
    // Sum the 32 per-dimension partials of each point (lanes sharing p0 form a half wave).
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float yv = yacc[j], xv = xacc[j];
#pragma unroll
      for (int off = 16; off > 0; off >>= 1) {
        yv += __shfl_xor(yv, off, 64);
        xv += __shfl_xor(xv, off, 64);
      }
      if (kk == 0) {
        sm.yn[p0 + 8 * j] = yv;
        sm.xn[p0 + 8 * j] = xv;
      }
    }
    __syncthreads();
  }
}

// Tree-order points split once into bf16 hi + lo (rows of dp values, zero past
// d): the same values mixed_tile forms when it stages uncentred coordinates.
__global__ void k_bf16_split(const double* __restrict__ Xt, int64_t N, int d, int dp, __bf16* __restrict__ hi,
                             __bf16* __restrict__ lo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * dp) return;
  const int64_t p = e / dp;
  const int k = (int)(e % dp);
  const double v = k < d ? Xt[p * d + k] : 0.0;
  const __bf16 h = (__bf16)(float)v;
  hi[e] = h;
  lo[e] = (__bf16)(float)(v - (double)(float)h);
}

// Squared norms of the tree-order points, summed in FP64 and rounded to FP32.
__global__ void k_point_norms(const double* __restrict__ Xt, int64_t N, int d, float* __restrict__ nrm) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const double* x = Xt + p * d;
  double s = 0.0;
  for (int k = 0; k < d; ++k) s = fma(x[k], x[k], s);
  nrm[p] = (float)s;
}

// The Gram tile of mixed_tile, uncentred, from the pre-split points: each
// thread stages one 16-byte group of 8 values of each of the four operands per
// 32-dimension chunk, and fetches the next chunk's groups while the matrix
// cores work on the current one. Same operands and chunk order as
// mixed_tile<false>, so the same bits. With nrm, the points' squared norms go
// to sm.yn / sm.xn for the distance epilogue.
__device__ void mixed_tile_split(const __bf16* __restrict__ Hh, const __bf16* __restrict__ Hl,
                                 const float* __restrict__ nrm, int dp, Idx rows, int nrows, Idx cols, int ncols,
                                 MixSmem& sm, f32x4 (&acc)[2][2]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int p = tid >> 2, part = (tid & 3) * 8;
  const int64_t yrow = p < nrows ? rows(p) : -1;
  const int64_t xrow = p < ncols ? cols(p) : -1;
  const u32x4 zero = {0u, 0u, 0u, 0u};
  if (nrm && (tid & 3) == 0) {
    sm.yn[p] = yrow >= 0 ? nrm[yrow] : 0.f;
    sm.xn[p] = xrow >= 0 ? nrm[xrow] : 0.f;
  }
  u32x4 yh, yl, xh, xl;   // native vectors: a choice between two structs would go through memory
  auto fetch = [&](int k0) {
    yh = yrow >= 0 ? *reinterpret_cast<const u32x4*>(Hh + yrow * dp + k0 + part) : zero;
    yl = yrow >= 0 ? *reinterpret_cast<const u32x4*>(Hl + yrow * dp + k0 + part) : zero;
    xh = xrow >= 0 ? *reinterpret_cast<const u32x4*>(Hh + xrow * dp + k0 + part) : zero;
    xl = xrow >= 0 ? *reinterpret_cast<const u32x4*>(Hl + xrow * dp + k0 + part) : zero;
  };
  fetch(0);
  for (int k0 = 0; k0 < dp; k0 += KCH) {
    *reinterpret_cast<u32x4*>(&sm.yh[p][part]) = yh;
    *reinterpret_cast<u32x4*>(&sm.yl[p][part]) = yl;
    *reinterpret_cast<u32x4*>(&sm.xh[p][part]) = xh;
    *reinterpret_cast<u32x4*>(&sm.xl[p][part]) = xl;
    __syncthreads();
    if (k0 + KCH < dp) fetch(k0 + KCH);
    const int kofs = (lane >> 4) * 8;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int xr = (w >> 1) * 32 + bi * 16 + (lane & 15);
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&sm.xh[xr][kofs]);
      const bf16x8 al = *reinterpret_cast<const bf16x8*>(&sm.xl[xr][kofs]);
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int yr = (w & 1) * 32 + bj * 16 + (lane & 15);
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&sm.yh[yr][kofs]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&sm.yl[yr][kofs]);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[bi][bj], 0, 0, 0);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[bi][bj], 0, 0, 0);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[bi][bj], 0, 0, 0);
      }
    }
    __syncthreads();
  }
}

// Tree-order points less the root centroid g, in float32 (rows of dp values,
// zero past d).
__global__ void k_offset_points(const double* __restrict__ Xt, int64_t N, int d, int dp,
                                const double* __restrict__ g, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * dp) return;
  const int64_t p = e / dp;
  const int k = (int)(e % dp);
  out[e] = k < d ? (float)(Xt[p * d + k] - g[k]) : 0.f;
}

// Node centres in the same frame: row a < nodes is centroid[a] - g, row
// nodes is -g (the origin).
__global__ void k_offset_centres(const double* __restrict__ centroid, int nodes, int d, int dp,
                                 float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)(nodes + 1) * dp) return;
  const int a = (int)(e / dp), k = (int)(e % dp);
  const double c = a < nodes ? centroid[(int64_t)a * d + k] : 0.0;
  out[e] = k < d ? (float)(c - centroid[k]) : 0.f;
}

// Splits eight centred values into bf16 hi and lo (16 bytes each) and adds
// their squares to nsum.
__device__ inline void split8(const f32x4& a, const f32x4& b, const f32x4& ca, const f32x4& cb, u32x4& hi,
                              u32x4& lo, float& nsum) {
  const float z[8] = {a.x - ca.x, a.y - ca.y, a.z - ca.z, a.w - ca.w, b.x - cb.x, b.y - cb.y, b.z - cb.z, b.w - cb.w};
  __bf16 h[8], l[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    h[i] = (__bf16)z[i];
    l[i] = (__bf16)(z[i] - (float)h[i]);
    nsum = fmaf(z[i], z[i], nsum);
  }
  hi = *reinterpret_cast<const u32x4*>(h);
  lo = *reinterpret_cast<const u32x4*>(l);
}

// The Gram tile of mixed_tile from the float32 points: both sets are centred
// on cen (a row of the centre table), split and staged 32 dimensions at a
// time; each thread handles 8 dimensions of one row point and one column
// point and fetches the next chunk's groups while the matrix cores work on
// the current one. With NORMS the centred points' squared norms go to sm.yn /
// sm.xn for the distance epilogue.
template <bool NORMS>
__device__ void mixed_tile_cached(const float* __restrict__ P, const float* __restrict__ cen, int dp, Idx rows,
                                  int nrows, Idx cols, int ncols, MixSmem& sm, f32x4 (&acc)[2][2]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int p = tid >> 2, part = (tid & 3) * 8;
  const int64_t yrow = p < nrows ? rows(p) : -1;
  const int64_t xrow = p < ncols ? cols(p) : -1;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 y0, y1, x0, x1, c0, c1;   // native vectors: a choice between two structs would go through memory
  auto fetch = [&](int k0) {
    const f32x4* yp = reinterpret_cast<const f32x4*>(P + yrow * dp + k0 + part);
    const f32x4* xp = reinterpret_cast<const f32x4*>(P + xrow * dp + k0 + part);
    const f32x4* cp = reinterpret_cast<const f32x4*>(cen + k0 + part);
    y0 = yrow >= 0 ? yp[0] : zero;
    y1 = yrow >= 0 ? yp[1] : zero;
    x0 = xrow >= 0 ? xp[0] : zero;
    x1 = xrow >= 0 ? xp[1] : zero;
    c0 = cp[0];
    c1 = cp[1];
  };
  float yn = 0.f, xn = 0.f;
  fetch(0);
  for (int k0 = 0; k0 < dp; k0 += KCH) {
    u32x4 h, l;
    // Padded rows stage zeros (not minus the centre) so they add nothing.
    split8(y0, y1, yrow >= 0 ? c0 : zero, yrow >= 0 ? c1 : zero, h, l, yn);
    *reinterpret_cast<u32x4*>(&sm.yh[p][part]) = h;
    *reinterpret_cast<u32x4*>(&sm.yl[p][part]) = l;
    split8(x0, x1, xrow >= 0 ? c0 : zero, xrow >= 0 ? c1 : zero, h, l, xn);
    *reinterpret_cast<u32x4*>(&sm.xh[p][part]) = h;
    *reinterpret_cast<u32x4*>(&sm.xl[p][part]) = l;
    __syncthreads();
    if (k0 + KCH < dp) fetch(k0 + KCH);
    const int kofs = (lane >> 4) * 8;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int xr = (w >> 1) * 32 + bi * 16 + (lane & 15);
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&sm.xh[xr][kofs]);
      const bf16x8 al = *reinterpret_cast<const bf16x8*>(&sm.xl[xr][kofs]);
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int yr = (w & 1) * 32 + bj * 16 + (lane & 15);
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&sm.yh[yr][kofs]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&sm.yl[yr][kofs]);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[bi][bj], 0, 0, 0);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[bi][bj], 0, 0, 0);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[bi][bj], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (NORMS) {
    // The four threads of a point are adjacent lanes.
    yn += __shfl_xor(yn, 1, 64);
    xn += __shfl_xor(xn, 1, 64);
    yn += __shfl_xor(yn, 2, 64);
    xn += __shfl_xor(xn, 2, 64);
    if ((tid & 3) == 0) {
      sm.yn[p] = yn;
      sm.xn[p] = xn;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// The Laplace kernel r^(2-d) on matrix cores. Its power turns a relative error
// e of r^2 into (d - 2) / 2 times e (31 e at d = 64), so its Gram products take
// three bf16 parts per coordinate, hi + mid + lo (the float32 value to about
// 2^-27), and the six products hh, hm, mh, hl, lh, mm (the others lie below
// float32 rounding), and a pair close enough for the Gram form to cancel
// takes explicit differences (laplace_value). Coordinates come from the
// float32 frame (points less the root centroid) and are centred on the tile's
// node; r^2 = |y - c|^2 + |x - c|^2 - 2 (y - c).(x - c) in float32 and the
// power in float64 (r^-62 spans more than float32's range). A pair of the same
// tree position, or with r^2 <= 0, contributes 0.
// ---------------------------------------------------------------------------
struct __attribute__((aligned(16))) LapSmem {
  __bf16 xh[TN][LROW], xm[TN][LROW], xl[TN][LROW];   // column points (A operand)
  __bf16 yh[TM][LROW], ym[TM][LROW], yl[TM][LROW];   // row points (B operand)
  float xn[TN], yn[TM];                               // squared norms of the centred points
};

__device__ inline void split8x3(const float4& a, const float4& b, const float4& ca, const float4& cb, uint4& hi,
                                uint4& mi, uint4& lo, float& nsum) {
  const float z[8] = {a.x - ca.x, a.y - ca.y, a.z - ca.z, a.w - ca.w, b.x - cb.x, b.y - cb.y, b.z - cb.z, b.w - cb.w};
  __bf16 h[8], m[8], l[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    h[i] = (__bf16)z[i];
    const float r1 = z[i] - (float)h[i];   // exact
    m[i] = (__bf16)r1;
    l[i] = (__bf16)(r1 - (float)m[i]);
    nsum = fmaf(z[i], z[i], nsum);
  }
  hi = *reinterpret_cast<const uint4*>(h);
  mi = *reinterpret_cast<const uint4*>(m);
  lo = *reinterpret_cast<const uint4*>(l);
}

// Gram tile of centred points from the float32 frame (the layout of
// mixed_tile_cached; norms always), three-part split, six products.
__device__ void laplace_tile(const float* __restrict__ P, const float* __restrict__ cen, int dp, Idx rows, int nrows,
                             Idx cols, int ncols, LapSmem& sm, f32x4 (&acc)[2][2]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int p = tid >> 2, part = (tid & 3) * 8;
  const int64_t yrow = p < nrows ? rows(p) : -1;
  const int64_t xrow = p < ncols ? cols(p) : -1;
  const float4 zero{0.f, 0.f, 0.f, 0.f};
  float4 y0, y1, x0, x1, c0, c1;
  auto fetch = [&](int k0) {
    const float4* yp = reinterpret_cast<const float4*>(P + yrow * dp + k0 + part);
    const float4* xp = reinterpret_cast<const float4*>(P + xrow * dp + k0 + part);
    const float4* cp = reinterpret_cast<const float4*>(cen + k0 + part);
    y0 = yrow >= 0 ? yp[0] : zero;
    y1 = yrow >= 0 ? yp[1] : zero;
    x0 = xrow >= 0 ? xp[0] : zero;
    x1 = xrow >= 0 ? xp[1] : zero;
    c0 = cp[0];
    c1 = cp[1];
  };
  float yn = 0.f, xn = 0.f;
  fetch(0);
  for (int k0 = 0; k0 < dp; k0 += KCH) {
    uint4 h, m, l;
    split8x3(y0, y1, yrow >= 0 ? c0 : zero, yrow >= 0 ? c1 : zero, h, m, l, yn);
    *reinterpret_cast<uint4*>(&sm.yh[p][part]) = h;
    *reinterpret_cast<uint4*>(&sm.ym[p][part]) = m;
    *reinterpret_cast<uint4*>(&sm.yl[p][part]) = l;
    split8x3(x0, x1, xrow >= 0 ? c0 : zero, xrow >= 0 ? c1 : zero, h, m, l, xn);
    *reinterpret_cast<uint4*>(&sm.xh[p][part]) = h;
    *reinterpret_cast<uint4*>(&sm.xm[p][part]) = m;
    *reinterpret_cast<uint4*>(&sm.xl[p][part]) = l;
    __syncthreads();
    if (k0 + KCH < dp) fetch(k0 + KCH);
    const int kofs = (lane >> 4) * 8;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int xr = (w >> 1) * 32 + bi * 16 + (lane & 15);
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&sm.xh[xr][kofs]);
      const bf16x8 am = *reinterpret_cast<const bf16x8*>(&sm.xm[xr][kofs]);
      const bf16x8 al = *reinterpret_cast<const bf16x8*>(&sm.xl[xr][kofs]);
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int yr = (w & 1) * 32 + bj * 16 + (lane & 15);
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&sm.yh[yr][kofs]);
        const bf16x8 bm = *reinterpret_cast<const bf16x8*>(&sm.ym[yr][kofs]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&sm.yl[yr][kofs]);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[bi][bj], 0, 0, 0);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, acc[bi][bj], 0, 0, 0);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, acc[bi][bj], 0, 0, 0);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[bi][bj], 0, 0, 0);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[bi][bj], 0, 0, 0);
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, acc[bi][bj], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  yn += __shfl_xor(yn, 1, 64);
  xn += __shfl_xor(xn, 1, 64);
  yn += __shfl_xor(yn, 2, 64);
  xn += __shfl_xor(xn, 2, 64);
  if ((tid & 3) == 0) {
    sm.yn[p] = yn;
    sm.xn[p] = xn;
  }
  __syncthreads();
}

// r^(2-d) = (1 / r^2)^((d - 2) / 2): an integer power by squaring, times
// sqrt(1 / r^2) for odd d; 0 for r^2 <= 0. The Gram form of r^2 loses
// about 2^-22 (|y - c|^2 + |x - c|^2) to cancellation, so a pair with r^2
// below 1/16 of that sum (rare: points much closer to each other than to the
// centre) takes r^2 from explicit float32 differences of its two points
// instead, which keeps every pair within about 2^-18 relative on r^2.
__device__ inline float exact_r2(const float* __restrict__ px, int dp, int64_t a, int64_t b) {
  const float4* pa = reinterpret_cast<const float4*>(px + a * dp);
  const float4* pb = reinterpret_cast<const float4*>(px + b * dp);
  float s = 0.f;
  for (int k = 0; k < dp / 4; ++k) {
    const float4 x = pa[k], y = pb[k];
    const float d0 = x.x - y.x, d1 = x.y - y.y, d2 = x.z - y.z, d3 = x.w - y.w;
    s = fmaf(d0, d0, s);
    s = fmaf(d1, d1, s);
    s = fmaf(d2, d2, s);
    s = fmaf(d3, d3, s);
  }
  return s;
}

__device__ inline double laplace_value(float g, float yn, float xn, int d, const float* __restrict__ px, int dp,
                                       int64_t prow, int64_t pcol) {
  float r2 = yn + xn - 2.f * g;
  if (r2 < 0.0625f * (yn + xn)) r2 = exact_r2(px, dp, prow, pcol);
  if (!(r2 > 0.f)) return 0.0;
  const double x = 1.0 / (double)r2;
  double p = 1.0, b = x;
  for (int e = (d - 2) >> 1; e; e >>= 1) {
    if (e & 1) p *= b;
    b *= b;
  }
  return (d & 1) ? p * sqrt(x) : p;
}

// Sampled blocks of a level, Laplace kernel (centred on the node's centroid).
__global__ void __launch_bounds__(NTH) k_level_kblock_laplace(int d, int first, int tiles_m, int tiles_n,
                                                              const int32_t* __restrict__ rows,
                                                              const int32_t* __restrict__ nrows_a, int s_cap,
                                                              const int32_t* __restrict__ cols,
                                                              const int32_t* __restrict__ ncols_a, int n_cap,
                                                              const unsigned char* __restrict__ mask,
                                                              const float* __restrict__ px,
                                                              const float* __restrict__ cc, int dp,
                                                              double* __restrict__ A, unsigned int* flag) {
  __shared__ LapSmem sm;
  const int tiles = tiles_m * tiles_n;
  const int ln = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  const int node = first + ln;
  if (mask && !mask[node]) return;
  const int s = nrows_a[node], n = ncols_a[node];
  const int r0 = (tile % tiles_m) * TM, c0 = (tile / tiles_m) * TN;
  if (r0 >= s || c0 >= n) return;
  const int32_t* rp = rows + (int64_t)node * s_cap + r0;
  const int32_t* cp = cols + (int64_t)node * n_cap + c0;
  f32x4 acc[2][2];
  laplace_tile(px, cc + (int64_t)node * dp, dp, Idx{rp, 0}, min(TM, s - r0), Idx{cp, 0}, min(TN, n - c0), sm, acc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double* out = A + (int64_t)ln * s_cap * n_cap;
  bool bad = false;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int yr = (w & 1) * 32 + bj * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int xc = (w >> 1) * 32 + bi * 16 + (lane >> 4) * 4 + e;
        if (r0 + yr < s && c0 + xc < n) {
          const double v = rp[yr] == cp[xc] ? 0.0
                                             : laplace_value(acc[bi][bj][e], sm.yn[yr], sm.xn[xc], d, px, dp, rp[yr],
                                                             cp[xc]);
          bad |= !isfinite(v);
          out[(int64_t)(c0 + xc) * s_cap + (r0 + yr)] = v;
        }
      }
    }
  if (bad) atomicOr(flag, 1u);
}

// part[bj] += sum_x K(y, x) q_x for the row point (w & 1) * 32 + bj * 16 + l % 16
// (row positions rbase + i, columns cols(j)), Laplace kernel, centred on cen.
__device__ inline void laplace_sum(const float* __restrict__ px, const float* __restrict__ cen, int dp, int d,
                                   int64_t rbase, int nrows, Idx cols, int ncols, const double* __restrict__ q,
                                   LapSmem& sm, double (&part)[2], bool& bad) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int c0 = 0; c0 < ncols; c0 += TN) {
    Idx cm{cols.idx ? cols.idx + c0 : nullptr, cols.base + c0};
    f32x4 acc[2][2];
    laplace_tile(px, cen, dp, Idx{nullptr, rbase}, nrows, cm, min(TN, ncols - c0), sm, acc);
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int yr = (w & 1) * 32 + bj * 16 + (lane & 15);
      double s = 0.0;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int xc = (w >> 1) * 32 + bi * 16 + (lane >> 4) * 4 + e;
          if (c0 + xc < ncols) {
            const int64_t pr = rbase + yr, pc = cm(xc);
            const double v = pr == pc ? 0.0 : laplace_value(acc[bi][bj][e], sm.yn[yr], sm.xn[xc], d, px, dp, pr, pc);
            bad |= !isfinite(v);
            s = fma(v, q[c0 + xc], s);
          }
        }
      part[bj] += s;
    }
    __syncthreads();   // norms in LDS are rewritten by the next tile
  }
}

// Operands of the tree's points for the matrix-core tiles: pre-split in the
// origin frame (hi, lo, with norms for the Gaussian), or in float32 with the
// centre table for tiles that centre while staging; all null: stage from
// float64.
struct Split {
  const __bf16* hi;
  const __bf16* lo;
  const float* nrm;
  const float* x;
  const float* cc;
  int dp;
  int origin;   // row of cc holding the origin
  // Centre row of a tile whose Gaussian centre is node a (the polynomial
  // kernel's inner products centre on the origin).
  template <bool DOT>
  __device__ inline const float* centre(int a) const { return cc + (int64_t)(DOT ? origin : a) * dp; }
};

template <bool DOT>
__device__ inline float kfun_mixed(float g, float yn, float xn, const KParams& kp) {
  if (DOT) {
    const float base = fmaf(g, (float)kp.inv_h, (float)kp.c);
    float r = 1.f;
    for (int i = 0; i < kp.p; ++i) r *= base;
    return r;
  }
  const float r2 = fmaxf(yn + xn - 2.f * g, 0.f);
  return expf(r2 * (float)kp.neg_inv_2h2);   // Gaussian (the Laplace kernel never comes here)
}

// Sampled blocks of a level in mixed precision (Gaussian: centred on the node
// centroid; polynomial: raw inner products).
template <bool DOT>
__global__ void __launch_bounds__(NTH) k_level_kblock_mixed(const double* __restrict__ Xt, int d, KParams kp,
                                                            int first, int tiles_m, int tiles_n,
                                                            const int32_t* __restrict__ rows,
                                                            const int32_t* __restrict__ nrows_a, int s_cap,
                                                            const int32_t* __restrict__ cols,
                                                            const int32_t* __restrict__ ncols_a, int n_cap,
                                                            const double* __restrict__ centroid,
                                                            const unsigned char* __restrict__ mask, Split sp,
                                                            double* __restrict__ A, unsigned int* flag) {
  __shared__ MixSmem sm;
  const int tiles = tiles_m * tiles_n;
  const int ln = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  const int node = first + ln;
  if (mask && !mask[node]) return;
  const int s = nrows_a[node], n = ncols_a[node];
  const int r0 = (tile % tiles_m) * TM, c0 = (tile / tiles_m) * TN;
  if (r0 >= s || c0 >= n) return;
  f32x4 acc[2][2];
  if (sp.hi)
    mixed_tile_split(sp.hi, sp.lo, sp.nrm, sp.dp, Idx{rows + (int64_t)node * s_cap + r0, 0}, min(TM, s - r0),
                     Idx{cols + (int64_t)node * n_cap + c0, 0}, min(TN, n - c0), sm, acc);
  else if (sp.x)
    mixed_tile_cached<!DOT>(sp.x, sp.centre<DOT>(node), sp.dp, Idx{rows + (int64_t)node * s_cap + r0, 0},
                            min(TM, s - r0), Idx{cols + (int64_t)node * n_cap + c0, 0}, min(TN, n - c0), sm, acc);
  else
    mixed_tile<!DOT>(Xt, Idx{rows + (int64_t)node * s_cap + r0, 0}, min(TM, s - r0), Xt,
                     Idx{cols + (int64_t)node * n_cap + c0, 0}, min(TN, n - c0), d, centroid + (int64_t)node * d, sm,
                     acc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double* out = A + (int64_t)ln * s_cap * n_cap;
  bool bad = false;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int yr = (w & 1) * 32 + bj * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int xc = (w >> 1) * 32 + bi * 16 + (lane >> 4) * 4 + e;
        if (r0 + yr < s && c0 + xc < n) {
          const float v = kfun_mixed<DOT>(acc[bi][bj][e], DOT ? 0.f : sm.yn[yr], DOT ? 0.f : sm.xn[xc], kp);
          bad |= !isfinite(v);
          out[(int64_t)(c0 + xc) * s_cap + (r0 + yr)] = (double)v;
        }
      }
    }
  if (bad) atomicOr(flag, 1u);
}

// Kernel sums in mixed precision: part[bj] accumulates sum_x K(y, x) q_x for
// the row point (w & 1) * 32 + bj * 16 + l % 16 of the tile.
template <bool DOT>
__device__ inline void mixed_sum(const double* __restrict__ Y, Idx rows, int nrows, const double* __restrict__ X,
                                 Idx cols, int ncols, const double* __restrict__ q, int d,
                                 const double* __restrict__ center, const KParams& kp, MixSmem& sm, double (&part)[2],
                                 bool& bad, Split sp = Split{}, int cen_node = 0) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int c0 = 0; c0 < ncols; c0 += TN) {
    Idx cm{cols.idx ? cols.idx + c0 : nullptr, cols.base + c0};
    f32x4 acc[2][2];
    if (sp.hi)
      mixed_tile_split(sp.hi, sp.lo, sp.nrm, sp.dp, rows, nrows, cm, min(TN, ncols - c0), sm, acc);
    else if (sp.x)
      mixed_tile_cached<!DOT>(sp.x, sp.centre<DOT>(cen_node), sp.dp, rows, nrows, cm, min(TN, ncols - c0), sm, acc);
    else mixed_tile<!DOT>(Y, rows, nrows, X, cm, min(TN, ncols - c0), d, center, sm, acc);
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int yr = (w & 1) * 32 + bj * 16 + (lane & 15);
      double s = 0.0;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int xc = (w >> 1) * 32 + bi * 16 + (lane >> 4) * 4 + e;
          if (c0 + xc < ncols) {
            const float v = kfun_mixed<DOT>(acc[bi][bj][e], DOT ? 0.f : sm.yn[yr], DOT ? 0.f : sm.xn[xc], kp);
            bad |= !isfinite(v);
            s = fma((double)v, q[c0 + xc], s);
          }
        }
      part[bj] += s;
    }
    __syncthreads();   // norms in LDS are rewritten by the next tile
  }
}

// Fixed-order reduction of part[] to one value per row point of the tile.
__device__ inline void mixed_reduce(double (&part)[2], double* red /* 4 waves x 2 x 64 */, double* rowsum) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) red[(w * 2 + bj) * 64 + lane] = part[bj];
  __syncthreads();
  if (threadIdx.x < TM) {
    const int yr = threadIdx.x;
    const int wy = yr / 32, bj = (yr % 32) / 16, l16 = yr % 16;
    double s = 0.0;
    for (int wx = 0; wx < 2; ++wx) {
      const int wv = wx * 2 + wy;
      for (int g = 0; g < 4; ++g) s += red[(wv * 2 + bj) * 64 + g * 16 + l16];
    }
    rowsum[yr] = s;
  }
  __syncthreads();
}

// (At most 168 registers, three workgroups per compute unit: the extra
// resident waves hide the tiles' load latencies; 15% faster than two.)
template <bool DOT>
__global__ void __launch_bounds__(NTH, 3) k_evaluate_mixed(const double* __restrict__ Xt, int d, KParams kp, int depth,
                                                        const int32_t* __restrict__ tile_leaf,
                                                        const int32_t* __restrict__ tile_start,
                                                        const int32_t* __restrict__ nb, const int32_t* __restrict__ ne,
                                                        const double* __restrict__ q_tree,
                                                        const int32_t* __restrict__ rank,
                                                        const int32_t* __restrict__ skel, int r_cap,
                                                        const double* __restrict__ qt,
                                                        const double* __restrict__ centroid,
                                                        const int32_t* __restrict__ perm, Split sp,
                                                        double* __restrict__ u, double* __restrict__ u_far,
                                                        unsigned int* flag) {
  __shared__ MixSmem sm;
  __shared__ double red[8 * 64];
  __shared__ double far_sum[TM], near_sum[TM];
  const int leaf = tile_leaf[blockIdx.x];
  const int start = tile_start[blockIdx.x];
  const int nrows = min(TM, ne[leaf] - start);
  const Idx rmap{nullptr, start};
  const double* cen = centroid + (int64_t)leaf * d;
  bool bad = false;
  double part[2] = {0.0, 0.0};
  int a = leaf;
  for (int lev = depth; lev >= 1; --lev) {
    const int sib = (a & 1) ? a + 1 : a - 1;
    const int r = rank[sib];
    if (r > 0)
      mixed_sum<DOT>(Xt, rmap, nrows, Xt, Idx{skel + (int64_t)sib * r_cap, 0}, r, qt + (int64_t)sib * r_cap, d, cen,
                     kp, sm, part, bad, sp, leaf);
    a = (a - 1) >> 1;
  }
  mixed_reduce(part, red, far_sum);
  double npart[2] = {0.0, 0.0};
  const int lb = nb[leaf];
  mixed_sum<DOT>(Xt, rmap, nrows, Xt, Idx{nullptr, lb}, ne[leaf] - lb, q_tree + lb, d, cen, kp, sm, npart, bad, sp,
                 leaf);
  mixed_reduce(npart, red, near_sum);
  if (threadIdx.x < nrows) {
    const int ci = perm[start + threadIdx.x];
    const double f = far_sum[threadIdx.x];
    u[ci] = f + near_sum[threadIdx.x];
    if (u_far) u_far[ci] = f;
  }
  if (bad) atomicOr(flag, 1u);
}

// k_evaluate_mixed on the pre-split operands for rows of at most 64
// dimensions, staged per workgroup. The 64 target rows and their norms go to
// LDS once for all tiles. Each 64-point column tile (a sibling's skeleton
// points at every level from the leaf up, then the leaf's own points) is staged
// at full width with its norms and charges, and the next tiles' loads are in
// flight while a tile is multiplied: the points of tile t + 1 and the skeleton
// indices of tile t + 2 during tile t. Same products in the same order and the
// same sums as k_evaluate_mixed, so the same bits.
constexpr int kStagedTiles = 96;   // column tiles a workgroup's list holds

template <int NC>
struct __attribute__((aligned(16))) StagedSmem {
  __bf16 yh[TM][NC * KCH + 8], yl[TM][NC * KCH + 8];   // target rows (B operand), 16-byte rows
  __bf16 xh[TN][NC * KCH + 8], xl[TN][NC * KCH + 8];   // column points (A operand)
  double xq[TN];                                       // the column points' charges
  float yn[TM], xn[TN];
  int64_t tb[kStagedTiles];   // tile base: skeleton slot (far field) or point position (near field)
  int tn[kStagedTiles];       // points in the tile; negative for the near field
  int nt, nfar;
};

// The skeleton position of point p of a far-field tile t of k_evaluate_staged,
// as loaded (from a clamped slot; anything for other tiles). The caller does
// not touch it until it loads the tile's points, a tile later: any arithmetic
// on it here would wait for the load.
__device__ __attribute__((always_inline)) inline int32_t staged_index(int t, int nt, const int* tn, const int64_t* tb,
                                                                      const int32_t* __restrict__ skel, int p) {
  int32_t raw = 0;
  if (t < nt) {
    const int n = tn[t];
    if (n > 0) raw = skel[tb[t] + min(p, n - 1)];
  }
  return raw;
}

// The operands of tile t for point p and group part into registers: groups 0
// and (NC = 2) 1 of the part's 8 NC values of each split, the point's norm and
// charge, and whether the point exists. Every load reads a valid address (row
// or slot 0 stands in for a missing point); the values are masked only when
// they are stored, a tile later. (Plain functions and named registers: a
// lambda's captured pointers and an array carried around the loop both ended
// up in scratch memory.)
template <int NC>
__device__ __attribute__((always_inline)) inline void staged_load_tile(
    int t, int32_t raw, int nt, const int* tn, const int64_t* tb, int p, int part, const __bf16* __restrict__ Hh,
    const __bf16* __restrict__ Hl, const float* __restrict__ nrm, const double* __restrict__ qt,
    const double* __restrict__ q_tree, u32x4& xh0, u32x4& xh1, u32x4& xl0, u32x4& xl1, float& xn, double& xq,
    bool& xv) {
  constexpr int DP = NC * KCH, PW = NC * 8;
  int64_t pt = 0, qi = 0;
  bool far = false, valid = false;
  if (t < nt) {
    const int n = tn[t];
    const int64_t base = tb[t];
    far = n > 0;
    const int cnt = far ? n : -n;
    valid = p < cnt;
    qi = base + min(p, cnt - 1);
    pt = far ? (int64_t)raw : qi;
  }
  const __bf16* hp = Hh + pt * DP + part * PW;
  const __bf16* lp = Hl + pt * DP + part * PW;
  xh0 = *reinterpret_cast<const u32x4*>(hp);
  xl0 = *reinterpret_cast<const u32x4*>(lp);
  if constexpr (NC == 2) {
    xh1 = *reinterpret_cast<const u32x4*>(hp + 8);
    xl1 = *reinterpret_cast<const u32x4*>(lp + 8);
  }
  xn = nrm ? nrm[pt] : 0.f;
  const double* qb = far ? qt : q_tree;
  xq = qb[qi];
  xv = valid;
}

template <bool DOT, int NC>
__global__ void __launch_bounds__(NTH, 3)
k_evaluate_staged(const __bf16* __restrict__ Hh, const __bf16* __restrict__ Hl, const float* __restrict__ nrm,
                  KParams kp, int depth, const int32_t* __restrict__ tile_leaf, const int32_t* __restrict__ tile_start,
                  const int32_t* __restrict__ nb, const int32_t* __restrict__ ne, const double* __restrict__ q_tree,
                  const int32_t* __restrict__ rank, const int32_t* __restrict__ skel, int r_cap,
                  const double* __restrict__ qt, const int32_t* __restrict__ perm, double* __restrict__ u,
                  double* __restrict__ u_far, unsigned int* flag) {
  constexpr int DP = NC * KCH;   // row length of the split operands
  constexpr int PW = NC * 8;     // values a thread stages per row
  __shared__ StagedSmem<NC> sm;
  __shared__ double red[8 * 64];
  __shared__ double far_sum[TM], near_sum[TM];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int leaf = tile_leaf[blockIdx.x];
  const int start = tile_start[blockIdx.x];
  const int nrows = min(TM, ne[leaf] - start);
  const int lb = nb[leaf];
  // Tile list: lane l < depth takes the sibling of the leaf's ancestor l
  // levels up, lane depth the leaf itself; an exclusive scan of the tile counts
  // places them in the order of k_evaluate_mixed.
  if (w == 0) {
    int a = leaf;
    for (int i = 0; i < lane && i < depth; ++i) a = (a - 1) >> 1;
    int cnt = 0, r = 0;
    int64_t base = 0;
    if (lane < depth) {
      const int sib = (a & 1) ? a + 1 : a - 1;
      r = rank[sib];
      base = (int64_t)sib * r_cap;
    } else if (lane == depth) {
      r = ne[leaf] - lb;
      base = lb;
    }
    if (lane <= depth && r > 0) cnt = (r + TN - 1) / TN;
    int incl = cnt;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off, 64);
      if (lane >= off) incl += y;
    }
    const int off0 = incl - cnt;
    for (int j = 0; j < cnt; ++j) {
      const int np = min(TN, r - j * TN);
      sm.tb[off0 + j] = base + j * TN;
      sm.tn[off0 + j] = lane < depth ? np : -np;
    }
    if (lane == depth) {
      sm.nt = incl;
      sm.nfar = off0;
    }
  }
  const int p = tid >> 2, part = tid & 3;
  const u32x4 zero = {0u, 0u, 0u, 0u};
  {
    const bool yv = p < nrows;
    const int64_t yrow = (int64_t)start + (yv ? p : 0);
    const __bf16* hp = Hh + yrow * DP + part * PW;
    const __bf16* lp = Hl + yrow * DP + part * PW;
    const u32x4 h0 = *reinterpret_cast<const u32x4*>(hp);
    const u32x4 l0 = *reinterpret_cast<const u32x4*>(lp);
    u32x4 h1 = zero, l1 = zero;
    if constexpr (NC == 2) {
      h1 = *reinterpret_cast<const u32x4*>(hp + 8);
      l1 = *reinterpret_cast<const u32x4*>(lp + 8);
    }
    const float yn = nrm ? nrm[yrow] : 0.f;
    *reinterpret_cast<u32x4*>(&sm.yh[p][part * PW]) = yv ? h0 : zero;
    *reinterpret_cast<u32x4*>(&sm.yl[p][part * PW]) = yv ? l0 : zero;
    if constexpr (NC == 2) {
      *reinterpret_cast<u32x4*>(&sm.yh[p][part * PW + 8]) = yv ? h1 : zero;
      *reinterpret_cast<u32x4*>(&sm.yl[p][part * PW + 8]) = yv ? l1 : zero;
    }
    if (part == 0) sm.yn[p] = yv ? yn : 0.f;
  }
  __syncthreads();   // tile list and target rows
  const int nt = sm.nt, nfar = sm.nfar;
  // The staged tile's operands in registers (see staged_load_tile).
  u32x4 xh0 = zero, xh1 = zero, xl0 = zero, xl1 = zero;
  float xn_r = 0.f;
  double xq_r = 0.0;
  bool xv = false;
  staged_load_tile<NC>(0, staged_index(0, nt, sm.tn, sm.tb, skel, p), nt, sm.tn, sm.tb, p, part, Hh, Hl, nrm, qt,
                       q_tree, xh0, xh1, xl0, xl1, xn_r, xq_r, xv);
  int32_t raw_next = staged_index(1, nt, sm.tn, sm.tb, skel, p);
  double part_f[2] = {0.0, 0.0}, part_n[2] = {0.0, 0.0};
  bool bad = false;
  for (int t = 0; t < nt; ++t) {
    *reinterpret_cast<u32x4*>(&sm.xh[p][part * PW]) = xv ? xh0 : zero;
    *reinterpret_cast<u32x4*>(&sm.xl[p][part * PW]) = xv ? xl0 : zero;
    if constexpr (NC == 2) {
      *reinterpret_cast<u32x4*>(&sm.xh[p][part * PW + 8]) = xv ? xh1 : zero;
      *reinterpret_cast<u32x4*>(&sm.xl[p][part * PW + 8]) = xv ? xl1 : zero;
    }
    if (part == 0) {
      sm.xn[p] = xv ? xn_r : 0.f;
      sm.xq[p] = xv ? xq_r : 0.0;
    }
    const int n_t = sm.tn[t];
    __syncthreads();
    // The next tile's points (their positions were loaded one tile ago),
    // then the positions of the tile after it.
    staged_load_tile<NC>(t + 1, raw_next, nt, sm.tn, sm.tb, p, part, Hh, Hl, nrm, qt, q_tree, xh0, xh1, xl0, xl1,
                         xn_r, xq_r, xv);
    raw_next = staged_index(t + 2, nt, sm.tn, sm.tb, skel, p);
    f32x4 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < NC; ++kc) {
      const int kofs = kc * KCH + (lane >> 4) * 8;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const int xr = (w >> 1) * 32 + bi * 16 + (lane & 15);
        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&sm.xh[xr][kofs]);
        const bf16x8 al = *reinterpret_cast<const bf16x8*>(&sm.xl[xr][kofs]);
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          const int yr = (w & 1) * 32 + bj * 16 + (lane & 15);
          const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&sm.yh[yr][kofs]);
          const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&sm.yl[yr][kofs]);
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[bi][bj], 0, 0, 0);
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[bi][bj], 0, 0, 0);
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[bi][bj], 0, 0, 0);
        }
      }
    }
    const int ncols = n_t > 0 ? n_t : -n_t;
    const bool far = t < nfar;
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int yr = (w & 1) * 32 + bj * 16 + (lane & 15);
      double s = 0.0;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int xc = (w >> 1) * 32 + bi * 16 + (lane >> 4) * 4 + e;
          if (xc < ncols) {
            const float v = kfun_mixed<DOT>(acc[bi][bj][e], DOT ? 0.f : sm.yn[yr], DOT ? 0.f : sm.xn[xc], kp);
            bad |= !isfinite(v);
            s = fma((double)v, sm.xq[xc], s);
          }
        }
      if (far) part_f[bj] += s;
      else part_n[bj] += s;
    }
    __syncthreads();   // the tile's operands are rewritten by the next one
  }
  mixed_reduce(part_f, red, far_sum);
  mixed_reduce(part_n, red, near_sum);
  if (threadIdx.x < nrows) {
    const int ci = perm[start + threadIdx.x];
    const double f = far_sum[threadIdx.x];
    u[ci] = f + near_sum[threadIdx.x];
    if (u_far) u_far[ci] = f;
  }
  if (bad) atomicOr(flag, 1u);
}

// k_level_kblock_mixed on the pre-split operands for rows of at most 64
// dimensions, staged per workgroup: one workgroup computes tpw consecutive
// 64-column tiles of one 64-row tile of a node's block. The rows and their
// norms go to LDS once; the column points of the next tile and the column
// positions of the one after are loaded while a tile is multiplied. Same
// products and kernel values as k_level_kblock_mixed, so the same bits.
template <int NC>
struct __attribute__((aligned(16))) KbSmem {
  __bf16 yh[TM][NC * KCH + 8], yl[TM][NC * KCH + 8];
  __bf16 xh[TN][NC * KCH + 8], xl[TN][NC * KCH + 8];
  float yn[TM], xn[TN];
};

template <bool DOT, int NC>
__global__ void __launch_bounds__(NTH, 3)
k_kblock_staged(const __bf16* __restrict__ Hh, const __bf16* __restrict__ Hl, const float* __restrict__ nrm, KParams kp,
                int first, int tiles_m, int groups_n, int tpw, const int32_t* __restrict__ rows,
                const int32_t* __restrict__ nrows_a, int s_cap, const int32_t* __restrict__ cols,
                const int32_t* __restrict__ ncols_a, int n_cap, const unsigned char* __restrict__ mask,
                double* __restrict__ A, unsigned int* flag) {
  constexpr int DP = NC * KCH, PW = NC * 8;
  __shared__ KbSmem<NC> sm;
  const int per = tiles_m * groups_n;
  const int ln = blockIdx.x / per, rem = blockIdx.x % per;
  const int node = first + ln;
  if (mask && !mask[node]) return;
  const int s = nrows_a[node], n = ncols_a[node];
  const int r0 = (rem % tiles_m) * TM, cb = (rem / tiles_m) * tpw * TN;   // first row, first column
  if (r0 >= s || cb >= n) return;
  const int nt = min(tpw, (n - cb + TN - 1) / TN);   // column tiles of this workgroup
  const int ncol = n - cb;                           // columns from cb to the node's last
  const int32_t* rix = rows + (int64_t)node * s_cap + r0;
  const int32_t* cix = cols + (int64_t)node * n_cap + cb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int p = tid >> 2, part = tid & 3;
  const u32x4 zero = {0u, 0u, 0u, 0u};
  {
    const bool yv = r0 + p < s;
    const int64_t yrow = rix[yv ? p : 0];
    const __bf16* hp = Hh + yrow * DP + part * PW;
    const __bf16* lp = Hl + yrow * DP + part * PW;
    const u32x4 h0 = *reinterpret_cast<const u32x4*>(hp);
    const u32x4 l0 = *reinterpret_cast<const u32x4*>(lp);
    u32x4 h1 = zero, l1 = zero;
    if constexpr (NC == 2) {
      h1 = *reinterpret_cast<const u32x4*>(hp + 8);
      l1 = *reinterpret_cast<const u32x4*>(lp + 8);
    }
    const float yn = nrm ? nrm[yrow] : 0.f;
    *reinterpret_cast<u32x4*>(&sm.yh[p][part * PW]) = yv ? h0 : zero;
    *reinterpret_cast<u32x4*>(&sm.yl[p][part * PW]) = yv ? l0 : zero;
    if constexpr (NC == 2) {
      *reinterpret_cast<u32x4*>(&sm.yh[p][part * PW + 8]) = yv ? h1 : zero;
      *reinterpret_cast<u32x4*>(&sm.yl[p][part * PW + 8]) = yv ? l1 : zero;
    }
    if (part == 0) sm.yn[p] = yv ? yn : 0.f;
  }
  // Column position of this thread's point in tile t, from a clamped slot (the
  // node's last column stands in past it); masked when the tile is stored.
  int32_t raw_cur = cix[min(p, ncol - 1)];
  int32_t raw_next = nt > 1 ? cix[min(TN + p, ncol - 1)] : 0;
  u32x4 xh0, xh1 = zero, xl0, xl1 = zero;
  float xn_r;
  {
    const int64_t pt = raw_cur;
    const __bf16* hp = Hh + pt * DP + part * PW;
    const __bf16* lp = Hl + pt * DP + part * PW;
    xh0 = *reinterpret_cast<const u32x4*>(hp);
    xl0 = *reinterpret_cast<const u32x4*>(lp);
    if constexpr (NC == 2) {
      xh1 = *reinterpret_cast<const u32x4*>(hp + 8);
      xl1 = *reinterpret_cast<const u32x4*>(lp + 8);
    }
    xn_r = nrm ? nrm[pt] : 0.f;
  }
  double* out = A + (int64_t)ln * s_cap * n_cap;
  bool bad = false;
  for (int t = 0; t < nt; ++t) {
    const int c0 = cb + t * TN;
    const bool xv = c0 + p < n;
    *reinterpret_cast<u32x4*>(&sm.xh[p][part * PW]) = xv ? xh0 : zero;
    *reinterpret_cast<u32x4*>(&sm.xl[p][part * PW]) = xv ? xl0 : zero;
    if constexpr (NC == 2) {
      *reinterpret_cast<u32x4*>(&sm.xh[p][part * PW + 8]) = xv ? xh1 : zero;
      *reinterpret_cast<u32x4*>(&sm.xl[p][part * PW + 8]) = xv ? xl1 : zero;
    }
    if (part == 0) sm.xn[p] = xv ? xn_r : 0.f;
    __syncthreads();
    if (t + 1 < nt) {
      // The next tile's points (positions loaded one tile ago), then the
      // positions of the tile after it.
      const int64_t pt = raw_next;
      const __bf16* hp = Hh + pt * DP + part * PW;
      const __bf16* lp = Hl + pt * DP + part * PW;
      xh0 = *reinterpret_cast<const u32x4*>(hp);
      xl0 = *reinterpret_cast<const u32x4*>(lp);
      if constexpr (NC == 2) {
        xh1 = *reinterpret_cast<const u32x4*>(hp + 8);
        xl1 = *reinterpret_cast<const u32x4*>(lp + 8);
      }
      xn_r = nrm ? nrm[pt] : 0.f;
      if (t + 2 < nt) raw_next = cix[min((t + 2) * TN + p, ncol - 1)];
    }
    f32x4 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < NC; ++kc) {
      const int kofs = kc * KCH + (lane >> 4) * 8;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const int xr = (w >> 1) * 32 + bi * 16 + (lane & 15);
        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&sm.xh[xr][kofs]);
        const bf16x8 al = *reinterpret_cast<const bf16x8*>(&sm.xl[xr][kofs]);
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          const int yr = (w & 1) * 32 + bj * 16 + (lane & 15);
          const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&sm.yh[yr][kofs]);
          const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&sm.yl[yr][kofs]);
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[bi][bj], 0, 0, 0);
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[bi][bj], 0, 0, 0);
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[bi][bj], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int yr = (w & 1) * 32 + bj * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int xc = (w >> 1) * 32 + bi * 16 + (lane >> 4) * 4 + e;
          if (r0 + yr < s && c0 + xc < n) {
            const float v = kfun_mixed<DOT>(acc[bi][bj][e], DOT ? 0.f : sm.yn[yr], DOT ? 0.f : sm.xn[xc], kp);
            bad |= !isfinite(v);
            out[(int64_t)(c0 + xc) * s_cap + (r0 + yr)] = (double)v;
          }
        }
      }
    __syncthreads();   // the tile's operands are rewritten by the next one
  }
  if (bad) atomicOr(flag, 1u);
}

// Column tiles a workgroup of k_evaluate_staged may list: every level's
// sibling skeleton plus the largest leaf.
int staged_tile_bound(const ffc_tree* t, const ffc_skel* sk) {
  int max_leaf = 0;
  const int first = (1 << t->depth) - 1;
  for (int a = first; a < t->num_nodes; ++a) max_leaf = std::max(max_leaf, t->end_h[a] - t->begin_h[a]);
  return t->depth * ((sk->r_cap + TN - 1) / TN) + (max_leaf + TN - 1) / TN;
}

// Far + near field of the Laplace kernel for one 64-target tile of a leaf
// (the layout of k_evaluate_mixed), every tile centred on the target leaf.
__global__ void __launch_bounds__(NTH) k_evaluate_laplace(int d, int depth, const int32_t* __restrict__ tile_leaf,
                                                          const int32_t* __restrict__ tile_start,
                                                          const int32_t* __restrict__ nb,
                                                          const int32_t* __restrict__ ne,
                                                          const double* __restrict__ q_tree,
                                                          const int32_t* __restrict__ rank,
                                                          const int32_t* __restrict__ skel, int r_cap,
                                                          const double* __restrict__ qt,
                                                          const int32_t* __restrict__ perm,
                                                          const float* __restrict__ px, const float* __restrict__ cc,
                                                          int dp, double* __restrict__ u, double* __restrict__ u_far,
                                                          unsigned int* flag) {
  __shared__ LapSmem sm;
  __shared__ double red[8 * 64];
  __shared__ double far_sum[TM], near_sum[TM];
  const int leaf = tile_leaf[blockIdx.x];
  const int start = tile_start[blockIdx.x];
  const int nrows = min(TM, ne[leaf] - start);
  const float* cen = cc + (int64_t)leaf * dp;
  bool bad = false;
  double part[2] = {0.0, 0.0};
  int a = leaf;
  for (int lev = depth; lev >= 1; --lev) {
    const int sib = (a & 1) ? a + 1 : a - 1;
    const int r = rank[sib];
    if (r > 0)
      laplace_sum(px, cen, dp, d, start, nrows, Idx{skel + (int64_t)sib * r_cap, 0}, r, qt + (int64_t)sib * r_cap, sm,
                  part, bad);
    a = (a - 1) >> 1;
  }
  mixed_reduce(part, red, far_sum);
  double npart[2] = {0.0, 0.0};
  const int lb = nb[leaf];
  laplace_sum(px, cen, dp, d, start, nrows, Idx{nullptr, lb}, ne[leaf] - lb, q_tree + lb, sm, npart, bad);
  mixed_reduce(npart, red, near_sum);
  if (threadIdx.x < nrows) {
    const int ci = perm[start + threadIdx.x];
    const double f = far_sum[threadIdx.x];
    u[ci] = f + near_sum[threadIdx.x];
    if (u_far) u_far[ci] = f;
  }
  if (bad) atomicOr(flag, 1u);
}

template <bool DOT>
__global__ void __launch_bounds__(NTH) k_direct_mixed(const double* __restrict__ Y, int64_t m,
                                                      const double* __restrict__ X, int64_t n, int d, KParams kp,
                                                      const double* __restrict__ q, double* __restrict__ u,
                                                      unsigned int* flag) {
  __shared__ MixSmem sm;
  __shared__ double red[8 * 64];
  __shared__ double rowsum[TM];
  __shared__ double cen[1024];
  const int64_t r0 = (int64_t)blockIdx.x * TM;
  const int nrows = (int)min<int64_t>(TM, m - r0);
  // Centre on the first target of the tile (any common point works for distances).
  const int dc = min(d, 1024);
  for (int k = threadIdx.x; k < dc; k += NTH) cen[k] = Y[r0 * d + k];
  __syncthreads();
  bool bad = false;
  double part[2] = {0.0, 0.0};
  mixed_sum<DOT>(Y, Idx{nullptr, r0}, nrows, X, Idx{nullptr, 0}, (int)n, q, d, cen, kp, sm, part, bad);
  mixed_reduce(part, red, rowsum);
  if (threadIdx.x < nrows) u[r0 + threadIdx.x] = rowsum[threadIdx.x];
  if (bad) atomicOr(flag, 1u);
}

}  // namespace

namespace {
// Whether the Gaussian can take the split coordinates as they are. The
// split's error on a squared distance grows with the two points' norms, so
// they are taken only where every leaf's centroid lies within four leaf radii
// of the origin: near pairs' norms then exceed what centring on their leaf
// would give at most 25-fold (about 4.6 of the split's 16 bits). Otherwise
// every tile centres while staging. Reads the leaves' centroids and radii
// back once.
ffc_status gaussian_frame_ok(const ffc_tree* t, hipStream_t st, bool& ok) {
  const int first = (1 << t->depth) - 1, leaves = 1 << t->depth;
  std::vector<double> c((size_t)leaves * t->d), r(leaves);
  FFC_HIP_TRY(hipMemcpyAsync(c.data(), t->centroid.ptr + (int64_t)first * t->d, c.size() * sizeof(double),
                             hipMemcpyDeviceToHost, st));
  FFC_HIP_TRY(hipMemcpyAsync(r.data(), t->radius.ptr + first, r.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));
  ok = true;
  for (int l = 0; l < leaves && ok; ++l) {
    double n2 = 0.0;
    for (int k = 0; k < t->d; ++k) n2 += c[(size_t)l * t->d + k] * c[(size_t)l * t->d + k];
    ok = n2 <= 16.0 * r[l] * r[l];
  }
  return FFC_OK;
}

// The tree's matrix-core operands (made on first use; a stream being captured
// must find them made).
ffc_status tree_split(const ffc_tree* t, const KParams& kp, hipStream_t st, Split& sp) {
  sp = Split{};
  ffc_tree* tm = const_cast<ffc_tree*>(t);
  const int dp = (t->d + KCH - 1) / KCH * KCH;
  const size_t n = (size_t)t->N * dp, nc = (size_t)(t->num_nodes + 1) * dp;
  if (kp.kind == FFC_LAPLACE) {
    // The float32 frame only (every Laplace tile centres while staging).
    if (tm->bf_x.count != n || tm->bf_cc.count != nc) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      FFC_HIP_TRY(hipStreamIsCapturing(st, &cs));
      if (cs != hipStreamCaptureStatusNone) {
        set_error("mixed precision: skeletonize or evaluate once in mixed precision with this kernel function on "
                  "this tree before capturing (the matrix-core operands are prepared then)");
        return FFC_ERR_STATE;
      }
      FFC_TRY(tm->bf_x.alloc(n));
      FFC_TRY(tm->bf_cc.alloc(nc));
      hipLaunchKernelGGL(k_offset_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, t->Xt.ptr, t->N, t->d,
                         dp, t->centroid.ptr, tm->bf_x.ptr);
      FFC_LAUNCH_CHECK("k_offset_points");
      hipLaunchKernelGGL(k_offset_centres, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, t->centroid.ptr,
                         t->num_nodes, t->d, dp, tm->bf_cc.ptr);
      FFC_LAUNCH_CHECK("k_offset_centres");
    }
    sp.x = t->bf_x.ptr;
    sp.cc = t->bf_cc.ptr;
    sp.origin = t->num_nodes;
    sp.dp = dp;
    return FFC_OK;
  }
  const bool make = tm->bf_dp != dp || tm->bf_hi.count != n;
  if (make || (kp.kind == FFC_GAUSSIAN && tm->bf_frame < 0)) {
    // Made once, eagerly: a captured graph would only make them when replayed.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    FFC_HIP_TRY(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) {
      set_error("mixed precision: skeletonize or evaluate once in mixed precision with this kernel function on "
                "this tree before capturing (the matrix-core operands are prepared then)");
      return FFC_ERR_STATE;
    }
  }
  if (make) {
    tm->bf_dp = 0;
    tm->bf_frame = -1;
    FFC_TRY(tm->bf_hi.alloc(n));
    FFC_TRY(tm->bf_lo.alloc(n));
    FFC_TRY(tm->bf_nrm.alloc((size_t)t->N));
    hipLaunchKernelGGL(k_bf16_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, t->Xt.ptr, t->N, t->d, dp,
                       reinterpret_cast<__bf16*>(tm->bf_hi.ptr), reinterpret_cast<__bf16*>(tm->bf_lo.ptr));
    FFC_LAUNCH_CHECK("k_bf16_split");
    hipLaunchKernelGGL(k_point_norms, dim3((unsigned)((t->N + 255) / 256)), dim3(256), 0, st, t->Xt.ptr, t->N, t->d,
                       tm->bf_nrm.ptr);
    FFC_LAUNCH_CHECK("k_point_norms");
    tm->bf_dp = dp;
  }
  if (kp.kind == FFC_GAUSSIAN && tm->bf_frame < 0) {
    bool ok = false;
    FFC_TRY(gaussian_frame_ok(t, st, ok));
    if (!ok) {
      FFC_TRY(tm->bf_x.alloc(n));
      FFC_TRY(tm->bf_cc.alloc(nc));
      hipLaunchKernelGGL(k_offset_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, t->Xt.ptr, t->N, t->d,
                         dp, t->centroid.ptr, tm->bf_x.ptr);
      FFC_LAUNCH_CHECK("k_offset_points");
      hipLaunchKernelGGL(k_offset_centres, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, t->centroid.ptr,
                         t->num_nodes, t->d, dp, tm->bf_cc.ptr);
      FFC_LAUNCH_CHECK("k_offset_centres");
    }
    tm->bf_frame = ok ? 1 : 0;
  }
  if (kp.kind == FFC_GAUSSIAN && tm->bf_frame == 0) {
    sp.x = t->bf_x.ptr;
    sp.cc = t->bf_cc.ptr;
    sp.origin = t->num_nodes;
  } else {
    sp.hi = reinterpret_cast<const __bf16*>(t->bf_hi.ptr);
    sp.lo = reinterpret_cast<const __bf16*>(t->bf_lo.ptr);
    sp.nrm = kp.kind == FFC_GAUSSIAN ? t->bf_nrm.ptr : nullptr;
  }
  sp.dp = dp;
  return FFC_OK;
}
}  // namespace

ffc_status launch_kblock_batch_mixed(const ffc_tree* t, const KParams& kp, const int32_t* rows, const int32_t* nrows,
                                     int s_cap, const int32_t* cols, const int32_t* ncols, int n_cap, int first,
                                     int count, const double* centroid, double* A, hipStream_t st,
                                     const unsigned char* mask) {
  const int tiles_m = (s_cap + TM - 1) / TM, tiles_n = (n_cap + TN - 1) / TN;
  const int64_t blocks = (int64_t)count * tiles_m * tiles_n;
  if (blocks == 0) return FFC_OK;
  Split sp;
  FFC_TRY(tree_split(t, kp, st, sp));
  if (kp.kind == FFC_LAPLACE) {
    hipLaunchKernelGGL(k_level_kblock_laplace, dim3((unsigned)blocks), dim3(NTH), 0, st, t->d, first, tiles_m, tiles_n,
                       rows, nrows, s_cap, cols, ncols, n_cap, mask, sp.x, sp.cc, sp.dp, A, device_flag());
    FFC_LAUNCH_CHECK("k_level_kblock_laplace");
    return FFC_OK;
  }
  if (sp.hi && (sp.dp == KCH || sp.dp == 2 * KCH)) {
    // Column tiles per workgroup: enough workgroups (about 4096) to fill the
    // chip, the rest of the tiles in sequence behind each.
    const int tpw = (int)std::max<int64_t>(1, std::min<int64_t>(tiles_n, blocks / 4096));
    const int groups_n = (tiles_n + tpw - 1) / tpw;
    const int64_t wgs = (int64_t)count * tiles_m * groups_n;
    const bool dot = kp.kind == FFC_POLYNOMIAL;
    auto kern = dot ? (sp.dp == KCH ? &k_kblock_staged<true, 1> : &k_kblock_staged<true, 2>)
                    : (sp.dp == KCH ? &k_kblock_staged<false, 1> : &k_kblock_staged<false, 2>);
    hipLaunchKernelGGL(kern, dim3((unsigned)wgs), dim3(NTH), 0, st, sp.hi, sp.lo, sp.nrm, kp, first, tiles_m,
                       groups_n, tpw, rows, nrows, s_cap, cols, ncols, n_cap, mask, A, device_flag());
    FFC_LAUNCH_CHECK("k_kblock_staged");
    return FFC_OK;
  }
  if (kp.kind == FFC_POLYNOMIAL)
    hipLaunchKernelGGL(k_level_kblock_mixed<true>, dim3((unsigned)blocks), dim3(NTH), 0, st, t->Xt.ptr, t->d, kp,
                       first, tiles_m, tiles_n, rows, nrows, s_cap, cols, ncols, n_cap, centroid, mask, sp, A,
                       device_flag());
  else
    hipLaunchKernelGGL(k_level_kblock_mixed<false>, dim3((unsigned)blocks), dim3(NTH), 0, st, t->Xt.ptr, t->d, kp,
                       first, tiles_m, tiles_n, rows, nrows, s_cap, cols, ncols, n_cap, centroid, mask, sp, A,
                       device_flag());
  FFC_LAUNCH_CHECK("k_level_kblock_mixed");
  return FFC_OK;
}

ffc_status launch_evaluate_mixed(const ffc_tree* t, const ffc_skel* sk, const KParams& kp, double* u, double* u_far,
                                 hipStream_t st) {
  Split sp;
  FFC_TRY(tree_split(t, kp, st, sp));
  if (kp.kind == FFC_LAPLACE) {
    hipLaunchKernelGGL(k_evaluate_laplace, dim3((unsigned)t->num_tiles), dim3(NTH), 0, st, t->d, t->depth,
                       t->tile_leaf.ptr, t->tile_start.ptr, t->begin.ptr, t->end.ptr, t->q_tree.ptr, sk->rank.ptr,
                       sk->skel.ptr, sk->r_cap, sk->qt.ptr, t->perm.ptr, sp.x, sp.cc, sp.dp, u, u_far,
                       device_flag());
    FFC_LAUNCH_CHECK("k_evaluate_laplace");
    return FFC_OK;
  }
  if (sp.hi && (sp.dp == KCH || sp.dp == 2 * KCH) && t->depth < 63 && (int64_t)t->num_nodes == (2LL << t->depth) - 1 &&
      staged_tile_bound(t, sk) <= kStagedTiles) {
    const bool dot = kp.kind == FFC_POLYNOMIAL;
    auto kern = dot ? (sp.dp == KCH ? &k_evaluate_staged<true, 1> : &k_evaluate_staged<true, 2>)
                    : (sp.dp == KCH ? &k_evaluate_staged<false, 1> : &k_evaluate_staged<false, 2>);
    hipLaunchKernelGGL(kern, dim3((unsigned)t->num_tiles), dim3(NTH), 0, st, sp.hi, sp.lo, sp.nrm, kp, t->depth,
                       t->tile_leaf.ptr, t->tile_start.ptr, t->begin.ptr, t->end.ptr, t->q_tree.ptr, sk->rank.ptr,
                       sk->skel.ptr, sk->r_cap, sk->qt.ptr, t->perm.ptr, u, u_far, device_flag());
    FFC_LAUNCH_CHECK("k_evaluate_staged");
    return FFC_OK;
  }
  if (kp.kind == FFC_POLYNOMIAL)
    hipLaunchKernelGGL(k_evaluate_mixed<true>, dim3((unsigned)t->num_tiles), dim3(NTH), 0, st, t->Xt.ptr, t->d, kp,
                       t->depth, t->tile_leaf.ptr, t->tile_start.ptr, t->begin.ptr, t->end.ptr, t->q_tree.ptr,
                       sk->rank.ptr, sk->skel.ptr, sk->r_cap, sk->qt.ptr, t->centroid.ptr, t->perm.ptr, sp, u, u_far,
                       device_flag());
  else
    hipLaunchKernelGGL(k_evaluate_mixed<false>, dim3((unsigned)t->num_tiles), dim3(NTH), 0, st, t->Xt.ptr, t->d, kp,
                       t->depth, t->tile_leaf.ptr, t->tile_start.ptr, t->begin.ptr, t->end.ptr, t->q_tree.ptr,
                       sk->rank.ptr, sk->skel.ptr, sk->r_cap, sk->qt.ptr, t->centroid.ptr, t->perm.ptr, sp, u, u_far,
                       device_flag());
  FFC_LAUNCH_CHECK("k_evaluate_mixed");
  return FFC_OK;
}

ffc_status launch_direct_mixed(const double* Y, int64_t m, const double* X, int64_t n, int d, const KParams& kp,
                               const double* q, double* u, hipStream_t st) {
  if (m == 0) return FFC_OK;
  if (kp.kind != FFC_POLYNOMIAL && d > 1024) {
    set_error("mixed-precision direct sum supports d <= 1024");
    return FFC_ERR_INVALID_ARG;
  }
  const unsigned blocks = (unsigned)((m + TM - 1) / TM);
  if (kp.kind == FFC_POLYNOMIAL)
    hipLaunchKernelGGL(k_direct_mixed<true>, dim3(blocks), dim3(NTH), 0, st, Y, m, X, n, d, kp, q, u, device_flag());
  else
    hipLaunchKernelGGL(k_direct_mixed<false>, dim3(blocks), dim3(NTH), 0, st, Y, m, X, n, d, kp, q, u, device_flag());
  FFC_LAUNCH_CHECK("k_direct_mixed");
  return FFC_OK;
}

}  // namespace ffc
