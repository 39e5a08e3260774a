// Ridge leverage scores of the rows of sampled kernel blocks: the training
// labels of the learned row proposal.
//
// Statistical leverage (Section 3, definition of statistical leverage) is the
// squared row norm of the top left singular vectors; its ridge form
//   l_i = b_i^T (B^T B + lambda I)^{-1} b_i,  lambda = eps^2 ||B||_F^2,
// weights each singular direction by sigma^2 / (sigma^2 + lambda) and needs no
// rank choice. With the Cholesky factor L L^T = B^T B + lambda I and
// W = B L^{-T}, l_i = |W(i, :)|^2.
//
// Blocks are row-major m x n (row i = the kernel values of target i against the
// n columns), count of them back to back. Four kernels, all FP64:
//   k_gram_rm   G = B^T B, lower-triangle 64 x 64 tiles, rows staged in LDS;
//   k_chol      one workgroup per block: lambda from the trace, then a
//               right-looking blocked Cholesky (32-column panels: LDS
//               factorization of the diagonal block, row-wise triangular solve
//               of the panel, 64 x 64 tiled update of the trailing matrix);
//   k_lev       W = B L^{-T} in place, 64 rows per workgroup, 32-column panels
//               (tiled update from solved columns, then an in-panel solve),
//               accumulating |W(i, :)|^2;
//   k_targets   t_i = ln(max(l_i, 1e-12) m / sum(l)).
// All reductions run in a fixed order, so results are deterministic.
//
// Pivoted (rank-r) leverage, the definition of Section 3 taken from the
// method's own factorization: the column-pivoted QR of B (largest trailing
// column norm first, stopped at the first rho_k < eps rho_0) picks r columns
// J, and l_i is the squared norm of row i of an orthonormal basis of
// span(B(:, J)), i.e. of B(i, J) R11^{-1}. Its pivots and R equal those of a
// Cholesky factorization of G = B^T B with diagonal pivoting (the trailing
// squared column norms are the Schur complement's diagonal), so:
//   k_gram_rm   G as above;
//   k_pchol     one workgroup per block: diagonal-pivoted Cholesky of G,
//               without moving rows (pivot order kept in perm); 16-column
//               panels of L in LDS, lower-triangle trailing update in global
//               memory after each panel; stops by the rank rule;
//   k_lev<true> W = B(:, J) L11^{-T} with L11(a, c) = L(J_a, c), l_i = |W(i,:)|^2.
#include <climits>

#include "ffc_internal.h"

namespace ffc {
namespace {

constexpr int TB = 64, KC = 32, NT = 256, PB = 32;

// G_b(lower tiles) = B_b^T B_b; B_b row-major m x n.
__global__ void __launch_bounds__(NT) k_gram_rm(const double* __restrict__ B, int64_t m, int n, int tiles,
                                                int tri, double* __restrict__ G) {
  __shared__ double ar[KC][TB + 1], ac[KC][TB + 1];
  const int b = blockIdx.x / tri;
  int t = blockIdx.x % tri;
  int ti = 0;
  while (t > ti) { t -= ti + 1; ++ti; }   // lower-triangle tile (ti, tj), tj <= ti
  const int tj = t;
  const int r0 = ti * TB, c0 = tj * TB;
  const double* Bb = B + (int64_t)b * m * n;
  const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;
  double acc[4][4] = {};
  for (int64_t i0 = 0; i0 < m; i0 += KC) {
    for (int e = tid; e < KC * TB; e += NT) {
      const int kk = e / TB, r = e % TB;
      const int64_t i = i0 + kk;
      ar[kk][r] = (i < m && r0 + r < n) ? Bb[i * n + r0 + r] : 0.0;
      ac[kk][r] = (i < m && c0 + r < n) ? Bb[i * n + c0 + r] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < KC; ++kk) {
      double a[4], c[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) { a[q] = ar[kk][tr + 16 * q]; c[q] = ac[kk][tc + 16 * q]; }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[q][w] = fma(a[q], c[w], acc[q][w]);
    }
    __syncthreads();
  }
  double* Gb = G + (int64_t)b * n * n;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int r = r0 + tr + 16 * q, c = c0 + tc + 16 * w;
      if (r < n && c < n) Gb[(int64_t)r * n + c] = acc[q][w];
    }
}

// In-place Cholesky of G_b + eps^2 tr(G_b) I (lower triangle, row-major n x n).
// status[b]: 0 factorized, 1 zero block (all leverages 0), 2 not positive definite.
__global__ void __launch_bounds__(NT) k_chol(double* __restrict__ G, int n, double eps2, int* __restrict__ status) {
  __shared__ double D[PB][PB + 1];
  __shared__ double lr[PB][TB + 1], lc[PB][TB + 1];
  __shared__ double s_lam;
  __shared__ int s_bad;
  const int b = blockIdx.x, tid = threadIdx.x;
  double* A = G + (int64_t)b * n * n;
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += A[(int64_t)i * n + i];
    s_lam = eps2 * tr;
    s_bad = !(tr > 0.0) ? 1 : 0;
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0) status[b] = 1;
    return;
  }
  const double lam = s_lam;
  for (int i = tid; i < n; i += NT) A[(int64_t)i * n + i] += lam;
  __syncthreads();
  for (int p0 = 0; p0 < n; p0 += PB) {
    const int nb = min(PB, n - p0);
    // (a) diagonal block in LDS.
    for (int e = tid; e < PB * PB; e += NT) {
      const int i = e / PB, j = e % PB;
      D[i][j] = (i < nb && j <= i) ? A[(int64_t)(p0 + i) * n + p0 + j] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
      const double dj = D[j][j];
      if (!(dj > 0.0) || !isfinite(dj)) {
        if (tid == 0) s_bad = 2;
      }
      const double sd = sqrt(fmax(dj, 0.0));
      __syncthreads();
      if (tid == 0) D[j][j] = sd;
      if (tid > j && tid < nb) D[tid][j] = sd > 0.0 ? D[tid][j] / sd : 0.0;
      __syncthreads();
      for (int e = tid; e < PB * PB; e += NT) {
        const int i = e / PB, k = e % PB;
        if (i > j && k > j && k <= i && i < nb) D[i][k] = fma(-D[i][j], D[k][j], D[i][k]);
      }
      __syncthreads();
    }
    if (s_bad) {
      if (tid == 0) status[b] = 2;
      return;
    }
    for (int e = tid; e < PB * PB; e += NT) {
      const int i = e / PB, j = e % PB;
      if (i < nb && j <= i) A[(int64_t)(p0 + i) * n + p0 + j] = D[i][j];
    }
    // (b) panel rows below: x L_pp^T = a, one thread per row, in place (the
    // row's 32 values stay in the L1 cache).
    for (int i = p0 + nb + tid; i < n; i += NT) {
      double* row = A + (int64_t)i * n + p0;
      for (int j = 0; j < nb; ++j) {
        double v = row[j];
        for (int k = 0; k < j; ++k) v = fma(-row[k], D[j][k], v);
        row[j] = v / D[j][j];
      }
    }
    __syncthreads();
    // (c) trailing update of the lower triangle.
    const int q0 = p0 + nb;
    const int rem = n - q0;
    const int tiles = (rem + TB - 1) / TB;
    const int tr = tid & 15, tc = tid >> 4;
    for (int ti = 0; ti < tiles; ++ti)
      for (int tj = 0; tj <= ti; ++tj) {
        const int r0 = q0 + ti * TB, c0 = q0 + tj * TB;
        for (int e = tid; e < PB * TB; e += NT) {
          const int r = e / PB, kk = e % PB;
          lr[kk][r] = (r0 + r < n && kk < nb) ? A[(int64_t)(r0 + r) * n + p0 + kk] : 0.0;
          lc[kk][r] = (c0 + r < n && kk < nb) ? A[(int64_t)(c0 + r) * n + p0 + kk] : 0.0;
        }
        __syncthreads();
        double acc[4][4] = {};
        for (int kk = 0; kk < nb; ++kk) {
          double a[4], c[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) { a[q] = lr[kk][tr + 16 * q]; c[q] = lc[kk][tc + 16 * q]; }
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int w = 0; w < 4; ++w) acc[q][w] = fma(a[q], c[w], acc[q][w]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int r = r0 + tr + 16 * q, c = c0 + tc + 16 * w;
            if (r < n && c <= r) A[(int64_t)r * n + c] -= acc[q][w];
          }
        __syncthreads();
      }
  }
  if (tid == 0) status[b] = 0;
}

// W = B L^{-T} in place and lev_i = |W(i, :)|^2, 64 rows per workgroup.
// PIV: column a of the solve is B's column perm[a] (W's column a is stored
// there), only the first rank[b] columns are solved, and L(a, c) is read from
// the column-major pivoted factor L[c * n + perm[a]].
template <bool PIV>
__global__ void __launch_bounds__(NT) k_lev(double* __restrict__ B, int64_t m, int n, int row_tiles,
                                            const double* __restrict__ G, const int* __restrict__ status,
                                            double* __restrict__ lev, const int* __restrict__ perm,
                                            const int* __restrict__ rank) {
  __shared__ double ws[PB][TB + 1];
  __shared__ double ls[PB][PB + 1];
  __shared__ double pan[TB][PB + 1];
  const int b = blockIdx.x / row_tiles;
  const int64_t i0 = (int64_t)(blockIdx.x % row_tiles) * TB;
  const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;
  double* Bb = B + (int64_t)b * m * n;
  const double* L = G + (int64_t)b * n * n;
  const int* pv = PIV ? perm + (int64_t)b * n : nullptr;
  // Column a of the solve lives at position col(a) of B; L(a, c) below the diagonal.
  auto col = [&](int a) { return PIV ? pv[a] : a; };
  auto Lat = [&](int a, int c) { return PIV ? L[(int64_t)c * n + pv[a]] : L[(int64_t)a * n + c]; };
  const int nsolve = PIV ? rank[b] : n;
  if (status[b] != 0) {   // zero block: leverage 0 (a failed factorization is reported by the host)
    for (int r = tid; r < TB; r += NT)
      if (i0 + r < m) lev[(int64_t)b * m + i0 + r] = 0.0;
    return;
  }
  double lsum = 0.0;   // row i0 + tid (tid < 64)
  for (int p0 = 0; p0 < nsolve; p0 += PB) {
    const int nb = min(PB, nsolve - p0);
    // acc(r, c) for rows tr + 16 q, panel columns tc + 16 w (w < 2).
    double acc[4][2];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const int64_t i = i0 + tr + 16 * q;
        const int c = tc + 16 * w;
        acc[q][w] = (i < m && c < nb) ? Bb[i * n + col(p0 + c)] : 0.0;
      }
    for (int k0 = 0; k0 < p0; k0 += PB) {
      for (int e = tid; e < PB * TB; e += NT) {
        const int r = e / PB, kk = e % PB;
        ws[kk][r] = i0 + r < m ? Bb[(i0 + r) * n + col(k0 + kk)] : 0.0;
      }
      for (int e = tid; e < PB * PB; e += NT) {
        const int c = e / PB, kk = e % PB;
        ls[kk][c] = c < nb ? Lat(p0 + c, k0 + kk) : 0.0;
      }
      __syncthreads();
#pragma unroll 8
      for (int kk = 0; kk < PB; ++kk) {
        double a[4], c[2];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = ws[kk][tr + 16 * q];
#pragma unroll
        for (int w = 0; w < 2; ++w) c[w] = ls[kk][tc + 16 * w];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int w = 0; w < 2; ++w) acc[q][w] = fma(-a[q], c[w], acc[q][w]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int w = 0; w < 2; ++w) pan[tr + 16 * q][tc + 16 * w] = acc[q][w];
    for (int e = tid; e < PB * PB; e += NT) {
      const int j = e / PB, k = e % PB;
      ls[j][k] = (j < nb && k <= j) ? Lat(p0 + j, p0 + k) : 0.0;
    }
    __syncthreads();
    if (tid < TB) {
      for (int j = 0; j < nb; ++j) {
        double v = pan[tid][j];
        for (int k = 0; k < j; ++k) v = fma(-pan[tid][k], ls[j][k], v);
        v /= ls[j][j];
        pan[tid][j] = v;
        lsum = fma(v, v, lsum);
      }
    }
    __syncthreads();
    for (int e = tid; e < TB * PB; e += NT) {
      const int r = e / PB, c = e % PB;
      if (i0 + r < m && c < nb) Bb[(i0 + r) * n + col(p0 + c)] = pan[r][c];
    }
    __syncthreads();
  }
  if (tid < TB && i0 + tid < m) lev[(int64_t)b * m + i0 + tid] = lsum;
}

// Diagonal-pivoted Cholesky of G_b (lower triangle of a row-major n x n
// matrix, n <= 1024; overwritten by trailing Schur complements). Step k takes
// the unpivoted index p of largest residual diagonal d_p (ties to the smaller
// index), stops when sqrt(d_p) < tol sqrt(d_first) or d_p <= 0 or k = kmax,
// else L(p, k) = sqrt(d_p) and L(i, k) = (G'(i, p) - sum over the current
// panel's earlier columns of L(i, l) L(p, l)) / L(p, k) for the other unpivoted i
// (0 for pivoted ones), d_i -= L(i, k)^2. G' is G less the finished panels,
// applied to its lower triangle after each panel. L is stored column-major
// (L[k * n + i]), perm[k] = p, rank[b] = the number of pivots.
constexpr int PN = 512, PR = 2;   // threads, rows per thread (n <= PN * PR)
// Panel columns held in LDS: at most 16, and at most 60 KB of them.
__host__ __device__ inline int panel_width(int n) { return n <= 480 ? 16 : 7680 / n; }
__global__ void __launch_bounds__(PN) k_pchol(double* __restrict__ G, int n, int kmax, double tol,
                                              double* __restrict__ Lc, int* __restrict__ perm,
                                              int* __restrict__ rank, int* __restrict__ status) {
  extern __shared__ double colbuf[];   // panel columns: colbuf[l * n + i]
  __shared__ double redv[2][PN / 64];
  __shared__ int redi[2][PN / 64];
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pb = panel_width(n);
  double* A = G + (int64_t)b * n * n;
  double* L = Lc + (int64_t)b * n * n;
  int* pv = perm + (int64_t)b * n;
  double d[PR];
  bool done[PR];
#pragma unroll
  for (int q = 0; q < PR; ++q) {
    const int i = tid + q * PN;
    done[q] = i >= n;
    d[q] = done[q] ? 0.0 : A[(int64_t)i * n + i];
  }
  double d0 = 0.0;
  int r = 0;
  bool stop = false;
  for (int k0 = 0; k0 < kmax && !stop; k0 += pb) {
    int j = 0;
    for (; j < pb && k0 + j < kmax; ++j) {
      const int k = k0 + j;
      double bv = -1.0;
      int bi = INT_MAX;
#pragma unroll
      for (int q = 0; q < PR; ++q) {
        const int i = tid + q * PN;
        if (!done[q] && (d[q] > bv || (d[q] == bv && i < bi))) {
          bv = d[q];
          bi = i;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        redv[k & 1][wave] = bv;
        redi[k & 1][wave] = bi;
      }
      __syncthreads();   // also publishes the previous step's panel column
      bv = redv[k & 1][0];
      bi = redi[k & 1][0];
      for (int w = 1; w < PN / 64; ++w) {
        const double ov = redv[k & 1][w];
        const int oi = redi[k & 1][w];
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (k == 0) d0 = bv;
      if (bi == INT_MAX || !(bv > 0.0) || sqrt(bv) < tol * sqrt(d0)) {
        stop = true;
        break;
      }
      const int p = bi;
      const double lkk = sqrt(bv);
      if (tid == 0) pv[k] = p;
#pragma unroll
      for (int q = 0; q < PR; ++q) {
        const int i = tid + q * PN;
        if (i >= n) continue;
        double lik = 0.0;
        if (i == p) {
          lik = lkk;
          done[q] = true;
        } else if (!done[q]) {
          double g = i >= p ? A[(int64_t)i * n + p] : A[(int64_t)p * n + i];
          for (int l = 0; l < j; ++l) g = fma(-colbuf[l * n + i], colbuf[l * n + p], g);
          lik = g / lkk;
          d[q] = fma(-lik, lik, d[q]);
        }
        colbuf[j * n + i] = lik;
        L[(int64_t)k * n + i] = lik;
      }
      r = k + 1;
    }
    __syncthreads();   // the panel's j columns are complete
    if (stop || j == 0 || k0 + j >= kmax) break;   // nothing left to update for
    // Lower-triangle update A(i, c) -= sum_l L(i, l) L(c, l) over this panel, 64 x 64 tiles.
    const int tiles = (n + TB - 1) / TB;
    const int tr = tid & 15, tc = tid >> 4;   // rows tr + 16 q (q < 4), columns tc + 32 w (w < 2)
    for (int ti = 0; ti < tiles; ++ti)
      for (int tj = 0; tj <= ti; ++tj) {
        double acc[4][2] = {};
        for (int l = 0; l < j; ++l) {
          double a[4], c[2];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = ti * TB + tr + 16 * q;
            a[q] = i < n ? colbuf[l * n + i] : 0.0;
          }
#pragma unroll
          for (int w = 0; w < 2; ++w) {
            const int c0 = tj * TB + tc + 32 * w;
            c[w] = c0 < n ? colbuf[l * n + c0] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int w = 0; w < 2; ++w) acc[q][w] = fma(a[q], c[w], acc[q][w]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int w = 0; w < 2; ++w) {
            const int i = ti * TB + tr + 16 * q, c0 = tj * TB + tc + 32 * w;
            if (i < n && c0 <= i) A[(int64_t)i * n + c0] -= acc[q][w];
          }
      }
    __syncthreads();   // updates visible before the next panel reads G'
  }
  if (tid == 0) {
    rank[b] = r;
    status[b] = d0 > 0.0 ? 0 : 1;
  }
}

// t_i = ln(max(l_i, 1e-12) m / max(sum l, 1e-300)); one workgroup per block.
__global__ void __launch_bounds__(NT) k_targets(const double* __restrict__ lev, int64_t m, float* __restrict__ target) {
  __shared__ double red[NT];
  const int b = blockIdx.x, tid = threadIdx.x;
  const double* l = lev + (int64_t)b * m;
  double s = 0.0;
  for (int64_t i = tid; i < m; i += NT) s += l[i];
  red[tid] = s;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  const double tot = fmax(red[0], 1e-300);
  for (int64_t i = tid; i < m; i += NT) target[(int64_t)b * m + i] = (float)log(fmax(l[i], 1e-12) * (double)m / tot);
}

}  // namespace

ffc_status launch_ridge_leverage(double* B, int64_t m, int n, int count, double* G, double eps, double* lev,
                                 float* target, int* status, hipStream_t st) {
  if (count <= 0 || m <= 0 || n <= 0) return FFC_OK;
  const int tiles = (n + TB - 1) / TB;
  const int tri = tiles * (tiles + 1) / 2;
  hipLaunchKernelGGL(k_gram_rm, dim3((unsigned)((int64_t)count * tri)), dim3(NT), 0, st, B, m, n, tiles, tri, G);
  FFC_LAUNCH_CHECK("k_gram_rm");
  hipLaunchKernelGGL(k_chol, dim3(count), dim3(NT), 0, st, G, n, eps * eps, status);
  FFC_LAUNCH_CHECK("k_chol");
  const int row_tiles = (int)((m + TB - 1) / TB);
  hipLaunchKernelGGL(k_lev<false>, dim3((unsigned)((int64_t)count * row_tiles)), dim3(NT), 0, st, B, m, n, row_tiles,
                     G, status, lev, nullptr, nullptr);
  FFC_LAUNCH_CHECK("k_lev");
  if (target) {
    hipLaunchKernelGGL(k_targets, dim3(count), dim3(NT), 0, st, lev, m, target);
    FFC_LAUNCH_CHECK("k_targets");
  }
  return FFC_OK;
}

ffc_status launch_pivoted_leverage(double* B, int64_t m, int n, int count, double* G, double* Lc, int* perm,
                                   int* rank, double eps, double* lev, float* target, int* status, hipStream_t st) {
  if (count <= 0 || m <= 0 || n <= 0) return FFC_OK;
  if (n > PN * PR) {
    set_error("pivoted leverage: at most 1024 columns per block");
    return FFC_ERR_INVALID_ARG;
  }
  const int tiles = (n + TB - 1) / TB;
  const int tri = tiles * (tiles + 1) / 2;
  hipLaunchKernelGGL(k_gram_rm, dim3((unsigned)((int64_t)count * tri)), dim3(NT), 0, st, B, m, n, tiles, tri, G);
  FFC_LAUNCH_CHECK("k_gram_rm");
  const int pb = panel_width(n);
  const int kmax = (int)std::min<int64_t>(m, n);
  hipLaunchKernelGGL(k_pchol, dim3(count), dim3(PN), (size_t)pb * n * sizeof(double), st, G, n, kmax, eps, Lc, perm,
                     rank, status);
  FFC_LAUNCH_CHECK("k_pchol");
  const int row_tiles = (int)((m + TB - 1) / TB);
  hipLaunchKernelGGL(k_lev<true>, dim3((unsigned)((int64_t)count * row_tiles)), dim3(NT), 0, st, B, m, n, row_tiles,
                     Lc, status, lev, perm, rank);
  FFC_LAUNCH_CHECK("k_lev");
  if (target) {
    hipLaunchKernelGGL(k_targets, dim3(count), dim3(NT), 0, st, lev, m, target);
    FFC_LAUNCH_CHECK("k_targets");
  }
  return FFC_OK;
}

}  // namespace ffc
