// Batched interpolative decomposition by column-pivoted Householder QR.
//
// For each block A (s x n, column major) the kernel computes A Pi = Q [R11
// R12; 0 R22] with Businger-Golub pivoting and stops at the first step k
// whose pivot column norm rho_k falls below tol * rho_0 or is zero (or at
// min(s, n, max_rank)); then T = R11^{-1} R12 by back substitution and the
// interpolation matrix P = [I T] Pi^T, whose columns on the skeleton are the
// identity (Section 2.1.3, Definition of the ID; Theorem thm_compute_id;
// Appendix 6.1). Q is never formed.
//
// One workgroup factors one block; every block of a batch runs at once. Each
// step makes one pass over the trailing columns: a wavefront takes a column,
// forms w = v^T a_j, applies the reflector and recomputes the column's
// trailing norm exactly from the updated values (no downdating), so the
// pivot order is that of exact norms. Pivot ties go to the smaller original
// column index.
#include <climits>

#include "ffc_internal.h"
#include "lane_ops.h"

namespace ffc {
namespace {

constexpr int NT = 1024;
constexpr int NW = NT / 64;
// Columns a wavefront updates at once: CPW * MAXR doubles stay in registers.
template <int MAXR>
struct ColsPerWave { static constexpr int value = MAXR <= 8 ? 4 : 2; };

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline bool better(double v, int pv, double bv, int bp) {
  return v > bv || (v == bv && pv < bp);
}

struct Arg {
  double v;
  int orig;
  int pos;
};

__device__ inline Arg wave_argmax(Arg a) {
  for (int off = 32; off > 0; off >>= 1) {
    Arg o;
    o.v = __shfl_xor(a.v, off, 64);
    o.orig = __shfl_xor(a.orig, off, 64);
    o.pos = __shfl_xor(a.pos, off, 64);
    if (better(o.v, o.orig, a.v, a.orig)) a = o;
  }
  return a;
}

__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NW; ++i) s += red[i];
  return s;
}

// Apply the reflector (v, beta) to CPW columns starting at j0 (a wavefront's
// share) and recompute their norms over rows k+1..s-1. Rows per lane are
// cached in registers when s - k <= 64 * MAXR.
template <int MAXR, int CPW>
__device__ inline void update_columns(double* __restrict__ A, int lda, int s, int k, int j0, int ncol,
                                      const double* __restrict__ v, double beta, double* __restrict__ norms,
                                      int lane) {
  double a[CPW][MAXR];
  double dot[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) dot[c] = 0.0;
#pragma unroll
  for (int m = 0; m < MAXR; ++m) {
    const int i = k + lane + 64 * m;
    const bool in = i < s;
    const double vi = in ? v[i] : 0.0;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      a[c][m] = (in && c < ncol) ? A[(int64_t)(j0 + c) * lda + i] : 0.0;
      dot[c] = fma(vi, a[c][m], dot[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) dot[c] = wave_sum(dot[c]) * beta;
  double nrm[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) nrm[c] = 0.0;
#pragma unroll
  for (int m = 0; m < MAXR; ++m) {
    const int i = k + lane + 64 * m;
    if (i < s) {
      const double vi = v[i];
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        if (c < ncol) {
          const double x = fma(-vi, dot[c], a[c][m]);
          A[(int64_t)(j0 + c) * lda + i] = x;
          if (i > k) nrm[c] = fma(x, x, nrm[c]);
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    nrm[c] = wave_sum(nrm[c]);
    if (lane == 0 && c < ncol) norms[j0 + c] = nrm[c];
  }
}

// Same without the register cache (any s): two passes over the column.
__device__ inline void update_columns_any(double* __restrict__ A, int lda, int s, int k, int j0, int ncol,
                                          const double* __restrict__ v, double beta, double* __restrict__ norms,
                                          int lane) {
  for (int c = 0; c < ncol; ++c) {
    double* cj = A + (int64_t)(j0 + c) * lda;
    double dot = 0.0;
    for (int i = k + lane; i < s; i += 64) dot = fma(v[i], cj[i], dot);
    dot = wave_sum(dot) * beta;
    double nrm = 0.0;
    for (int i = k + lane; i < s; i += 64) {
      const double x = fma(-v[i], dot, cj[i]);
      cj[i] = x;
      if (i > k) nrm = fma(x, x, nrm);
    }
    nrm = wave_sum(nrm);
    if (lane == 0) norms[j0 + c] = nrm;
  }
}

template <int MAXR>
__global__ void __launch_bounds__(NT) k_cpqr_id(IdBatch bt) {
  extern __shared__ double smem[];
  const int b = blockIdx.x;
  if (bt.mask && !bt.mask[b]) return;
  const int s = bt.s_arr ? bt.s_arr[b] : bt.s_uniform;
  const int n = bt.n_arr ? bt.n_arr[b] : bt.n_uniform;
  double* A = bt.A + (int64_t)b * bt.a_stride;
  const int lda = bt.lda;
  int32_t* piv_out = bt.piv + (int64_t)b * bt.piv_stride;
  double* norms = smem;                          // n_max
  double* v = norms + bt.n_max;                  // s_max
  double* red = v + bt.s_max;                    // NW
  Arg* wbest = reinterpret_cast<Arg*>(red + NW); // NW
  int* piv = reinterpret_cast<int*>(wbest + NW); // n_max
  __shared__ int s_r;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

  // Initial column norms.
  for (int j = w; j < n; j += NW) {
    const double* col = A + (int64_t)j * lda;
    double acc = 0.0;
    for (int i = lane; i < s; i += 64) acc = fma(col[i], col[i], acc);
    acc = wave_sum(acc);
    if (lane == 0) { norms[j] = acc; piv[j] = j; }
  }
  __syncthreads();

  const int kmax = min(min(s, n), bt.max_rank);
  double rho0 = 0.0;
  int k = 0;
  for (; k < kmax; ++k) {
    // Pivot: largest trailing norm, ties to the smaller original column.
    Arg best{-1.0, INT_MAX, -1};
    for (int j = k + tid; j < n; j += NT) {
      const Arg c{norms[j], piv[j], j};
      if (better(c.v, c.orig, best.v, best.orig)) best = c;
    }
    best = wave_argmax(best);
    if (lane == 0) wbest[w] = best;
    __syncthreads();
    best = wbest[0];
    for (int i = 1; i < NW; ++i)
      if (better(wbest[i].v, wbest[i].orig, best.v, best.orig)) best = wbest[i];
    const double rho = sqrt(best.v);
    if (k == 0) rho0 = rho;
    if (rho == 0.0 || rho < bt.tol * rho0) break;
    const int p = best.pos;
    __syncthreads();   // every thread has read wbest
    // Swap columns k and p.
    if (p != k) {
      double* ck = A + (int64_t)k * lda;
      double* cp = A + (int64_t)p * lda;
      for (int i = tid; i < s; i += NT) {
        const double t = ck[i];
        ck[i] = cp[i];
        cp[i] = t;
      }
      if (tid == 0) {
        const double tn = norms[k]; norms[k] = norms[p]; norms[p] = tn;
        const int tp = piv[k]; piv[k] = piv[p]; piv[p] = tp;
      }
    }
    __syncthreads();
    // Householder reflector for x = A(k:s, k): v = x - alpha e1, alpha = -sign(x0) rho.
    double* ck = A + (int64_t)k * lda;
    const double x0 = ck[k];
    const double alpha = x0 != 0.0 ? -copysign(rho, x0) : -rho;
    double part = 0.0;
    for (int i = k + tid; i < s; i += NT) {
      const double vi = i == k ? x0 - alpha : ck[i];
      v[i] = vi;
      part = fma(vi, vi, part);
    }
    const double vv = block_sum(part, red);
    const double beta = vv > 0.0 ? 2.0 / vv : 0.0;
    __syncthreads();
    for (int i = k + tid; i < s; i += NT) ck[i] = i == k ? alpha : 0.0;
    // Apply to the trailing columns; each wavefront takes CPW columns at a time.
    const int first = k + 1;
    constexpr int CPW = ColsPerWave<MAXR>::value;
    const bool cached = MAXR > 0 && (s - k) <= 64 * MAXR;
    for (int j0 = first + w * CPW; j0 < n; j0 += NW * CPW) {
      const int ncol = min(CPW, n - j0);
      if (cached) update_columns<(MAXR > 0 ? MAXR : 1), CPW>(A, lda, s, k, j0, ncol, v, beta, norms, lane);
      else update_columns_any(A, lda, s, k, j0, ncol, v, beta, norms, lane);
    }
    __syncthreads();
  }
  if (tid == 0) s_r = k;
  __syncthreads();
  const int r = s_r;
  for (int j = tid; j < n; j += NT) piv_out[j] = piv[j];
  if (tid == 0) bt.rank[b] = r;

  // T = R11^{-1} R12, one thread per column of R12, in place (column-major A).
  for (int c = r + tid; c < n; c += NT) {
    double* col = A + (int64_t)c * lda;
    for (int i = r - 1; i >= 0; --i) {
      double acc = col[i];
      for (int l = i + 1; l < r; ++l) acc = fma(-A[(int64_t)l * lda + i], col[l], acc);
      col[i] = acc / A[(int64_t)i * lda + i];
    }
  }
  __syncthreads();
  // P (r x n, row-major with leading dimension p_ld): P(:, piv[j]) = e_j for
  // j < r, P(:, piv[j]) = T(:, j - r) otherwise.
  double* P = bt.P + (int64_t)b * bt.p_stride;
  for (int e = tid; e < r * n; e += NT) {
    const int i = e / n, j = e % n;
    double val;
    if (j < r) val = (i == j) ? 1.0 : 0.0;
    else val = A[(int64_t)j * lda + i];
    P[(int64_t)i * bt.p_ld + piv[j]] = val;
  }
}

__global__ void k_skeleton_ids(int first, int n_cap, int r_cap, const int32_t* __restrict__ rank,
                               const int32_t* __restrict__ piv, const int32_t* __restrict__ cols,
                               int32_t* __restrict__ skel, const unsigned char* __restrict__ mask) {
  const int node = first + blockIdx.x;
  if (mask && !mask[node]) return;
  const int r = rank[node];
  for (int i = threadIdx.x; i < r; i += blockDim.x)
    skel[(int64_t)node * r_cap + i] = cols[(int64_t)node * n_cap + piv[(int64_t)node * n_cap + i]];
}

// q~ = P q_alpha; q_alpha = the node's own charges (leaf) or the children's
// equivalent charges, left then right (internal node). Workgroup (node, y)
// forms rows 16 y .. 16 y + 15; each of its wavefronts four of them at once
// (lanes stride the columns), reduced in a fixed order by DPP within rows of
// 16 lanes and then across the four rows.
__global__ void __launch_bounds__(256) k_upward(int first, int leaves, const int32_t* __restrict__ nb, int n_cap,
                                                int r_cap, const int32_t* __restrict__ rank,
                                                const int32_t* __restrict__ ncols, const double* __restrict__ P,
                                                const double* __restrict__ q_tree, double* __restrict__ qt) {
  const int node = first + blockIdx.x;
  const int r = rank[node], n = ncols[node];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const double* Pn = P + (int64_t)node * r_cap * n_cap;
  const int l = 2 * node + 1;
  const int rl = leaves ? 0 : rank[l];
  const double* ql = leaves ? q_tree + nb[node] : qt + (int64_t)l * r_cap;
  const double* qr = leaves ? nullptr : qt + (int64_t)(l + 1) * r_cap;
  for (int i0 = 16 * (int)blockIdx.y + 4 * w; i0 < min(r, 16 * (int)blockIdx.y + 16); i0 += 4 * nw) {
    const int nr = min(4, r - i0);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    // Four passes at a time with their loads issued first (rows past nr
    // read row i0), then the products in pass order, so each sum keeps its
    // order.
    int j = lane;
    for (; j + 192 < n; j += 256) {
      double qv[4], pv[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int jj = j + 64 * u;
        qv[u] = *((leaves || jj < rl) ? ql + jj : qr + (jj - rl));
#pragma unroll
        for (int t = 0; t < 4; ++t) pv[u][t] = Pn[(int64_t)(i0 + (t < nr ? t : 0)) * n_cap + jj];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (t < nr) acc[t] = fma(pv[u][t], qv[u], acc[t]);
    }
    for (; j < n; j += 64) {
      const double qj = (leaves || j < rl) ? ql[j] : qr[j - rl];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < nr) acc[t] = fma(Pn[(int64_t)(i0 + t) * n_cap + j], qj, acc[t]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double v = wave_sum_dpp(acc[t]);
      if (lane == 0 && t < nr) qt[(int64_t)node * r_cap + i0 + t] = v;
    }
  }
}

__global__ void k_charges_to_tree(const double* __restrict__ q, const int32_t* __restrict__ perm, int64_t N,
                                  double* __restrict__ q_tree) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N) q_tree[i] = q[perm[i]];
}

}  // namespace

ffc_status launch_interp_decomp(const IdBatch& bt, int batch, hipStream_t st) {
  if (batch <= 0) return FFC_OK;
  const size_t lds = (size_t)bt.n_max * sizeof(double) + (size_t)bt.s_max * sizeof(double) + NW * sizeof(double) +
                     NW * sizeof(Arg) + (size_t)bt.n_max * sizeof(int);
  if (lds > 150 * 1024) {
    set_error("interpolative decomposition: block too large for LDS (s + n too big)");
    return FFC_ERR_INVALID_ARG;
  }
  auto launch = [&](auto kern) -> ffc_status {
    if (lds > 64 * 1024)
      FFC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(batch), dim3(NT), lds, st, bt);
    return FFC_OK;
  };
  if (bt.s_max <= 64 * 8) FFC_TRY(launch(k_cpqr_id<8>));
  else if (bt.s_max <= 64 * 16) FFC_TRY(launch(k_cpqr_id<16>));
  else FFC_TRY(launch(k_cpqr_id<0>));
  FFC_LAUNCH_CHECK("k_cpqr_id");
  return FFC_OK;
}

ffc_status launch_skeleton_ids(ffc_skel* sk, int first, int count, hipStream_t st, const unsigned char* mask) {
  hipLaunchKernelGGL(k_skeleton_ids, dim3(count), dim3(256), 0, st, first, sk->n_cap, sk->r_cap, sk->rank.ptr,
                     sk->piv.ptr, sk->cols.ptr, sk->skel.ptr, mask);
  FFC_LAUNCH_CHECK("k_skeleton_ids");
  return FFC_OK;
}

ffc_status launch_upward(const ffc_tree* t, ffc_skel* sk, int first, int count, bool leaves, hipStream_t st) {
  hipLaunchKernelGGL(k_upward, dim3(count, (sk->r_cap + 15) / 16), dim3(256), 0, st, first, leaves ? 1 : 0,
                     t->begin.ptr, sk->n_cap,
                     sk->r_cap, sk->rank.ptr, sk->ncols.ptr, sk->P.ptr, t->q_tree.ptr, sk->qt.ptr);
  FFC_LAUNCH_CHECK("k_upward");
  return FFC_OK;
}

ffc_status launch_charges_to_tree(ffc_tree* t, const double* q, hipStream_t st) {
  hipLaunchKernelGGL(k_charges_to_tree, dim3((unsigned)((t->N + 255) / 256)), dim3(256), 0, st, q, t->perm.ptr, t->N,
                     t->q_tree.ptr);
  FFC_LAUNCH_CHECK("k_charges_to_tree");
  return FFC_OK;
}

}  // namespace ffc
