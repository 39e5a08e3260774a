// Kernel-function tiles: sampled blocks K', far/near-field evaluation (the
// sibling cover, and the treecode with separation of Section 2 together with
// its per-node separation bitmaps) and the direct sum. Kernel values and the
// tile sums live in tile_sums.h, shared with the FMM-style kernels (fmm.hip).
//
// Every stage that evaluates the kernel shares one tile engine: a 256-thread
// workgroup computes a 64 x 64 tile of squared distances (Gaussian, Laplace)
// or inner products (polynomial) between a row set and a column set of
// points. Coordinates are staged through LDS in chunks of 32 dimensions,
// transposed so that each thread reads 4 row values and 4 column values per
// dimension and owns a 4 x 4 block of the tile. Squared distances are formed
// from explicit coordinate differences, so they carry no cancellation.
//
// Epilogues:
//   * sampled block K'_{ij} = K(y_rows[i], x_cols[j]) stored column major
//     (Section 2.2, the s x n matrix whose ID is taken);
//   * kernel sums u_i = sum_j K(y_i, x_j) q_j (Section 1, eq. e:sum; eq. e:id
//     with the skeleton points and equivalent charges), reduced across the
//     16 threads sharing a row in a fixed order, so results are deterministic.
// Precision: FP64 tiles in double; FP32 tiles (and the direct sum of the
// Laplace kernel in the mixed mode) in float with the Laplace power taken in
// double; the mixed mode of the sampled blocks and the evaluation runs on
// matrix cores for every kernel function (gram_mfma.hip).
#include "ffc_internal.h"
#include "tile_engine.h"
#include "tile_sums.h"

namespace ffc {
namespace {

using namespace tile;

// ---------------------------------------------------------------------------
// Sampled blocks for all nodes of a level.
// ---------------------------------------------------------------------------
template <typename T, int KF>
__global__ void __launch_bounds__(NT) k_level_kblock(const double* __restrict__ Xt, int d, KParams kp, int first,
                                                     int tiles_m, int tiles_n, const int32_t* __restrict__ rows,
                                                     const int32_t* __restrict__ nrows, int s_cap,
                                                     const int32_t* __restrict__ cols,
                                                     const int32_t* __restrict__ ncols, int n_cap,
                                                     const unsigned char* __restrict__ mask,
                                                     double* __restrict__ A, unsigned int* flag) {
  __shared__ TileSmem<T> sm;
  const int tiles = tiles_m * tiles_n;
  const int ln = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  const int node = first + ln;
  if (mask && !mask[node]) return;
  const int s = nrows[node], n = ncols[node];
  const int r0 = (tile % tiles_m) * BM, c0 = (tile / tiles_m) * BN;
  if (r0 >= s || c0 >= n) return;
  const IdxMap rmap{rows + (int64_t)node * s_cap + r0, 0};
  const IdxMap cmap{cols + (int64_t)node * n_cap + c0, 0};
  T acc[4][4];
  tile_accumulate<T, KF == FFC_POLYNOMIAL>(Xt, rmap, s - r0, Xt, cmap, n - c0, d, sm, acc);
  double* out = A + (int64_t)ln * s_cap * n_cap;
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  bool bad = false;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = c0 + tc + 16 * j;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + tr + 16 * i;
      if (r < s && c < n) {
        const double v = kfun<KF>(acc[i][j], kp);
        bad |= !isfinite(v);
        out[(int64_t)c * s_cap + r] = v;
      }
    }
  }
  if (bad) flag_nonfinite(flag);
}

// Standalone sampled block: rows/cols are explicit lists of tree positions.
template <typename T, int KF>
__global__ void __launch_bounds__(NT) k_sampled_block(const double* __restrict__ Xt, int d, KParams kp,
                                                      const int32_t* __restrict__ rows, int s,
                                                      const int32_t* __restrict__ cols, int n, int tiles_m,
                                                      double* __restrict__ out, unsigned int* flag) {
  __shared__ TileSmem<T> sm;
  const int r0 = (blockIdx.x % tiles_m) * BM, c0 = (blockIdx.x / tiles_m) * BN;
  T acc[4][4];
  tile_accumulate<T, KF == FFC_POLYNOMIAL>(Xt, IdxMap{rows + r0, 0}, s - r0, Xt, IdxMap{cols + c0, 0}, n - c0, d, sm, acc);
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  bool bad = false;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + tr + 16 * i, c = c0 + tc + 16 * j;
      if (r < s && c < n) {
        const double v = kfun<KF>(acc[i][j], kp);
        bad |= !isfinite(v);
        out[(int64_t)c * s + r] = v;
      }
    }
  if (bad) flag_nonfinite(flag);
}


// Far field (sibling cover) + near field (own leaf) for a tile of targets.
template <typename T, int KF, int DM>
__global__ void __launch_bounds__(NT) k_evaluate(const double* __restrict__ Xt, int d, KParams kp, int depth,
                                                 const int32_t* __restrict__ tile_leaf,
                                                 const int32_t* __restrict__ tile_start,
                                                 const int32_t* __restrict__ nb, const int32_t* __restrict__ ne,
                                                 const double* __restrict__ q_tree,
                                                 const int32_t* __restrict__ rank, const int32_t* __restrict__ skel,
                                                 int r_cap, const double* __restrict__ qt,
                                                 const int32_t* __restrict__ perm, double* __restrict__ u,
                                                 double* __restrict__ u_far, unsigned int* flag) {
  __shared__ EvalSmem<T, DM> sm;
  __shared__ double red[16 * BM];
  __shared__ double far_sum[BM], near_sum[BM];
  const int leaf = tile_leaf[blockIdx.x];
  const int start = tile_start[blockIdx.x];
  const int nrows = min(BM, ne[leaf] - start);
  const IdxMap rmap{nullptr, start};
  if constexpr (DM > 0) stage_rows<T, DM>(Xt, rmap, nrows, d, sm);
  bool bad = false;
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  // Far field: one cover node per level (the sibling of each ancestor).
  int a = leaf;
  for (int lev = depth; lev >= 1; --lev) {
    const int sib = (a & 1) ? a + 1 : a - 1;
    const int r = rank[sib];
    if (r > 0)
      sum_sources<T, KF, DM>(Xt, rmap, nrows, Xt, IdxMap{skel + (int64_t)sib * r_cap, 0}, r,
                          qt + (int64_t)sib * r_cap, d, kp, sm, part, bad);
    a = (a - 1) >> 1;
  }
  reduce_rows(part, red, far_sum);
  double npart[4] = {0.0, 0.0, 0.0, 0.0};
  const int lb = nb[leaf];
  sum_sources<T, KF, DM>(Xt, rmap, nrows, Xt, IdxMap{nullptr, lb}, ne[leaf] - lb, q_tree + lb, d, kp, sm, npart,
                      bad);
  reduce_rows(npart, red, near_sum);
  if (threadIdx.x < nrows) {
    const int pos = start + threadIdx.x;
    const int ci = perm[pos];
    const double f = far_sum[threadIdx.x];
    u[ci] = f + near_sum[threadIdx.x];
    if (u_far) u_far[ci] = f;
  }
  if (bad) flag_nonfinite(flag);
}

// ---------------------------------------------------------------------------
// Separation (Section 2, eq. e:separated, with the source ball of Section 4.1):
// tree position p is separated from node a when it lies outside a and
// |x_p - c_a|^2 >= (xi rho_a)^2. One 64 x 64 tile covers 64 consecutive
// positions (one bitmap word) against 64 nodes; the squared distances come
// from the tile engine in FP64 and each wavefront packs its predicates with
// ballots: lane 16 w' + tr of a wavefront holds row tr of column 4 w + w', so
// the 16 bits of column tc for rows tr + 16 i sit at bits 16 (tc % 4) of the
// ballot of (i, j).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) k_sep_bitmap(const double* __restrict__ Xt, int64_t N, int d,
                                                   const double* __restrict__ centroid,
                                                   const double* __restrict__ radius, const int32_t* __restrict__ nb,
                                                   const int32_t* __restrict__ ne, int num_nodes, double xi,
                                                   int words, int tiles_n, uint64_t* __restrict__ bits) {
  __shared__ TileSmem<double> sm;
  const int64_t r0 = (int64_t)(blockIdx.x / tiles_n) * BM;
  const int c0 = (blockIdx.x % tiles_n) * BN;
  double acc[4][4];
  tile_accumulate<double, false>(Xt, IdxMap{nullptr, r0}, (int)min<int64_t>(BM, N - r0), centroid,
                                 IdxMap{nullptr, c0}, num_nodes - c0, d, sm, acc);
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  const int sub = tc & 3;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = c0 + tc + 16 * j;
    const bool col = c < num_nodes;
    const double thr = col ? xi * radius[c] : 0.0;
    const double thr2 = thr * thr;
    const int b = col ? nb[c] : 0, e = col ? ne[c] : 0;
    uint64_t word = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t p = r0 + tr + 16 * i;
      const bool sep = col && p < N && (p < b || p >= e) && acc[i][j] >= thr2;
      const uint64_t bal = __ballot(sep);
      word |= ((bal >> (16 * sub)) & 0xFFFFull) << (16 * i);
    }
    if (col && tr == 0) bits[(int64_t)c * words + (r0 >> 6)] = word;
  }
}

// Exclusive prefix of the set-bit counts over each node's words:
// pre[a * (words + 1) + w] = bits set in words 0..w-1 (w = words: all of them).
constexpr int kPreThreads = 256;
__global__ void __launch_bounds__(kPreThreads) k_sep_prefix(const uint64_t* __restrict__ bits, int words,
                                                            int32_t* __restrict__ pre) {
  __shared__ int wsum[kPreThreads / 64];
  const int a = blockIdx.x, tid = threadIdx.x;
  const uint64_t* bw = bits + (int64_t)a * words;
  int32_t* out = pre + (int64_t)a * (words + 1);
  const int per = (words + kPreThreads - 1) / kPreThreads;
  const int w0 = min(words, tid * per), w1 = min(words, w0 + per);
  int cnt = 0;
  for (int w = w0; w < w1; ++w) cnt += __popcll((unsigned long long)bw[w]);
  const int lane = tid & 63, wid = tid >> 6;
  int incl = cnt;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int pos = incl - cnt;
  for (int w = 0; w < wid; ++w) pos += wsum[w];
  for (int w = w0; w < w1; ++w) {
    out[w] = pos;
    pos += __popcll((unsigned long long)bw[w]);
  }
  if (tid == kPreThreads - 1) out[words] = pos;
}

// Treecode evaluation with separation for a tile of 64 targets of one leaf.
// The workgroup walks the tree depth first from the root's children with a
// stack in LDS. Per node and target row the choice is: apply the node's
// skeleton (the row reaches the node, the node does not contain it and the
// separation bit is set), pass the row on (children, or a direct sum at a
// leaf), or nothing (the row was served higher up). Bit l of arrive[row] says
// whether the row reaches the node of level l on the current path; a node of
// level l sets bit l + 1 for its children, and nodes visited before its second
// child are all deeper, so that bit still holds when the second child is popped.
template <typename T, int KF, int DM>
__global__ void __launch_bounds__(NT) k_treecode(const double* __restrict__ Xt, int d, KParams kp, int depth,
                                                 const int32_t* __restrict__ tile_leaf,
                                                 const int32_t* __restrict__ tile_start,
                                                 const int32_t* __restrict__ nb, const int32_t* __restrict__ ne,
                                                 const double* __restrict__ q_tree,
                                                 const int32_t* __restrict__ rank, const int32_t* __restrict__ skel,
                                                 int r_cap, const double* __restrict__ qt,
                                                 const uint64_t* __restrict__ sep_bits, int words,
                                                 const int32_t* __restrict__ perm, double* __restrict__ u,
                                                 double* __restrict__ u_far, unsigned int* flag) {
  __shared__ EvalSmem<T, DM> sm;
  __shared__ double red[16 * BM];
  __shared__ double far_sum[BM], near_sum[BM];
  __shared__ int stack[64];
  __shared__ uint32_t arrive[BM];
  __shared__ unsigned char take[BM];   // 1: skeleton sum, 2: passed on / direct sum, 0: neither
  const int leaf = tile_leaf[blockIdx.x];
  const int start = tile_start[blockIdx.x];
  const int nrows = min(BM, ne[leaf] - start);
  const IdxMap rmap{nullptr, start};
  if constexpr (DM > 0) stage_rows<T, DM>(Xt, rmap, nrows, d, sm);
  const int tid = threadIdx.x, tr = tid & 15;
  bool bad = false;
  double fpart[4] = {0.0, 0.0, 0.0, 0.0}, npart[4] = {0.0, 0.0, 0.0, 0.0};
  if (tid < BM) arrive[tid] = tid < nrows ? 2u : 0u;   // every row reaches level 1
  if (tid == 0) {
    stack[0] = 2;
    stack[1] = 1;
  }
  int sp = 2;   // the same in every thread
  __syncthreads();
  while (sp > 0) {
    const int a = stack[--sp];
    const int lev = 31 - __clz(a + 1);
    const bool is_leaf = lev == depth;
    const bool contains = ((leaf + 1) >> (depth - lev)) == a + 1;
    int k = 0;
    if (tid < BM) {
      if ((arrive[tid] >> lev) & 1u) {
        bool sep = false;
        if (!contains) {
          const int64_t p = start + tid;
          sep = (sep_bits[(int64_t)a * words + (p >> 6)] >> (p & 63)) & 1ull;
        }
        k = sep ? 1 : 2;
      }
      take[tid] = (unsigned char)k;
      if (!is_leaf) arrive[tid] = (arrive[tid] & ~(2u << lev)) | (k == 2 ? (2u << lev) : 0u);
    }
    const int any_far = __syncthreads_or(k == 1);
    const int any_rest = __syncthreads_or(k == 2);
    if (any_far && rank[a] > 0) {
      double tmp[4] = {0.0, 0.0, 0.0, 0.0};
      sum_sources<T, KF, DM>(Xt, rmap, nrows, Xt, IdxMap{skel + (int64_t)a * r_cap, 0}, rank[a],
                          qt + (int64_t)a * r_cap, d, kp, sm, tmp, bad);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (take[tr + 16 * i] == 1) fpart[i] += tmp[i];
    }
    if (any_rest) {
      if (is_leaf) {
        const int lb = nb[a];
        double tmp[4] = {0.0, 0.0, 0.0, 0.0};
        sum_sources<T, KF, DM>(Xt, rmap, nrows, Xt, IdxMap{nullptr, lb}, ne[a] - lb, q_tree + lb, d, kp, sm, tmp,
                            bad);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (take[tr + 16 * i] == 2) npart[i] += tmp[i];
      } else {
        if (tid == 0) {   // right child below the left one: the left subtree is walked first
          stack[sp] = 2 * a + 2;
          stack[sp + 1] = 2 * a + 1;
        }
        sp += 2;
      }
    }
    __syncthreads();
  }
  reduce_rows(fpart, red, far_sum);
  reduce_rows(npart, red, near_sum);
  if (threadIdx.x < nrows) {
    const int pos = start + threadIdx.x;
    const int ci = perm[pos];
    const double f = far_sum[threadIdx.x];
    u[ci] = f + near_sum[threadIdx.x];
    if (u_far) u_far[ci] = f;
  }
  if (bad) flag_nonfinite(flag);
}

// Direct sum over all sources for a tile of 64 targets.
template <typename T, int KF, int DM>
__global__ void __launch_bounds__(NT) k_direct(const double* __restrict__ Y, int64_t m, const double* __restrict__ X,
                                               int64_t n, int d, KParams kp, const double* __restrict__ q,
                                               double* __restrict__ u, unsigned int* flag) {
  __shared__ EvalSmem<T, DM> sm;
  __shared__ double red[16 * BM];
  __shared__ double rowsum[BM];
  const int64_t r0 = (int64_t)blockIdx.x * BM;
  const int nrows = (int)min<int64_t>(BM, m - r0);
  bool bad = false;
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  if constexpr (DM > 0) stage_rows<T, DM>(Y, IdxMap{nullptr, r0}, nrows, d, sm);
  sum_sources<T, KF, DM>(Y, IdxMap{nullptr, r0}, nrows, X, IdxMap{nullptr, 0}, (int)n, q, d, kp, sm, part, bad);
  reduce_rows(part, red, rowsum);
  if (threadIdx.x < nrows) u[r0 + threadIdx.x] = rowsum[threadIdx.x];
  if (bad) flag_nonfinite(flag);
}

template <typename F>
ffc_status dispatch(int precision, const KParams& kp, F&& f) {
  return with_kind(kp, [&](auto kv) -> ffc_status {
    if (precision == FFC_FP64) return f(double(), kv);
    return f(float(), kv);
  });
}

}  // namespace

ffc_status launch_kblock_batch(const ffc_tree* t, const KParams& kp, int precision, const int32_t* rows,
                               const int32_t* nrows, int s_cap, const int32_t* cols, const int32_t* ncols, int n_cap,
                               int first, int count, const double* centroid, double* A, hipStream_t st,
                               const unsigned char* mask) {
  if (precision == FFC_MIXED_BF16X3)
    return launch_kblock_batch_mixed(t, kp, rows, nrows, s_cap, cols, ncols, n_cap, first, count, centroid, A, st,
                                     mask);
  const int tiles_m = (s_cap + BM - 1) / BM, tiles_n = (n_cap + BN - 1) / BN;
  const int64_t blocks = (int64_t)count * tiles_m * tiles_n;
  if (blocks == 0) return FFC_OK;
  return dispatch(precision, kp, [&](auto tv, auto kv) -> ffc_status {
    using T = decltype(tv);
    constexpr int KF = decltype(kv)::value;
    hipLaunchKernelGGL((k_level_kblock<T, KF>), dim3((unsigned)blocks), dim3(NT), 0, st, t->Xt.ptr, t->d, kp, first,
                       tiles_m, tiles_n, rows, nrows, s_cap, cols, ncols, n_cap, mask, A, device_flag());
    FFC_LAUNCH_CHECK("k_level_kblock");
    return FFC_OK;
  });
}

ffc_status launch_level_kblock(const ffc_tree* t, const ffc_skel* sk, const KParams& kp, int precision, int first,
                               int count, double* A, hipStream_t st, const unsigned char* mask) {
  return launch_kblock_batch(t, kp, precision, sk->rows.ptr, sk->nrows.ptr, sk->s_cap, sk->cols.ptr, sk->ncols.ptr,
                             sk->n_cap, first, count, t->centroid.ptr, A, st, mask);
}

// Gram matrices G_b = B_b^T B_b of column-major m x n blocks (B_b at B + b * m * n):
// column i of B_b is an m-dimensional point, so the inner-product tile engine applies.
__global__ void __launch_bounds__(NT) k_gram(const double* __restrict__ B, int m, int n, int tiles,
                                             double* __restrict__ G) {
  __shared__ TileSmem<double> sm;
  const int b = blockIdx.x / (tiles * tiles), tile = blockIdx.x % (tiles * tiles);
  const int r0 = (tile % tiles) * BM, c0 = (tile / tiles) * BN;
  const double* Bb = B + (int64_t)b * m * n;
  double acc[4][4];
  tile_accumulate<double, true>(Bb, IdxMap{nullptr, r0}, n - r0, Bb, IdxMap{nullptr, c0}, n - c0, m, sm, acc);
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  double* Gb = G + (int64_t)b * n * n;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + tr + 16 * i, c = c0 + tc + 16 * j;
      if (r < n && c < n) Gb[(int64_t)r * n + c] = acc[i][j];
    }
}

ffc_status launch_gram(const double* B, int m, int n, int count, double* G, hipStream_t st) {
  const int tiles = (n + BM - 1) / BM;
  const int64_t blocks = (int64_t)count * tiles * tiles;
  if (blocks == 0) return FFC_OK;
  hipLaunchKernelGGL(k_gram, dim3((unsigned)blocks), dim3(NT), 0, st, B, m, n, tiles, G);
  FFC_LAUNCH_CHECK("k_gram");
  return FFC_OK;
}

ffc_status launch_sampled_block(const ffc_tree* t, const KParams& kp, int precision, const int32_t* rows, int s,
                                const int32_t* cols, int n, double* out, hipStream_t st) {
  const int tiles_m = (s + BM - 1) / BM, tiles_n = (n + BN - 1) / BN;
  return dispatch(precision, kp, [&](auto tv, auto kv) -> ffc_status {
    using T = decltype(tv);
    constexpr int KF = decltype(kv)::value;
    hipLaunchKernelGGL((k_sampled_block<T, KF>), dim3((unsigned)(tiles_m * tiles_n)), dim3(NT), 0, st, t->Xt.ptr,
                       t->d, kp, rows, s, cols, n, tiles_m, out, device_flag());
    FFC_LAUNCH_CHECK("k_sampled_block");
    return FFC_OK;
  });
}

ffc_status launch_evaluate(const ffc_tree* t, const ffc_skel* sk, const KParams& kp, int precision, double* u,
                           double* u_far, hipStream_t st) {
  if (precision == FFC_MIXED_BF16X3) return launch_evaluate_mixed(t, sk, kp, u, u_far, st);
  return dispatch(precision, kp, [&](auto tv, auto kv) -> ffc_status {
    using T = decltype(tv);
    constexpr int KF = decltype(kv)::value;
    return with_dims(t->d, [&](auto dm) -> ffc_status {
      constexpr int DM = decltype(dm)::value;
      hipLaunchKernelGGL((k_evaluate<T, KF, DM>), dim3((unsigned)t->num_tiles), dim3(NT), 0, st, t->Xt.ptr, t->d, kp,
                         t->depth, t->tile_leaf.ptr, t->tile_start.ptr, t->begin.ptr, t->end.ptr, t->q_tree.ptr,
                         sk->rank.ptr, sk->skel.ptr, sk->r_cap, sk->qt.ptr, t->perm.ptr, u, u_far, device_flag());
      FFC_LAUNCH_CHECK("k_evaluate");
      return FFC_OK;
    });
  });
}

ffc_status launch_separation(const ffc_tree* t, ffc_skel* sk, double xi, hipStream_t st) {
  const int words = (int)((t->N + 63) / 64);
  const size_t nn = (size_t)t->num_nodes;
  if (sk->sep_words != words || sk->sep_bits.count != nn * words) {
    FFC_TRY(sk->sep_bits.alloc(nn * words));
    FFC_TRY(sk->sep_pre.alloc(nn * (words + 1)));
    sk->sep_words = words;
  }
  const int tiles_n = (t->num_nodes + BN - 1) / BN;
  const int64_t blocks = (int64_t)words * tiles_n;
  hipLaunchKernelGGL(k_sep_bitmap, dim3((unsigned)blocks), dim3(NT), 0, st, t->Xt.ptr, t->N, t->d, t->centroid.ptr,
                     t->radius.ptr, t->begin.ptr, t->end.ptr, t->num_nodes, xi, words, tiles_n, sk->sep_bits.ptr);
  FFC_LAUNCH_CHECK("k_sep_bitmap");
  hipLaunchKernelGGL(k_sep_prefix, dim3((unsigned)t->num_nodes), dim3(kPreThreads), 0, st, sk->sep_bits.ptr, words,
                     sk->sep_pre.ptr);
  FFC_LAUNCH_CHECK("k_sep_prefix");
  return FFC_OK;
}

ffc_status launch_treecode(const ffc_tree* t, const ffc_skel* sk, const KParams& kp, int precision, double* u,
                           double* u_far, hipStream_t st) {
  if (precision == FFC_MIXED_BF16X3) {
    set_error("a treecode (separation > 0) evaluates in FFC_FP64 or FFC_FP32");
    return FFC_ERR_INVALID_ARG;
  }
  if (!sk->sep_bits.ptr || sk->sep_words != (int)((t->N + 63) / 64) || t->depth > 30) {
    set_error("separation bitmaps are missing");
    return FFC_ERR_STATE;
  }
  return dispatch(precision, kp, [&](auto tv, auto kv) -> ffc_status {
    using T = decltype(tv);
    constexpr int KF = decltype(kv)::value;
    return with_dims(t->d, [&](auto dm) -> ffc_status {
      constexpr int DM = decltype(dm)::value;
      hipLaunchKernelGGL((k_treecode<T, KF, DM>), dim3((unsigned)t->num_tiles), dim3(NT), 0, st, t->Xt.ptr, t->d, kp,
                         t->depth, t->tile_leaf.ptr, t->tile_start.ptr, t->begin.ptr, t->end.ptr, t->q_tree.ptr,
                         sk->rank.ptr, sk->skel.ptr, sk->r_cap, sk->qt.ptr, sk->sep_bits.ptr, sk->sep_words,
                         t->perm.ptr, u, u_far, device_flag());
      FFC_LAUNCH_CHECK("k_treecode");
      return FFC_OK;
    });
  });
}

ffc_status launch_direct_sum(const double* Y, int64_t m, const double* X, int64_t n, int d, const KParams& kp,
                             int precision, const double* q, double* u, hipStream_t st) {
  if (m == 0) return FFC_OK;
  if (precision == FFC_MIXED_BF16X3 && kp.kind != FFC_LAPLACE) return launch_direct_mixed(Y, m, X, n, d, kp, q, u, st);
  return dispatch(precision, kp, [&](auto tv, auto kv) -> ffc_status {
    using T = decltype(tv);
    constexpr int KF = decltype(kv)::value;
    return with_dims(d, [&](auto dm) -> ffc_status {
      constexpr int DM = decltype(dm)::value;
      hipLaunchKernelGGL((k_direct<T, KF, DM>), dim3((unsigned)((m + BM - 1) / BM)), dim3(NT), 0, st, Y, m, X, n, d,
                         kp, q, u, device_flag());
      FFC_LAUNCH_CHECK("k_direct");
      return FFC_OK;
    });
  });
}

}  // namespace ffc
