// Ball-tree construction on the GPU.
//
// The paper groups points hierarchically with a space-partitioning tree
// (Section 2) and leaves its construction open. This tree is perfect (all
// leaves at one depth); a node is split at the median of the projections of
// its points onto (p2 - p1), p1 the point farthest from the node centroid, p2
// the point farthest from p1, with ties broken by the smaller caller index.
//
// Every level is processed for all of its nodes at once:
//   1. per-chunk partial sums of coordinates  -> centroid (fixed-order reduce)
//   2. per-chunk farthest point from centroid -> p1 and the node radius
//   3. per-chunk farthest point from p1       -> p2
//   4. sort keys (projection, caller index) into one padded segment per node
//   5. segmented bitonic sort (global passes for long strides, LDS otherwise)
//   6. write the sorted caller indices back as the node's part of perm.
// All reductions run in a fixed order, so the tree is deterministic.
#include <climits>

#include "ffc_internal.h"

namespace ffc {
namespace {

constexpr int kChunk = 1024;     // points per partial-reduction block
constexpr int kThreads = 256;
constexpr int kSortTile = 2048;  // elements per LDS bitonic tile

struct BestPt {
  double val;
  int idx;   // caller index
  int pos;   // tree position
};

struct SortKey {
  unsigned long long key;
  int idx;
  int pad;
};

__device__ inline bool better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

__device__ inline bool key_less(const SortKey& a, const SortKey& b) {
  return a.key < b.key || (a.key == b.key && a.idx < b.idx);
}

__device__ inline unsigned long long orderable(double v) {
  v = v + 0.0;  // -0 -> +0
  unsigned long long u = __double_as_longlong(v);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void k_iota(int32_t* perm, int64_t N) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N) perm[i] = (int32_t)i;
}

// Partial coordinate sums of one chunk of a node.
__global__ void k_centroid_partial(const double* __restrict__ X, const int32_t* __restrict__ perm, int d,
                                   const int32_t* __restrict__ ch_begin, const int32_t* __restrict__ ch_end,
                                   double* __restrict__ partial) {
  __shared__ double red[kThreads];
  const int ch = blockIdx.x;
  const int b = ch_begin[ch], e = ch_end[ch];
  const int lane_k = threadIdx.x & 63, pl = threadIdx.x >> 6;
  for (int k0 = 0; k0 < d; k0 += 64) {
    const int k = k0 + lane_k;
    double acc = 0.0;
    if (k < d)
      for (int i = b + pl; i < e; i += 4) acc += X[(int64_t)perm[i] * d + k];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (pl == 0 && k < d)
      partial[(int64_t)ch * d + k] = ((red[lane_k] + red[64 + lane_k]) + red[128 + lane_k]) + red[192 + lane_k];
    __syncthreads();
  }
}

// centroid[node] = (sum of the node's chunk partials, in chunk order) / n.
__global__ void k_centroid_final(const double* __restrict__ partial, int d, int first,
                                 const int32_t* __restrict__ node_ch_first, const int32_t* __restrict__ node_ch_count,
                                 const int32_t* __restrict__ nb, const int32_t* __restrict__ ne,
                                 double* __restrict__ centroid) {
  const int ln = blockIdx.x, node = first + ln;
  const int n = ne[node] - nb[node];
  const int c0 = node_ch_first[ln], cc = node_ch_count[ln];
  for (int k = threadIdx.x; k < d; k += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < cc; ++c) s += partial[(int64_t)(c0 + c) * d + k];
    centroid[(int64_t)node * d + k] = n > 0 ? s / (double)n : 0.0;
  }
}

// Farthest point of a chunk from a per-node reference point. ref_mode 0: the
// node centroid; 1: the point X[ref_idx[node - first]].
__global__ void k_farthest_partial(const double* __restrict__ X, const int32_t* __restrict__ perm, int d,
                                   const int32_t* __restrict__ ch_begin, const int32_t* __restrict__ ch_end,
                                   const int32_t* __restrict__ ch_node, int first, int ref_mode,
                                   const double* __restrict__ centroid, const int32_t* __restrict__ ref_idx,
                                   BestPt* __restrict__ partial) {
  __shared__ BestPt wbest[kThreads / 64];
  const int ch = blockIdx.x;
  const int b = ch_begin[ch], e = ch_end[ch], node = ch_node[ch];
  const double* ref = ref_mode == 0 ? centroid + (int64_t)node * d : X + (int64_t)ref_idx[node - first] * d;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double bv = -1.0;
  int bi = INT_MAX, bp = -1;
  for (int i = b + w; i < e; i += kThreads / 64) {
    const int ci = perm[i];
    const double* x = X + (int64_t)ci * d;
    double acc = 0.0;
    for (int k = lane; k < d; k += 64) {
      const double df = x[k] - ref[k];
      acc += df * df;
    }
    acc = wave_sum(acc);
    if (better(acc, ci, bv, bi)) { bv = acc; bi = ci; bp = i; }
  }
  if (lane == 0) wbest[w] = BestPt{bv, bi, bp};
  __syncthreads();
  if (threadIdx.x == 0) {
    BestPt best = wbest[0];
    for (int j = 1; j < kThreads / 64; ++j)
      if (better(wbest[j].val, wbest[j].idx, best.val, best.idx)) best = wbest[j];
    partial[ch] = best;
  }
}

__global__ void k_farthest_final(const BestPt* __restrict__ partial, int first,
                                 const int32_t* __restrict__ node_ch_first, const int32_t* __restrict__ node_ch_count,
                                 int32_t* __restrict__ out_idx, double* __restrict__ radius_or_null) {
  const int ln = blockIdx.x;
  if (threadIdx.x != 0) return;
  const int cc = node_ch_count[ln];
  BestPt best{-1.0, INT_MAX, -1};
  for (int c = 0; c < cc; ++c) {
    const BestPt p = partial[node_ch_first[ln] + c];
    if (better(p.val, p.idx, best.val, best.idx)) best = p;
  }
  out_idx[ln] = best.idx == INT_MAX ? -1 : best.idx;
  if (radius_or_null) radius_or_null[first + ln] = best.val > 0.0 ? sqrt(best.val) : 0.0;
}

// Sort keys: one wave per tree position of the level.
__global__ void k_proj_keys(const double* __restrict__ X, const int32_t* __restrict__ perm, int d, int first,
                            int count, const int32_t* __restrict__ nb, const int32_t* __restrict__ ne,
                            const double* __restrict__ centroid, const int32_t* __restrict__ p1,
                            const int32_t* __restrict__ p2, int P, int64_t lo, int64_t hi,
                            SortKey* __restrict__ keys) {
  const int64_t pos = lo + (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 64;
  const int lane = threadIdx.x & 63;
  if (pos >= hi) return;
  // Locate the node of `pos` (nodes of a level are contiguous and ordered).
  int a = 0, bsz = count;
  while (bsz > 1) {
    const int half = bsz >> 1;
    if (nb[first + a + half] <= pos) { a += half; bsz -= half; } else bsz = half;
  }
  while (a + 1 < count && nb[first + a + 1] <= pos) ++a;
  const int node = first + a;
  const int ci = perm[pos];
  const double* x = X + (int64_t)ci * d;
  const double* c = centroid + (int64_t)node * d;
  const double* x1 = X + (int64_t)p1[a] * d;
  const double* x2 = X + (int64_t)p2[a] * d;
  double acc = 0.0;
  for (int k = lane; k < d; k += 64) acc += (x[k] - c[k]) * (x2[k] - x1[k]);
  acc = wave_sum(acc);
  if (lane == 0) keys[(int64_t)a * P + (pos - nb[node])] = SortKey{orderable(acc), ci, 0};
}

__global__ void k_fill_pad(SortKey* keys, int64_t total) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < total) keys[i] = SortKey{~0ull, INT_MAX, 0};
}

// One global compare-exchange pass of a bitonic network on segments of size P.
__global__ void k_bitonic_global(SortKey* keys, int64_t total, int P, int k, int j) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t i = (t / j) * 2 * j + (t % j);
  const int64_t pj = i + j;
  if (pj >= total) return;
  const bool asc = ((i % P) & k) == 0;
  SortKey a = keys[i], b = keys[pj];
  if (key_less(b, a) == asc) { keys[i] = b; keys[pj] = a; }
}

// Compare-exchange passes j_start, j_start/2, ..., 1 inside LDS tiles.
__global__ void k_bitonic_local(SortKey* keys, int P, int k, int j_start) {
  __shared__ SortKey tile[kSortTile];
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int i = threadIdx.x; i < kSortTile; i += blockDim.x) tile[i] = keys[base + i];
  __syncthreads();
  for (int j = j_start; j >= 1; j >>= 1) {
    for (int t = threadIdx.x; t < kSortTile / 2; t += blockDim.x) {
      const int i = (t / j) * 2 * j + (t % j);
      const bool asc = (((base + i) % P) & k) == 0;
      SortKey a = tile[i], b = tile[i + j];
      if (key_less(b, a) == asc) { tile[i] = b; tile[i + j] = a; }
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < kSortTile; i += blockDim.x) keys[base + i] = tile[i];
}

__global__ void k_write_perm(const SortKey* __restrict__ keys, int first, int count, const int32_t* __restrict__ nb,
                             const int32_t* __restrict__ ne, int P, int maxn, int32_t* __restrict__ perm) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)count * maxn) return;
  const int a = (int)(t / maxn), i = (int)(t % maxn);
  const int node = first + a;
  const int b = nb[node], n = ne[node] - b;
  if (i < n) perm[b + i] = keys[(int64_t)a * P + i].idx;
}

__global__ void k_gather_rows(const double* __restrict__ X, const int32_t* __restrict__ perm, int64_t N, int d,
                              double* __restrict__ Xt) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= N * d) return;
  const int64_t pos = e / d, k = e % d;
  Xt[e] = X[(int64_t)perm[pos] * d + k];
}

struct LevelChunks {
  std::vector<int32_t> ch_begin, ch_end, ch_node, node_first, node_count;
};

LevelChunks make_chunks(const ffc_tree* t, int first, int count) {
  LevelChunks c;
  for (int a = 0; a < count; ++a) {
    const int b = t->begin_h[first + a], e = t->end_h[first + a];
    c.node_first.push_back((int32_t)c.ch_begin.size());
    int nch = 0;
    for (int x = b; x < e; x += kChunk) {
      c.ch_begin.push_back(x);
      c.ch_end.push_back(std::min(e, x + kChunk));
      c.ch_node.push_back(first + a);
      ++nch;
    }
    c.node_count.push_back(nch);
  }
  return c;
}

struct Scratch {
  DevBuf<int32_t> ch_begin, ch_end, ch_node, node_first, node_count, p1, p2;
  DevBuf<double> psum;
  DevBuf<BestPt> pbest;
};

ffc_status upload(DevBuf<int32_t>& dst, const std::vector<int32_t>& src, hipStream_t st) {
  if (dst.count < src.size() || dst.ptr == nullptr) FFC_TRY(dst.alloc(std::max<size_t>(src.size(), 1)));
  if (!src.empty())
    FFC_HIP_TRY(hipMemcpyAsync(dst.ptr, src.data(), src.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  // The host vectors die at return: make the copy complete before that.
  FFC_HIP_TRY(hipStreamSynchronize(st));
  return FFC_OK;
}

// Centroid, p1 (farthest from centroid) and radius for the nodes of a level.
ffc_status centroid_and_p1(ffc_tree* t, int first, int count, Scratch& s, const LevelChunks& lc,
                           hipStream_t st, bool want_p2) {
  const int nch = (int)lc.ch_begin.size();
  const int d = t->d;
  FFC_TRY(upload(s.ch_begin, lc.ch_begin, st));
  FFC_TRY(upload(s.ch_end, lc.ch_end, st));
  FFC_TRY(upload(s.ch_node, lc.ch_node, st));
  FFC_TRY(upload(s.node_first, lc.node_first, st));
  FFC_TRY(upload(s.node_count, lc.node_count, st));
  if (s.psum.count < (size_t)std::max(1, nch) * d) FFC_TRY(s.psum.alloc((size_t)std::max(1, nch) * d));
  if (s.pbest.count < (size_t)std::max(1, nch)) FFC_TRY(s.pbest.alloc(std::max(1, nch)));
  if (s.p1.count < (size_t)count) FFC_TRY(s.p1.alloc(count));
  if (s.p2.count < (size_t)count) FFC_TRY(s.p2.alloc(count));
  if (nch > 0) {
    hipLaunchKernelGGL(k_centroid_partial, dim3(nch), dim3(kThreads), 0, st, t->X.ptr, t->perm.ptr, d,
                       s.ch_begin.ptr, s.ch_end.ptr, s.psum.ptr);
    FFC_LAUNCH_CHECK("k_centroid_partial");
  }
  hipLaunchKernelGGL(k_centroid_final, dim3(count), dim3(64), 0, st, s.psum.ptr, d, first, s.node_first.ptr,
                     s.node_count.ptr, t->begin.ptr, t->end.ptr, t->centroid.ptr);
  FFC_LAUNCH_CHECK("k_centroid_final");
  if (nch > 0) {
    hipLaunchKernelGGL(k_farthest_partial, dim3(nch), dim3(kThreads), 0, st, t->X.ptr, t->perm.ptr, d,
                       s.ch_begin.ptr, s.ch_end.ptr, s.ch_node.ptr, first, 0, t->centroid.ptr, s.p1.ptr,
                       s.pbest.ptr);
    FFC_LAUNCH_CHECK("k_farthest_partial");
  }
  hipLaunchKernelGGL(k_farthest_final, dim3(count), dim3(1), 0, st, s.pbest.ptr, first, s.node_first.ptr,
                     s.node_count.ptr, s.p1.ptr, t->radius.ptr);
  FFC_LAUNCH_CHECK("k_farthest_final");
  if (want_p2 && nch > 0) {
    hipLaunchKernelGGL(k_farthest_partial, dim3(nch), dim3(kThreads), 0, st, t->X.ptr, t->perm.ptr, d,
                       s.ch_begin.ptr, s.ch_end.ptr, s.ch_node.ptr, first, 1, t->centroid.ptr, s.p1.ptr,
                       s.pbest.ptr);
    FFC_LAUNCH_CHECK("k_farthest_partial");
    hipLaunchKernelGGL(k_farthest_final, dim3(count), dim3(1), 0, st, s.pbest.ptr, first, s.node_first.ptr,
                       s.node_count.ptr, s.p2.ptr, (double*)nullptr);
    FFC_LAUNCH_CHECK("k_farthest_final");
  }
  return FFC_OK;
}

int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

}  // namespace

ffc_status launch_build_tree(ffc_tree* t, int32_t /*leaf_size*/, hipStream_t st) {
  const int64_t N = t->N;
  hipLaunchKernelGGL(k_iota, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, t->perm.ptr, N);
  FFC_LAUNCH_CHECK("k_iota");
  Scratch s;
  DevBuf<SortKey> keys;
  for (int level = 0; level < t->depth; ++level) {
    const int first = (1 << level) - 1, count = 1 << level;
    LevelChunks lc = make_chunks(t, first, count);
    FFC_TRY(centroid_and_p1(t, first, count, s, lc, st, true));
    int maxn = 1;
    for (int a = 0; a < count; ++a) maxn = std::max(maxn, t->end_h[first + a] - t->begin_h[first + a]);
    const int P = next_pow2(maxn);
    const int64_t total = ((int64_t)count * P + kSortTile - 1) / kSortTile * kSortTile;
    if (keys.count < (size_t)total) FFC_TRY(keys.alloc(total));
    hipLaunchKernelGGL(k_fill_pad, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, keys.ptr, total);
    FFC_LAUNCH_CHECK("k_fill_pad");
    const int64_t lo = t->begin_h[first], hi = t->end_h[first + count - 1];
    if (hi > lo) {
      const int64_t threads = (hi - lo) * 64;
      hipLaunchKernelGGL(k_proj_keys, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, t->X.ptr,
                         t->perm.ptr, t->d, first, count, t->begin.ptr, t->end.ptr, t->centroid.ptr, s.p1.ptr,
                         s.p2.ptr, P, lo, hi, keys.ptr);
      FFC_LAUNCH_CHECK("k_proj_keys");
    }
    for (int k = 2; k <= P; k <<= 1) {
      int j = k >> 1;
      for (; j > kSortTile / 2; j >>= 1) {
        const int64_t pairs = total / 2;
        hipLaunchKernelGGL(k_bitonic_global, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, st, keys.ptr,
                           total, P, k, j);
        FFC_LAUNCH_CHECK("k_bitonic_global");
      }
      hipLaunchKernelGGL(k_bitonic_local, dim3((unsigned)(total / kSortTile)), dim3(256), 0, st, keys.ptr, P, k, j);
      FFC_LAUNCH_CHECK("k_bitonic_local");
    }
    const int64_t wthreads = (int64_t)count * maxn;
    hipLaunchKernelGGL(k_write_perm, dim3((unsigned)((wthreads + 255) / 256)), dim3(256), 0, st, keys.ptr, first,
                       count, t->begin.ptr, t->end.ptr, P, maxn, t->perm.ptr);
    FFC_LAUNCH_CHECK("k_write_perm");
  }
  // Leaf-level centroids and radii.
  {
    const int first = (1 << t->depth) - 1, count = 1 << t->depth;
    LevelChunks lc = make_chunks(t, first, count);
    FFC_TRY(centroid_and_p1(t, first, count, s, lc, st, false));
  }
  FFC_TRY(launch_gather_tree_points(t, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));  // scratch buffers are freed on return
  return FFC_OK;
}

ffc_status launch_node_stats(ffc_tree* t, int level, hipStream_t st) {
  const int first = (1 << level) - 1, count = 1 << level;
  Scratch s;
  LevelChunks lc = make_chunks(t, first, count);
  FFC_TRY(centroid_and_p1(t, first, count, s, lc, st, false));
  FFC_HIP_TRY(hipStreamSynchronize(st));
  return FFC_OK;
}

ffc_status launch_gather_tree_points(ffc_tree* t, hipStream_t st) {
  const int64_t total = t->N * t->d;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, t->X.ptr, t->perm.ptr,
                     t->N, t->d, t->Xt.ptr);
  FFC_LAUNCH_CHECK("k_gather_rows");
  return FFC_OK;
}

}  // namespace ffc
