// FMM-style evaluation with incoming representations built from the same
// skeletons (Section 2: the Fast Multipole Method adds incoming
// representations, and the construction of outgoing ones serves for them too).
// For a symmetric kernel on one point set, the ID of node b fitted on its
// separated far field gives outgoing K(F, cols) ~ K(F, J) P and incoming
// K(cols, S) ~ P^T K(J, S) for sources S in that far field.
//
//   * admissibility: nodes b != a of one level are admissible when every point
//     of b is separated from a and every point of a from b: two range tests on
//     the separation bitmaps (k_fmm_admissible, every pair of every level);
//   * lists: the dual-tree recursion from the pairs of the root's children, on
//     the host from the copied admissibility bytes (the first call with a
//     skeleton set synchronizes once): admissible pairs are multipole-to-local
//     pairs, other leaf pairs are direct pairs, other pairs recurse into their
//     four child pairs. Pairs are visited in (target, source) order;
//   * k_m2l: v_b = sum over b's list of K(x_{J_b}, x_{J_a}) q~_a, one workgroup
//     per (node, 64 skeleton points, quarter of the list: entries e with
//     e mod 4 = part), whose partial sums k_m2l_fold adds in part order;
//   * k_l2l (top-down, one launch per level): P_b^T v_b is added to the
//     children's v at their skeleton points, or is the far field at a leaf's
//     points; one thread per column, the rank loop in a fixed order;
//   * k_p2p: per 64-target tile, the direct sums over the leaf's direct list,
//     plus the far field, written in caller order.
#include <algorithm>
#include <utility>
#include <vector>

#include "ffc_internal.h"
#include "tile_engine.h"
#include "tile_sums.h"

namespace ffc {
namespace {

using namespace tile;

// Bits [lo, hi) of one node's bitmap are all set.
__device__ inline bool all_set(const uint64_t* __restrict__ bits, int lo, int hi) {
  for (int p = lo; p < hi;) {
    const int off = p & 63;
    const int n = min(64 - off, hi - p);
    const uint64_t mask = (n == 64 ? ~0ull : ((1ull << n) - 1ull)) << off;
    if ((bits[p >> 6] & mask) != mask) return false;
    p += n;
  }
  return true;
}

// adm[base + bi * count + ai] for the pairs (first + bi, first + ai) of one level.
__global__ void k_fmm_admissible(const uint64_t* __restrict__ bits, int words, const int32_t* __restrict__ nb,
                                 const int32_t* __restrict__ ne, int first, int count,
                                 unsigned char* __restrict__ adm) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)count * count) return;
  const int b = first + (int)(p / count), a = first + (int)(p % count);
  bool ok = false;
  if (a != b)
    ok = all_set(bits + (int64_t)a * words, nb[b], ne[b]) && all_set(bits + (int64_t)b * words, nb[a], ne[a]);
  adm[p] = ok ? 1 : 0;
}

constexpr int kM2lParts = 4;

template <typename T, int KF, int DM>
__global__ void __launch_bounds__(NT) k_m2l(const double* __restrict__ Xt, int d, KParams kp, int chunks,
                                            int num_nodes, const int32_t* __restrict__ rank,
                                            const int32_t* __restrict__ skel, int r_cap,
                                            const double* __restrict__ qt, const int32_t* __restrict__ off,
                                            const int32_t* __restrict__ src, double* __restrict__ vpart,
                                            unsigned int* flag) {
  __shared__ EvalSmem<T, DM> sm;
  __shared__ double red[16 * BM];
  __shared__ double rowsum[BM];
  const int part = blockIdx.x % kM2lParts;
  const int bc = blockIdx.x / kM2lParts;
  const int b = 1 + bc / chunks, c = bc % chunks;
  const int nrows = min(BM, rank[b] - c * BM);
  if (nrows <= 0) return;
  const IdxMap rmap{skel + (int64_t)b * r_cap + c * BM, 0};
  if constexpr (DM > 0) stage_rows<T, DM>(Xt, rmap, nrows, d, sm);
  bool bad = false;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int e = off[b] + part; e < off[b + 1]; e += kM2lParts) {
    const int a = src[e];
    if (rank[a] > 0)
      sum_sources<T, KF, DM>(Xt, rmap, nrows, Xt, IdxMap{skel + (int64_t)a * r_cap, 0}, rank[a],
                          qt + (int64_t)a * r_cap, d, kp, sm, acc, bad);
  }
  reduce_rows(acc, red, rowsum);
  if (threadIdx.x < nrows)
    vpart[((int64_t)part * num_nodes + b) * r_cap + c * BM + threadIdx.x] = rowsum[threadIdx.x];
  if (bad) flag_nonfinite(flag);
}

// v_b = the partial sums of b's list quarters, in part order.
__global__ void k_m2l_fold(int num_nodes, int r_cap, const int32_t* __restrict__ rank,
                           const double* __restrict__ vpart, double* __restrict__ v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)num_nodes * r_cap) return;
  const int b = (int)(e / r_cap), i = (int)(e % r_cap);
  if (b == 0 || i >= rank[b]) return;
  double s = 0.0;
  for (int p = 0; p < kM2lParts; ++p) s += vpart[(int64_t)p * num_nodes * r_cap + e];
  v[e] = s;
}

// Nodes [first, first + count) of one level: w = P_b^T v_b at b's columns, added
// to the children's v (internal nodes) or stored as the far field of the leaf's
// points (tree order).
__global__ void __launch_bounds__(256) k_l2l(int first, int leaves, const int32_t* __restrict__ rank,
                                             const int32_t* __restrict__ ncols, const double* __restrict__ P,
                                             int r_cap, int n_cap, const int32_t* __restrict__ nb,
                                             double* __restrict__ v, double* __restrict__ ufar) {
  const int b = first + blockIdx.x;
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= ncols[b]) return;
  const int r = rank[b];
  const double* Pb = P + (int64_t)b * r_cap * n_cap + j;
  const double* vb = v + (int64_t)b * r_cap;
  double w = 0.0;
  for (int i = 0; i < r; ++i) w = fma(Pb[(int64_t)i * n_cap], vb[i], w);
  if (leaves) {
    ufar[nb[b] + j] = w;
    return;
  }
  const int l = 2 * b + 1, rl = rank[l];
  if (j < rl) v[(int64_t)l * r_cap + j] += w;
  else v[(int64_t)(l + 1) * r_cap + (j - rl)] += w;
}

template <typename T, int KF, int DM>
__global__ void __launch_bounds__(NT) k_p2p(const double* __restrict__ Xt, int d, KParams kp,
                                            const int32_t* __restrict__ tile_leaf,
                                            const int32_t* __restrict__ tile_start, const int32_t* __restrict__ nb,
                                            const int32_t* __restrict__ ne, const double* __restrict__ q_tree,
                                            int leaf0, const int32_t* __restrict__ off,
                                            const int32_t* __restrict__ src, const double* __restrict__ ufar,
                                            const int32_t* __restrict__ perm, double* __restrict__ u,
                                            double* __restrict__ u_far, unsigned int* flag) {
  __shared__ EvalSmem<T, DM> sm;
  __shared__ double red[16 * BM];
  __shared__ double near_sum[BM];
  const int leaf = tile_leaf[blockIdx.x];
  const int start = tile_start[blockIdx.x];
  const int nrows = min(BM, ne[leaf] - start);
  const IdxMap rmap{nullptr, start};
  if constexpr (DM > 0) stage_rows<T, DM>(Xt, rmap, nrows, d, sm);
  bool bad = false;
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  const int li = leaf - leaf0;
  for (int e = off[li]; e < off[li + 1]; ++e) {
    const int a = src[e];
    const int ab = nb[a];
    sum_sources<T, KF, DM>(Xt, rmap, nrows, Xt, IdxMap{nullptr, ab}, ne[a] - ab, q_tree + ab, d, kp, sm, part,
                        bad);
  }
  reduce_rows(part, red, near_sum);
  if (threadIdx.x < nrows) {
    const int pos = start + threadIdx.x;
    const int ci = perm[pos];
    const double f = ufar[pos];
    u[ci] = f + near_sum[threadIdx.x];
    if (u_far) u_far[ci] = f;
  }
  if (bad) flag_nonfinite(flag);
}

template <typename F>
ffc_status dispatch_tiles(int precision, const KParams& kp, F&& f) {
  return with_kind(kp, [&](auto kv) -> ffc_status {
    if (precision == FFC_FP64) return f(double(), kv);
    return f(float(), kv);
  });
}

// Interaction lists of the skeleton set's separation (synchronizes `st`).
ffc_status build_fmm_lists(const ffc_tree* t, ffc_skel* sk, hipStream_t st) {
  const int depth = t->depth;
  std::vector<int64_t> base(depth + 2, 0);
  for (int l = 1; l <= depth; ++l) base[l + 1] = base[l] + ((int64_t)1 << (2 * l));
  DevBuf<unsigned char> adm;
  FFC_TRY(adm.alloc((size_t)base[depth + 1]));
  for (int l = 1; l <= depth; ++l) {
    const int first = (1 << l) - 1, count = 1 << l;
    const int64_t pairs = (int64_t)count * count;
    hipLaunchKernelGGL(k_fmm_admissible, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, st, sk->sep_bits.ptr,
                       sk->sep_words, t->begin.ptr, t->end.ptr, first, count, adm.ptr + base[l]);
    FFC_LAUNCH_CHECK("k_fmm_admissible");
  }
  std::vector<unsigned char> h((size_t)base[depth + 1]);
  FFC_HIP_TRY(hipMemcpyAsync(h.data(), adm.ptr, h.size(), hipMemcpyDeviceToHost, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));
  const int nn = t->num_nodes, leaf0 = (1 << depth) - 1, nleaves = 1 << depth;
  std::vector<std::vector<int32_t>> far(nn), near(nleaves);
  std::vector<std::pair<int, int>> pairs = {{1, 1}, {1, 2}, {2, 1}, {2, 2}}, next;
  for (int l = 1; l <= depth; ++l) {
    const int first = (1 << l) - 1, count = 1 << l;
    std::sort(pairs.begin(), pairs.end());
    next.clear();
    for (const auto& pr : pairs) {
      const int b = pr.first, a = pr.second;
      if (h[(size_t)(base[l] + (int64_t)(b - first) * count + (a - first))]) {
        far[b].push_back(a);
      } else if (l == depth) {
        near[b - leaf0].push_back(a);
      } else {
        for (int cb = 2 * b + 1; cb <= 2 * b + 2; ++cb)
          for (int ca = 2 * a + 1; ca <= 2 * a + 2; ++ca) next.emplace_back(cb, ca);
      }
    }
    pairs.swap(next);
  }
  std::vector<int32_t> far_off(nn + 1, 0), near_off(nleaves + 1, 0), far_src, near_src;
  for (int b = 0; b < nn; ++b) {
    far_off[b + 1] = far_off[b] + (int32_t)far[b].size();
    far_src.insert(far_src.end(), far[b].begin(), far[b].end());
  }
  for (int L = 0; L < nleaves; ++L) {
    near_off[L + 1] = near_off[L] + (int32_t)near[L].size();
    near_src.insert(near_src.end(), near[L].begin(), near[L].end());
  }
  FFC_TRY(sk->fmm_far_off.alloc(far_off.size()));
  FFC_TRY(sk->fmm_near_off.alloc(near_off.size()));
  FFC_TRY(sk->fmm_far_src.alloc(std::max<size_t>(1, far_src.size())));
  FFC_TRY(sk->fmm_near_src.alloc(std::max<size_t>(1, near_src.size())));
  FFC_HIP_TRY(hipMemcpyAsync(sk->fmm_far_off.ptr, far_off.data(), far_off.size() * 4, hipMemcpyHostToDevice, st));
  FFC_HIP_TRY(hipMemcpyAsync(sk->fmm_near_off.ptr, near_off.data(), near_off.size() * 4, hipMemcpyHostToDevice, st));
  if (!far_src.empty())
    FFC_HIP_TRY(hipMemcpyAsync(sk->fmm_far_src.ptr, far_src.data(), far_src.size() * 4, hipMemcpyHostToDevice, st));
  if (!near_src.empty())
    FFC_HIP_TRY(
        hipMemcpyAsync(sk->fmm_near_src.ptr, near_src.data(), near_src.size() * 4, hipMemcpyHostToDevice, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));   // the host vectors go out of scope
  sk->fmm_far_pairs = (int64_t)far_src.size();
  sk->fmm_near_pairs = (int64_t)near_src.size();
  sk->fmm_xi = sk->opts.separation;
  return FFC_OK;
}

}  // namespace

ffc_status launch_fmm(const ffc_tree* t, ffc_skel* sk, const KParams& kp, int precision, double* u, double* u_far,
                      hipStream_t st) {
  if (precision == FFC_MIXED_BF16X3) {
    set_error("the FMM-style evaluation runs in FFC_FP64 or FFC_FP32");
    return FFC_ERR_INVALID_ARG;
  }
  if (!(sk->opts.separation > 0.0) || !sk->sep_bits.ptr || sk->sep_words != (int)((t->N + 63) / 64)) {
    set_error("the FMM-style evaluation needs a skeleton set built with separation > 0");
    return FFC_ERR_STATE;
  }
  if (t->depth > 11) {
    set_error("the FMM-style evaluation supports trees of depth <= 11");
    return FFC_ERR_INVALID_ARG;
  }
  if (sk->fmm_xi != sk->opts.separation || !sk->fmm_far_off.ptr) FFC_TRY(build_fmm_lists(t, sk, st));
  const size_t nv = (size_t)t->num_nodes * sk->r_cap;
  if (sk->fmm_v.count != nv) FFC_TRY(sk->fmm_v.alloc(nv));
  if (sk->fmm_vpart.count != nv * kM2lParts) FFC_TRY(sk->fmm_vpart.alloc(nv * kM2lParts));
  if (sk->fmm_ufar.count != (size_t)t->N) FFC_TRY(sk->fmm_ufar.alloc((size_t)t->N));
  const int chunks = (sk->r_cap + BM - 1) / BM;
  const int leaf0 = (1 << t->depth) - 1;
  return dispatch_tiles(precision, kp, [&](auto tv, auto kv) -> ffc_status {
    using T = decltype(tv);
    constexpr int KF = decltype(kv)::value;
    return with_dims(t->d, [&](auto dm) -> ffc_status {
      constexpr int DM = decltype(dm)::value;
      hipLaunchKernelGGL((k_m2l<T, KF, DM>), dim3((unsigned)((t->num_nodes - 1) * chunks * kM2lParts)), dim3(NT), 0, st,
                         t->Xt.ptr, t->d, kp, chunks, t->num_nodes, sk->rank.ptr, sk->skel.ptr, sk->r_cap, sk->qt.ptr,
                         sk->fmm_far_off.ptr, sk->fmm_far_src.ptr, sk->fmm_vpart.ptr, device_flag());
      FFC_LAUNCH_CHECK("k_m2l");
      const int64_t nv = (int64_t)t->num_nodes * sk->r_cap;
      hipLaunchKernelGGL(k_m2l_fold, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st, t->num_nodes, sk->r_cap,
                         sk->rank.ptr, sk->fmm_vpart.ptr, sk->fmm_v.ptr);
      FFC_LAUNCH_CHECK("k_m2l_fold");
      for (int l = 1; l <= t->depth; ++l) {
        const int first = (1 << l) - 1, count = 1 << l;
        hipLaunchKernelGGL(k_l2l, dim3((unsigned)count, (unsigned)((sk->n_cap + 255) / 256)), dim3(256), 0, st, first,
                           l == t->depth ? 1 : 0, sk->rank.ptr, sk->ncols.ptr, sk->P.ptr, sk->r_cap, sk->n_cap,
                           t->begin.ptr, sk->fmm_v.ptr, sk->fmm_ufar.ptr);
        FFC_LAUNCH_CHECK("k_l2l");
      }
      hipLaunchKernelGGL((k_p2p<T, KF, DM>), dim3((unsigned)t->num_tiles), dim3(NT), 0, st, t->Xt.ptr, t->d, kp,
                         t->tile_leaf.ptr, t->tile_start.ptr, t->begin.ptr, t->end.ptr, t->q_tree.ptr, leaf0,
                         sk->fmm_near_off.ptr, sk->fmm_near_src.ptr, sk->fmm_ufar.ptr, t->perm.ptr, u, u_far,
                         device_flag());
      FFC_LAUNCH_CHECK("k_p2p");
      return FFC_OK;
    });
  });
}

}  // namespace ffc
