// C ABI of the learned row proposal: handles, features, scores, gradients,
// Adam, ridge leverage labels, the training set and the training loop, plus
// the per-level steps of skeletonization with the learned sampler.
//
// Counter streams (seed ^ (stream << 32) ^ counter, first SplitMix64 output):
//   node                   uniform rows of a node (Section 4.1.3, uniform sampling)
//   node | 2^29            held-out rows of the fallback check
//   node | 2^30            subsample of a node's column set (features)
//   node | 2^31            candidate pool of the learned sampler
//   node | 3 * 2^30        Efraimidis-Spirakis keys
//   g | 5 * 2^29           training block g: columns inside its leaf
//   g | 5 * 2^29 | 2^28    training block g: targets outside its leaf
//   7 * 2^29, counter g    training block g: its leaf
//   7 * 2^29 | 2^28, e     epoch e: the stride of its visiting order
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "ffc_internal.h"

namespace ffc {

namespace {

constexpr int kNF = FFC_PROPOSAL_NFEAT;
constexpr int kNParam = FFC_PROPOSAL_NPARAM;
constexpr int kHeld = 32;
constexpr int kGradBatch = 64;   // samples per workgroup of the gradient kernel
constexpr uint32_t kStreamHeldout = 1u << 29, kStreamPool = 1u << 31;
constexpr uint32_t kStreamTrainCols = 5u << 29, kStreamTrainRows = (5u << 29) | (1u << 28);
constexpr uint32_t kStreamTrainLeaf = 7u << 29, kStreamTrainShuffle = (7u << 29) | (1u << 28);

ffc_status fail(ffc_status code, const std::string& msg) {
  set_error(msg);
  return code;
}

uint64_t host_counter_u64(uint64_t seed, uint64_t stream, uint64_t j) {
  uint64_t z = (seed ^ (stream << 32) ^ j) + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t uniform_below(uint64_t u, uint64_t bound) {
  return (uint64_t)(((unsigned __int128)u * bound) >> 64);
}

// Multiplier of epoch e's visiting order p -> (p k) mod C, coprime with C.
int64_t epoch_stride(int64_t C, uint64_t seed, int e) {
  if (C <= 1) return 1;
  int64_t k = 1 + (int64_t)uniform_below(host_counter_u64(seed, kStreamTrainShuffle, (uint64_t)e), (uint64_t)(C - 1));
  while (std::gcd(k, C) != 1) k = k + 1 < C ? k + 1 : 1;
  return k;
}

bool all_finite(const float* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// Geometry scratch for `count` column sets.
struct GeomScratch {
  DevBuf<double> cen, rho, U, subn2;
  DevBuf<int32_t> sub, nsub;
  ffc_status alloc(int count, int d) {
    FFC_TRY(cen.alloc((size_t)count * d));
    FFC_TRY(subn2.alloc((size_t)count * 256));
    FFC_TRY(rho.alloc(count));
    FFC_TRY(U.alloc((size_t)count * 7 * d));
    FFC_TRY(sub.alloc((size_t)count * 256));
    FFC_TRY(nsub.alloc(count));
    return FFC_OK;
  }
  GeomArgs args(const int32_t* cols, int64_t stride, const int32_t* ncols, const int32_t* ids, uint64_t seed) {
    return GeomArgs{cols, stride, ncols, ids, seed, cen.ptr, rho.ptr, sub.ptr, nsub.ptr, U.ptr, subn2.ptr};
  }
};

// Full-batch (or one mini-batch) gradient into partial sums, then reduced.
ffc_status grad_step(const ffc_proposal* p, float* theta, float* m1, float* m2, const float* feat, const float* target,
                     int64_t count, int64_t p0, int64_t stride, int64_t total, DevBuf<float>& partial, float* gsum,
                     float* loss, bool adam, float lr, int step, hipStream_t st) {
  const int nwg = (int)((total + kGradBatch - 1) / kGradBatch);
  if (partial.count < (size_t)nwg * (kNParam + 1)) FFC_TRY(partial.alloc((size_t)nwg * (kNParam + 1)));
  FFC_TRY(launch_mlp_grad(theta, p->mu.ptr, p->sd.ptr, feat, target, count, p0, stride, total, partial.ptr, st));
  FFC_TRY(launch_grad_reduce_adam(partial.ptr, nwg, theta, m1, m2, gsum, loss, adam, lr, step, total, st));
  return FFC_OK;
}

// The training set: leaves, columns, targets, features, leverages and label targets.
struct TrainSet {
  int n = 0, m = 0, G = 0;
  std::vector<int32_t> leaves_h;
  DevBuf<int32_t> leaves, lo, hi, cols, ncols, rows, nrows;
  DevBuf<float> feat, target;
  DevBuf<double> lev;
};

ffc_status check_train_opts(const ffc_tree* t, const ffc_kernel* k, const ffc_train_opts* o) {
  if (!t || !k || !o) return fail(FFC_ERR_INVALID_ARG, "tree, kernel or options is NULL");
  if (o->num_blocks < 1 || o->num_blocks >= (1 << 28)) return fail(FFC_ERR_INVALID_ARG, "num_blocks must be in [1, 2^28)");
  if (o->block_cols < 1 || o->block_rows < 1) return fail(FFC_ERR_INVALID_ARG, "block sizes must be >= 1");
  if (!(o->eps > 0.0) || !std::isfinite(o->eps)) return fail(FFC_ERR_INVALID_ARG, "eps must be > 0");
  if (o->epochs < 0 || o->batch < 1) return fail(FFC_ERR_INVALID_ARG, "epochs must be >= 0 and batch >= 1");
  if (!(o->lr > 0.f) || !std::isfinite(o->lr)) return fail(FFC_ERR_INVALID_ARG, "lr must be > 0");
  if (o->label != FFC_LABEL_PIVOTED && o->label != FFC_LABEL_RIDGE) return fail(FFC_ERR_INVALID_ARG, "unknown label kind");
  return validate_kernel(k, t->d);
}

ffc_status train_sizes(const ffc_tree* t, const ffc_train_opts* o, int& n, int& m) {
  const int first = (1 << t->depth) - 1;
  int min_leaf = INT32_MAX, max_leaf = 0;
  for (int a = first; a < t->num_nodes; ++a) {
    min_leaf = std::min(min_leaf, t->end_h[a] - t->begin_h[a]);
    max_leaf = std::max(max_leaf, t->end_h[a] - t->begin_h[a]);
  }
  n = std::min(o->block_cols, min_leaf);
  m = (int)std::min<int64_t>(o->block_rows, t->N - max_leaf);
  if (n < 1 || m < 1) return fail(FFC_ERR_INVALID_ARG, "tree too small for training blocks (needs two non-empty leaves)");
  if (n > 4096) return fail(FFC_ERR_INVALID_ARG, "block_cols above 4096 is not supported");
  if (o->label == FFC_LABEL_PIVOTED && n > 1024)
    return fail(FFC_ERR_INVALID_ARG, "pivoted leverage labels support block_cols <= 1024");
  if ((int64_t)m > 65536) return fail(FFC_ERR_INVALID_ARG, "block_rows above 65536 is not supported");
  return FFC_OK;
}

ffc_status build_training_set(const ffc_tree* t, const ffc_kernel* k, const ffc_train_opts* o, TrainSet& ts,
                              hipStream_t st) {
  FFC_TRY(train_sizes(t, o, ts.n, ts.m));
  const int G = ts.G = o->num_blocks, n = ts.n, m = ts.m;
  const int first = (1 << t->depth) - 1, nleaves = 1 << t->depth;
  ts.leaves_h.resize(G);
  std::vector<int32_t> lo(G), hi(G);
  for (int g = 0; g < G; ++g) {
    const int leaf = first + (int)uniform_below(host_counter_u64(o->seed, kStreamTrainLeaf, (uint64_t)g), nleaves);
    ts.leaves_h[g] = leaf;
    lo[g] = t->begin_h[leaf];
    hi[g] = t->end_h[leaf];
  }
  FFC_TRY(ts.leaves.alloc(G));
  FFC_TRY(ts.lo.alloc(G));
  FFC_TRY(ts.hi.alloc(G));
  FFC_HIP_TRY(hipMemcpyAsync(ts.leaves.ptr, ts.leaves_h.data(), G * sizeof(int32_t), hipMemcpyHostToDevice, st));
  FFC_HIP_TRY(hipMemcpyAsync(ts.lo.ptr, lo.data(), G * sizeof(int32_t), hipMemcpyHostToDevice, st));
  FFC_HIP_TRY(hipMemcpyAsync(ts.hi.ptr, hi.data(), G * sizeof(int32_t), hipMemcpyHostToDevice, st));
  FFC_TRY(ts.cols.alloc((size_t)G * n));
  FFC_TRY(ts.ncols.alloc(G));
  FFC_TRY(ts.rows.alloc((size_t)G * m));
  FFC_TRY(ts.nrows.alloc(G));
  FFC_TRY(launch_draw(ts.lo.ptr, ts.hi.ptr, t->N, true, ts.cols.ptr, ts.ncols.ptr, n, 0, G, n, o->seed,
                      kStreamTrainCols, nullptr, st));
  FFC_TRY(launch_draw(ts.lo.ptr, ts.hi.ptr, t->N, false, ts.rows.ptr, ts.nrows.ptr, m, 0, G, m, o->seed,
                      kStreamTrainRows, nullptr, st));
  const int64_t C = (int64_t)G * m;
  FFC_TRY(ts.feat.alloc((size_t)C * kNF));
  FFC_TRY(ts.target.alloc(C));
  FFC_TRY(ts.lev.alloc(C));
  // Labels in chunks of blocks (about 1 GiB of blocks and Gram matrices each).
  const KParams kp = make_kparams(*k, t->d);
  const bool pivoted = o->label == FFC_LABEL_PIVOTED;
  const size_t per_block = (size_t)m * n + (size_t)n * n * (pivoted ? 2 : 1);
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(G, ((size_t)1 << 27) / per_block));
  DevBuf<double> B, Gm, Lc;
  DevBuf<int> status, perm, rank;
  FFC_TRY(B.alloc((size_t)chunk * m * n));
  FFC_TRY(Gm.alloc((size_t)chunk * n * n));
  FFC_TRY(status.alloc(G));
  if (pivoted) {
    FFC_TRY(Lc.alloc((size_t)chunk * n * n));
    FFC_TRY(perm.alloc((size_t)chunk * n));
    FFC_TRY(rank.alloc(chunk));
  }
  GeomScratch gs;   // outlives the launches below (freed after the synchronization)
  FFC_TRY(gs.alloc(G, t->d));
  {
    StageTimer timer(FFC_STAGE_LABELS, st);
    for (int g0 = 0; g0 < G; g0 += chunk) {
      const int c = std::min(chunk, G - g0);
      // Row-major m x n blocks: the "rows" of the tile engine are the block's
      // columns, its "columns" the targets (the kernels are symmetric).
      FFC_TRY(launch_kblock_batch(t, kp, FFC_FP64, ts.cols.ptr + (int64_t)g0 * n, ts.ncols.ptr + g0, n,
                                  ts.rows.ptr + (int64_t)g0 * m, ts.nrows.ptr + g0, m, 0, c, nullptr, B.ptr, st));
      if (pivoted)
        FFC_TRY(launch_pivoted_leverage(B.ptr, m, n, c, Gm.ptr, Lc.ptr, perm.ptr, rank.ptr, o->eps,
                                        ts.lev.ptr + (int64_t)g0 * m, ts.target.ptr + (int64_t)g0 * m,
                                        status.ptr + g0, st));
      else
        FFC_TRY(launch_ridge_leverage(B.ptr, m, n, c, Gm.ptr, o->eps, ts.lev.ptr + (int64_t)g0 * m,
                                      ts.target.ptr + (int64_t)g0 * m, status.ptr + g0, st));
    }
    // Features of every target against its block's columns.
    const GeomArgs ga = gs.args(ts.cols.ptr, n, ts.ncols.ptr, ts.leaves.ptr, o->seed);
    FFC_TRY(launch_geometry(t->Xt.ptr, t->d, ga, G, st));
    FFC_TRY(launch_features(t->Xt.ptr, t->d, ga, ts.rows.ptr, m, ts.nrows.ptr, G, ts.feat.ptr, (int64_t)m * kNF,
                            st));
  }
  std::vector<int> st_h(G);
  FFC_HIP_TRY(hipMemcpyAsync(st_h.data(), status.ptr, G * sizeof(int), hipMemcpyDeviceToHost, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));
  for (int g = 0; g < G; ++g)
    if (st_h[g] == 2) return fail(FFC_ERR_NONFINITE, "leverage labels: Cholesky factorization failed");
  return FFC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Learned sampler inside skeletonization
// ---------------------------------------------------------------------------
ffc_status learned_alloc(const ffc_tree* t, ffc_skel* sk, int pool_factor) {
  LearnedScratch& L = sk->learned;
  const int p_cap = (int)std::min<int64_t>((int64_t)pool_factor * sk->s_cap, t->N);
  if (L.p_cap == p_cap && L.ids.ptr) return FFC_OK;
  if (p_cap > 8192)
    return fail(FFC_ERR_INVALID_ARG, "the learned sampler's candidate pool (pool_factor * samples) is limited to 8192");
  const size_t nn = t->num_nodes, widest = (size_t)1 << t->depth, d = t->d;
  FFC_TRY(L.ids.alloc(nn));
  std::vector<int32_t> iota(nn);
  std::iota(iota.begin(), iota.end(), 0);
  FFC_HIP_TRY(hipMemcpy(L.ids.ptr, iota.data(), nn * sizeof(int32_t), hipMemcpyHostToDevice));
  FFC_TRY(L.pool.alloc(nn * p_cap));
  FFC_TRY(L.npool.alloc(nn));
  FFC_TRY(L.cen.alloc(widest * d));
  FFC_TRY(L.rho.alloc(widest));
  FFC_TRY(L.U.alloc(widest * 7 * d));
  FFC_TRY(L.subn2.alloc(widest * 256));
  FFC_TRY(L.sub.alloc(widest * 256));
  FFC_TRY(L.nsub.alloc(widest));
  FFC_TRY(L.feat.alloc(widest * p_cap * kNF));
  FFC_TRY(L.score.alloc(widest * p_cap));
  FFC_TRY(L.hrows.alloc(nn * kHeld));
  FFC_TRY(L.nheld.alloc(nn));
  FFC_TRY(L.Kh.alloc(widest * kHeld * sk->n_cap));
  FFC_TRY(L.mask.alloc(nn));
  FFC_TRY(L.counter.alloc(1));
  L.p_cap = p_cap;   // only once every buffer has its new size
  return FFC_OK;
}

ffc_status learned_rows_level(const ffc_tree* t, ffc_skel* sk, int sampler, const ffc_proposal* p, int first,
                              int count, int s, uint64_t seed, hipStream_t st) {
  LearnedScratch& L = sk->learned;
  const int pc = L.p_cap;
  FFC_TRY(launch_sample_rows_into(t, L.pool.ptr, L.npool.ptr, pc, first, count, pc, seed, kStreamPool, nullptr, st));
  const GeomArgs ga{sk->cols.ptr + (int64_t)first * sk->n_cap, sk->n_cap, sk->ncols.ptr + first, L.ids.ptr + first,
                    seed, L.cen.ptr, L.rho.ptr, L.sub.ptr, L.nsub.ptr, L.U.ptr, L.subn2.ptr};
  FFC_TRY(launch_geometry(t->Xt.ptr, t->d, ga, count, st));
  FFC_TRY(launch_features(t->Xt.ptr, t->d, ga, L.pool.ptr + (int64_t)first * pc, pc, L.npool.ptr + first, count,
                          L.feat.ptr, (int64_t)pc * kNF, st));
  if (sampler == FFC_SAMPLE_LEARNED) {
    FFC_TRY(launch_mlp_score(p->theta.ptr, p->mu.ptr, p->sd.ptr, L.feat.ptr, (int64_t)count * pc, L.score.ptr, st));
    return launch_select_rows(L.score.ptr, pc, 1, 0, L.pool.ptr + (int64_t)first * pc, pc, L.npool.ptr + first, first,
                              count, s, seed, sk->ncols.ptr, nullptr, sk->rows.ptr, sk->s_cap, sk->nrows.ptr, st);
  }
  // The paper's heuristics (Sections 3.2, 4.1.3) on the same pool: distance
  // weights from f0 = |y - c| / rho, nearest neighbours by f2 = distance to the
  // nearest point of the column subsample / rho.
  const bool dist = sampler == FFC_SAMPLE_DISTANCE;
  return launch_select_rows(L.feat.ptr + (dist ? 0 : 2), (int64_t)pc * kNF, kNF, dist ? 1 : 2,
                            L.pool.ptr + (int64_t)first * pc, pc, L.npool.ptr + first, first, count, s, seed,
                            sk->ncols.ptr, nullptr, sk->rows.ptr, sk->s_cap, sk->nrows.ptr, st);
}

ffc_status learned_heldout_level(const ffc_tree* t, ffc_skel* sk, const KParams& kp, int precision, int first,
                                 int count, int s, uint64_t seed, double tol, int& redo, hipStream_t st) {
  LearnedScratch& L = sk->learned;
  redo = 0;
  FFC_TRY(launch_sample_rows_into(t, L.hrows.ptr, L.nheld.ptr, kHeld, first, count, kHeld, seed, kStreamHeldout,
                                  nullptr, st));
  FFC_TRY(launch_kblock_batch(t, kp, precision, L.hrows.ptr, L.nheld.ptr, kHeld, sk->cols.ptr, sk->ncols.ptr,
                              sk->n_cap, first, count, t->centroid.ptr, L.Kh.ptr, st));
  FFC_HIP_TRY(hipMemsetAsync(L.counter.ptr, 0, sizeof(unsigned int), st));
  FFC_TRY(launch_heldout_check(L.Kh.ptr, L.nheld.ptr, kHeld, sk, first, count, tol, L.mask.ptr, L.counter.ptr,
                               HeldoutGrow{}, st));
  unsigned int h = 0;
  FFC_HIP_TRY(hipMemcpyAsync(&h, L.counter.ptr, sizeof(unsigned int), hipMemcpyDeviceToHost, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));
  redo = (int)h;
  if (h)
    FFC_TRY(launch_sample_rows_into(t, sk->rows.ptr, sk->nrows.ptr, sk->s_cap, first, count, s, seed, 0u, L.mask.ptr,
                                    st));
  return FFC_OK;
}

ffc_status heldout_alloc(const ffc_tree* t, ffc_skel* sk) {
  LearnedScratch& L = sk->learned;
  if (L.hrows.ptr) return FFC_OK;
  const size_t nn = t->num_nodes, widest = (size_t)1 << t->depth;
  FFC_TRY(L.hrows.alloc(nn * kHeld));
  FFC_TRY(L.nheld.alloc(nn));
  FFC_TRY(L.Kh.alloc(widest * kHeld * sk->n_cap));
  FFC_TRY(L.mask.alloc(nn));
  FFC_TRY(L.counter.alloc(1));
  return FFC_OK;
}

ffc_status heldout_prepare_level(const ffc_tree* t, ffc_skel* sk, const KParams& kp, int precision, int first,
                                 int count, uint64_t seed, hipStream_t st) {
  LearnedScratch& L = sk->learned;
  FFC_TRY(launch_sample_rows_into(t, L.hrows.ptr, L.nheld.ptr, kHeld, first, count, kHeld, seed, kStreamHeldout,
                                  nullptr, st));
  return launch_kblock_batch(t, kp, precision, L.hrows.ptr, L.nheld.ptr, kHeld, sk->cols.ptr, sk->ncols.ptr,
                             sk->n_cap, first, count, t->centroid.ptr, L.Kh.ptr, st);
}

ffc_status adaptive_round_level(const ffc_tree* t, ffc_skel* sk, int first, int count, uint64_t seed, double tol,
                                int s_limit, int s_next, int& redo, hipStream_t st) {
  LearnedScratch& L = sk->learned;
  redo = 0;
  FFC_HIP_TRY(hipMemsetAsync(L.counter.ptr, 0, sizeof(unsigned int), st));
  HeldoutGrow grow;
  grow.nrows = sk->nrows.ptr;
  grow.nb = t->begin.ptr;
  grow.ne = t->end.ptr;
  grow.N = t->N;
  grow.s_limit = s_limit;
  FFC_TRY(launch_heldout_check(L.Kh.ptr, L.nheld.ptr, kHeld, sk, first, count, tol, L.mask.ptr, L.counter.ptr, grow,
                               st));
  unsigned int h = 0;
  FFC_HIP_TRY(hipMemcpyAsync(&h, L.counter.ptr, sizeof(unsigned int), hipMemcpyDeviceToHost, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));
  redo = (int)h;
  if (h)
    FFC_TRY(launch_sample_rows_into(t, sk->rows.ptr, sk->nrows.ptr, sk->s_cap, first, count, s_next, seed, 0u,
                                    L.mask.ptr, st));
  return FFC_OK;
}

}  // namespace ffc

using namespace ffc;

extern "C" {

ffc_status ffc_proposal_create(const float* theta_host, const float* mu_host, const float* sd_host,
                               ffc_proposal** out) {
  if (!theta_host || !out) return fail(FFC_ERR_INVALID_ARG, "theta or out is NULL");
  if (!all_finite(theta_host, kNParam) || (mu_host && !all_finite(mu_host, kNF)) ||
      (sd_host && !all_finite(sd_host, kNF)))
    return fail(FFC_ERR_INVALID_ARG, "proposal parameters must be finite");
  if (sd_host)
    for (int f = 0; f < kNF; ++f)
      if (!(sd_host[f] > 0.f)) return fail(FFC_ERR_INVALID_ARG, "standard deviations must be > 0");
  ffc_proposal* p = new ffc_proposal();
  std::vector<float> mu(kNF, 0.f), sd(kNF, 1.f), zeros(kNParam, 0.f);
  if (mu_host) std::copy(mu_host, mu_host + kNF, mu.begin());
  if (sd_host) std::copy(sd_host, sd_host + kNF, sd.begin());
  auto init = [&]() -> ffc_status {
    FFC_TRY(p->theta.alloc(kNParam));
    FFC_TRY(p->mu.alloc(kNF));
    FFC_TRY(p->sd.alloc(kNF));
    FFC_TRY(p->m1.alloc(kNParam));
    FFC_TRY(p->m2.alloc(kNParam));
    FFC_HIP_TRY(hipMemcpy(p->theta.ptr, theta_host, kNParam * sizeof(float), hipMemcpyHostToDevice));
    FFC_HIP_TRY(hipMemcpy(p->mu.ptr, mu.data(), kNF * sizeof(float), hipMemcpyHostToDevice));
    FFC_HIP_TRY(hipMemcpy(p->sd.ptr, sd.data(), kNF * sizeof(float), hipMemcpyHostToDevice));
    FFC_HIP_TRY(hipMemcpy(p->m1.ptr, zeros.data(), kNParam * sizeof(float), hipMemcpyHostToDevice));
    FFC_HIP_TRY(hipMemcpy(p->m2.ptr, zeros.data(), kNParam * sizeof(float), hipMemcpyHostToDevice));
    return FFC_OK;
  };
  const ffc_status s = init();
  if (s != FFC_OK) {
    delete p;
    return s;
  }
  *out = p;
  return FFC_OK;
}

ffc_status ffc_proposal_get_adam(const ffc_proposal* p, float* m1_host, float* m2_host, int32_t* step) {
  if (!p) return fail(FFC_ERR_INVALID_ARG, "proposal is NULL");
  FFC_HIP_TRY(hipDeviceSynchronize());
  if (m1_host) FFC_HIP_TRY(hipMemcpy(m1_host, p->m1.ptr, kNParam * sizeof(float), hipMemcpyDeviceToHost));
  if (m2_host) FFC_HIP_TRY(hipMemcpy(m2_host, p->m2.ptr, kNParam * sizeof(float), hipMemcpyDeviceToHost));
  if (step) *step = p->step;
  return FFC_OK;
}

ffc_status ffc_proposal_set_adam(ffc_proposal* p, const float* m1_host, const float* m2_host, int32_t step) {
  if (!p || !m1_host || !m2_host) return fail(FFC_ERR_INVALID_ARG, "proposal or moments are NULL");
  if (step < 0) return fail(FFC_ERR_INVALID_ARG, "step must be >= 0");
  if (!all_finite(m1_host, kNParam) || !all_finite(m2_host, kNParam))
    return fail(FFC_ERR_INVALID_ARG, "Adam moments must be finite");
  for (int i = 0; i < kNParam; ++i)
    if (m2_host[i] < 0.f) return fail(FFC_ERR_INVALID_ARG, "second moments must be >= 0");
  FFC_HIP_TRY(hipDeviceSynchronize());
  FFC_HIP_TRY(hipMemcpy(p->m1.ptr, m1_host, kNParam * sizeof(float), hipMemcpyHostToDevice));
  FFC_HIP_TRY(hipMemcpy(p->m2.ptr, m2_host, kNParam * sizeof(float), hipMemcpyHostToDevice));
  p->step = step;
  return FFC_OK;
}

ffc_status ffc_proposal_get(const ffc_proposal* p, float* theta_host, float* mu_host, float* sd_host) {
  if (!p) return fail(FFC_ERR_INVALID_ARG, "proposal is NULL");
  FFC_HIP_TRY(hipDeviceSynchronize());
  if (theta_host) FFC_HIP_TRY(hipMemcpy(theta_host, p->theta.ptr, kNParam * sizeof(float), hipMemcpyDeviceToHost));
  if (mu_host) FFC_HIP_TRY(hipMemcpy(mu_host, p->mu.ptr, kNF * sizeof(float), hipMemcpyDeviceToHost));
  if (sd_host) FFC_HIP_TRY(hipMemcpy(sd_host, p->sd.ptr, kNF * sizeof(float), hipMemcpyDeviceToHost));
  return FFC_OK;
}

void ffc_proposal_free(ffc_proposal* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  delete p;
}

// Proposal checkpoint file, version 1 (little-endian): 8-byte magic
// "FFCPROP1", uint32 version, uint32 parameter count, uint32 feature count,
// int32 Adam step, then float32 theta, mu, sd, m1, m2, then the 64-bit FNV-1a
// hash of every preceding byte.
}  // extern "C"

namespace {
constexpr char kPropMagic[8] = {'F', 'F', 'C', 'P', 'R', 'O', 'P', '1'};
constexpr uint32_t kPropVersion = 1;

uint64_t fnv1a(const unsigned char* b, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

template <typename T>
void put(std::vector<unsigned char>& buf, const T* v, size_t n) {
  const size_t at = buf.size();
  buf.resize(at + n * sizeof(T));
  std::memcpy(buf.data() + at, v, n * sizeof(T));
}
}  // namespace

extern "C" {

ffc_status ffc_proposal_save(const ffc_proposal* p, const char* path) {
  if (!p || !path) return fail(FFC_ERR_INVALID_ARG, "proposal or path is NULL");
  std::vector<float> th(kNParam), mu(kNF), sd(kNF), m1(kNParam), m2(kNParam);
  FFC_TRY(ffc_proposal_get(p, th.data(), mu.data(), sd.data()));
  int32_t step = 0;
  FFC_TRY(ffc_proposal_get_adam(p, m1.data(), m2.data(), &step));
  std::vector<unsigned char> buf;
  put(buf, kPropMagic, 8);
  const uint32_t hdr[3] = {kPropVersion, (uint32_t)kNParam, (uint32_t)kNF};
  put(buf, hdr, 3);
  put(buf, &step, 1);
  put(buf, th.data(), kNParam);
  put(buf, mu.data(), kNF);
  put(buf, sd.data(), kNF);
  put(buf, m1.data(), kNParam);
  put(buf, m2.data(), kNParam);
  const uint64_t h = fnv1a(buf.data(), buf.size());
  put(buf, &h, 1);
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(FFC_ERR_INVALID_ARG, std::string("cannot open ") + path + " for writing");
  const bool ok = std::fwrite(buf.data(), 1, buf.size(), f) == buf.size();
  if (std::fclose(f) != 0 || !ok) return fail(FFC_ERR_INVALID_ARG, std::string("cannot write ") + path);
  return FFC_OK;
}

ffc_status ffc_proposal_load(const char* path, ffc_proposal** out) {
  if (!path || !out) return fail(FFC_ERR_INVALID_ARG, "path or out is NULL");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(FFC_ERR_INVALID_ARG, std::string("cannot open ") + path);
  const size_t want = 8 + 4 * sizeof(uint32_t) + (3 * (size_t)kNParam + 2 * kNF) * sizeof(float) + sizeof(uint64_t);
  std::vector<unsigned char> buf(want + 1);
  const size_t got = std::fread(buf.data(), 1, buf.size(), f);
  std::fclose(f);
  if (got != want) return fail(FFC_ERR_INVALID_ARG, std::string(path) + ": not a proposal checkpoint (wrong size)");
  if (std::memcmp(buf.data(), kPropMagic, 8) != 0)
    return fail(FFC_ERR_INVALID_ARG, std::string(path) + ": not a proposal checkpoint (bad magic)");
  uint32_t hdr[3];
  std::memcpy(hdr, buf.data() + 8, sizeof(hdr));
  if (hdr[0] != kPropVersion)
    return fail(FFC_ERR_INVALID_ARG, std::string(path) + ": unsupported checkpoint version " + std::to_string(hdr[0]));
  if (hdr[1] != (uint32_t)kNParam || hdr[2] != (uint32_t)kNF)
    return fail(FFC_ERR_INVALID_ARG, std::string(path) + ": network shape does not match this library");
  uint64_t h = 0;
  std::memcpy(&h, buf.data() + want - sizeof(uint64_t), sizeof(h));
  if (h != fnv1a(buf.data(), want - sizeof(uint64_t)))
    return fail(FFC_ERR_INVALID_ARG, std::string(path) + ": checksum mismatch (corrupt checkpoint)");
  const unsigned char* c = buf.data() + 8 + sizeof(hdr);
  int32_t step = 0;
  std::memcpy(&step, c, sizeof(step));
  c += sizeof(step);
  std::vector<float> th(kNParam), mu(kNF), sd(kNF), m1(kNParam), m2(kNParam);
  for (std::vector<float>* v : {&th, &mu, &sd, &m1, &m2}) {
    std::memcpy(v->data(), c, v->size() * sizeof(float));
    c += v->size() * sizeof(float);
  }
  ffc_proposal* p = nullptr;
  FFC_TRY(ffc_proposal_create(th.data(), mu.data(), sd.data(), &p));
  const ffc_status s = ffc_proposal_set_adam(p, m1.data(), m2.data(), step);
  if (s != FFC_OK) {
    ffc_proposal_free(p);
    return s;
  }
  *out = p;
  return FFC_OK;
}

ffc_status ffc_proposal_features(const ffc_tree* t, const int32_t* cols_dev, int32_t col_stride,
                                 const int32_t* ncols_dev, const int32_t* ids_dev, const int32_t* tgt_dev,
                                 int32_t tgt_stride, const int32_t* ntgt_dev, int32_t count, uint64_t seed,
                                 float* feat_dev, void* stream) {
  if (!t) return fail(FFC_ERR_INVALID_ARG, "tree is NULL");
  if (count < 0 || col_stride < 1 || tgt_stride < 1) return fail(FFC_ERR_INVALID_ARG, "bad count or strides");
  if (count == 0) return FFC_OK;
  if (!cols_dev || !ncols_dev || !ids_dev || !tgt_dev || !ntgt_dev || !feat_dev)
    return fail(FFC_ERR_INVALID_ARG, "NULL array");
  hipStream_t st = (hipStream_t)stream;
  GeomScratch gs;
  FFC_TRY(gs.alloc(count, t->d));
  const GeomArgs ga = gs.args(cols_dev, col_stride, ncols_dev, ids_dev, seed);
  FFC_TRY(launch_geometry(t->Xt.ptr, t->d, ga, count, st));
  FFC_TRY(launch_features(t->Xt.ptr, t->d, ga, tgt_dev, tgt_stride, ntgt_dev, count, feat_dev,
                          (int64_t)tgt_stride * kNF, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));
  return FFC_OK;
}

ffc_status ffc_proposal_fit_standardization(ffc_proposal* p, const float* feat_dev, int64_t count, void* stream) {
  if (!p || !feat_dev) return fail(FFC_ERR_INVALID_ARG, "proposal or features is NULL");
  if (count < 1) return fail(FFC_ERR_INVALID_ARG, "count must be >= 1");
  return launch_feature_stats(feat_dev, count, p->mu.ptr, p->sd.ptr, (hipStream_t)stream);
}

ffc_status ffc_proposal_score(const ffc_proposal* p, const float* feat_dev, int64_t count, float* score_dev,
                              void* stream) {
  if (!p) return fail(FFC_ERR_INVALID_ARG, "proposal is NULL");
  if (count < 0) return fail(FFC_ERR_INVALID_ARG, "count must be >= 0");
  if (count == 0) return FFC_OK;
  if (!feat_dev || !score_dev) return fail(FFC_ERR_INVALID_ARG, "NULL array");
  return launch_mlp_score(p->theta.ptr, p->mu.ptr, p->sd.ptr, feat_dev, count, score_dev, (hipStream_t)stream);
}

ffc_status ffc_proposal_gradient(const ffc_proposal* p, const float* feat_dev, const float* target_dev,
                                 int64_t count, float* grad_dev, float* loss_dev, void* stream) {
  if (!p) return fail(FFC_ERR_INVALID_ARG, "proposal is NULL");
  if (count < 1) return fail(FFC_ERR_INVALID_ARG, "count must be >= 1");
  if (!feat_dev || !target_dev || !grad_dev || !loss_dev) return fail(FFC_ERR_INVALID_ARG, "NULL array");
  hipStream_t st = (hipStream_t)stream;
  DevBuf<float> partial;
  ffc_proposal* pm = const_cast<ffc_proposal*>(p);   // parameters are read only (adam = false)
  FFC_TRY(grad_step(p, pm->theta.ptr, nullptr, nullptr, feat_dev, target_dev, count, 0, 1, count, partial, grad_dev,
                    loss_dev, false, 0.f, 1, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));
  return FFC_OK;
}

ffc_status ffc_proposal_adam(ffc_proposal* p, const float* grad_dev, float lr, void* stream) {
  if (!p || !grad_dev) return fail(FFC_ERR_INVALID_ARG, "proposal or gradient is NULL");
  if (!(lr > 0.f) || !std::isfinite(lr)) return fail(FFC_ERR_INVALID_ARG, "lr must be > 0");
  // One "workgroup" row: the kernel reads grad_dev[0 .. NPARAM).
  return launch_grad_reduce_adam(grad_dev, 1, p->theta.ptr, p->m1.ptr, p->m2.ptr, nullptr, nullptr, true, lr,
                                 ++p->step, 1, (hipStream_t)stream);
}

ffc_status ffc_leverage_labels(const double* B_dev, int64_t m, int32_t n, int32_t count, double eps,
                               double* lev_dev, float* target_dev, void* stream) {
  if (m < 1 || n < 1 || count < 0) return fail(FFC_ERR_INVALID_ARG, "m and n must be >= 1, count >= 0");
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(FFC_ERR_INVALID_ARG, "eps must be > 0");
  if (count == 0) return FFC_OK;
  if (!B_dev || !lev_dev) return fail(FFC_ERR_INVALID_ARG, "B or lev is NULL");
  hipStream_t st = (hipStream_t)stream;
  DevBuf<double> B, G;
  DevBuf<int> status;
  FFC_TRY(B.alloc((size_t)count * m * n));
  FFC_TRY(G.alloc((size_t)count * n * n));
  FFC_TRY(status.alloc(count));
  FFC_HIP_TRY(hipMemcpyAsync(B.ptr, B_dev, (size_t)count * m * n * sizeof(double), hipMemcpyDeviceToDevice, st));
  FFC_TRY(launch_ridge_leverage(B.ptr, m, n, count, G.ptr, eps, lev_dev, target_dev, status.ptr, st));
  std::vector<int> sh(count);
  FFC_HIP_TRY(hipMemcpyAsync(sh.data(), status.ptr, count * sizeof(int), hipMemcpyDeviceToHost, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));
  for (int g = 0; g < count; ++g)
    if (sh[g] == 2) return fail(FFC_ERR_NONFINITE, "leverage labels: Cholesky factorization failed");
  return FFC_OK;
}

ffc_status ffc_pivoted_leverage_labels(const double* B_dev, int64_t m, int32_t n, int32_t count, double eps,
                                       double* lev_dev, float* target_dev, int32_t* rank_host, int32_t* piv_host,
                                       void* stream) {
  if (m < 1 || n < 1 || count < 0) return fail(FFC_ERR_INVALID_ARG, "m and n must be >= 1, count >= 0");
  if (n > 1024) return fail(FFC_ERR_INVALID_ARG, "pivoted leverage supports n <= 1024");
  if (!(eps > 0.0) || !(eps < 1.0)) return fail(FFC_ERR_INVALID_ARG, "eps must be in (0, 1)");
  if (count == 0) return FFC_OK;
  if (!B_dev || !lev_dev) return fail(FFC_ERR_INVALID_ARG, "B or lev is NULL");
  hipStream_t st = (hipStream_t)stream;
  DevBuf<double> B, G, Lc;
  DevBuf<int> status, perm, rank;
  FFC_TRY(B.alloc((size_t)count * m * n));
  FFC_TRY(G.alloc((size_t)count * n * n));
  FFC_TRY(Lc.alloc((size_t)count * n * n));
  FFC_TRY(status.alloc(count));
  FFC_TRY(perm.alloc((size_t)count * n));
  FFC_TRY(rank.alloc(count));
  FFC_HIP_TRY(hipMemcpyAsync(B.ptr, B_dev, (size_t)count * m * n * sizeof(double), hipMemcpyDeviceToDevice, st));
  FFC_TRY(launch_pivoted_leverage(B.ptr, m, n, count, G.ptr, Lc.ptr, perm.ptr, rank.ptr, eps, lev_dev, target_dev,
                                  status.ptr, st));
  std::vector<int> rh(count);
  FFC_HIP_TRY(hipMemcpyAsync(rh.data(), rank.ptr, count * sizeof(int), hipMemcpyDeviceToHost, st));
  if (piv_host)
    FFC_HIP_TRY(hipMemcpyAsync(piv_host, perm.ptr, (size_t)count * n * sizeof(int), hipMemcpyDeviceToHost, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));
  if (rank_host) std::copy(rh.begin(), rh.end(), rank_host);
  return FFC_OK;
}

ffc_status ffc_proposal_training_set(const ffc_tree* t, const ffc_kernel* k, const ffc_train_opts* o,
                                     int32_t* n_out, int32_t* m_out, int32_t* leaves_dev, int32_t* cols_dev,
                                     int32_t* rows_dev, float* feat_dev, float* target_dev, double* lev_dev,
                                     void* stream) {
  FFC_TRY(check_train_opts(t, k, o));
  int n = 0, m = 0;
  FFC_TRY(train_sizes(t, o, n, m));
  if (n_out) *n_out = n;
  if (m_out) *m_out = m;
  if (!leaves_dev && !cols_dev && !rows_dev && !feat_dev && !target_dev && !lev_dev) return FFC_OK;
  hipStream_t st = (hipStream_t)stream;
  TrainSet ts;
  FFC_TRY(build_training_set(t, k, o, ts, st));
  const size_t G = ts.G, C = G * m;
  if (leaves_dev) FFC_HIP_TRY(hipMemcpyAsync(leaves_dev, ts.leaves.ptr, G * 4, hipMemcpyDeviceToDevice, st));
  if (cols_dev) FFC_HIP_TRY(hipMemcpyAsync(cols_dev, ts.cols.ptr, G * n * 4, hipMemcpyDeviceToDevice, st));
  if (rows_dev) FFC_HIP_TRY(hipMemcpyAsync(rows_dev, ts.rows.ptr, G * m * 4, hipMemcpyDeviceToDevice, st));
  if (feat_dev) FFC_HIP_TRY(hipMemcpyAsync(feat_dev, ts.feat.ptr, C * kNF * 4, hipMemcpyDeviceToDevice, st));
  if (target_dev) FFC_HIP_TRY(hipMemcpyAsync(target_dev, ts.target.ptr, C * 4, hipMemcpyDeviceToDevice, st));
  if (lev_dev) FFC_HIP_TRY(hipMemcpyAsync(lev_dev, ts.lev.ptr, C * 8, hipMemcpyDeviceToDevice, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));
  return FFC_OK;
}

ffc_status ffc_proposal_train(ffc_proposal* p, const ffc_tree* t, const ffc_kernel* k, const ffc_train_opts* o,
                              float* loss_host, void* stream) {
  if (!p) return fail(FFC_ERR_INVALID_ARG, "proposal is NULL");
  FFC_TRY(check_train_opts(t, k, o));
  hipStream_t st = (hipStream_t)stream;
  TrainSet ts;
  FFC_TRY(build_training_set(t, k, o, ts, st));
  const int64_t C = (int64_t)ts.G * ts.m;
  FFC_TRY(launch_feature_stats(ts.feat.ptr, C, p->mu.ptr, p->sd.ptr, st));
  const int64_t steps_per_epoch = (C + o->batch - 1) / o->batch;
  DevBuf<float> step_loss, partial;
  FFC_TRY(step_loss.alloc((size_t)std::max<int64_t>(1, steps_per_epoch * o->epochs)));
  int64_t si = 0;
  FFC_TRY(partial.alloc((size_t)((std::min<int64_t>(o->batch, C) + kGradBatch - 1) / kGradBatch) * (kNParam + 1)));
  {
    StageTimer timer(FFC_STAGE_TRAIN, st);
    for (int e = 0; e < o->epochs; ++e) {
      const int64_t stride = epoch_stride(C, o->seed, e);
      for (int64_t p0 = 0; p0 < C; p0 += o->batch, ++si) {
        const int64_t bs = std::min<int64_t>(o->batch, C - p0);
        FFC_TRY(grad_step(p, p->theta.ptr, p->m1.ptr, p->m2.ptr, ts.feat.ptr, ts.target.ptr, C, p0, stride, bs,
                          partial, nullptr, step_loss.ptr + si, true, o->lr, ++p->step, st));
      }
    }
  }
  std::vector<float> sl((size_t)si);
  if (si) FFC_HIP_TRY(hipMemcpyAsync(sl.data(), step_loss.ptr, si * sizeof(float), hipMemcpyDeviceToHost, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));
  if (loss_host) {
    for (int e = 0; e < o->epochs; ++e) {
      double acc = 0.0;
      for (int64_t j = 0; j < steps_per_epoch; ++j) {
        const int64_t bs = std::min<int64_t>(o->batch, C - j * o->batch);
        acc += (double)sl[e * steps_per_epoch + j] * bs;
      }
      loss_host[e] = (float)(acc / C);
    }
  }
  return FFC_OK;
}

}  // extern "C"
