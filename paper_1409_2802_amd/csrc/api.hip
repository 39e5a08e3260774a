// C ABI of the far-field compression library: argument validation, handle
// management and the level-by-level schedule of the skeletonization.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "ffc_internal.h"

namespace ffc {

namespace {
thread_local std::string g_error;
std::mutex g_flag_mu;
unsigned int* g_flags[64] = {};   // per device: address of g_device_flag
// The device error flag word (bit 0: a non-finite kernel value, bit 1: a QR
// wait timed out). A file-scope device variable, so reading the flag never
// allocates; each device holds its own copy, zero at load.
__device__ unsigned int g_device_flag = 0u;

ffc_status fail(ffc_status code, const std::string& msg) {
  set_error(msg);
  return code;
}

ffc_status check_kernel(const ffc_kernel* k, int d) {
  if (!k) return fail(FFC_ERR_INVALID_ARG, "kernel is NULL");
  if (k->kind != FFC_GAUSSIAN && k->kind != FFC_LAPLACE && k->kind != FFC_POLYNOMIAL)
    return fail(FFC_ERR_INVALID_ARG, "unknown kernel kind");
  if (k->kind != FFC_LAPLACE && !(k->h > 0.0) )
    return fail(FFC_ERR_INVALID_ARG, "kernel bandwidth h must be > 0");
  if (k->kind == FFC_POLYNOMIAL && k->p < 1) return fail(FFC_ERR_INVALID_ARG, "polynomial degree p must be >= 1");
  if (k->kind == FFC_LAPLACE && d < 3)
    return fail(FFC_ERR_INVALID_ARG, "the Laplace kernel needs d >= 3 (the d = 2 logarithmic form is not provided)");
  return FFC_OK;
}

ffc_status check_precision(int p) {
  if (p != FFC_FP64 && p != FFC_FP32 && p != FFC_MIXED_BF16X3) return fail(FFC_ERR_INVALID_ARG, "unknown precision");
  return FFC_OK;
}

int tree_depth(int64_t N, int leaf) {
  int D = 0;
  while ((N + (int64_t(1) << D) - 1) / (int64_t(1) << D) > leaf) ++D;
  return D;
}

ffc_status finish_tree_common(ffc_tree* t, hipStream_t st) {
  FFC_TRY(t->begin.alloc(t->num_nodes));
  FFC_TRY(t->end.alloc(t->num_nodes));
  FFC_HIP_TRY(hipMemcpyAsync(t->begin.ptr, t->begin_h.data(), t->num_nodes * sizeof(int32_t), hipMemcpyHostToDevice, st));
  FFC_HIP_TRY(hipMemcpyAsync(t->end.ptr, t->end_h.data(), t->num_nodes * sizeof(int32_t), hipMemcpyHostToDevice, st));
  FFC_TRY(t->perm.alloc(t->N));
  FFC_TRY(t->Xt.alloc((size_t)t->N * t->d));
  FFC_TRY(t->centroid.alloc((size_t)t->num_nodes * t->d));
  FFC_TRY(t->radius.alloc(t->num_nodes));
  FFC_TRY(t->q_tree.alloc(t->N));
  // Evaluation tiles: blocks of up to 64 consecutive targets inside one leaf.
  t->tile_rows = 64;
  std::vector<int32_t> tl, ts;
  const int first_leaf = (1 << t->depth) - 1;
  for (int a = first_leaf; a < t->num_nodes; ++a)
    for (int x = t->begin_h[a]; x < t->end_h[a]; x += t->tile_rows) {
      tl.push_back(a);
      ts.push_back(x);
    }
  t->num_tiles = (int32_t)tl.size();
  FFC_TRY(t->tile_leaf.alloc(std::max<size_t>(1, tl.size())));
  FFC_TRY(t->tile_start.alloc(std::max<size_t>(1, ts.size())));
  FFC_HIP_TRY(hipMemcpyAsync(t->tile_leaf.ptr, tl.data(), tl.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  FFC_HIP_TRY(hipMemcpyAsync(t->tile_start.ptr, ts.data(), ts.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));   // host vectors go out of scope
  return FFC_OK;
}

}  // namespace

void set_error(const std::string& msg) { g_error = msg; }

ffc_status refuse_pinned_alloc() {
  set_error("a step graph holds this handle's device buffers: free the graph (ffc_graph_free) before a call that "
            "would resize or replace them (another separation, sampler, pool or sample count, new FMM lists)");
  return FFC_ERR_STATE;
}

ffc_status validate_kernel(const ffc_kernel* k, int d) { return check_kernel(k, d); }

bool alloc_forced_to_fail() {
  const char* e = std::getenv("FFC_FAIL_ALLOC");
  return e && e[0] == '1';
}

KParams make_kparams(const ffc_kernel& k, int d) {
  KParams p{};
  p.kind = k.kind;
  p.p = k.p;
  p.inv_h = k.kind == FFC_LAPLACE ? 1.0 : 1.0 / k.h;
  p.c = k.c;
  p.neg_inv_2h2 = k.kind == FFC_LAPLACE ? 0.0 : -1.0 / (2.0 * k.h * k.h);
  p.lap_expo = (2.0 - d) / 2.0;
  p.lap_small = k.kind == FFC_LAPLACE && d <= 7;
  p.lap_m = (d & 1) ? d - 2 : (d - 2) / 2;
  p.lap_odd = d & 1;
  return p;
}

unsigned int* device_flag() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  std::lock_guard<std::mutex> lock(g_flag_mu);
  if (!g_flags[dev]) {   // this device's copy of the file-scope word (nothing is allocated)
    unsigned int* p = nullptr;
    if (hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(g_device_flag)) != hipSuccess || !p)
      return nullptr;
    g_flags[dev] = p;
  }
  return g_flags[dev];
}

}  // namespace ffc

using namespace ffc;

extern "C" {

const char* ffc_last_error(void) { return g_error.c_str(); }

ffc_status ffc_build_tree(const double* X_dev, int64_t N, int32_t d, int32_t leaf_size, void* stream,
                          ffc_tree** out) {
  if (!out) return fail(FFC_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!X_dev) return fail(FFC_ERR_INVALID_ARG, "X is NULL");
  if (N < 1 || N > INT32_MAX / 2) return fail(FFC_ERR_INVALID_ARG, "N must be in [1, 2^30]");
  if (d < 1) return fail(FFC_ERR_INVALID_ARG, "d must be >= 1");
  if (leaf_size < 1) return fail(FFC_ERR_INVALID_ARG, "leaf_size must be >= 1");
  const int D = tree_depth(N, leaf_size);
  if (D > 24) return fail(FFC_ERR_INVALID_ARG, "tree deeper than 24 levels: increase leaf_size");
  if (!device_flag()) return fail(FFC_ERR_HIP, "cannot allocate the device flag");
  hipStream_t st = (hipStream_t)stream;
  auto t = new ffc_tree();
  t->N = N;
  t->d = d;
  t->depth = D;
  t->num_nodes = (1 << (D + 1)) - 1;
  t->begin_h.assign(t->num_nodes, 0);
  t->end_h.assign(t->num_nodes, 0);
  t->end_h[0] = (int32_t)N;
  for (int a = 0; a < (1 << D) - 1; ++a) {
    const int b = t->begin_h[a], e = t->end_h[a], nl = (e - b + 1) / 2;
    t->begin_h[2 * a + 1] = b;
    t->end_h[2 * a + 1] = b + nl;
    t->begin_h[2 * a + 2] = b + nl;
    t->end_h[2 * a + 2] = e;
  }
  ffc_status s = t->X.alloc((size_t)N * d);
  if (s == FFC_OK) {
    hipError_t e = hipMemcpyAsync(t->X.ptr, X_dev, (size_t)N * d * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) s = fail(FFC_ERR_HIP, std::string("copy of X: ") + hipGetErrorString(e));
  }
  if (s == FFC_OK) s = finish_tree_common(t, st);
  if (s == FFC_OK) {
    StageTimer timer(FFC_STAGE_TREE, st);
    s = launch_build_tree(t, leaf_size, st);
  }
  if (s != FFC_OK) {
    delete t;
    return s;
  }
  t->last_stream = st;
  *out = t;
  return FFC_OK;
}

ffc_status ffc_build_partition(const double* X_dev, int64_t N, int32_t d, int64_t n_left, void* stream,
                               ffc_tree** out) {
  if (!out) return fail(FFC_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!X_dev) return fail(FFC_ERR_INVALID_ARG, "X is NULL");
  if (N < 2 || N > INT32_MAX / 2) return fail(FFC_ERR_INVALID_ARG, "N must be in [2, 2^30]");
  if (d < 1) return fail(FFC_ERR_INVALID_ARG, "d must be >= 1");
  if (n_left < 1 || n_left >= N) return fail(FFC_ERR_INVALID_ARG, "n_left must be in [1, N)");
  if (!device_flag()) return fail(FFC_ERR_HIP, "cannot allocate the device flag");
  hipStream_t st = (hipStream_t)stream;
  auto t = new ffc_tree();
  t->N = N;
  t->d = d;
  t->depth = 1;
  t->num_nodes = 3;
  t->begin_h = {0, 0, (int32_t)n_left};
  t->end_h = {(int32_t)N, (int32_t)n_left, (int32_t)N};
  ffc_status s = t->X.alloc((size_t)N * d);
  if (s == FFC_OK) {
    hipError_t e = hipMemcpyAsync(t->X.ptr, X_dev, (size_t)N * d * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) s = fail(FFC_ERR_HIP, std::string("copy of X: ") + hipGetErrorString(e));
  }
  if (s == FFC_OK) s = finish_tree_common(t, st);
  if (s == FFC_OK) {
    std::vector<int32_t> iota(N);
    for (int64_t i = 0; i < N; ++i) iota[i] = (int32_t)i;
    hipError_t e = hipMemcpy(t->perm.ptr, iota.data(), N * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) s = fail(FFC_ERR_HIP, std::string("perm upload: ") + hipGetErrorString(e));
  }
  if (s == FFC_OK) s = launch_node_stats(t, 0, st);
  if (s == FFC_OK) s = launch_node_stats(t, 1, st);
  if (s == FFC_OK) s = launch_gather_tree_points(t, st);
  if (s != FFC_OK) {
    delete t;
    return s;
  }
  t->last_stream = st;
  *out = t;
  return FFC_OK;
}

ffc_status ffc_tree_info(const ffc_tree* t, int32_t* depth, int32_t* num_nodes, int64_t* N, int32_t* d) {
  if (!t) return fail(FFC_ERR_INVALID_ARG, "tree is NULL");
  if (depth) *depth = t->depth;
  if (num_nodes) *num_nodes = t->num_nodes;
  if (N) *N = t->N;
  if (d) *d = t->d;
  return FFC_OK;
}

ffc_status ffc_tree_arrays(const ffc_tree* t, int32_t* perm_host, int64_t* begin_host, int64_t* end_host,
                           double* centroid_host, double* radius_host) {
  if (!t) return fail(FFC_ERR_INVALID_ARG, "tree is NULL");
  FFC_HIP_TRY(hipStreamSynchronize(t->last_stream));
  if (perm_host) FFC_HIP_TRY(hipMemcpy(perm_host, t->perm.ptr, t->N * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int a = 0; a < t->num_nodes; ++a) {
    if (begin_host) begin_host[a] = t->begin_h[a];
    if (end_host) end_host[a] = t->end_h[a];
  }
  if (centroid_host)
    FFC_HIP_TRY(hipMemcpy(centroid_host, t->centroid.ptr, (size_t)t->num_nodes * t->d * sizeof(double),
                          hipMemcpyDeviceToHost));
  if (radius_host)
    FFC_HIP_TRY(hipMemcpy(radius_host, t->radius.ptr, t->num_nodes * sizeof(double), hipMemcpyDeviceToHost));
  return FFC_OK;
}

ffc_status ffc_skeletonize_nodes(const ffc_tree* t, const ffc_kernel* k, const ffc_skel_opts* o,
                                 const int32_t* node_ids_host, int32_t num_ids, void* stream, ffc_skel** out) {
  if (!t) return fail(FFC_ERR_INVALID_ARG, "tree is NULL");
  if (!o) return fail(FFC_ERR_INVALID_ARG, "options are NULL");
  if (!out) return fail(FFC_ERR_INVALID_ARG, "out is NULL");
  FFC_TRY(check_kernel(k, t->d));
  FFC_TRY(check_precision(o->precision));
  if (!(o->tol >= 0.0)) return fail(FFC_ERR_INVALID_ARG, "tol must be >= 0");
  if (o->max_rank < 1) return fail(FFC_ERR_INVALID_ARG, "max_rank must be >= 1");
  if (o->num_samples < 0) return fail(FFC_ERR_INVALID_ARG, "num_samples must be >= 0");
  if (o->sampler < FFC_SAMPLE_UNIFORM || o->sampler > FFC_SAMPLE_NEAREST)
    return fail(FFC_ERR_INVALID_ARG, "unknown sampler");
  // Every sampler but the uniform one draws from a candidate pool (learned proposal, distance, nearest).
  const bool learned = o->sampler != FFC_SAMPLE_UNIFORM;
  if (o->sampler == FFC_SAMPLE_LEARNED && !o->proposal)
    return fail(FFC_ERR_INVALID_ARG, "the learned sampler needs a proposal");
  if (learned && !std::isfinite(o->fallback_tol)) return fail(FFC_ERR_INVALID_ARG, "fallback_tol must be finite");
  if (learned && o->pool_factor < 0) return fail(FFC_ERR_INVALID_ARG, "pool_factor must be >= 0");
  if (!std::isfinite(o->adaptive_tol)) return fail(FFC_ERR_INVALID_ARG, "adaptive_tol must be finite");
  const bool adaptive = o->adaptive_tol > 0.0;
  if (adaptive && learned)
    return fail(FFC_ERR_INVALID_ARG, "the adaptive sample count works with the uniform sampler only");
  if (o->max_samples < 0) return fail(FFC_ERR_INVALID_ARG, "max_samples must be >= 0");
  if (!(o->separation >= 0.0)) return fail(FFC_ERR_INVALID_ARG, "separation must be >= 0");
  const bool separated = o->separation > 0.0;
  if (separated && (learned || adaptive))
    return fail(FFC_ERR_INVALID_ARG, "separation works with the uniform sampler and a fixed sample count only");
  if (separated && t->depth > 30) return fail(FFC_ERR_INVALID_ARG, "separation supports trees of depth <= 30");
  // Node subset: a host byte per node, set for the listed ones.
  const bool subset = node_ids_host != nullptr;
  std::vector<unsigned char> listed;
  std::vector<int> level_listed(t->depth + 1, 0);
  if (subset) {
    if (num_ids < 1) return fail(FFC_ERR_INVALID_ARG, "num_ids must be >= 1 with a node list");
    if (learned || adaptive)
      return fail(FFC_ERR_INVALID_ARG, "a node subset works with the uniform sampler and a fixed sample count only");
    listed.assign(t->num_nodes, 0);
    for (int32_t i = 0; i < num_ids; ++i) {
      const int32_t a = node_ids_host[i];
      if (a < 1 || a >= t->num_nodes) return fail(FFC_ERR_INVALID_ARG, "node id out of range (the root has no far field)");
      if (listed[a]) return fail(FFC_ERR_INVALID_ARG, "node id listed twice");
      listed[a] = 1;
      int lev = 0;
      while (((2 << lev) - 1) <= a) ++lev;
      level_listed[lev] += 1;
    }
  } else if (num_ids != 0) {
    return fail(FFC_ERR_INVALID_ARG, "num_ids must be 0 without a node list");
  }
  hipStream_t st = (hipStream_t)stream;

  const int64_t s_req = o->num_samples > 0 ? o->num_samples : 2 * (int64_t)o->max_rank;
  // Adaptive sample count: rows start at s_req and double up to s_lim.
  const int64_t s_lim = adaptive ? (o->max_samples > 0 ? o->max_samples : 4 * s_req) : s_req;
  if (s_lim < s_req) return fail(FFC_ERR_INVALID_ARG, "max_samples must be >= the initial sample count");
  int max_leaf = 0;
  for (int a = (1 << t->depth) - 1; a < t->num_nodes; ++a) max_leaf = std::max(max_leaf, t->end_h[a] - t->begin_h[a]);
  int max_nonroot = 0;
  for (int a = 1; a < t->num_nodes; ++a) max_nonroot = std::max(max_nonroot, t->end_h[a] - t->begin_h[a]);
  const int64_t M_max = t->N - 0;   // largest complement (an empty node)
  if (s_lim > 8192) return fail(FFC_ERR_INVALID_ARG, "num_samples (or max_samples) above 8192 is not supported");
  const int s_cap = (int)std::min<int64_t>(s_lim, M_max);
  const int s0 = (int)std::min<int64_t>(s_req, M_max);   // rows drawn first
  const int r_cap = std::max(1, std::min(o->max_rank, s_cap));
  const int n_cap = std::max(max_leaf, 2 * r_cap);
  if ((size_t)n_cap * 12 + (size_t)s_cap * 8 > 140 * 1024)
    return fail(FFC_ERR_INVALID_ARG, "node too large for the QR kernel (leaf_size or 2*max_rank above ~11000)");

  ffc_skel* sk = *out;
  const bool reuse = sk != nullptr;
  if (reuse && !(sk->num_nodes == t->num_nodes && sk->depth == t->depth && sk->s_cap == s_cap &&
                 sk->n_cap == n_cap && sk->r_cap == r_cap))
    return fail(FFC_ERR_STATE, "the skeleton handle passed in was made for another tree or sample count / rank cap");
  if (!reuse) {
    sk = new ffc_skel();
    sk->num_nodes = t->num_nodes;
    sk->depth = t->depth;
    sk->s_cap = s_cap;
    sk->n_cap = n_cap;
    sk->r_cap = r_cap;
    const size_t nn = t->num_nodes;
    ffc_status s = FFC_OK;
    if (s == FFC_OK) s = sk->rank.alloc(nn);
    if (s == FFC_OK) s = sk->ncols.alloc(nn);
    if (s == FFC_OK) s = sk->nrows.alloc(nn);
    if (s == FFC_OK) s = sk->cols.alloc(nn * n_cap);
    if (s == FFC_OK) s = sk->rows.alloc(nn * s_cap);
    if (s == FFC_OK) s = sk->piv.alloc(nn * n_cap);
    if (s == FFC_OK) s = sk->skel.alloc(nn * r_cap);
    if (s == FFC_OK) s = sk->P.alloc(nn * r_cap * n_cap);
    if (s == FFC_OK) s = sk->qt.alloc(nn * r_cap);
    size_t work = 0;
    for (int lev = 1; lev <= t->depth; ++lev) work = std::max(work, ((size_t)1 << lev) * s_cap * n_cap);
    if (s == FFC_OK) s = sk->work.alloc(work);
    if (s != FFC_OK) {
      delete sk;
      return s;
    }
    FFC_HIP_TRY(hipMemsetAsync(sk->rank.ptr, 0, nn * sizeof(int32_t), st));
    FFC_HIP_TRY(hipMemsetAsync(sk->ncols.ptr, 0, nn * sizeof(int32_t), st));
    FFC_HIP_TRY(hipMemsetAsync(sk->nrows.ptr, 0, nn * sizeof(int32_t), st));
  }
  const unsigned char* smask = nullptr;   // device copy of `listed`
  if (subset) {
    if (sk->subset.count != (size_t)t->num_nodes) {
      const ffc_status sa = sk->subset.alloc(t->num_nodes);
      if (sa != FFC_OK) {
        if (!reuse) delete sk;
        return sa;
      }
    }
    FFC_HIP_TRY(hipMemcpyAsync(sk->subset.ptr, listed.data(), listed.size(), hipMemcpyHostToDevice, st));
    FFC_HIP_TRY(hipStreamSynchronize(st));   // `listed` is pageable host memory that ends with this call
    smask = sk->subset.ptr;
  }
  sk->kernel = *k;
  sk->opts = *o;
  sk->fallbacks = 0;
  sk->resampled = 0;
  const KParams kp = make_kparams(*k, t->d);
  const int max_rank = std::min(o->max_rank, r_cap);
  // Sampled blocks, interpolative decompositions and skeleton ids of one level
  // (rows and columns already in place).
  // With a mask (indexed by node) only the nodes whose entry is set are redone.
  auto skeletonize_level = [&](int first, int count, const unsigned char* mask = nullptr) -> ffc_status {
    {
      StageTimer tm(FFC_STAGE_KBLOCK, st);
      FFC_TRY(launch_level_kblock(t, sk, kp, o->precision, first, count, sk->work.ptr, st, mask));
    }
    IdBatch bt{};
    bt.A = sk->work.ptr;
    bt.a_stride = (int64_t)s_cap * n_cap;
    bt.lda = s_cap;
    bt.s_arr = sk->nrows.ptr + first;
    bt.n_arr = sk->ncols.ptr + first;
    bt.s_max = s_cap;
    bt.n_max = n_cap;
    bt.tol = o->tol;
    bt.max_rank = max_rank;
    bt.rank = sk->rank.ptr + first;
    bt.piv = sk->piv.ptr + (int64_t)first * n_cap;
    bt.piv_stride = n_cap;
    bt.P = sk->P.ptr + (int64_t)first * r_cap * n_cap;
    bt.p_stride = (int64_t)r_cap * n_cap;
    bt.p_ld = n_cap;
    bt.mask = mask ? mask + first : nullptr;
    {
      bool used = false;
      FFC_TRY(launch_interp_decomp_coop(bt, count, sk->qr_scratch, st, used));
      if (!used) {
        StageTimer tm(FFC_STAGE_CPQR, st);
        FFC_TRY(launch_interp_decomp(bt, count, st));
      }
    }
    {
      StageTimer tm(FFC_STAGE_SKEL, st);
      FFC_TRY(launch_skeleton_ids(sk, first, count, st, mask));
    }
    return FFC_OK;
  };
  auto run = [&]() -> ffc_status {
    if (learned) FFC_TRY(learned_alloc(t, sk, o->pool_factor > 0 ? o->pool_factor : 8));
    if (adaptive) FFC_TRY(heldout_alloc(t, sk));
    if (separated) {
      StageTimer tm(FFC_STAGE_SAMPLE, st);
      FFC_TRY(launch_separation(t, sk, o->separation, st));
    }
    for (int lev = t->depth; lev >= 1; --lev) {
      const int first = (1 << lev) - 1, count = 1 << lev;
      if (subset && !level_listed[lev]) continue;
      {
        StageTimer tm(FFC_STAGE_COLUMNS, st);
        FFC_TRY(launch_level_columns(t, sk, first, count, lev == t->depth, st, smask));
      }
      if (learned) {
        StageTimer tm(FFC_STAGE_PROPOSAL, st);
        FFC_TRY(learned_rows_level(t, sk, o->sampler, o->proposal, first, count, s_cap, o->seed, st));
      } else if (separated) {
        StageTimer tm(FFC_STAGE_SAMPLE, st);
        FFC_TRY(launch_sample_rows_sep(t, sk, first, count, s0, o->seed, st, smask));
      } else {
        StageTimer tm(FFC_STAGE_SAMPLE, st);
        FFC_TRY(launch_sample_rows(t, sk, first, count, s0, o->seed, st, smask));
      }
      FFC_TRY(skeletonize_level(first, count, smask));
      if (adaptive) {
        // Double the rows of the nodes whose held-out estimate is too large
        // until all pass or reach the cap; a round redoes only those nodes
        // (mask). They all had the previous round's count (the others passed
        // earlier and keep their skeletons), so one count per round serves.
        {
          StageTimer tm(FFC_STAGE_HELDOUT, st);
          FFC_TRY(heldout_prepare_level(t, sk, kp, o->precision, first, count, o->seed, st));
        }
        for (int s_round = s0;;) {
          const int s_next = (int)std::min<int64_t>(2 * (int64_t)s_round, s_cap);
          int redo = 0;
          {
            StageTimer tm(FFC_STAGE_HELDOUT, st);
            FFC_TRY(adaptive_round_level(t, sk, first, count, o->seed, o->adaptive_tol, s_cap, s_next, redo, st));
          }
          if (!redo) break;
          sk->resampled += redo;
          s_round = s_next;
          FFC_TRY(skeletonize_level(first, count, sk->learned.mask.ptr));
        }
      }
      if (learned && o->fallback_tol > 0.0) {
        int redo = 0;
        {
          StageTimer tm(FFC_STAGE_HELDOUT, st);
          FFC_TRY(learned_heldout_level(t, sk, kp, o->precision, first, count, s_cap, o->seed, o->fallback_tol, redo,
                                        st));
        }
        if (redo) {   // failed nodes now hold uniform rows and are redone alone (mask)
          sk->fallbacks += redo;
          FFC_TRY(skeletonize_level(first, count, sk->learned.mask.ptr));
        }
      }
    }
    return FFC_OK;
  };
  ffc_status s = run();
  if (s != FFC_OK) {
    if (!reuse) delete sk;
    return s;
  }
  sk->last_stream = st;
  *out = sk;
  return FFC_OK;
}

ffc_status ffc_evaluate_sum(const ffc_tree* t, const ffc_skel* sk, const ffc_kernel* k, const double* q_dev,
                            double* u_dev, double* u_far_dev, int32_t precision, void* stream) {
  if (!t || !sk) return fail(FFC_ERR_INVALID_ARG, "tree or skeleton is NULL");
  if (!q_dev || !u_dev) return fail(FFC_ERR_INVALID_ARG, "q or u is NULL");
  if (sk->num_nodes != t->num_nodes || sk->depth != t->depth)
    return fail(FFC_ERR_STATE, "skeleton set does not belong to this tree");
  FFC_TRY(check_kernel(k, t->d));
  FFC_TRY(check_precision(precision));
  hipStream_t st = (hipStream_t)stream;
  ffc_tree* tm = const_cast<ffc_tree*>(t);
  ffc_skel* sm = const_cast<ffc_skel*>(sk);
  {
    StageTimer timer(FFC_STAGE_UPWARD, st);
    FFC_TRY(launch_charges_to_tree(tm, q_dev, st));
    for (int lev = t->depth; lev >= 1; --lev)
      FFC_TRY(launch_upward(t, sm, (1 << lev) - 1, 1 << lev, lev == t->depth, st));
  }
  {
    StageTimer timer(FFC_STAGE_EVALUATE, st);
    if (sk->opts.separation > 0.0)
      FFC_TRY(launch_treecode(t, sk, make_kparams(*k, t->d), precision, u_dev, u_far_dev, st));
    else
      FFC_TRY(launch_evaluate(t, sk, make_kparams(*k, t->d), precision, u_dev, u_far_dev, st));
  }
  tm->last_stream = st;
  return FFC_OK;
}

ffc_status ffc_evaluate_fmm(const ffc_tree* t, ffc_skel* sk, const ffc_kernel* k, const double* q_dev,
                            double* u_dev, double* u_far_dev, int32_t precision, void* stream) {
  if (!t || !sk) return fail(FFC_ERR_INVALID_ARG, "tree or skeleton is NULL");
  if (!q_dev || !u_dev) return fail(FFC_ERR_INVALID_ARG, "q or u is NULL");
  if (sk->num_nodes != t->num_nodes || sk->depth != t->depth)
    return fail(FFC_ERR_STATE, "skeleton set does not belong to this tree");
  FFC_TRY(check_kernel(k, t->d));
  FFC_TRY(check_precision(precision));
  hipStream_t st = (hipStream_t)stream;
  ffc_tree* tm = const_cast<ffc_tree*>(t);
  {
    StageTimer timer(FFC_STAGE_UPWARD, st);
    FFC_TRY(launch_charges_to_tree(tm, q_dev, st));
    for (int lev = t->depth; lev >= 1; --lev)
      FFC_TRY(launch_upward(t, sk, (1 << lev) - 1, 1 << lev, lev == t->depth, st));
  }
  {
    StageTimer timer(FFC_STAGE_EVALUATE, st);
    FFC_TRY(launch_fmm(t, sk, make_kparams(*k, t->d), precision, u_dev, u_far_dev, st));
  }
  tm->last_stream = st;
  return FFC_OK;
}

ffc_status ffc_direct_sum(const double* Y_dev, int64_t m, const double* X_dev, int64_t n, int32_t d,
                          const ffc_kernel* k, const double* q_dev, double* u_dev, int32_t precision, void* stream) {
  if (m < 0 || n < 0 || n > INT32_MAX) return fail(FFC_ERR_INVALID_ARG, "m, n must be >= 0 (n < 2^31)");
  if (d < 1) return fail(FFC_ERR_INVALID_ARG, "d must be >= 1");
  if ((m > 0 && (!Y_dev || !u_dev)) || (n > 0 && (!X_dev || !q_dev)))
    return fail(FFC_ERR_INVALID_ARG, "NULL pointer with nonzero size");
  FFC_TRY(check_kernel(k, d));
  FFC_TRY(check_precision(precision));
  if (!device_flag()) return fail(FFC_ERR_HIP, "cannot allocate the device flag");
  StageTimer timer(FFC_STAGE_DIRECT, (hipStream_t)stream);
  return launch_direct_sum(Y_dev, m, X_dev, n, d, make_kparams(*k, d), precision, q_dev, u_dev, (hipStream_t)stream);
}

ffc_status ffc_sampled_block(const ffc_tree* t, const ffc_kernel* k, int32_t precision, const int32_t* rows_dev,
                             int32_t s, const int32_t* cols_dev, int32_t n, double* out_dev, void* stream) {
  if (!t) return fail(FFC_ERR_INVALID_ARG, "tree is NULL");
  if (s < 0 || n < 0) return fail(FFC_ERR_INVALID_ARG, "s, n must be >= 0");
  if ((s > 0 && !rows_dev) || (n > 0 && !cols_dev) || (s > 0 && n > 0 && !out_dev))
    return fail(FFC_ERR_INVALID_ARG, "NULL pointer with nonzero size");
  FFC_TRY(check_kernel(k, t->d));
  FFC_TRY(check_precision(precision));
  if (precision == FFC_MIXED_BF16X3)
    return fail(FFC_ERR_INVALID_ARG, "ffc_sampled_block supports FFC_FP64 and FFC_FP32 only");
  if (s == 0 || n == 0) return FFC_OK;
  return launch_sampled_block(t, make_kparams(*k, t->d), precision, rows_dev, s, cols_dev, n, out_dev,
                              (hipStream_t)stream);
}

ffc_status ffc_interp_decomp(double* A_dev, int32_t batch, int32_t s, int32_t n, double tol, int32_t max_rank,
                             int32_t* rank_dev, int32_t* piv_dev, double* P_dev, void* stream) {
  if (batch < 0) return fail(FFC_ERR_INVALID_ARG, "batch must be >= 0");
  if (s < 1 || n < 1) return fail(FFC_ERR_INVALID_ARG, "s and n must be >= 1");
  if (max_rank < 1) return fail(FFC_ERR_INVALID_ARG, "max_rank must be >= 1");
  if (!(tol >= 0.0)) return fail(FFC_ERR_INVALID_ARG, "tol must be >= 0");
  if (batch > 0 && (!A_dev || !rank_dev || !piv_dev || !P_dev)) return fail(FFC_ERR_INVALID_ARG, "NULL pointer");
  IdBatch bt{};
  bt.A = A_dev;
  bt.a_stride = (int64_t)s * n;
  bt.lda = s;
  bt.s_uniform = s;
  bt.n_uniform = n;
  bt.s_max = s;
  bt.n_max = n;
  bt.tol = tol;
  bt.max_rank = max_rank;
  bt.rank = rank_dev;
  bt.piv = piv_dev;
  bt.piv_stride = n;
  bt.P = P_dev;
  bt.p_stride = (int64_t)max_rank * n;
  bt.p_ld = n;
  hipStream_t st = (hipStream_t)stream;
  DevBuf<unsigned char> scratch;
  bool used = false;
  FFC_TRY(launch_interp_decomp_coop(bt, batch, scratch, st, used));
  if (!used) FFC_TRY(launch_interp_decomp(bt, batch, st));
  FFC_HIP_TRY(hipStreamSynchronize(st));   // the scratch is released on return
  return FFC_OK;
}

ffc_status ffc_skel_node(const ffc_skel* sk, int32_t node, int32_t* rank, int32_t* n_cols, int32_t* n_rows,
                         int32_t* cols_host, int32_t* rows_host, int32_t* skel_host, double* P_host) {
  if (!sk) return fail(FFC_ERR_INVALID_ARG, "skeleton is NULL");
  if (node < 1 || node >= sk->num_nodes) return fail(FFC_ERR_INVALID_ARG, "node out of range");
  if (!rank || !n_cols || !n_rows) return fail(FFC_ERR_INVALID_ARG, "rank, n_cols and n_rows are required");
  FFC_HIP_TRY(hipStreamSynchronize(sk->last_stream));
  FFC_HIP_TRY(hipMemcpy(rank, sk->rank.ptr + node, sizeof(int32_t), hipMemcpyDeviceToHost));
  FFC_HIP_TRY(hipMemcpy(n_cols, sk->ncols.ptr + node, sizeof(int32_t), hipMemcpyDeviceToHost));
  FFC_HIP_TRY(hipMemcpy(n_rows, sk->nrows.ptr + node, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (cols_host && *n_cols > 0)
    FFC_HIP_TRY(hipMemcpy(cols_host, sk->cols.ptr + (int64_t)node * sk->n_cap, *n_cols * sizeof(int32_t),
                          hipMemcpyDeviceToHost));
  if (rows_host && *n_rows > 0)
    FFC_HIP_TRY(hipMemcpy(rows_host, sk->rows.ptr + (int64_t)node * sk->s_cap, *n_rows * sizeof(int32_t),
                          hipMemcpyDeviceToHost));
  if (skel_host && *rank > 0)
    FFC_HIP_TRY(hipMemcpy(skel_host, sk->skel.ptr + (int64_t)node * sk->r_cap, *rank * sizeof(int32_t),
                          hipMemcpyDeviceToHost));
  if (P_host && *rank > 0 && *n_cols > 0)
    FFC_HIP_TRY(hipMemcpy2D(P_host, *n_cols * sizeof(double), sk->P.ptr + (int64_t)node * sk->r_cap * sk->n_cap,
                            sk->n_cap * sizeof(double), *n_cols * sizeof(double), *rank, hipMemcpyDeviceToHost));
  return FFC_OK;
}

ffc_status ffc_skel_load(const ffc_tree* t, const ffc_skel_opts* o, const int32_t* rank_host,
                         const int32_t* ncols_host, const int32_t* skel_host, const double* P_host, int32_t r_max,
                         int32_t n_max, void* stream, ffc_skel** out) {
  if (!t || !o || !rank_host || !ncols_host || !skel_host || !P_host || !out)
    return fail(FFC_ERR_INVALID_ARG, "NULL argument");
  if (r_max < 1 || n_max < 1) return fail(FFC_ERR_INVALID_ARG, "r_max and n_max must be >= 1");
  if (!(o->separation >= 0.0)) return fail(FFC_ERR_INVALID_ARG, "separation must be >= 0");
  if (o->separation > 0.0 && t->depth > 30)
    return fail(FFC_ERR_INVALID_ARG, "separation supports trees of depth <= 30");
  const int nn = t->num_nodes, leaf0 = (1 << t->depth) - 1;
  for (int a = 1; a < nn; ++a) {
    const int n = ncols_host[a], r = rank_host[a];
    const int want = a >= leaf0 ? t->end_h[a] - t->begin_h[a] : rank_host[2 * a + 1] + rank_host[2 * a + 2];
    if (n != want || n > n_max)
      return fail(FFC_ERR_INVALID_ARG, "node " + std::to_string(a) + ": ncols must be the leaf size or the sum "
                                       "of the children's ranks, and at most n_max");
    if (r < 0 || r > std::min(r_max, n))
      return fail(FFC_ERR_INVALID_ARG, "node " + std::to_string(a) + ": rank outside [0, min(r_max, ncols)]");
    for (int i = 0; i < r; ++i) {
      const int32_t j = skel_host[(int64_t)a * r_max + i];
      if (j < 0 || j >= t->N) return fail(FFC_ERR_INVALID_ARG, "skeleton id outside [0, N)");
      for (int c = 0; c < n; ++c)
        if (!std::isfinite(P_host[((int64_t)a * r_max + i) * n_max + c]))
          return fail(FFC_ERR_INVALID_ARG, "P entries must be finite");
    }
  }
  hipStream_t st = (hipStream_t)stream;
  ffc_skel* sk = new ffc_skel();
  sk->num_nodes = nn;
  sk->depth = t->depth;
  sk->s_cap = 1;
  sk->r_cap = r_max;
  sk->n_cap = n_max;
  sk->opts = *o;
  sk->opts.max_rank = r_max;
  auto load = [&]() -> ffc_status {
    std::vector<int32_t> nrows(nn, 0), rank(rank_host, rank_host + nn), ncols(ncols_host, ncols_host + nn);
    rank[0] = ncols[0] = 0;
    // Column lists implied by the nesting (for ffc_skel_node): leaf ranges,
    // else the children's skeletons.
    std::vector<int32_t> cols((size_t)nn * n_max, 0);
    for (int a = 1; a < nn; ++a) {
      int32_t* c = cols.data() + (int64_t)a * n_max;
      if (a >= leaf0) {
        for (int j = 0; j < ncols[a]; ++j) c[j] = t->begin_h[a] + j;
      } else {
        const int l = 2 * a + 1;
        std::copy(skel_host + (int64_t)l * r_max, skel_host + (int64_t)l * r_max + rank[l], c);
        std::copy(skel_host + (int64_t)(l + 1) * r_max, skel_host + (int64_t)(l + 1) * r_max + rank[l + 1],
                  c + rank[l]);
      }
    }
    FFC_TRY(sk->rank.alloc(nn));
    FFC_TRY(sk->ncols.alloc(nn));
    FFC_TRY(sk->nrows.alloc(nn));
    FFC_TRY(sk->cols.alloc((size_t)nn * n_max));
    FFC_TRY(sk->rows.alloc((size_t)nn));
    FFC_TRY(sk->piv.alloc((size_t)nn * n_max));
    FFC_TRY(sk->skel.alloc((size_t)nn * r_max));
    FFC_TRY(sk->P.alloc((size_t)nn * r_max * n_max));
    FFC_TRY(sk->qt.alloc((size_t)nn * r_max));
    FFC_HIP_TRY(hipMemcpy(sk->rank.ptr, rank.data(), nn * sizeof(int32_t), hipMemcpyHostToDevice));
    FFC_HIP_TRY(hipMemcpy(sk->ncols.ptr, ncols.data(), nn * sizeof(int32_t), hipMemcpyHostToDevice));
    FFC_HIP_TRY(hipMemcpy(sk->nrows.ptr, nrows.data(), nn * sizeof(int32_t), hipMemcpyHostToDevice));
    FFC_HIP_TRY(hipMemcpy(sk->cols.ptr, cols.data(), cols.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    FFC_HIP_TRY(hipMemcpy(sk->skel.ptr, skel_host, (size_t)nn * r_max * sizeof(int32_t), hipMemcpyHostToDevice));
    FFC_HIP_TRY(hipMemcpy(sk->P.ptr, P_host, (size_t)nn * r_max * n_max * sizeof(double), hipMemcpyHostToDevice));
    if (o->separation > 0.0) FFC_TRY(launch_separation(t, sk, o->separation, st));
    FFC_HIP_TRY(hipStreamSynchronize(st));
    return FFC_OK;
  };
  const ffc_status s = load();
  if (s != FFC_OK) {
    delete sk;
    return s;
  }
  sk->last_stream = st;
  *out = sk;
  return FFC_OK;
}

ffc_status ffc_skel_stats(const ffc_skel* sk, ffc_stats* out) {
  if (!sk || !out) return fail(FFC_ERR_INVALID_ARG, "NULL argument");
  FFC_HIP_TRY(hipStreamSynchronize(sk->last_stream));
  std::vector<int32_t> rank(sk->num_nodes), nc(sk->num_nodes), nr(sk->num_nodes);
  FFC_HIP_TRY(hipMemcpy(rank.data(), sk->rank.ptr, rank.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  FFC_HIP_TRY(hipMemcpy(nc.data(), sk->ncols.ptr, nc.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  FFC_HIP_TRY(hipMemcpy(nr.data(), sk->nrows.ptr, nr.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof(*out));
  out->num_nodes = sk->num_nodes - 1;
  out->rank_min = INT32_MAX;
  double sum = 0.0, evals = 0.0;
  const int cap = std::min(sk->opts.max_rank, sk->r_cap);
  for (int a = 1; a < sk->num_nodes; ++a) {
    out->rank_min = std::min(out->rank_min, rank[a]);
    out->rank_max = std::max(out->rank_max, rank[a]);
    sum += rank[a];
    out->rank_cap_hits += rank[a] >= cap ? 1 : 0;
    evals += (double)nr[a] * nc[a];
  }
  if (out->num_nodes == 0) out->rank_min = 0;
  out->rank_mean = out->num_nodes ? sum / out->num_nodes : 0.0;
  out->fallbacks = sk->fallbacks;
  out->kernel_evals = evals;
  out->resampled = sk->resampled;
  for (int a = 1; a < sk->num_nodes; ++a) out->rows_max = std::max(out->rows_max, nr[a]);
  return FFC_OK;
}

ffc_status ffc_check_device(void* stream) {
  FFC_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  unsigned int* f = device_flag();
  if (!f) return fail(FFC_ERR_HIP, "cannot allocate the device flag");
  unsigned int h = 0;
  FFC_HIP_TRY(hipMemcpy(&h, f, sizeof(h), hipMemcpyDeviceToHost));
  if (h) {
    FFC_HIP_TRY(hipMemset(f, 0, sizeof(unsigned int)));
    if (h & 2u) return fail(FFC_ERR_HIP, "a QR workgroup group barrier timed out (results are invalid)");
    return fail(FFC_ERR_NONFINITE, "a kernel evaluation was not finite");
  }
  return FFC_OK;
}

void ffc_shutdown(void) {
  (void)hipDeviceSynchronize();
  ffc::profiler_release();
}

void ffc_free_tree(ffc_tree* t) {
  if (!t) return;
  if (t->graphs > 0) {   // a step graph still reads its buffers: the last ffc_graph_free deletes it
    t->orphaned = true;
    return;
  }
  (void)hipStreamSynchronize(t->last_stream);
  delete t;
}

void ffc_free_skel(ffc_skel* sk) {
  if (!sk) return;
  if (sk->graphs > 0) {
    sk->orphaned = true;
    return;
  }
  (void)hipStreamSynchronize(sk->last_stream);
  delete sk;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Step graphs
// ---------------------------------------------------------------------------
struct ffc_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ffc_tree* tree = nullptr;   // handles whose buffers the graph has baked in
  ffc_skel* skel = nullptr;
};

namespace {

// One captured step: skeletonize with reuse, then the sibling-cover or
// treecode evaluation (fmm false) or the FMM-style evaluation (fmm true).
ffc_status create_step_graph(const ffc_tree* t, ffc_skel* sk, const ffc_kernel* k, const ffc_skel_opts* o,
                             const double* q_dev, double* u_dev, double* u_far_dev, int32_t precision,
                             void* stream, bool fmm, ffc_graph** out) {
  using namespace ffc;
  if (!t || !sk || !k || !o || !q_dev || !u_dev || !out) {
    set_error("NULL argument (a skeleton set from a previous skeletonization is required)");
    return FFC_ERR_INVALID_ARG;
  }
  if (!stream) {
    set_error("graphs need a non-null stream");
    return FFC_ERR_INVALID_ARG;
  }
  if (t->orphaned || sk->orphaned) {
    set_error("the tree or skeleton set has been freed");
    return FFC_ERR_STATE;
  }
  if (o->sampler != FFC_SAMPLE_UNIFORM && o->fallback_tol > 0.0) {
    set_error("the pool samplers' fallback check synchronizes and cannot be captured");
    return FFC_ERR_INVALID_ARG;
  }
  if (o->adaptive_tol > 0.0) {
    set_error("the adaptive sample count synchronizes after every round and cannot be captured");
    return FFC_ERR_INVALID_ARG;
  }
  if (o->separation > 0.0 && (!sk->sep_bits.ptr || sk->sep_words != (int)((t->N + 63) / 64))) {
    set_error("separation: skeletonize once with a separation > 0 before capturing (its bitmaps are allocated then)");
    return FFC_ERR_STATE;
  }
  if (fmm && !(o->separation > 0.0)) {
    set_error("the FMM-style evaluation needs a separation > 0");
    return FFC_ERR_INVALID_ARG;
  }
  if (fmm && (sk->fmm_xi != o->separation || !sk->fmm_far_off.ptr || !sk->fmm_ufar.ptr)) {
    set_error("FMM-style graph: evaluate once eagerly with ffc_evaluate_fmm at this separation before capturing "
              "(its interaction lists and buffers are made then)");
    return FFC_ERR_STATE;
  }
  hipStream_t st = (hipStream_t)stream;
  FFC_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
  ffc_skel* skp = sk;
  ffc_status s1 = ffc_skeletonize_nodes(t, k, o, nullptr, 0, stream, &skp);
  ffc_status s2 = s1;
  if (s1 == FFC_OK)
    s2 = fmm ? ffc_evaluate_fmm(t, sk, k, q_dev, u_dev, u_far_dev, precision, stream)
             : ffc_evaluate_sum(t, sk, k, q_dev, u_dev, u_far_dev, precision, stream);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(st, &graph);
  if (s2 != FFC_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s2;
  }
  if (ec != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    return FFC_ERR_HIP;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(graph);
    set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    return FFC_ERR_HIP;
  }
  ffc_graph* g = new ffc_graph();
  g->graph = graph;
  g->exec = exec;
  g->tree = const_cast<ffc_tree*>(t);
  g->skel = sk;
  g->tree->graphs += 1;
  g->skel->graphs += 1;
  *out = g;
  return FFC_OK;
}

}  // namespace

extern "C" {

ffc_status ffc_step_graph_create(const ffc_tree* t, ffc_skel* sk, const ffc_kernel* k, const ffc_skel_opts* o,
                                 const double* q_dev, double* u_dev, double* u_far_dev, int32_t precision,
                                 void* stream, ffc_graph** out) {
  return create_step_graph(t, sk, k, o, q_dev, u_dev, u_far_dev, precision, stream, false, out);
}

ffc_status ffc_step_graph_create_fmm(const ffc_tree* t, ffc_skel* sk, const ffc_kernel* k, const ffc_skel_opts* o,
                                     const double* q_dev, double* u_dev, double* u_far_dev, int32_t precision,
                                     void* stream, ffc_graph** out) {
  return create_step_graph(t, sk, k, o, q_dev, u_dev, u_far_dev, precision, stream, true, out);
}

ffc_status ffc_graph_launch(ffc_graph* g, void* stream) {
  if (!g) {
    ffc::set_error("graph is NULL");
    return FFC_ERR_INVALID_ARG;
  }
  FFC_HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return FFC_OK;
}

void ffc_graph_free(ffc_graph* g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->skel && --g->skel->graphs == 0 && g->skel->orphaned) delete g->skel;
  if (g->tree && --g->tree->graphs == 0 && g->tree->orphaned) delete g->tree;
  delete g;
}

}  // extern "C"
