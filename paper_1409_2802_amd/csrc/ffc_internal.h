// Internal declarations of the far-field compression library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ffc.h"

namespace ffc {

// ---------------------------------------------------------------------------
// Error handling
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);

struct Status {
  ffc_status code = FFC_OK;
  bool ok() const { return code == FFC_OK; }
};

#define FFC_HIP_TRY(expr)                                                            \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ::ffc::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));           \
      return e_ == hipErrorOutOfMemory ? FFC_ERR_OOM : FFC_ERR_HIP;                  \
    }                                                                                \
  } while (0)

#define FFC_LAUNCH_CHECK(name)                                                       \
  do {                                                                               \
    hipError_t e_ = hipGetLastError();                                               \
    if (e_ != hipSuccess) {                                                          \
      ::ffc::set_error(std::string("launch of ") + name + ": " + hipGetErrorString(e_)); \
      return FFC_ERR_HIP;                                                            \
    }                                                                                \
  } while (0)

#define FFC_TRY(expr)                 \
  do {                                \
    ffc_status s_ = (expr);           \
    if (s_ != FFC_OK) return s_;      \
  } while (0)

// ---------------------------------------------------------------------------
// Kernel-function parameters as seen by device code
// ---------------------------------------------------------------------------
struct KParams {
  int kind;        // ffc_kernel_kind
  int p;           // polynomial degree
  double inv_h;    // 1 / h
  double c;        // polynomial constant
  double neg_inv_2h2;  // -1 / (2 h^2)
  double lap_expo;     // (2 - d) / 2
  // Laplace for d <= 7: r^(2-d) = (1/r)^m for odd d (m = d - 2), (1/r^2)^m for even d (m = (d - 2) / 2).
  int lap_small;
  int lap_m;
  int lap_odd;
};

KParams make_kparams(const ffc_kernel& k, int d);
// Validates a kernel description for dimension d (sets the error message).
ffc_status validate_kernel(const ffc_kernel* k, int d);

// Stage profiler: a StageTimer brackets the launches of one stage with events
// on the stage's stream while profiling is enabled.
bool profiling();
// Destroys the profiler's pooled events (ffc_shutdown).
void profiler_release();
class StageTimer {
 public:
  StageTimer(int stage, hipStream_t st);
  ~StageTimer();
  StageTimer(const StageTimer&) = delete;
  StageTimer& operator=(const StageTimer&) = delete;

 private:
  int stage_;
  hipStream_t st_;
  hipEvent_t start_{}, stop_{};
  bool active_ = false;
};

// Device flag word (bit 0: a kernel value was not finite). One per process.
unsigned int* device_flag();

// ---------------------------------------------------------------------------
// Opaque handle layouts
// ---------------------------------------------------------------------------
// Failure injection for tests: with FFC_FAIL_ALLOC=1 in the environment every
// device allocation of the library fails with FFC_ERR_OOM.
bool alloc_forced_to_fail();

// Buffers of a handle that a step graph has baked in must not move while the
// graph exists: `pin` points at the handle's live-graph count, and a
// (re)allocation while it is non-zero fails with FFC_ERR_STATE.
ffc_status refuse_pinned_alloc();

template <typename T>
struct DevBuf {
  T* ptr = nullptr;
  size_t count = 0;
  const int32_t* pin = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    count = 0;
  }
  ffc_status alloc(size_t n) {
    if (pin && *pin > 0) return refuse_pinned_alloc();
    release();
    if (n == 0) return FFC_OK;
    if (alloc_forced_to_fail()) {
      set_error("device allocation refused (FFC_FAIL_ALLOC is set)");
      return FFC_ERR_OOM;
    }
    hipError_t e = hipMalloc(&ptr, n * sizeof(T));
    if (e != hipSuccess) {
      ptr = nullptr;
      set_error(std::string("hipMalloc of ") + std::to_string(n * sizeof(T)) + " bytes: " + hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? FFC_ERR_OOM : FFC_ERR_HIP;
    }
    count = n;
    return FFC_OK;
  }
};

template <typename... B>
void pin_buffers(const int32_t* count, B&... bufs) {
  ((bufs.pin = count), ...);
}

// Column geometry of node blocks for the learned proposal (proposal.hip).
struct GeomArgs {
  const int32_t* cols;      // block b's columns at cols + b * col_stride (tree positions)
  int64_t col_stride;
  const int32_t* ncols;     // [count]
  const int32_t* node_ids;  // [count] stream ids of the blocks
  uint64_t seed;
  double* cen;              // [count][d]
  double* rho;              // [count]
  int32_t* sub;             // [count][256] subsample (tree positions)
  int32_t* nsub;            // [count]
  double* U;                // [count][7][d] anchor directions
  double* subn2;            // [count][256] squared norms of the subsample points (0 past nsub)
};

}  // namespace ffc

struct ffc_tree {
  int64_t N = 0;
  int32_t d = 0;
  int32_t depth = 0;
  int32_t num_nodes = 0;
  std::vector<int32_t> begin_h, end_h;      // node ranges (host copy)
  ffc::DevBuf<double> X;                    // caller order copy, N x d
  ffc::DevBuf<double> Xt;                   // tree order, N x d
  ffc::DevBuf<int32_t> perm;                // perm[pos] = caller index
  ffc::DevBuf<int32_t> begin, end;          // node ranges (device)
  ffc::DevBuf<double> centroid;             // num_nodes x d
  ffc::DevBuf<double> radius;               // num_nodes
  ffc::DevBuf<double> q_tree;               // charges in tree order (evaluation scratch)
  // Evaluation target tiles: (leaf node, first position) for blocks of targets.
  ffc::DevBuf<int32_t> tile_leaf, tile_start;
  int32_t num_tiles = 0;
  int32_t tile_rows = 0;
  // Operands of the matrix-core kernels, made on their first use (rows padded
  // with zeros to bf_dp, a multiple of 32): the tree-order coordinates split
  // into bfloat16 hi + lo with their squared norms; and, where distances need
  // centring on each tile (bf_frame == 0), the coordinates less the root
  // centroid in float32 with every node's centroid in the same frame plus one
  // last row holding the origin. bf_frame: -1 not yet decided, 1 the split
  // coordinates serve the Gaussian too, 0 the Gaussian centres per tile.
  ffc::DevBuf<uint16_t> bf_hi, bf_lo;
  ffc::DevBuf<float> bf_nrm;
  ffc::DevBuf<float> bf_x, bf_cc;
  int32_t bf_dp = 0;
  int32_t bf_frame = -1;
  hipStream_t last_stream = nullptr;
  // Step graphs holding this tree's buffers; ffc_free_tree while some exist
  // only marks the tree, and the last ffc_graph_free deletes it.
  int32_t graphs = 0;
  bool orphaned = false;
  ffc_tree() {
    ffc::pin_buffers(&graphs, X, Xt, perm, begin, end, centroid, radius, q_tree, tile_leaf, tile_start, bf_hi, bf_lo,
                     bf_nrm, bf_x, bf_cc);
  }
};

struct ffc_proposal {
  ffc::DevBuf<float> theta, mu, sd;   // parameters and standardization
  ffc::DevBuf<float> m1, m2;          // Adam moments
  int32_t step = 0;                   // Adam steps taken
};

namespace ffc {
// Scratch of the learned sampler, sized for the widest level of one tree.
struct LearnedScratch {
  int32_t p_cap = 0;                  // candidate pool capacity per node
  DevBuf<int32_t> ids;                // node ids 0..num_nodes-1
  DevBuf<int32_t> pool, npool;        // num_nodes x p_cap
  DevBuf<double> cen, rho, U, subn2;  // geometry of one level
  DevBuf<int32_t> sub, nsub;          // 256-point column subsamples
  DevBuf<float> feat, score;          // level x p_cap (x 16)
  DevBuf<int32_t> hrows, nheld;       // num_nodes x 32 held-out rows
  DevBuf<double> Kh;                  // level x 32 x n_cap
  DevBuf<unsigned char> mask;         // num_nodes
  DevBuf<unsigned int> counter;       // fallbacks of the current level
};
}  // namespace ffc

struct ffc_skel {
  int32_t num_nodes = 0;
  int32_t depth = 0;
  int32_t s_cap = 0;      // row capacity per node
  int32_t n_cap = 0;      // column capacity per node
  int32_t r_cap = 0;      // rank capacity per node
  ffc_kernel kernel{};
  ffc_skel_opts opts{};
  ffc::DevBuf<int32_t> rank, ncols, nrows;  // per node
  ffc::DevBuf<int32_t> cols;                // num_nodes x n_cap (tree positions)
  ffc::DevBuf<int32_t> rows;                // num_nodes x s_cap (tree positions)
  ffc::DevBuf<int32_t> piv;                 // num_nodes x n_cap (column slots)
  ffc::DevBuf<int32_t> skel;                // num_nodes x r_cap (tree positions)
  ffc::DevBuf<double> P;                    // num_nodes x r_cap x n_cap
  ffc::DevBuf<double> qt;                   // num_nodes x r_cap (equivalent charges)
  ffc::DevBuf<double> work;                 // sampled blocks of the widest level
  ffc::DevBuf<unsigned char> qr_scratch;    // group slots / counters of the QR kernel
  ffc::LearnedScratch learned;              // learned sampler (allocated on first use)
  ffc::DevBuf<unsigned char> subset;        // node subset of the last call (num_nodes bytes)
  int32_t fallbacks = 0;
  int32_t resampled = 0;                    // adaptive sample count: node redos
  // Separation (opts.separation > 0): bit p of sep_bits[a * sep_words + p / 64]
  // is set when tree position p is outside node a and separated from it;
  // sep_pre[a * (sep_words + 1) + w] counts the set bits of words 0..w-1.
  ffc::DevBuf<uint64_t> sep_bits;
  ffc::DevBuf<int32_t> sep_pre;
  int32_t sep_words = 0;
  // FMM-style evaluation: multipole-to-local lists per node and direct lists
  // per leaf (CSR, built for separation fmm_xi), incoming values v at the
  // skeleton points (num_nodes x r_cap) and the far field in tree order.
  double fmm_xi = -1.0;
  ffc::DevBuf<int32_t> fmm_far_off, fmm_far_src, fmm_near_off, fmm_near_src;
  ffc::DevBuf<double> fmm_v, fmm_vpart, fmm_ufar;   // vpart: partial sums of the list quarters
  int64_t fmm_far_pairs = 0, fmm_near_pairs = 0;
  hipStream_t last_stream = nullptr;
  // Step graphs holding this set's buffers (see ffc_tree::graphs).
  int32_t graphs = 0;
  bool orphaned = false;
  ffc_skel() {
    ffc::pin_buffers(&graphs, rank, ncols, nrows, cols, rows, piv, skel, P, qt, work, qr_scratch, subset, sep_bits,
                     sep_pre,
                     fmm_far_off, fmm_far_src, fmm_near_off, fmm_near_src, fmm_v, fmm_vpart, fmm_ufar);
    ffc::LearnedScratch& L = learned;
    ffc::pin_buffers(&graphs, L.ids, L.pool, L.npool, L.cen, L.rho, L.U, L.sub, L.nsub, L.feat, L.score, L.hrows,
                     L.nheld, L.Kh, L.mask, L.counter);
  }
};

namespace ffc {

// ---------------------------------------------------------------------------
// Launchers (one per device stage). All are asynchronous on `st`.
// ---------------------------------------------------------------------------

// Tree construction (tree.hip).
ffc_status launch_build_tree(ffc_tree* t, int32_t leaf_size, hipStream_t st);
ffc_status launch_node_stats(ffc_tree* t, int level, hipStream_t st);
ffc_status launch_gather_tree_points(ffc_tree* t, hipStream_t st);

// Uniform row sampling (sample.hip): rows[node] for nodes [first, first+count).
ffc_status launch_sample_rows(const ffc_tree* t, ffc_skel* sk, int first, int count, int s,
                              uint64_t seed, hipStream_t st, const unsigned char* mask = nullptr);
// General form: draws into rows + node * cap (counts in nrows[node]) with the
// Floyd stream node | stream_or; nodes with mask[node] == 0 are skipped when
// mask is non-null.
ffc_status launch_sample_rows_into(const ffc_tree* t, int32_t* rows, int32_t* nrows, int cap, int first, int count,
                                   int s, uint64_t seed, uint32_t stream_or, const unsigned char* mask,
                                   hipStream_t st);
// Raw form: range g = [nb[g], ne[g]) of tree positions; draws s of the M
// positions inside it (inside) or outside it in [0, N), Floyd stream g | stream_or.
ffc_status launch_draw(const int32_t* nb, const int32_t* ne, int64_t N, bool inside, int32_t* rows, int32_t* nrows,
                       int cap, int first, int count, int s, uint64_t seed, uint32_t stream_or,
                       const unsigned char* mask, hipStream_t st);

// Separated far sets (bits == nullptr: none). A draw outside node g then takes
// the M = pre[g * (words + 1) + words] separated positions (all outside points
// when M is 0), candidate t being the t-th set bit of g's bitmap.
struct SepView {
  const uint64_t* bits = nullptr;
  const int32_t* pre = nullptr;
  int words = 0;
};
ffc_status launch_sample_rows_sep(const ffc_tree* t, ffc_skel* sk, int first, int count, int s, uint64_t seed,
                                  hipStream_t st, const unsigned char* mask = nullptr);

// Column lists of a level (sample.hip); with a mask (indexed by node) only
// the nodes whose entry is set.
ffc_status launch_level_columns(const ffc_tree* t, ffc_skel* sk, int first, int count, bool leaves,
                                hipStream_t st, const unsigned char* mask = nullptr);

// Sampled kernel blocks for nodes [first, first+count) into A (node-major,
// each s_cap x n_cap column-major with leading dimension s_cap); with a mask
// (indexed by node) only the nodes whose entry is set (kblock.hip).
ffc_status launch_level_kblock(const ffc_tree* t, const ffc_skel* sk, const KParams& kp, int precision,
                               int first, int count, double* A, hipStream_t st,
                               const unsigned char* mask = nullptr);

// Sampled blocks for nodes [first, first+count) given raw row/column lists
// (node b: rows + b * s_cap, nrows[b], cols + b * n_cap, ncols[b]; the mixed
// mode centres block b on centroid + (first + b) * d) (kblock.hip).
ffc_status launch_kblock_batch(const ffc_tree* t, const KParams& kp, int precision, const int32_t* rows,
                               const int32_t* nrows, int s_cap, const int32_t* cols, const int32_t* ncols, int n_cap,
                               int first, int count, const double* centroid, double* A, hipStream_t st,
                               const unsigned char* mask = nullptr);

// Gram matrices of column-major m x n blocks, n x n row-major each (kblock.hip).
ffc_status launch_gram(const double* B, int m, int n, int count, double* G, hipStream_t st);

// Standalone sampled block (kblock.hip).
ffc_status launch_sampled_block(const ffc_tree* t, const KParams& kp, int precision, const int32_t* rows,
                                int s, const int32_t* cols, int n, double* out, hipStream_t st);

// Batched CPQR + interpolation solve (cpqr.hip). Per batch entry b: block at
// A + b * a_stride (column-major, leading dim lda), dims from s_arr/n_arr (or
// uniform s/n when the arrays are null).
struct IdBatch {
  double* A;
  int64_t a_stride;
  int lda;
  const int32_t* s_arr;   // may be null -> s_uniform
  const int32_t* n_arr;   // may be null -> n_uniform
  int s_uniform, n_uniform;
  int s_max, n_max;
  double tol;
  int max_rank;
  int32_t* rank;          // [batch]
  int32_t* piv;           // [batch][piv_stride]
  int64_t piv_stride;
  double* P;              // [batch][p_stride], row-major rank x n with row stride n_max? (p_ld)
  int64_t p_stride;
  int p_ld;               // leading dimension of P rows
  const unsigned char* mask = nullptr;   // [batch]: only entries set are factored (all when null)
};
ffc_status launch_interp_decomp(const IdBatch& b, int batch, hipStream_t st);

// Register-resident variant (cpqr_coop.hip) for s <= 512: sets used = false
// (and launches nothing) when a block does not fit, so the caller can fall
// back to launch_interp_decomp. scratch grows as needed and must stay alive
// until the stream has passed the call.
// Autotuner choices of the QR kernel so far: 8 int32 per entry (s_max, n_max,
// batch, rank cap, rows per lane, threads, best us, first candidate's us);
// writes at most cap entries, returns the number of entries (cpqr_coop.hip).
int autotune_entries(int32_t* out, int cap);
void autotune_reset();
ffc_status launch_interp_decomp_coop(const IdBatch& b, int batch, DevBuf<unsigned char>& scratch, hipStream_t st,
                                     bool& used);
// The same without any allocation: the QR's slots and the solve's scratch
// come from `fixed` (fixed_bytes long), the variant is the autotuner's earlier
// choice for this shape or else the first that fits, and nothing is timed.
// FFC_ERR_INVALID_ARG when no variant fits s_max or the scratch is too small.
ffc_status launch_interp_decomp_fixed(const IdBatch& b, int batch, unsigned char* fixed, size_t fixed_bytes,
                                      hipStream_t st);

// Skeleton ids from pivots: skel[node][i] = cols[node][piv[node][i]] (cpqr.hip).
ffc_status launch_skeleton_ids(ffc_skel* sk, int first, int count, hipStream_t st,
                               const unsigned char* mask = nullptr);

// Equivalent charges for a level (cpqr.hip).
ffc_status launch_upward(const ffc_tree* t, ffc_skel* sk, int first, int count, bool leaves, hipStream_t st);
ffc_status launch_charges_to_tree(ffc_tree* t, const double* q, hipStream_t st);

// Learned sampler for one level (api_proposal.hip): candidate pool, geometry,
// features, scores and selection into sk->rows / sk->nrows.
ffc_status learned_rows_level(const ffc_tree* t, ffc_skel* sk, int sampler, const ffc_proposal* p, int first,
                              int count, int s, uint64_t seed, hipStream_t st);
// Held-out check of a skeletonized level; returns in `redo` the number of nodes
// that failed (their mask is set and their rows redrawn uniformly). Synchronizes.
ffc_status learned_heldout_level(const ffc_tree* t, ffc_skel* sk, const KParams& kp, int precision, int first,
                                 int count, int s, uint64_t seed, double tol, int& redo, hipStream_t st);
ffc_status learned_alloc(const ffc_tree* t, ffc_skel* sk, int pool_factor);
// Adaptive sample count (held-out rows and blocks in sk->learned).
ffc_status heldout_alloc(const ffc_tree* t, ffc_skel* sk);
// Held-out rows and their kernel block for the nodes of a level (once per level).
ffc_status heldout_prepare_level(const ffc_tree* t, ffc_skel* sk, const KParams& kp, int precision, int first,
                                 int count, uint64_t seed, hipStream_t st);
// One round: nodes whose held-out error exceeds tol and whose rows can grow
// (below s_limit) get s_next fresh uniform rows; their number goes to `redo`.
// Synchronizes.
ffc_status adaptive_round_level(const ffc_tree* t, ffc_skel* sk, int first, int count, uint64_t seed, double tol,
                                int s_limit, int s_next, int& redo, hipStream_t st);

// Learned proposal (proposal.hip).
ffc_status launch_geometry(const double* Xt, int d, const GeomArgs& ga, int count, hipStream_t st);
ffc_status launch_features(const double* Xt, int d, const GeomArgs& ga, const int32_t* tgt, int tgt_stride,
                           const int32_t* ntgt, int count, float* feat, int64_t feat_stride, hipStream_t st);
ffc_status launch_mlp_score(const float* theta, const float* mu, const float* sdv, const float* feat, int64_t count,
                            float* score, hipStream_t st);
ffc_status launch_mlp_grad(const float* theta, const float* mu, const float* sdv, const float* feat,
                           const float* target, int64_t count, int64_t p0, int64_t stride_mul, int64_t total,
                           float* grads, hipStream_t st);
ffc_status launch_grad_reduce_adam(const float* grads, int nwg, float* theta, float* m1, float* m2, float* gsum,
                                   float* loss_out, bool adam, float lr, int step, int64_t total, hipStream_t st);
ffc_status launch_feature_stats(const float* feat, int64_t count, float* mu, float* sdv, hipStream_t st);
// Selection for nodes [first, first+count): pool / npool / values indexed by
// b = node - first (value i at score[b * score_stride + i * elem_stride]),
// rows / nrows / ncols / mask by node; nodes with an empty column set get
// nrows = 0. mode 0: learned weights from scores; 1: weights proportional to
// 1 / value; 2: the s smallest values.
ffc_status launch_select_rows(const float* score, int64_t score_stride, int elem_stride, int mode,
                              const int32_t* pool, int pool_stride, const int32_t* npool, int first, int count, int s,
                              uint64_t seed, const int32_t* ncols, const unsigned char* mask, int32_t* rows, int s_cap,
                              int32_t* nrows, hipStream_t st);
// Held-out check of the nodes [first, first+count): err = |K_h - K_h(:, J) P|_F
// / |K_h|_F; mask[node] = err > tol, and with grow.nrows set also only when
// the node's row count can still grow (below grow.s_limit and the points
// outside the node); the number of masked nodes is added to *fallbacks.
struct HeldoutGrow {
  const int32_t* nrows = nullptr;
  const int32_t* nb = nullptr;
  const int32_t* ne = nullptr;
  int64_t N = 0;
  int s_limit = 0;
};
ffc_status launch_heldout_check(const double* Kh, const int32_t* nh, int h_cap, const ffc_skel* sk, int first,
                                int count, double tol, unsigned char* mask, unsigned int* fallbacks,
                                const HeldoutGrow& grow, hipStream_t st);

// Ridge leverage labels (leverage.hip) of row-major m x n blocks B_b: G_b =
// B_b^T B_b, its Cholesky factor with eps^2 tr(G_b) added to the diagonal,
// lev[b][i] = |B_b(i, :) L^{-T}|^2 (B overwritten by B L^{-T}) and, when target
// is non-null, target[b][i] = ln(max(lev, 1e-12) m / sum(lev)).
// status[b]: 0 factorized, 1 zero block (leverages 0), 2 not positive definite.
ffc_status launch_ridge_leverage(double* B, int64_t m, int n, int count, double* G, double eps, double* lev,
                                 float* target, int* status, hipStream_t st);

// Pivoted (rank-r) leverage labels (leverage.hip) of row-major m x n blocks
// (n <= 1024): G_b = B_b^T B_b, its diagonal-pivoted Cholesky factor (column-
// major in Lc, pivot order in perm, pivots in rank) stopped at sqrt(d_k) <
// eps sqrt(d_0), lev[b][i] = |B_b(i, J) L11^{-T}|^2 (B overwritten at the
// pivot columns) and, when target is non-null, the log targets as above.
// status[b]: 0 factorized, 1 zero block.
ffc_status launch_pivoted_leverage(double* B, int64_t m, int n, int count, double* G, double* Lc, int* perm,
                                   int* rank, double eps, double* lev, float* target, int* status, hipStream_t st);

// Far + near field evaluation (kblock.hip).
ffc_status launch_evaluate(const ffc_tree* t, const ffc_skel* sk, const KParams& kp, int precision,
                           double* u, double* u_far, hipStream_t st);
// Separation bitmaps and their word prefixes for every node (kblock.hip), and
// the treecode evaluation that reads them (FFC_FP64 / FFC_FP32).
ffc_status launch_separation(const ffc_tree* t, ffc_skel* sk, double xi, hipStream_t st);
ffc_status launch_treecode(const ffc_tree* t, const ffc_skel* sk, const KParams& kp, int precision, double* u,
                           double* u_far, hipStream_t st);
// FMM-style evaluation (fmm.hip); builds the interaction lists on first use
// (synchronizes the stream once).
ffc_status launch_fmm(const ffc_tree* t, ffc_skel* sk, const KParams& kp, int precision, double* u, double* u_far,
                      hipStream_t st);

// Mixed-precision (bf16 hi/lo Gram on matrix cores) variants of the sampled
// blocks, the evaluation and the direct sum for the Gaussian and polynomial
// kernels (gram_mfma.hip).
ffc_status launch_kblock_batch_mixed(const ffc_tree* t, const KParams& kp, const int32_t* rows, const int32_t* nrows,
                                     int s_cap, const int32_t* cols, const int32_t* ncols, int n_cap, int first,
                                     int count, const double* centroid, double* A, hipStream_t st,
                                     const unsigned char* mask);
ffc_status launch_evaluate_mixed(const ffc_tree* t, const ffc_skel* sk, const KParams& kp, double* u, double* u_far,
                                 hipStream_t st);
ffc_status launch_direct_mixed(const double* Y, int64_t m, const double* X, int64_t n, int d, const KParams& kp,
                               const double* q, double* u, hipStream_t st);

// Direct sum (kblock.hip).
ffc_status launch_direct_sum(const double* Y, int64_t m, const double* X, int64_t n, int d, const KParams& kp,
                             int precision, const double* q, double* u, hipStream_t st);

}  // namespace ffc
