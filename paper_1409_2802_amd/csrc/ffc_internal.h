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
};

KParams make_kparams(const ffc_kernel& k, int d);

// Stage profiler: a StageTimer brackets the launches of one stage with events
// on the stage's stream while profiling is enabled.
bool profiling();
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
template <typename T>
struct DevBuf {
  T* ptr = nullptr;
  size_t count = 0;
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
    release();
    if (n == 0) return FFC_OK;
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
  hipStream_t last_stream = nullptr;
};

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
  int32_t fallbacks = 0;
  hipStream_t last_stream = nullptr;
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
                              uint64_t seed, hipStream_t st);

// Column lists of a level (sample.hip).
ffc_status launch_level_columns(const ffc_tree* t, ffc_skel* sk, int first, int count, bool leaves,
                                hipStream_t st);

// Sampled kernel blocks for nodes [first, first+count) into A (node-major,
// each s_cap x n_cap column-major with leading dimension s_cap) (kblock.hip).
ffc_status launch_level_kblock(const ffc_tree* t, const ffc_skel* sk, const KParams& kp, int precision,
                               int first, int count, double* A, hipStream_t st);

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
};
ffc_status launch_interp_decomp(const IdBatch& b, int batch, hipStream_t st);

// Register-resident variant (cpqr_coop.hip) for s <= 512: sets used = false
// (and launches nothing) when a block does not fit, so the caller can fall
// back to launch_interp_decomp. scratch grows as needed and must stay alive
// until the stream has passed the call.
ffc_status launch_interp_decomp_coop(const IdBatch& b, int batch, DevBuf<unsigned char>& scratch, hipStream_t st,
                                     bool& used);

// Skeleton ids from pivots: skel[node][i] = cols[node][piv[node][i]] (cpqr.hip).
ffc_status launch_skeleton_ids(ffc_skel* sk, int first, int count, hipStream_t st);

// Equivalent charges for a level (cpqr.hip).
ffc_status launch_upward(const ffc_tree* t, ffc_skel* sk, int first, int count, bool leaves, hipStream_t st);
ffc_status launch_charges_to_tree(ffc_tree* t, const double* q, hipStream_t st);

// Far + near field evaluation (kblock.hip).
ffc_status launch_evaluate(const ffc_tree* t, const ffc_skel* sk, const KParams& kp, int precision,
                           double* u, double* u_far, hipStream_t st);

// Mixed-precision (bf16 hi/lo Gram on matrix cores) variants of the sampled
// blocks, the evaluation and the direct sum for the Gaussian and polynomial
// kernels (gram_mfma.hip).
ffc_status launch_level_kblock_mixed(const ffc_tree* t, const ffc_skel* sk, const KParams& kp, int first, int count,
                                     double* A, hipStream_t st);
ffc_status launch_evaluate_mixed(const ffc_tree* t, const ffc_skel* sk, const KParams& kp, double* u, double* u_far,
                                 hipStream_t st);
ffc_status launch_direct_mixed(const double* Y, int64_t m, const double* X, int64_t n, int d, const KParams& kp,
                               const double* q, double* u, hipStream_t st);

// Direct sum (kblock.hip).
ffc_status launch_direct_sum(const double* Y, int64_t m, const double* X, int64_t n, int d, const KParams& kp,
                             int precision, const double* q, double* u, hipStream_t st);

}  // namespace ffc
