/*
 * ffc.h - C ABI of the far-field compression library (HIP, gfx950).
 *
 * The library computes kernel sums u_i = sum_j K(y_i, x_j) q_j (March & Biros,
 * "Far-Field Compression for Fast Kernel Summation Methods in High
 * Dimensions", Section 1, eq. e:sum) with the paper's sampled-row
 * interpolative decomposition as the far-field representation (Section 2.2):
 * for every node of a tree over the points, sample target rows, form the
 * sampled kernel block K' (Section 2.2), take its interpolative decomposition
 * by column-pivoted QR (Section 2.1.3; Appendix 6.1) and apply the skeletons
 * in the sum (eq. e:id).
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device pointers (HIP global memory), *_host are
 *    host pointers. Coordinates are float64, row-major (point-major), N x d.
 *  - stream is a hipStream_t passed as void*; NULL means the null stream.
 *    Calls that launch work are asynchronous and stream ordered; the caller
 *    keeps device buffers alive until the stream has reached the call.
 *  - Every call returns ffc_status; nothing throws across the ABI. On error
 *    ffc_last_error() returns a thread-local message. Arguments are validated
 *    before anything is launched.
 *  - Handles (ffc_tree, ffc_skel) are opaque, owned by the library and released
 *    with ffc_free_tree / ffc_free_skel.
 *  - Kernel values that are not finite (for instance the Laplace kernel
 *    overflowing at tiny distances), and kernel sums that are not, raise a
 *    device flag that ffc_check_device reports as FFC_ERR_NONFINITE.
 */
#ifndef FFC_H
#define FFC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FFC_OK = 0,
  FFC_ERR_INVALID_ARG = 1,
  FFC_ERR_HIP = 2,
  FFC_ERR_OOM = 3,
  FFC_ERR_NONFINITE = 4,
  FFC_ERR_STATE = 5
} ffc_status;

/* Kernel functions (Section 4.2-4.4):
 *  FFC_GAUSSIAN    exp(-||x - y||^2 / (2 h^2))                 (eq. eqn_gaussian_kernel)
 *  FFC_LAPLACE     ||x - y||^(2 - d), d >= 3; pairs at zero distance give 0
 *  FFC_POLYNOMIAL  (x^T y / h + c)^p, integer p >= 1 (the paper sets c = 1)  */
typedef enum { FFC_GAUSSIAN = 0, FFC_LAPLACE = 1, FFC_POLYNOMIAL = 2 } ffc_kernel_kind;

typedef struct {
  int32_t kind;   /* ffc_kernel_kind */
  int32_t p;      /* polynomial degree */
  double h;       /* bandwidth (Gaussian, polynomial), > 0 */
  double c;       /* polynomial constant */
} ffc_kernel;

/* Arithmetic of the kernel evaluations (distances / inner products and the
 * kernel function). The QR, the interpolation solve and the charges are always
 * float64. FFC_MIXED_BF16X3 splits coordinates into bfloat16 hi + lo parts and
 * forms the Gram products hi*hi + hi*lo + lo*hi on matrix cores with float32
 * accumulation (Gaussian and polynomial kernels). The Laplace kernel's power
 * (d - 2) / 2 amplifies errors of r^2, so its sampled blocks and evaluation
 * split into three bf16 parts (six products, about float32 precision), take
 * r^2 of pairs much closer to each other than to the tile's centre from
 * explicit float32 differences, and form the power in float64; its direct sum
 * uses float32 differences. For the Gaussian,
 * coordinates are centred on each tile's node (or target leaf) before the
 * split unless every leaf of the tree lies within four of its radii of the
 * origin; the Laplace kernel always centres. The first mixed-precision call
 * on a tree prepares these operands
 * (4 N dp bytes of device memory kept with the tree, 8 N dp with per-tile
 * centring; dp = d rounded up to a multiple of 32) and cannot be made while
 * the stream is captured (FFC_ERR_STATE). */
typedef enum { FFC_FP64 = 0, FFC_FP32 = 1, FFC_MIXED_BF16X3 = 2 } ffc_precision;

/* Row samplers. UNIFORM: uniform without replacement over the points outside
 * the node (Section 4.1.3). The others choose s rows from a pool of
 * min(M, pool_factor * s) uniform far points, with the node's column
 * geometry (centroid c, radius rho, a 256-point column subsample):
 *  LEARNED   weights from the proposal network's scores (importance sampling
 *            by predicted leverage, Section 3);
 *  DISTANCE  the paper's distance sampling (Sections 3.2, 4.1.3): without
 *            replacement, weights inversely proportional to |y - c| (the
 *            motivation of Section 3.2; Section 4.1.3's "proportional" would
 *            favour the least significant rows);
 *  NEAREST   the paper's nearest neighbours, deterministic: the s pool points
 *            nearest to the node's columns (distance to the nearest point of
 *            the column subsample; exact for nodes of at most 256 columns).
 * All pool samplers support the held-out fallback (fallback_tol). */
typedef enum {
  FFC_SAMPLE_UNIFORM = 0,
  FFC_SAMPLE_LEARNED = 1,
  FFC_SAMPLE_DISTANCE = 2,
  FFC_SAMPLE_NEAREST = 3
} ffc_sampler;

typedef struct ffc_tree ffc_tree;
typedef struct ffc_skel ffc_skel;
typedef struct ffc_proposal ffc_proposal;

/* Skeletonization options.
 *  tol          relative rank tolerance: the QR stops at the first pivot whose
 *               column norm is below tol times the first pivot's (> 0 or 0 for
 *               full rank)
 *  max_rank     rank cap, >= 1
 *  num_samples  sampled target rows per node; 0 means 2 * max_rank. Capped at
 *               the number of points outside the node.
 *  precision    ffc_precision of the sampled kernel block
 *  sampler      ffc_sampler; FFC_SAMPLE_LEARNED needs `proposal` (kept by
 *               reference: it must outlive the call)
 *  seed         seed of the counter-based row sampler
 *  fallback_tol pool samplers only: a node whose held-out error estimate
 *               exceeds it is redone with uniform rows (<= 0 disables; the
 *               check synchronizes the stream once per level)
 *  pool_factor  pool samplers only: the candidate pool of a node is
 *               min(M, pool_factor * samples) uniform far points (0 means 8;
 *               the pool is limited to 8192)
 *  adaptive_tol uniform sampler only; > 0 turns on the adaptive sample count
 *               (the integration question of Section 5): after a level is
 *               skeletonized, every node whose error estimate on 32 held-out
 *               uniform far rows, |K_h - K_h(:, J) P|_F / |K_h|_F, exceeds
 *               adaptive_tol and whose row count can still grow is redone with
 *               twice the rows (a fresh uniform draw), until all pass or reach
 *               the cap; each round synchronizes the stream once. <= 0: off.
 *  max_samples  cap of the adaptive sample count (0 means 4 * the initial
 *               count); rows never exceed the points outside the node
 *  separation   xi >= 0, the separation of sources and targets (Section 2,
 *               eq. e:separated; Section 4.1 measures it as a multiple of the
 *               source ball's radius). A point y outside node a is separated
 *               from a when |y - c_a|^2 >= (xi rho_a)^2, with c_a and rho_a the
 *               node's centroid and radius (ffc_tree_arrays). xi > 0 draws the
 *               rows of every node uniformly from its separated points in
 *               ascending tree order (Floyd on their count; a node with none
 *               draws from all points outside it, as xi = 0 does) and makes
 *               ffc_evaluate_sum a treecode with the same test. 0: the plain
 *               method. Uniform sampler only, no adaptive count. */
typedef struct {
  double tol;
  int32_t max_rank;
  int32_t num_samples;
  int32_t precision;
  int32_t sampler;
  uint64_t seed;
  const ffc_proposal* proposal;
  double fallback_tol;
  int32_t pool_factor;
  double adaptive_tol;
  int32_t max_samples;
  double separation;
} ffc_skel_opts;

/* Build a binary ball tree over X (Section 2: hierarchical groupings of the
 * points). Depth D is the least D with ceil(N / 2^D) <= leaf_size; all leaves
 * sit at level D. Each node is split at the median of the projections onto
 * (p2 - p1), p1 the point farthest from the node centroid, p2 the point
 * farthest from p1; points are ordered by (projection, caller index) and the
 * left child takes the first ceil(n/2). Node ids are breadth first (root 0,
 * children 2a+1, 2a+2). The points are copied, so X_dev may be freed after
 * the stream passes the call. Errors: N < 1, d < 1, leaf_size < 1, NULL
 * pointers -> FFC_ERR_INVALID_ARG. */
ffc_status ffc_build_tree(const double* X_dev, int64_t N, int32_t d, int32_t leaf_size,
                          void* stream, ffc_tree** out);

/* Two-part "tree": root plus leaves [0, n_left) and [n_left, N) in caller order
 * (one source node against the remaining targets, Section 4.1 set-up).
 * Errors: n_left < 1 or n_left >= N -> FFC_ERR_INVALID_ARG. */
ffc_status ffc_build_partition(const double* X_dev, int64_t N, int32_t d, int64_t n_left,
                               void* stream, ffc_tree** out);

/* Tree shape: depth, number of nodes (2^(depth+1) - 1), N and d. */
ffc_status ffc_tree_info(const ffc_tree* t, int32_t* depth, int32_t* num_nodes,
                         int64_t* N, int32_t* d);

/* Copies to host: perm_host[pos] = caller index of the point at tree position
 * pos (N entries); begin/end of every node (num_nodes entries each); centroid
 * (num_nodes x d) and radius (num_nodes). Any output may be NULL. Synchronizes
 * with the stream of the last call on the tree. */
ffc_status ffc_tree_arrays(const ffc_tree* t, int32_t* perm_host, int64_t* begin_host,
                           int64_t* end_host, double* centroid_host, double* radius_host);

/* Skeletonize every non-root node (Section 2.2), deepest level first. A leaf's
 * columns are its points; an internal node's columns are the skeleton of its
 * left child followed by that of its right child. Target rows are sampled from
 * the points outside the node. Per node: sampled block K' (s x n), column-
 * pivoted QR to tolerance (Appendix 6.1), R11 T = R12, P = [I T] Pi^T, skeleton
 * = first r pivots (Section 2.1.3). All nodes of a level run in one launch per
 * stage. *out must be NULL (a new handle is returned) or a handle from an
 * earlier call on the same tree with the same sample count and rank cap,
 * whose storage is then reused and overwritten (FFC_ERR_STATE otherwise).
 * node_ids_host: NULL (every non-root node; num_ids must be 0) or num_ids >= 1
 * distinct node ids in [1, num_nodes) (host memory, read during the call):
 * only those nodes are skeletonized (outgoing representations per source
 * node, Section 2.2), deepest level first; the others keep what the handle
 * holds (rank 0 and no columns in a new handle). A listed internal node takes
 * as columns its children's skeletons as they stand when its level is
 * reached, so listing a node together with its descendants gives exactly what
 * the full call gives for it. Subsets work with the uniform sampler (also
 * with separation) and a fixed sample count; the call copies the list to the
 * device and synchronizes the stream once, so it cannot be captured.
 * Errors: invalid kernel (h <= 0, p < 1, Laplace with d = 2), tol < 0,
 * max_rank < 1, num_samples < 0, learned sampler without proposal, a bad
 * node list (out of range, repeated, num_ids inconsistent with the pointer,
 * another sampler or the adaptive count) -> FFC_ERR_INVALID_ARG. */
ffc_status ffc_skeletonize_nodes(const ffc_tree* t, const ffc_kernel* k, const ffc_skel_opts* o,
                                 const int32_t* node_ids_host, int32_t num_ids, void* stream, ffc_skel** out);

/* u = K q with the compressed far field (eq. e:id): equivalent charges
 * q~ = P q upward through the tree, then for every target the skeletons of
 * the siblings of its leaf's ancestors (far field) plus its own leaf directly
 * (near field). A skeleton set built with separation xi > 0 is evaluated as a
 * treecode (Section 2): each target walks down from the root's children; a
 * node that does not contain it and from which it is separated (the test of
 * ffc_skel_opts.separation) contributes its skeleton sum and ends that branch,
 * any other node passes the target to its children, and leaves reached that
 * way (the target's own among them) are summed directly. q_dev and u_dev are
 * N-vectors in caller order; u_far_dev (nullable) receives the far-field part
 * only. precision: ffc_precision of the kernel evaluations (a treecode takes
 * FFC_FP64 or FFC_FP32). The skeleton must come from the same tree. */
ffc_status ffc_evaluate_sum(const ffc_tree* t, const ffc_skel* sk, const ffc_kernel* k,
                            const double* q_dev, double* u_dev, double* u_far_dev,
                            int32_t precision, void* stream);

/* u = K q by the FMM-style scheme that Section 2 sets beside the treecode:
 * incoming representations from the same skeletons (for the symmetric kernel on
 * one point set, node b's ID gives K(cols_b, S) ~ P_b^T K(J_b, S) for sources
 * S in its separated far field). Nodes b != a of one level are admissible when
 * every point of each is separated from the other (the test of
 * ffc_skel_opts.separation both ways). From the pairs of the root's children,
 * an admissible pair contributes K(x_{J_b}, x_{J_a}) q~_a at b's skeleton
 * points, any other pair of leaves is summed directly, and any other pair
 * recurses into its four child pairs. The values at skeleton points are passed
 * down by P^T to the children's skeleton points and, at the leaves, to the
 * points (far field); direct pairs give the near field. q_dev, u_dev, u_far_dev
 * as in ffc_evaluate_sum. The interaction lists are built on the first call
 * with a skeleton set (or after its separation changed), which synchronizes
 * `stream` once. Errors: a skeleton set built without separation ->
 * FFC_ERR_STATE; precision other than FFC_FP64 / FFC_FP32, tree depth above
 * 11 -> FFC_ERR_INVALID_ARG. */
ffc_status ffc_evaluate_fmm(const ffc_tree* t, ffc_skel* sk, const ffc_kernel* k,
                            const double* q_dev, double* u_dev, double* u_far_dev,
                            int32_t precision, void* stream);

/* Direct summation u_i = sum_j K(y_i, x_j) q_j (Section 1, eq. e:sum) for m
 * targets Y (m x d) and n sources X (n x d). Laplace pairs at zero distance
 * contribute 0. Errors: m, n < 0, d < 1, NULL pointers with nonzero sizes. */
ffc_status ffc_direct_sum(const double* Y_dev, int64_t m, const double* X_dev, int64_t n,
                          int32_t d, const ffc_kernel* k, const double* q_dev, double* u_dev,
                          int32_t precision, void* stream);

/* Sampled kernel block of a tree: out[j * s + i] = K(x_rows[i], x_cols[j]) for
 * tree positions rows_dev (s) and cols_dev (n), column-major s x n (the block
 * K' of Section 2.2, computed by the same kernels the skeletonization uses).
 * precision: FFC_FP64 or FFC_FP32. */
ffc_status ffc_sampled_block(const ffc_tree* t, const ffc_kernel* k, int32_t precision,
                             const int32_t* rows_dev, int32_t s, const int32_t* cols_dev,
                             int32_t n, double* out_dev, void* stream);

/* Interpolative decompositions of `batch` column-major s x n blocks A_dev
 * (block b at A_dev + b * s * n; overwritten by the factorization). Outputs:
 * rank_dev[b]; piv_dev[b * n + k] = column of the k-th pivot; P_dev[b *
 * max_rank * n + i * n + j] = P (rank x n, row-major, original column order);
 * rows i >= rank are left untouched. Same QR and solve as the skeletonization
 * (Appendix 6.1; Theorem thm_compute_id). piv_dev entries k >= rank list the
 * remaining columns. Returns after the stream has finished the work (the call
 * owns temporary device scratch). Errors: s, n < 1, max_rank < 1.
 * The QR (here and in the skeletonization) is a cooperative launch when the
 * blocks fit in registers (s <= 1024). A process that has made one holds the
 * device's cooperative-launch resource until it exits; while it does, the
 * same call in another process on that device falls back to the
 * one-workgroup-per-block kernel (slower; results within the same parity
 * bar, not bitwise the same). */
ffc_status ffc_interp_decomp(double* A_dev, int32_t batch, int32_t s, int32_t n, double tol,
                             int32_t max_rank, int32_t* rank_dev, int32_t* piv_dev,
                             double* P_dev, void* stream);

/* The same decompositions for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): nothing is allocated, freed or synchronized. The QR's exchange
 * slots, task counter and the solve's diagonal inverses live in a file-scope
 * device array of FFC_NOALLOC_SCRATCH_BYTES bytes that each GPU holds once
 * for the life of the process; the call clears what must start at zero. The
 * QR variant is the one the autotuner picked earlier for the same shape (via
 * ffc_interp_decomp or a skeletonization), else the first that fits; nothing
 * is timed. Limits: s <= 1024 (the register-resident QR; no streamed fallback)
 * and the blocks' scratch within the array (about 66 KB per 512 x 512 block,
 * so up to ~250 such blocks). The call is asynchronous on `stream`: inputs
 * and outputs must stay valid until the stream passes it. Calls that overlap
 * on one GPU (other streams, other threads) share the array and race: order
 * them on one stream. Errors: as ffc_interp_decomp, plus s > 1024 or blocks
 * beyond the scratch -> FFC_ERR_INVALID_ARG (nothing launched); the
 * cooperative launch refused because another process holds the device's
 * cooperative-launch resource -> FFC_ERR_STATE (there is no fallback here). */
#define FFC_NOALLOC_SCRATCH_BYTES (16u << 20)
ffc_status ffc_interp_decomp_noalloc(double* A_dev, int32_t batch, int32_t s, int32_t n, double tol,
                                     int32_t max_rank, int32_t* rank_dev, int32_t* piv_dev, double* P_dev,
                                     void* stream);

/* Per-node results copied to host (synchronizes). node in [1, num_nodes).
 * rank, n_cols, n_rows are required; cols/rows/skel (tree positions) and P
 * (rank x n_cols, row-major) may be NULL; buffers must hold n_cols, n_rows,
 * rank and rank * n_cols entries. */
ffc_status ffc_skel_node(const ffc_skel* sk, int32_t node, int32_t* rank, int32_t* n_cols,
                         int32_t* n_rows, int32_t* cols_host, int32_t* rows_host,
                         int32_t* skel_host, double* P_host);

/* A skeleton set from host arrays, such as a checkpoint written with
 * ffc_skel_node, for evaluation without skeletonizing. For every node a in
 * [1, num_nodes): rank_host[a] and ncols_host[a]; skel_host[a * r_max + i]
 * (i < rank, tree positions) and P_host[(a * r_max + i) * n_max + j]
 * (i < rank, j < ncols; entries past them are ignored). The columns are
 * implied by the tree: a leaf's points, an internal node's children's
 * skeletons (left, then right), so ncols must be the leaf's size or the sum of
 * the children's ranks. Only opts->separation is read (> 0 prepares the
 * separation bitmaps for the treecode and FMM-style evaluations); no rows are
 * stored, so the set cannot be passed back to ffc_skeletonize_nodes. Copies
 * the arrays (they may be freed on return) and synchronizes `stream`.
 * Errors: NULL arguments, r_max or n_max < 1, a rank outside [0,
 * min(r_max, ncols)], an ncols that breaks the nesting or exceeds n_max, a
 * skeleton id outside [0, N), a non-finite P entry, separation < 0 ->
 * FFC_ERR_INVALID_ARG. */
ffc_status ffc_skel_load(const ffc_tree* t, const ffc_skel_opts* o, const int32_t* rank_host,
                         const int32_t* ncols_host, const int32_t* skel_host, const double* P_host,
                         int32_t r_max, int32_t n_max, void* stream, ffc_skel** out);

typedef struct {
  int32_t num_nodes;        /* skeletonized nodes (all non-root nodes) */
  int32_t rank_min, rank_max;
  double rank_mean;
  int32_t rank_cap_hits;    /* nodes whose rank equals max_rank */
  int32_t fallbacks;        /* learned sampler: nodes redone with uniform rows */
  double kernel_evals;      /* sum over nodes of s * n_cols (final row counts) */
  int32_t resampled;        /* adaptive sample count: node redos with doubled rows */
  int32_t rows_max;         /* largest final row count of a node */
} ffc_stats;

/* Rank statistics of a skeleton set (synchronizes). */
ffc_status ffc_skel_stats(const ffc_skel* sk, ffc_stats* out);

/* One step of the hot path as a HIP graph: ffc_skeletonize_nodes (reusing `sk`,
 * with options `o`) followed by ffc_evaluate_sum, captured once on `stream` and
 * replayed by ffc_graph_launch. Every node of a level still runs in one
 * persistent cooperative launch; the graph removes the host-side launch work
 * of the ~40 kernels of a step. `sk` must come from a previous
 * ffc_skeletonize_nodes call with the same tree, kernel and options (so no
 * buffer is allocated inside the graph), and keeps being written by every
 * replay; q_dev, u_dev, u_far_dev (may be NULL) are baked into the graph and
 * must stay valid while it exists. Not for the learned sampler with a fallback
 * (its check synchronizes). `stream` must not be the null stream.
 * Errors: NULL arguments, a null stream, a fallback -> FFC_ERR_INVALID_ARG; a
 * failed capture -> FFC_ERR_HIP (the stream is left usable). */
typedef struct ffc_graph ffc_graph;
ffc_status ffc_step_graph_create(const ffc_tree* t, ffc_skel* sk, const ffc_kernel* k, const ffc_skel_opts* o,
                                 const double* q_dev, double* u_dev, double* u_far_dev, int32_t precision,
                                 void* stream, ffc_graph** out);
/* The same with the FMM-style evaluation (ffc_evaluate_fmm) in place of
 * ffc_evaluate_sum: o->separation must be > 0 (FFC_ERR_INVALID_ARG), and one
 * eager ffc_evaluate_fmm with this skeleton set at that separation must come
 * first, since it builds the interaction lists on the host (FFC_ERR_STATE
 * otherwise). */
ffc_status ffc_step_graph_create_fmm(const ffc_tree* t, ffc_skel* sk, const ffc_kernel* k, const ffc_skel_opts* o,
                                     const double* q_dev, double* u_dev, double* u_far_dev, int32_t precision,
                                     void* stream, ffc_graph** out);
ffc_status ffc_graph_launch(ffc_graph* g, void* stream);
/* Lifetime: a graph bakes in device buffers of its tree and skeleton set.
 * While it exists, a call that would allocate, resize or replace any of them
 * (an eager ffc_skeletonize_nodes with another separation, sampler, pool or
 * sample count; ffc_evaluate_fmm at another separation, which rebuilds the
 * FMM lists) fails with FFC_ERR_STATE and changes nothing; calls that reuse
 * the buffers as they are stay allowed. ffc_free_tree / ffc_free_skel on a
 * handle that a graph still holds only mark it: the last ffc_graph_free of
 * those graphs deletes it. ffc_graph_free synchronizes the device. */
void ffc_graph_free(ffc_graph* g);

/* ---------------------------------------------------------------------------
 * Learned row proposal.
 *
 * Leverage-score sampling of target rows (Section 3, importance sampling) is
 * the most reliable choice of rows but needs the whole block; the paper's
 * cheap alternatives are geometric heuristics (Section 3.2). The proposal
 * learns the map from 16 cheap geometric features of a target (against the
 * node's column set: distances to its centroid, to a 256-point subsample and
 * projections on 7 far anchors) to the log of its ridge leverage, with a
 * 16 -> 64 -> 64 -> 1 ReLU network in float32. Skeletonization then draws s
 * rows from a uniform pool of min(M, c s) candidates (c = pool_factor) with weights 0.9
 * softmax(score) + 0.1 / pool, without replacement (Efraimidis-Spirakis keys),
 * and redoes a node with uniform rows when the error on 32 held-out rows
 * exceeds fallback_tol.
 *
 * Parameters theta (FFC_PROPOSAL_NPARAM float32): W1 (16 x 64, row-major), b1
 * (64), W2 (64 x 64), b2 (64), w3 (64), b3. Standardization mu, sd (16 each):
 * the network sees (f - mu) / sd, with the constant feature 15 left at 1.
 * A proposal handle owns device copies of theta, mu, sd and the Adam moments.
 * ------------------------------------------------------------------------- */
#define FFC_PROPOSAL_NPARAM 5313
#define FFC_PROPOSAL_NFEAT 16

/* theta_host required; mu_host / sd_host may be NULL (0 and 1). Synchronous.
 * Errors: NULL theta or out, non-finite values -> FFC_ERR_INVALID_ARG. */
ffc_status ffc_proposal_create(const float* theta_host, const float* mu_host, const float* sd_host,
                               ffc_proposal** out);
/* Copies the current theta / mu / sd to the host (any may be NULL); synchronizes
 * the device. */
ffc_status ffc_proposal_get(const ffc_proposal* p, float* theta_host, float* mu_host, float* sd_host);
/* Adam state, for checkpoints that resume training: the first and second
 * moments (FFC_PROPOSAL_NPARAM float32 each) and the number of steps taken.
 * get: any output may be NULL; synchronizes the device. set: m1_host and
 * m2_host required, step >= 0; synchronous. Errors: NULL handle, NULL moments
 * (set), step < 0 or non-finite moments -> FFC_ERR_INVALID_ARG. */
ffc_status ffc_proposal_get_adam(const ffc_proposal* p, float* m1_host, float* m2_host, int32_t* step);
ffc_status ffc_proposal_set_adam(ffc_proposal* p, const float* m1_host, const float* m2_host, int32_t step);
void ffc_proposal_free(ffc_proposal* p);
/* Checkpoint of a proposal (the learned sampler of Section 3's importance
 * sampling; the network itself is this library's): parameters,
 * standardization and Adam state in a versioned binary file (version 1,
 * little-endian: magic "FFCPROP1", uint32 version, uint32 parameter count,
 * uint32 feature count, int32 Adam step, float32 theta, mu, sd, m1, m2, then
 * a 64-bit FNV-1a hash of all preceding bytes). save synchronizes the device
 * and writes `path` (host file name, overwritten); load reads it and returns a
 * new handle (free with ffc_proposal_free) whose scores, training and Adam
 * steps continue exactly where the saved one stood. Errors: NULL arguments, a
 * file that cannot be opened or written, a wrong size, magic, version,
 * network shape or hash -> FFC_ERR_INVALID_ARG (nothing is created). */
ffc_status ffc_proposal_save(const ffc_proposal* p, const char* path);
ffc_status ffc_proposal_load(const char* path, ffc_proposal** out);

/* Features of target rows against column sets, for `count` blocks: block g
 * has columns cols_dev[g * col_stride + j], j < ncols_dev[g] (tree positions,
 * at least 1), stream id ids_dev[g] (the node id in skeletonization) and
 * targets tgt_dev[g * tgt_stride + i], i < ntgt_dev[g] (tree positions); the
 * features go to feat_dev[(g * tgt_stride + i) * 16 + f] (other slots are not
 * written). All arrays are device arrays. Synchronizes (geometry scratch).
 * FFC_ERR_INVALID_ARG when col_stride > 16384 or when the column geometry does
 * not fit in a compute unit's LDS (8 d + 4 col_stride above about 114000
 * bytes for d > 64). */
ffc_status ffc_proposal_features(const ffc_tree* t, const int32_t* cols_dev, int32_t col_stride,
                                 const int32_t* ncols_dev, const int32_t* ids_dev, const int32_t* tgt_dev,
                                 int32_t tgt_stride, const int32_t* ntgt_dev, int32_t count, uint64_t seed,
                                 float* feat_dev, void* stream);
/* Sets mu, sd from `count` feature rows (population std floored at 1e-6). */
ffc_status ffc_proposal_fit_standardization(ffc_proposal* p, const float* feat_dev, int64_t count, void* stream);
/* score_dev[i] = network output for feature row i (feat_dev: count x 16 floats,
 * 16-byte aligned, as device allocations are; FP32 matrix-core arithmetic). */
ffc_status ffc_proposal_score(const ffc_proposal* p, const float* feat_dev, int64_t count, float* score_dev,
                              void* stream);
/* Mean squared error of the scores against target_dev over `count` rows and
 * its gradient (grad_dev: FFC_PROPOSAL_NPARAM floats, loss_dev: 1 float, both
 * device). Synchronizes (partial sums scratch). */
ffc_status ffc_proposal_gradient(const ffc_proposal* p, const float* feat_dev, const float* target_dev,
                                 int64_t count, float* grad_dev, float* loss_dev, void* stream);
/* One Adam step (beta 0.9, 0.999, eps 1e-8, bias-corrected; the handle counts
 * its steps) with the gradient grad_dev. */
ffc_status ffc_proposal_adam(ffc_proposal* p, const float* grad_dev, float lr, void* stream);

/* Ridge leverage of the rows of `count` row-major m x n blocks (B_dev, back
 * to back, not modified): l_i = b_i^T (B^T B + eps^2 ||B||_F^2 I)^{-1} b_i,
 * the smoothed form of the leverage of Section 3 that needs no rank choice;
 * target_dev (may be NULL) gets ln(max(l_i, 1e-12) m / sum(l)). A zero block
 * gives zeros. Errors: a factorization that fails (not positive definite)
 * -> FFC_ERR_NONFINITE. Synchronizes (scratch). */
ffc_status ffc_leverage_labels(const double* B_dev, int64_t m, int32_t n, int32_t count, double eps,
                               double* lev_dev, float* target_dev, void* stream);

/* Statistical leverage at the block's rank (Section 3, definition of
 * statistical leverage), from the method's own factorization: the column-
 * pivoted QR of each row-major m x n block B (largest trailing column norm
 * first, ties to the smaller column; stopped at the first pivot whose norm
 * is below eps times the first one's, else at min(m, n)) picks r columns J,
 * and l_i is the squared norm of row i of an orthonormal basis of
 * span(B(:, J)); sum(l) = r, and for a block of exact rank r this is the
 * leverage of its top r singular vectors. Computed through B^T B, whose
 * diagonal-pivoted Cholesky factorization has the same pivots and R.
 * B_dev (count blocks back to back) is not modified; lev_dev gets count x m
 * scores, target_dev (may be NULL) ln(max(l_i, 1e-12) m / sum(l));
 * rank_host (may be NULL) the r of each block, piv_host (may be NULL,
 * count x n) the pivot order (its first r entries are J). A zero block gives
 * zeros and rank 0. Errors: n > 1024, eps outside (0, 1), bad sizes or NULL
 * arrays -> FFC_ERR_INVALID_ARG. Synchronizes (scratch). */
ffc_status ffc_pivoted_leverage_labels(const double* B_dev, int64_t m, int32_t n, int32_t count, double eps,
                                       double* lev_dev, float* target_dev, int32_t* rank_host, int32_t* piv_host,
                                       void* stream);

/* Proposal training. Block g of the training set takes a random leaf of the
 * tree, n = min(block_cols, smallest leaf) of its points as columns and m =
 * min(block_rows, N - largest leaf) points outside it as targets (counter-based
 * draws from `seed`); its samples are the targets' features and the targets
 * of the leverage of K(targets, columns) in float64 (o->label: the pivoted
 * leverage at the block's eps-rank, or the ridge form). Training fits the
 * standardization on all samples, then runs `epochs` passes of mini-batch Adam
 * (`batch` samples per step, learning rate lr) on the mean squared error, the
 * epoch's order a seeded stride permutation. loss_host (epochs floats, may be
 * NULL) receives each epoch's mean loss. Synchronizes.
 * Errors: num_blocks < 1, block sizes < 1, batch < 1, epochs < 0 ->
 * FFC_ERR_INVALID_ARG. */
typedef enum {
  FFC_LABEL_PIVOTED = 0,   /* ffc_pivoted_leverage_labels: leverage at the block's eps-rank (default) */
  FFC_LABEL_RIDGE = 1      /* ffc_leverage_labels: ridge leverage with lambda = eps^2 ||B||_F^2 */
} ffc_label_kind;
typedef struct {
  int32_t num_blocks;
  int32_t block_cols;
  int32_t block_rows;
  int32_t epochs;
  int32_t batch;
  float lr;
  double eps;
  uint64_t seed;
  int32_t label;   /* ffc_label_kind of the targets */
} ffc_train_opts;
ffc_status ffc_proposal_train(ffc_proposal* p, const ffc_tree* t, const ffc_kernel* k, const ffc_train_opts* o,
                              float* loss_host, void* stream);
/* The training set of ffc_proposal_train without the training: block leaves,
 * columns (num_blocks x n), targets (num_blocks x m), features
 * (num_blocks * m x 16) and label targets (num_blocks * m) into device arrays
 * sized by the caller from n_out / m_out, which a first call with all arrays
 * NULL returns. Synchronizes. */
ffc_status ffc_proposal_training_set(const ffc_tree* t, const ffc_kernel* k, const ffc_train_opts* o,
                                     int32_t* n_out, int32_t* m_out, int32_t* leaves_dev, int32_t* cols_dev,
                                     int32_t* rows_dev, float* feat_dev, float* target_dev, double* lev_dev,
                                     void* stream);

/* Synchronizes `stream` and reports (then clears) the device error flag:
 * FFC_ERR_NONFINITE if a kernel value or sum was not finite since the last check,
 * FFC_ERR_HIP if a bounded wait inside the QR kernel gave up (its results
 * are then invalid). */
ffc_status ffc_check_device(void* stream);

/* Stage profiler (tracing). When enabled, every stage launch is bracketed by
 * two HIP events recorded on the stream the stage runs on; ffc_profile_read
 * waits for them and returns the accumulated milliseconds and launch counts
 * per stage (index = ffc_stage), optionally resetting the totals. */
typedef enum {
  FFC_STAGE_TREE = 0,      /* tree construction */
  FFC_STAGE_SAMPLE = 1,    /* target-row sampling */
  FFC_STAGE_COLUMNS = 2,   /* per-level column lists */
  FFC_STAGE_KBLOCK = 3,    /* sampled kernel blocks K' */
  FFC_STAGE_CPQR = 4,      /* column-pivoted QR factorization kernel */
  FFC_STAGE_SKEL = 5,      /* skeleton ids */
  FFC_STAGE_UPWARD = 6,    /* equivalent charges */
  FFC_STAGE_EVALUATE = 7,  /* far + near field sums */
  FFC_STAGE_DIRECT = 8,    /* direct sums */
  FFC_STAGE_SOLVE = 9,     /* QR set-up and interpolation solve R11 T = R12, P */
  FFC_STAGE_PROPOSAL = 10, /* learned sampler: pool, geometry, features, scores, selection */
  FFC_STAGE_HELDOUT = 11,  /* learned sampler: held-out rows, their block and the check */
  FFC_STAGE_LABELS = 12,   /* training set: blocks, ridge leverage, geometry and features */
  FFC_STAGE_TRAIN = 13,    /* proposal training: gradients and Adam steps */
  FFC_NUM_STAGES = 14
} ffc_stage;
ffc_status ffc_profile_enable(int32_t on);
/* Autotuner: the first pivoted-QR launch of each block shape times the kernel
 * variants (lanes and rows per column, workgroup size) that can hold the blocks on a copy of
 * them and keeps the fastest; FFC_AUTOTUNE=0 in the environment disables it.
 * Writes up to `cap` entries of 8 int32 (s_max, n_max, batch, rank cap, 100 x
 * the most rows the variant holds + columns per lane group, threads per workgroup, best time in
 * us, first candidate's time in us or -1 for a choice read from the cache) to
 * out_host and their total number to *count. With FFC_TUNE_CACHE=<file> in
 * the environment the choices persist: they are read from the file on first
 * use and each new one is appended (one text line per choice, keyed by the
 * device's architecture name and compute-unit count), so later processes on
 * the same kind of device skip the timing. */
ffc_status ffc_autotune_report(int32_t* out_host, int32_t cap, int32_t* count);
/* Forgets the autotuner's choices in this process; the next factorization
 * reads FFC_TUNE_CACHE again (when set) and times the shapes it does not find
 * there. Not to be called while another thread factors blocks. */
void ffc_autotune_reset(void);
ffc_status ffc_profile_read(double* ms_host, int64_t* launches_host, int32_t num_stages, int32_t reset);

void ffc_free_tree(ffc_tree* t);
void ffc_free_skel(ffc_skel* sk);
/* Releases the library's process-wide resources: synchronizes the device and
 * destroys the stage profiler's pooled HIP events (the device error flag is a
 * file-scope device word and needs no release). Call it after the last handle
 * is freed and before
 * the process exits, so that nothing of the library's is torn down by static
 * destructors or runtime teardown (the Python binding calls it at interpreter
 * exit, after freeing its live handles). Later calls of the library remain
 * valid and recreate what they need. */
void ffc_shutdown(void);
const char* ffc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FFC_H */
