// Register-resident batched column-pivoted QR (the ID of Section 2.1.3 /
// Appendix 6.1), distributed over a group of workgroups per block.
//
// Right-looking Householder QR with column pivoting re-reads the whole
// trailing block at every pivot step, so with the block in HBM it is bound by
// memory traffic. Here each block (s <= 1024 rows) is spread over G
// workgroups: a workgroup owns 8 wavefronts x 8 columns, each column held by
// 16 lanes (32 lanes and 4 columns per wavefront for blocks of more than 512
// rows) with up to 32 rows per lane in VGPRs for the whole factorization.
// One pivot step then needs no block traffic at all:
//   1. every workgroup loads the winning column (published at the end of the
//      previous step, one row per thread) into LDS and forms the reflector
//      v, beta = 2 / v^T v;
//   2. it applies the reflector to its own non-pivot columns in registers and
//      recomputes their trailing norms exactly (rows k+1..s-1);
//   3. it publishes its best column (largest norm, ties to the smaller
//      original column): norm, column id and rows k..s-1 go to the group's
//      double-buffered slot, one word per thread, with no wait;
//   4. one wave polls the G slots' norm and id words and picks the global
//      best, which every workgroup then applies alike (pivot and stop rule).
// Every published word carries the step's tag (1 + k mod 3) in its two lowest
// mantissa bits, so a reader accepts a word only once the current step's
// store has reached it and rereads otherwise: no store has to be waited for
// before another becomes visible. The tag perturbs a published value by at
// most 3 ulp (its two lowest bits are cleared after the check), the same on
// every workgroup, far below the rounding of the factorization. Slots are
// cleared before every launch; a slot read at step k can otherwise only hold
// step k - 2, whose tag differs.
// Row k of every active column is final after step k. The register block
// that holds row k is kept in its own register (cur) and is zero in the block
// array, as are the blocks above, so norms and reflector products over the
// array need no row masks, and the current block's finished rows are masked
// by lane; when the next block takes its place, the finished block goes to A
// as one contiguous segment per column. The pivot column of step k is frozen
// in place (its rows 0..k-1 go to A with their blocks, row k gets alpha), so
// no columns are swapped; the pivot order is recorded. A ends with
// R(0:l+1, l) in column piv[l] and R(0:r, j) in rows 0..r-1 of every other
// column j.
//
// Scheduling: the groups of a level form a flat task list (block 0's G_0
// parts, then block 1's, ...); the workgroups of a persistent grid, all
// co-resident (guaranteed by the cooperative launch), claim tasks in order
// from a counter as they become free. The claimed tasks are always a prefix
// of the list, so every block but the last claimed one has all its members
// running and finishes, freeing workgroups for the rest: no deadlock as long
// as G <= grid. Barrier waits are bounded; a timeout raises bit 1 of the
// device flag and the workgroup abandons its remaining work, so every wave
// exits.
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <mutex>
#include <type_traits>
#include <vector>

#include "ffc_internal.h"
#include "lane_ops.h"

namespace ffc {
namespace {

constexpr unsigned int kSpinLimit = 1u << 21;   // ~1 us per poll -> about 2 s

struct CoopArgs {
  double* A;
  int64_t a_stride;
  int lda;
  const int32_t* s_arr;
  const int32_t* n_arr;
  int s_uniform, n_uniform;
  int count;
  double tol;
  int max_rank;
  int32_t* rank;
  int32_t* piv;
  int64_t piv_stride;
  int32_t* task_start;       // [count + 1]
  const unsigned char* mask; // [count]: blocks to factor (all when null); the others get no tasks
  int32_t* claim;            // next unclaimed task
  double* slots;             // [count][2][gmax][s_max + 2]: norm, column id, rows (tagged words)
  int64_t slot_words;
  int gmax;
  int s_max;
  int cols_per_wg;
  unsigned int* flag;
};

struct Best {
  double v;
  int orig;
};

__device__ inline bool better(double v, int o, double bv, int bo) { return v > bv || (v == bv && o < bo); }

// Group tasks per block: G_b = ceil(n_b / cols_per_wg) (at least 1); prefix
// sums into task_start. Run by one 256-thread workgroup.
__device__ void coop_tasks(const CoopArgs& ca) {
  __shared__ int wtot[4];
  __shared__ int s_base;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) {
    *ca.claim = 0;
    s_base = 0;
  }
  __syncthreads();
  // Block-wide exclusive scan over chunks of 256 blocks: shuffle scan per
  // wavefront, then the totals of the wavefronts before this one.
  for (int b0 = 0; b0 < ca.count; b0 += 256) {
    const int b = b0 + (int)threadIdx.x;
    int g = 0;
    if (b < ca.count && !(ca.mask && !ca.mask[b])) {
      const int n = ca.n_arr ? ca.n_arr[b] : ca.n_uniform;
      g = max(1, (n + ca.cols_per_wg - 1) / ca.cols_per_wg);
    }
    int incl = g;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off);
      if (lane >= off) incl += y;
    }
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    int pos = s_base + incl - g;
    for (int v = 0; v < w; ++v) pos += wtot[v];
    if (b < ca.count) ca.task_start[b] = pos;
    __syncthreads();
    if (threadIdx.x == 0) s_base += wtot[0] + wtot[1] + wtot[2] + wtot[3];
    __syncthreads();
  }
  if (threadIdx.x == 0) ca.task_start[ca.count] = s_base;
}

// Set-up of a factorization launch: workgroup 0 computes the task offsets
// and resets the claim counter; all workgroups clear the slots (tag 0 is
// never a step's tag).
__global__ void __launch_bounds__(256) k_coop_setup(CoopArgs ca) {
  if (blockIdx.x == 0) coop_tasks(ca);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ca.slot_words;
       e += (int64_t)gridDim.x * blockDim.x)
    ca.slots[e] = 0.0;
}

__device__ inline double* slot_ptr(const CoopArgs& ca, int b, int buf, int g) {
  return ca.slots + (((int64_t)b * 2 + buf) * ca.gmax + g) * (int64_t)(ca.s_max + 2);
}

// Slot traffic uses relaxed agent-scope atomic loads and stores: they are
// performed coherently across the chiplets' L2 caches, so no cache-wide fence
// (L2 write-back / invalidate) is needed.
__device__ inline void slot_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double slot_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline long long step_tag(int k) { return 1 + k % 3; }
__device__ inline double tagged(double v, long long tag) {
  return __longlong_as_double((__double_as_longlong(v) & ~3ll) | tag);
}
__device__ inline long long tag_of(double v) { return __double_as_longlong(v) & 3ll; }
__device__ inline double untag(double v) { return __longlong_as_double(__double_as_longlong(v) & ~3ll); }

// Register layout: a wavefront is 64 / LG lane groups of LG lanes (16 or 32);
// a lane group owns CS columns and each of its lanes keeps RL rows
// (i = lg + LG m) of them, so a column's dot products and norms are LG-lane
// reductions (16-lane DPP, plus one exchange between row pairs for LG = 32).
// Variants: RL rows per lane (16 or 32), CS columns per lane group (2, or 1
// to halve the per-wave work of a step for small batches), NTC threads per
// workgroup (512, 256 or 128) and LG (32 for blocks of up to 1024 rows); all
// keep at most 256 VGPRs per lane.
template <int LG>
__device__ inline double group_sum(double x) {
  x = row16_sum(x);
  if constexpr (LG == 32) x += __shfl_xor(x, 16, 64);   // a + b = b + a: both rows end equal
  return x;
}

template <int RL, int CS, int NTC, int LG>
__global__ void __launch_bounds__(NTC, 2) k_cpqr_coop(CoopArgs ca) {
  static_assert(LG == 16 || LG == 32, "lane groups of 16 or 32 lanes");
  constexpr int NG = 64 / LG;          // lane groups per wavefront
  constexpr int CPW = NG * CS;         // columns per wavefront
  constexpr int ROWS = LG * RL;        // rows a lane group holds (LDS rows are padded to it)
  constexpr int NWVC = NTC / 64;       // wavefronts per workgroup
  __shared__ Best wb[NWVC];
  __shared__ int s_win[3];             // {ok, winner group, winner column}
  __shared__ double s_nv;              // winner's norm (tag cleared)
  __shared__ double s_xk;              // winner's row k
  __shared__ double s_vcb[LG];         // the reflector's rows in the current register block
  extern __shared__ double lds[];      // NWVC candidate columns, then the winner column (ROWS each)
  double* candcol = lds;
  double* wincol = lds + NWVC * ROWS;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int grp = lane / LG, lg = lane & (LG - 1);
  // Tasks (block b, part g) are taken in order from a counter by whichever
  // workgroup is free, so a level with more tasks than resident workgroups is
  // balanced by how long each block takes rather than in fixed rounds.
  __shared__ int s_task;
  const int T = ca.task_start[ca.count];
  for (;;) {
    if (threadIdx.x == 0) s_task = atomicAdd(ca.claim, 1);
    __syncthreads();
    const int task = s_task;
    __syncthreads();   // s_task is rewritten at the next claim
    if (task >= T) break;
    // Block of this task: largest b with task_start[b] <= task.
    int lo = 0, hi = ca.count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ca.task_start[mid] <= task) lo = mid; else hi = mid - 1;
    }
    const int b = lo;
    const int g = task - ca.task_start[b];
    const int G = ca.task_start[b + 1] - ca.task_start[b];
    const int s = ca.s_arr ? ca.s_arr[b] : ca.s_uniform;
    const int n = ca.n_arr ? ca.n_arr[b] : ca.n_uniform;
    double* A = ca.A + (int64_t)b * ca.a_stride;   // element offsets within a block fit in 32 bits
    const int col0 = g * ca.cols_per_wg + w * CPW + grp * CS;   // this lane group's first column
    int32_t* pivb = ca.piv + (int64_t)b * ca.piv_stride;

    // Row lg + LG m exists for m < mlim. (Comparing m, an immediate, with
    // one per-lane bound keeps the compiler from holding all RL row indices
    // in registers across the task loop.)
    const int mlim = s > lg ? (s - lg + LG - 1) / LG : 0;
    double a[CS][RL];
#pragma unroll
    for (int c = 0; c < CS; ++c) {
      const double* colp = A + (int64_t)(col0 + c) * ca.lda + lg;
      const bool jin = col0 + c < n;
#pragma unroll
      for (int m = 0; m < RL; ++m) a[c][m] = (jin && m < mlim) ? colp[LG * m] : 0.0;
    }
    unsigned int done = 0u;   // bit c: column col0 + c is a frozen pivot
    int kfz[CS];              // the step at which column col0 + c was frozen
#pragma unroll
    for (int c = 0; c < CS; ++c) kfz[c] = INT_MAX;

    // The register block that holds row k (block kb = k / LG, rows
    // LG kb + lg) lives in cur[] instead of a[][kb], which is kept zero
    // together with every block above it. Rows above the active ones thus
    // drop out of the norms and of the reflector products without a
    // register index that depends on k: R(k, j) is read from cur, and only
    // the move of a new block into cur, once every LG steps, indexes the
    // registers. The reflector's rows of the current block are staged apart
    // (s_vcb) and are zero in wincol, so the loops over a[][] never touch
    // them.
    double cur[CS];
#pragma unroll
    for (int c = 0; c < CS; ++c) {
      cur[c] = a[c][0];
      a[c][0] = 0.0;
    }
    int kb = 0;
    // R rows leave the registers a block at a time: the finished rows of the
    // current block (those below lim) go to A as one contiguous LG-row
    // segment per column, instead of one scattered word per row and step.
    auto store_block = [&](int lim) {
#pragma unroll
      for (int c = 0; c < CS; ++c) {
        const int j = col0 + c, row = LG * kb + lg;
        if (j < n && row < min(lim, kfz[c])) A[(uint32_t)(j * ca.lda + row)] = cur[c];
      }
    };
    // Norm of the rows at or below row kk (kk in the current block or the
    // first row of the next one).
    auto active_norm = [&](int c, int kk) -> double {
      double n2[2] = {0.0, 0.0};   // even and odd m: two chains of dependent FMAs
#pragma unroll
      for (int m = 0; m < RL; ++m) n2[m & 1] = fma(a[c][m], a[c][m], n2[m & 1]);
      const double y = LG * kb + lg >= kk ? cur[c] : 0.0;
      return group_sum<LG>(fma(y, y, n2[0] + n2[1]));
    };

    // Publish this workgroup's best column for step k (trailing norms over rows >= k).
    auto publish = [&](int k) {
      Best best{-1.0, INT_MAX};
      int bestc = -1;
#pragma unroll
      for (int c = 0; c < CS; ++c) {
        const double nrm = active_norm(c, k);
        const int j = col0 + c;
        if (j < n && !(done & (1u << c)) && better(nrm, j, best.v, best.orig)) {
          best = Best{nrm, j};
          bestc = c;
        }
      }
      // Best of the lane groups of the wavefront (same result in every lane).
      Best wbst{readlane_d(best.v, 0), __builtin_amdgcn_readlane(best.orig, 0)};
      int wg_owner = 0;
#pragma unroll
      for (int q = 1; q < NG; ++q) {
        const Best o{readlane_d(best.v, LG * q), __builtin_amdgcn_readlane(best.orig, LG * q)};
        if (better(o.v, o.orig, wbst.v, wbst.orig)) { wbst = o; wg_owner = q; }
      }
      // The wave's best column goes to its LDS candidate row (all ROWS rows;
      // only rows k..s-1 are published).
      // (The column is picked with selects, in the form that keeps a[][] in
      // registers: an index into it would move the array to scratch memory.)
      if (wbst.orig != INT_MAX && grp == wg_owner) {
#pragma unroll
        for (int m = 0; m < RL; ++m) {
          double x = a[0][m];
#pragma unroll
          for (int c = 1; c < CS; ++c) x = bestc == c ? a[c][m] : x;
          candcol[w * ROWS + lg + LG * m] = x;
        }
        double y = cur[0];
#pragma unroll
        for (int c = 1; c < CS; ++c) y = bestc == c ? cur[c] : y;
        candcol[w * ROWS + LG * kb + lg] = y;   // the current block (zero in a[][kb])
      }
      if (lane == 0) wb[w] = wbst;
      __syncthreads();
      Best gb = wb[0];
      int gw = 0;
      for (int i = 1; i < NWVC; ++i)
        if (better(wb[i].v, wb[i].orig, gb.v, gb.orig)) { gb = wb[i]; gw = i; }
      double* sl = slot_ptr(ca, b, k & 1, g);
      const long long tag = step_tag(k);
      if (gb.orig != INT_MAX) {
        constexpr int PER = (ROWS + NTC - 1) / NTC;   // rows per thread, all read before any store
        double x[PER];
#pragma unroll
        for (int t = 0; t < PER; ++t) x[t] = candcol[gw * ROWS + min(k + (int)threadIdx.x + t * NTC, ROWS - 1)];
#pragma unroll
        for (int t = 0; t < PER; ++t) {
          const int i = k + (int)threadIdx.x + t * NTC;
          if (i < s) slot_store(sl + 2 + i, tagged(x[t], tag));
        }
      }
      if (threadIdx.x == 0) {
        const bool any = gb.orig != INT_MAX;
        slot_store(sl + 1, tagged(any ? (double)gb.orig : -1.0, tag));
        slot_store(sl, tagged(any ? gb.v : -1.0, tag));
      }
    };
    // Wave 0 waits for the G norm / id words of step k and picks the winner;
    // the result is shared through LDS so every wave takes the same decisions.
    auto poll = [&](int k, int& gwin, int& orig) -> bool {
      if (w == 0) {
        const long long tag = step_tag(k);
        Best bb{-1.0, INT_MAX};
        int bq = -1;
        bool ok = true;
        for (int q0 = 0; q0 < G; q0 += 64) {
          const int q = q0 + lane;
          Best c{-1.0, INT_MAX};
          if (q < G) {
            const double* sq = slot_ptr(ca, b, k & 1, q);
            unsigned int spins = 0;
            double nv = 0.0, ov = 0.0;
            for (;;) {
              nv = slot_load(sq);
              ov = slot_load(sq + 1);
              if (tag_of(nv) == tag && tag_of(ov) == tag) break;
              if (++spins > kSpinLimit) { ok = false; break; }
              __builtin_amdgcn_s_sleep(1);
            }
            const double o = untag(ov);
            if (ok && o >= 0.0) c = Best{untag(nv), (int)rint(o)};
          }
          // Best of these 64 slots: the largest norm (DPP maximum within rows
          // of 16, then across the four rows), ties to the smallest column id
          // among the lanes that hold it (found by ballot; usually one).
          double vm = row16_max(c.v);
          vm = fmax(fmax(readlane_d(vm, 0), readlane_d(vm, 16)), fmax(readlane_d(vm, 32), readlane_d(vm, 48)));
          unsigned long long hit = __ballot(c.orig != INT_MAX && c.v == vm);
          while (hit) {
            const int L = __ffsll((long long)hit) - 1;
            hit &= hit - 1;
            const int o = __builtin_amdgcn_readlane(c.orig, L);
            if (better(vm, o, bb.v, bb.orig)) {
              bb = Best{vm, o};
              bq = q0 + L;
            }
          }
        }
        const bool all_ok = __all(ok);
        if (!all_ok && lane == 0) atomicOr(ca.flag, 2u);
        if (lane == 0) {
          s_win[0] = all_ok ? 1 : 0;
          s_win[1] = bq;
          s_win[2] = bb.orig;
          s_nv = bb.v;
        }
      }
      __syncthreads();
      gwin = s_win[1];
      orig = s_win[2];
      return s_win[0] != 0;
    };
    // The reflector v of step k into LDS: rows k+1..s-1 of the winner's column,
    // x_k - alpha in row k (x_k kept in s_xk), zero elsewhere (rows >= s are
    // cleared once per block, row k - 1 at step k). One row per thread,
    // reread until every word carries step k's tag. False on timeout.
    auto load_winner = [&](int k, int gwin) -> bool {
      const double* sl = slot_ptr(ca, b, k & 1, gwin);
      const long long tag = step_tag(k);
      const double rho = sqrt(s_nv);
      // Rows of block k / LG (the current register block at step k) go to
      // s_vcb and are zero in wincol; row k - 1, when it is in that block,
      // is cleared in s_vcb (the rows of earlier blocks are already zero).
      const int vb = k / LG * LG;   // first row of the current block
      if (k > vb && threadIdx.x == 0) s_vcb[(k - 1) & (LG - 1)] = 0.0;
      constexpr int PER = (ROWS + NTC - 1) / NTC;   // rows per thread, all loaded before any is used
      for (unsigned int spins = 0;; ++spins) {
        int stale = 0;
        double raw[PER];
#pragma unroll
        for (int t = 0; t < PER; ++t) {
          const int i = k + (int)threadIdx.x + t * NTC;
          raw[t] = i < s ? slot_load(sl + 2 + i) : 0.0;
        }
#pragma unroll
        for (int t = 0; t < PER; ++t) {
          const int i = k + (int)threadIdx.x + t * NTC;
          if (i < s) stale |= tag_of(raw[t]) != tag;
          double x = untag(raw[t]);   // 0 for rows >= s
          if (i == k) {
            s_xk = x;
            x = x - (x != 0.0 ? -copysign(rho, x) : -rho);
          }
          if (i < vb + LG) {
            s_vcb[i & (LG - 1)] = x;
            wincol[i] = 0.0;
          } else if (i < ROWS) {
            wincol[i] = x;
          }
        }
        if (!__syncthreads_or(stale)) return true;
        if (spins > kSpinLimit) {
          if (threadIdx.x == 0) atomicOr(ca.flag, 2u);
          return false;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    };

    for (int i = threadIdx.x; i < ROWS; i += NTC) wincol[i] = 0.0;
    if (threadIdx.x < LG) s_vcb[threadIdx.x] = 0.0;
    publish(0);   // its barrier also orders the clearing above
    int gwin, porig;
    bool alive = poll(0, gwin, porig);
    if (alive && porig != INT_MAX) alive = load_winner(0, gwin);
    const int kmax = min(min(s, n), ca.max_rank);
    double nv = s_nv;
    const double rho0 = (alive && porig != INT_MAX) ? sqrt(nv) : 0.0;
    int k = 0;
    for (; alive && k < kmax; ++k) {
      if (porig == INT_MAX) break;
      const double rho = sqrt(nv);
      if (rho == 0.0 || rho < ca.tol * rho0) break;
      const double xk = s_xk;
      const double alpha = xk != 0.0 ? -copysign(rho, xk) : -rho;
      if (k > 0 && k % LG == 0) {
        // Row k opens register block kb + 1: the old block's rows, all final,
        // go to A; the new block's rows move into cur and a[][kb + 1] becomes
        // zero, once every LG steps. Straight-line selects against a per-lane
        // copy of the block index: branches on it would merge every register
        // of a[][] at their joins.
        store_block(k);
        ++kb;
        int kbv;
        asm volatile("v_mov_b32 %0, %1" : "=v"(kbv) : "s"(kb));
#pragma unroll
        for (int c = 0; c < CS; ++c) {
          double y = 0.0;
#pragma unroll
          for (int m = 1; m < RL; ++m) {
            const bool hit = kbv == m;
            y = hit ? a[c][m] : y;
            a[c][m] = hit ? 0.0 : a[c][m];
          }
          cur[c] = y;
        }
      }
      const double vcur = s_vcb[lg];
      double v[RL];   // the reflector's rows of this lane, for the second pass
      // v^T a for each held column, in two partial sums (even and odd m).
      double dots[CS][2];
#pragma unroll
      for (int c = 0; c < CS; ++c) dots[c][0] = dots[c][1] = 0.0;
#pragma unroll
      for (int m = 0; m < RL; ++m) {   // wincol: the reflector below the current block, zero above
        v[m] = wincol[lg + LG * m];
#pragma unroll
        for (int c = 0; c < CS; ++c) dots[c][m & 1] = fma(v[m], a[c][m], dots[c][m & 1]);
      }
      // v^T v in closed form: v = x - alpha e_k with x^T x = rho^2 and
      // alpha = -sign(x_k) rho, so v^T v = 2 rho (rho + |x_k|).
      const double vv = 2.0 * rho * (rho + fabs(xk));
      const double beta = vv > 0.0 ? 2.0 / vv : 0.0;
      // Freeze the pivot column: its rows 0..k-1 go to A with their blocks,
      // row k gets alpha now.
      if (g == gwin) {
#pragma unroll
        for (int c = 0; c < CS; ++c)
          if (col0 + c == porig) {
            done |= 1u << c;
            kfz[c] = k;
            if (lg == (k & (LG - 1))) A[(uint32_t)(porig * ca.lda + k)] = alpha;
          }
        if (threadIdx.x == 0) pivb[k] = porig;
      }
      // Apply the reflector to the non-pivot columns (a frozen or absent
      // column gets a zero coefficient, which leaves it unchanged).
      double coef[CS];
#pragma unroll
      for (int c = 0; c < CS; ++c) {
        const double dot = group_sum<LG>(fma(vcur, cur[c], dots[c][0] + dots[c][1]));
        coef[c] = (col0 + c < n && !(done & (1u << c))) ? dot * beta : 0.0;
      }
#pragma unroll
      for (int m = 0; m < RL; ++m) {
#pragma unroll
        for (int c = 0; c < CS; ++c) a[c][m] = fma(-v[m], coef[c], a[c][m]);
      }
      // Row k of the active columns is now final, R(k, j). It stays in cur
      // (the norms and products of later steps leave it out) until its block
      // is stored.
#pragma unroll
      for (int c = 0; c < CS; ++c) cur[c] = fma(-vcur, coef[c], cur[c]);
      publish(k + 1);
      alive = poll(k + 1, gwin, porig);
      if (alive && porig != INT_MAX && k + 1 < kmax) alive = load_winner(k + 1, gwin);
      nv = s_nv;
    }
    if (!alive) return;   // timed out: the device flag reports it
    store_block(k);       // the rows 0..k-1 of the last block
    if (g == 0 && threadIdx.x == 0) ca.rank[b] = k;
  }
}


// ---------------------------------------------------------------------------
// T = R11^{-1} R12 on matrix cores (v_mfma_f64_16x16x4f64, FP64 operands and
// accumulation). Back substitution in blocks of 16 rows, bottom-up: the
// contribution of the rows already solved below a block is one 16 x K by
// K x 16 product, and the block is then solved by multiplying with the inverse
// of its 16 x 16 diagonal block of R (formed beforehand by k_diag_inv), one
// more 16 x 16 x 16 product. One wavefront per (block, 16-column chunk): it
// writes the identity part of P for the pivot columns among columns
// [16 ch, 16 ch + 16) and solves for the non-pivot columns whose place in the
// ascending non-pivot order is in that range, their right-hand sides held in
// LDS. Operand layouts of the 16x16x4 FP64 instruction (checked on the
// device): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives
// D[4 v + l / 16][l % 16] for v = 0..3.
// ---------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int MB = 16;    // rows per diagonal block, columns per chunk
constexpr int MTS = 17;   // LDS row stride of the right-hand sides, in doubles

int round_mb(int x) { return (x + MB - 1) / MB * MB; }
__device__ inline int round_mb_dev(int x) { return (x + MB - 1) / MB * MB; }

size_t mfma_solve_lds_bytes(int r_max, int n_max) {
  return (size_t)(round_mb(r_max) + MB) * MTS * sizeof(double) +
         ((size_t)r_max + MB + (n_max + 31) / 32 + 2 * MB) * sizeof(int);
}

int solve_rank_bound(const IdBatch& bt) { return std::max(1, std::min(bt.max_rank, std::min(bt.s_max, bt.n_max))); }

// Diagonal block inverses of the matrix-core solve: batch x blocks x 16 x 16.
size_t solve_scratch_bytes(const IdBatch& bt, int batch) {
  return (size_t)batch * (round_mb(solve_rank_bound(bt)) / MB) * MB * MB * sizeof(double);
}

// Inverse of each 16 x 16 diagonal block of R11, rows and columns past the
// rank padded with the identity; one wavefront per (block, diagonal block),
// lane c < 16 back-substituting U x = e_c. Dinv[b][kd] is row-major 16 x 16.
__global__ void __launch_bounds__(64)
k_diag_inv(const double* __restrict__ A, int64_t a_stride, int lda, const int32_t* __restrict__ rank,
           const int32_t* __restrict__ piv, int64_t piv_stride, double* __restrict__ Dinv, int nblk,
           const unsigned char* __restrict__ mask) {
  __shared__ double U[MB][MB + 1];
  const int b = blockIdx.x, kd = blockIdx.y, kb = MB * kd;
  if (mask && !mask[b]) return;
  const int r = rank[b];
  if (kb >= r) return;
  const int nii = min(MB, r - kb);
  const double* Ab = A + (int64_t)b * a_stride;
  const int32_t* pb = piv + (int64_t)b * piv_stride;
  for (int e = threadIdx.x; e < MB * MB; e += 64) {
    const int i = e % MB, j = e / MB;   // consecutive lanes walk down a column of R
    double v = i == j ? 1.0 : 0.0;
    if (i <= j && j < nii) v = Ab[(int64_t)pb[kb + j] * lda + kb + i];
    U[i][j] = v;
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < MB) {
    double x[MB];
#pragma unroll
    for (int i = MB - 1; i >= 0; --i) {
      double t = i == c ? 1.0 : 0.0;
#pragma unroll
      for (int j = i + 1; j < MB; ++j) t = fma(-U[i][j], x[j], t);
      x[i] = t / U[i][i];
    }
    double* D = Dinv + ((int64_t)b * nblk + kd) * MB * MB;
#pragma unroll
    for (int i = 0; i < MB; ++i) D[i * MB + c] = x[i];
  }
}

// The columns of a solve chunk, in LDS: pv = the pivot order (pv[r..r+15] =
// pv[0], a real column for the rows past the rank), isp = the pivot bitmap,
// npc = the chunk's non-pivot columns (place j0 + c in ascending non-pivot
// order), posl = the pivot position of column j0 + c or -1. One wavefront;
// synchronizes.
__device__ inline void solve_columns(const int32_t* __restrict__ pb, int r, int n, int j0, int* pv,
                                     unsigned int* isp, int* npc, int* posl) {
  const int lane = threadIdx.x;
  for (int w = lane; w < (n + 31) / 32; w += 64) isp[w] = 0u;
  if (lane < MB) posl[lane] = -1;
  __syncthreads();
  // (Pivot loads of up to 8 passes are issued together, then used: one
  // memory round trip instead of one per pass.)
  for (int l0 = 0; l0 < r; l0 += 64 * 8) {
    int jl[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int l = l0 + 64 * u + lane;
      jl[u] = l < r ? pb[l] : -1;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int l = l0 + 64 * u + lane, j = jl[u];
      if (l < r) {
        pv[l] = j;
        atomicOr(&isp[j >> 5], 1u << (j & 31));
        if (j >= j0 && j < j0 + MB) posl[j - j0] = l;
      }
    }
  }
  // Past the rank the trailing products read a real column of R against
  // zero right-hand sides, so no lane needs a bounds test.
  if (r > 0 && lane < MB) pv[r + lane] = pb[0];
  __syncthreads();
  // Non-pivot columns in ascending order (place = j minus the pivots below j).
  int base = 0;
  for (int c0 = 0; c0 < n && base < j0 + MB; c0 += 64) {
    const int j = c0 + lane;
    const bool f = j < n && !((isp[j >> 5] >> (j & 31)) & 1u);
    const unsigned long long m = __ballot(f);
    const int q = base + __popcll(m & ((1ull << lane) - 1ull));
    if (f && q >= j0 && q < j0 + MB) npc[q - j0] = j;
    base += __popcll(m);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(64)
k_id_solve_mfma(const double* __restrict__ A, int64_t a_stride, int lda, const int32_t* __restrict__ n_arr,
                int n_uniform, int n_max, const int32_t* __restrict__ rank, int32_t* __restrict__ piv,
                int64_t piv_stride, const double* __restrict__ Dinv, int nblk, double* __restrict__ P,
                int64_t p_stride, int p_ld, int r_max, const unsigned char* __restrict__ mask) {
  extern __shared__ double smm[];
  const int b = blockIdx.x, j0 = MB * (int)blockIdx.y;
  if (mask && !mask[b]) return;
  const int n = n_arr ? n_arr[b] : n_uniform;
  if (j0 >= n) return;
  const int r = rank[b], r16 = round_mb_dev(r);
  const int t_rows = round_mb_dev(r_max) + MB;
  double* T = smm;                                                   // t_rows x MTS
  int* pv = reinterpret_cast<int*>(T + (size_t)t_rows * MTS);        // r_max + MB pivot columns
  unsigned int* isp = reinterpret_cast<unsigned int*>(pv + r_max + MB);   // pivot bitmap
  int* npc = reinterpret_cast<int*>(isp + (n_max + 31) / 32);        // this chunk's non-pivot columns
  int* posl = npc + MB;                                  // pivot position of column j0 + c, or -1
  const int lane = threadIdx.x, i16 = lane & 15, g = lane >> 4;
  const double* Ab = A + (int64_t)b * a_stride;
  const int32_t* pb = piv + (int64_t)b * piv_stride;
  // Rows r .. r16 + MB - 1 stay zero: the padded part of the last diagonal
  // block and the tail of the last 16-row chunk of the trailing products.
  for (int e = lane; e < (r16 + MB) * MB; e += 64) T[(e >> 4) * MTS + (e & 15)] = 0.0;
  solve_columns(pb, r, n, j0, pv, isp, npc, posl);
  const int nq = min(MB, n - r - j0);
  // The right-hand sides (nq non-pivot columns x r rows) go to LDS, 16
  // elements per lane at a time, their loads in flight together.
  const int ne = nq * r;
  for (int e0 = 0; e0 < ne; e0 += 64 * 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + 64 * u + lane;
      const int c = e < ne ? e / r : 0, l = e < ne ? e - c * r : 0;
      v[u] = e < ne ? Ab[(int64_t)npc[c] * lda + l] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + 64 * u + lane;
      if (e < ne) {
        const int c = e / r, l = e - c * r;
        T[l * MTS + c] = v[u];
      }
    }
  }
  __syncthreads();
  if (nq > 0 && r > 0) {
    for (int kb = r16 - MB; kb >= 0; kb -= MB) {
      // This block's diagonal inverse (A operands of the last product),
      // fetched first so that its latency hides behind the trailing products.
      const double* D = Dinv + ((int64_t)b * nblk + kb / MB) * MB * MB + i16 * MB + g;
      double dv[MB / 4];
#pragma unroll
      for (int k4 = 0; k4 < MB / 4; ++k4) dv[k4] = D[4 * k4];
      dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
      // Trailing products over 16-row chunks of the solved rows below the
      // block, in batches of up to 16 chunks: a batch's R operands are all
      // loaded first (one memory round trip per batch instead of one per
      // chunk), then multiplied in chunk order. Rows at or past the rank read
      // the zero row r16 of T against a real column of R.
      const double* Ak = Ab + kb + i16;
      for (int l0 = kb + MB; l0 < r; l0 += 16 * MB) {
        const int nch = min(16, (r - l0 + MB - 1) / MB);
        double a[16][4];
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (c < nch)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const int l = l0 + MB * c + 4 * m + g;
              a[c][m] = Ak[(int64_t)pv[l < r ? l : r] * lda];
            }
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (c < nch) {
            double bq[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const int l = l0 + MB * c + 4 * m + g;
              bq[m] = T[(l < r ? l : r16) * MTS + i16];
            }
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][0], bq[0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][1], bq[1], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][2], bq[2], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][3], bq[3], acc1, 0, 0, 0);
          }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double* t = &T[(kb + 4 * v + g) * MTS + i16];
        *t = *t - (acc0[v] + acc1[v]);
      }
      __syncthreads();
      dbl4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k4 = 0; k4 < MB / 4; ++k4)
        x = __builtin_amdgcn_mfma_f64_16x16x4f64(dv[k4], T[(kb + 4 * k4 + g) * MTS + i16], x, 0, 0, 0);
      __syncthreads();
#pragma unroll
      for (int v = 0; v < 4; ++v) T[(kb + 4 * v + g) * MTS + i16] = x[v];
      __syncthreads();
    }
  }
  double* Pb = P + (int64_t)b * p_stride;
  for (int e = lane; e < r * MB; e += 64) {
    const int i = e >> 4, c = e & 15;
    if (c < nq) Pb[(int64_t)i * p_ld + npc[c]] = T[i * MTS + c];
    const int pl = posl[c];
    if (pl >= 0) Pb[(int64_t)i * p_ld + j0 + c] = pl == i ? 1.0 : 0.0;
  }
  for (int c = lane; c < nq; c += 64) piv[(int64_t)b * piv_stride + r + j0 + c] = npc[c];
}

// The same solve for ranks up to kRegSolveRank with the right-hand sides in
// registers: lane (i16, g) holds T[4 i + g][i16], i < 64. Those are exactly
// the B operands it supplies to the trailing products and to the product with
// the diagonal inverse, and the rows of the block it updates, so T needs
// neither LDS nor barriers, and two wavefronts share a SIMD (the LDS-resident
// version's 37 KB of T allowed one). The 16 blocks and their chunks are
// unrolled so that every register index is fixed; the products run in the
// same order as in k_id_solve_mfma, so the results are the same bits.
// BATCH chunks' R operands are loaded at a time: two for launches with many
// wavefronts (two per SIMD, which hide each other's loads; larger batches
// spilled), all fifteen for small launches (one wavefront per SIMD with 512
// registers: one load round trip per block instead of one per two chunks).
constexpr int kRegSolveRank = 256;

template <int BATCH>
__global__ void __launch_bounds__(64, BATCH > 2 ? 1 : 2)
k_id_solve_regs(const double* __restrict__ A, int64_t a_stride, int lda, const int32_t* __restrict__ n_arr,
                int n_uniform, int n_max, const int32_t* __restrict__ rank, int32_t* __restrict__ piv,
                int64_t piv_stride, const double* __restrict__ Dinv, int nblk, double* __restrict__ P,
                int64_t p_stride, int p_ld, int r_max, const unsigned char* __restrict__ mask) {
  extern __shared__ int smi[];
  const int b = blockIdx.x, j0 = MB * (int)blockIdx.y;
  if (mask && !mask[b]) return;
  const int n = n_arr ? n_arr[b] : n_uniform;
  if (j0 >= n) return;
  const int r = rank[b], r16 = round_mb_dev(r);
  int* pv = smi;                                                          // r_max + MB
  unsigned int* isp = reinterpret_cast<unsigned int*>(pv + r_max + MB);  // pivot bitmap
  int* npc = reinterpret_cast<int*>(isp + (n_max + 31) / 32);
  int* posl = npc + MB;
  const int lane = threadIdx.x, i16 = lane & 15, g = lane >> 4;
  const double* Ab = A + (int64_t)b * a_stride;
  const int32_t* pb = piv + (int64_t)b * piv_stride;
  solve_columns(pb, r, n, j0, pv, isp, npc, posl);
  const int nq = min(MB, n - r - j0);
  constexpr int NR = kRegSolveRank / 4;
  double T[NR];
  {
    const double* col = Ab + (int64_t)npc[i16 < nq ? i16 : 0] * lda;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int l = 4 * i + g;
      T[i] = (l < r && i16 < nq) ? col[l] : 0.0;
    }
  }
  if (nq > 0 && r > 0) {
#pragma unroll
    for (int bi = kRegSolveRank / MB - 1; bi >= 0; --bi) {
      if (MB * bi >= r16) continue;
      const int kb = MB * bi;
      const double* D = Dinv + ((int64_t)b * nblk + bi) * MB * MB + i16 * MB + g;
      double dv[MB / 4];
#pragma unroll
      for (int k4 = 0; k4 < MB / 4; ++k4) dv[k4] = D[4 * k4];
      dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
      // R operands are addressed by 32-bit byte offsets from the uniform
      // base of the block (the host keeps the block under 2^32 bytes).
      const char* Abc = reinterpret_cast<const char*>(Ab);
      const unsigned ko = (unsigned)(kb + i16);
      // Trailing products over the chunks cb > bi that start below the rank,
      // BATCH chunks' R operands loaded at a time.
#pragma unroll
      for (int c0 = bi + 1; c0 < kRegSolveRank / MB; c0 += BATCH) {
        if (MB * c0 >= r) break;
        double a[BATCH][4];
#pragma unroll
        for (int c = 0; c < BATCH; ++c)
          if (c0 + c < kRegSolveRank / MB && MB * (c0 + c) < r)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const int l = MB * (c0 + c) + 4 * m + g;
              const unsigned off = ((unsigned)pv[l < r ? l : r] * (unsigned)lda + ko) * 8u;
              a[c][m] = *reinterpret_cast<const double*>(Abc + off);
            }
#pragma unroll
        for (int c = 0; c < BATCH; ++c) {
          const int cb = c0 + c;
          if (cb < kRegSolveRank / MB && MB * cb < r) {
            double bq[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) bq[m] = MB * cb + 4 * m + g < r ? T[4 * cb + m] : 0.0;
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][0], bq[0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][1], bq[1], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][2], bq[2], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][3], bq[3], acc1, 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) T[4 * bi + v] = T[4 * bi + v] - (acc0[v] + acc1[v]);
      dbl4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k4 = 0; k4 < MB / 4; ++k4) x = __builtin_amdgcn_mfma_f64_16x16x4f64(dv[k4], T[4 * bi + k4], x, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) T[4 * bi + v] = x[v];
    }
  }
  double* Pb = P + (int64_t)b * p_stride;
  const int pl = posl[i16];
  const int npj = npc[i16 < nq ? i16 : 0];
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int l = 4 * i + g;
    if (l < r) {
      if (i16 < nq) Pb[(int64_t)l * p_ld + npj] = T[i];
      if (pl >= 0) Pb[(int64_t)l * p_ld + j0 + i16] = pl == l ? 1.0 : 0.0;
    }
  }
  for (int c = lane; c < nq; c += 64) piv[(int64_t)b * piv_stride + r + j0 + c] = npc[c];
}

// Set when a cooperative QR launch was refused on this thread (see launch_qr).
thread_local bool g_coop_refused = false;

int resident_grid(const void* kern, int threads, size_t lds) {
  int dev = 0, nb = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, threads, lds) != hipSuccess) return 0;
  return nb * cus;
}

// Scratch of a factorization launch: a growable buffer, or a fixed region
// that must already be large enough (nothing is allocated then).
struct QrScratch {
  DevBuf<unsigned char>* buf = nullptr;
  unsigned char* fixed = nullptr;
  size_t fixed_bytes = 0;
  ffc_status ensure(size_t bytes) {
    if (buf) return buf->count < bytes ? buf->alloc(bytes) : FFC_OK;
    if (bytes > fixed_bytes) {
      set_error("the blocks need " + std::to_string(bytes) + " bytes of QR scratch, above the fixed " +
                std::to_string(fixed_bytes));
      return FFC_ERR_INVALID_ARG;
    }
    return FFC_OK;
  }
  unsigned char* ptr() const { return buf ? buf->ptr : fixed; }
  size_t bytes() const { return buf ? buf->count : fixed_bytes; }
};

// Scratch bytes of variant (R, CS, NTC) for the blocks of bt: slots, task
// offsets and claim counter of the QR, or the solve's diagonal inverses,
// whichever is larger (the solve reuses the QR's scratch).
template <int R, int CS, int NTC, int LG>
size_t qr_scratch_bytes(const IdBatch& bt, int batch) {
  constexpr int CPW = 64 / LG * CS;
  const int cols_per_wg = CPW * (NTC / 64);
  const int gmax = std::max(1, (bt.n_max + cols_per_wg - 1) / cols_per_wg);
  const size_t slot_doubles = (size_t)batch * 2 * gmax * (bt.s_max + 2);
  return std::max(slot_doubles * sizeof(double) + ((size_t)batch + 2) * sizeof(int32_t),
                  solve_scratch_bytes(bt, batch));
}

// The factorization with variant (R, NTC) on the blocks of bt (in place);
// fits = false (nothing launched) when a block's group cannot be resident.
template <int R, int CS, int NTC, int LG>
ffc_status launch_qr(const IdBatch& bt, int batch, QrScratch scratch, hipStream_t st, bool& fits) {
  constexpr int CPW = 64 / LG * CS;   // columns per wavefront
  const int cols_per_wg = CPW * (NTC / 64);
  const int gmax = std::max(1, (bt.n_max + cols_per_wg - 1) / cols_per_wg);
  const void* kern = reinterpret_cast<const void*>(&k_cpqr_coop<R, CS, NTC, LG>);
  const size_t lds = (size_t)(NTC / 64 + 1) * LG * R * sizeof(double);
  if (lds > 64 * 1024)
    FFC_HIP_TRY(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const int grid_cap = resident_grid(kern, NTC, lds);
  fits = grid_cap >= gmax;
  if (!fits) return FFC_OK;
  const size_t slot_doubles = (size_t)batch * 2 * gmax * (bt.s_max + 2);
  // Slots, task offsets, claim counter. The solve that follows reuses the
  // scratch: size it for both up front.
  FFC_TRY(scratch.ensure(qr_scratch_bytes<R, CS, NTC, LG>(bt, batch)));
  CoopArgs ca{};
  ca.A = bt.A;
  ca.a_stride = bt.a_stride;
  ca.lda = bt.lda;
  ca.s_arr = bt.s_arr;
  ca.n_arr = bt.n_arr;
  ca.s_uniform = bt.s_uniform;
  ca.n_uniform = bt.n_uniform;
  ca.count = batch;
  ca.tol = bt.tol;
  ca.max_rank = bt.max_rank;
  ca.rank = bt.rank;
  ca.piv = bt.piv;
  ca.piv_stride = bt.piv_stride;
  ca.slots = reinterpret_cast<double*>(scratch.ptr());
  ca.slot_words = (int64_t)slot_doubles;
  ca.task_start = reinterpret_cast<int32_t*>(ca.slots + slot_doubles);
  ca.mask = bt.mask;
  ca.claim = ca.task_start + batch + 1;
  ca.gmax = gmax;
  ca.s_max = bt.s_max;
  ca.cols_per_wg = cols_per_wg;
  ca.flag = device_flag();
  {
    StageTimer tm(FFC_STAGE_SOLVE, st);
    const int cgrid = (int)std::min<int64_t>(1024, (ca.slot_words + 255) / 256);
    hipLaunchKernelGGL(k_coop_setup, dim3(std::max(1, cgrid)), dim3(256), 0, st, ca);
    FFC_LAUNCH_CHECK("k_coop_setup");
  }
  const int grid = std::min(grid_cap, batch * gmax);
  void* args[] = {&ca};
  hipError_t le;
  {
    StageTimer tm(FFC_STAGE_CPQR, st);
    le = hipLaunchCooperativeKernel(kern, dim3(grid), dim3(NTC), args, (unsigned int)lds, st);
  }
  if (le == hipErrorIllegalState || le == hipErrorCooperativeLaunchTooLarge) {
    // The device's cooperative-launch resource (global wave sync) belongs to
    // another process that has made such a launch, or the grid cannot be
    // co-resident after all: nothing was launched, and the caller falls back
    // to the one-workgroup-per-block kernel.
    (void)hipGetLastError();
    g_coop_refused = true;
    fits = false;
    return FFC_OK;
  }
  if (le != hipSuccess) {
    set_error(std::string("hipLaunchCooperativeKernel (QR): ") + hipGetErrorString(le));
    return le == hipErrorOutOfMemory ? FFC_ERR_OOM : FFC_ERR_HIP;
  }
  return FFC_OK;
}

// Blocks factored in place without swaps: column piv[l] holds R(0:l+1, l),
// every other column j holds R(0:r, j) in rows 0..r-1. The QR launch sized
// the scratch for the diagonal block inverses (it is done with it by now:
// same stream).
ffc_status launch_solve(const IdBatch& bt, int batch, QrScratch scratch, hipStream_t st) {
  const int r_max = solve_rank_bound(bt);
  const int nblk = round_mb(r_max) / MB;
  if (scratch.bytes() < solve_scratch_bytes(bt, batch)) {
    set_error("QR scratch smaller than the solve needs");
    return FFC_ERR_STATE;
  }
  double* Dinv = reinterpret_cast<double*>(scratch.ptr());
  const bool regs = r_max <= kRegSolveRank && (int64_t)bt.lda * bt.n_max * (int64_t)sizeof(double) < (INT64_C(1) << 32);
  const size_t lds = regs ? ((size_t)r_max + 3 * MB + (bt.n_max + 31) / 32) * sizeof(int)
                          : mfma_solve_lds_bytes(r_max, bt.n_max);
  if (!regs && lds > 64 * 1024)
    FFC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_id_solve_mfma),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  StageTimer tm(FFC_STAGE_SOLVE, st);
  hipLaunchKernelGGL(k_diag_inv, dim3(batch, nblk), dim3(64), 0, st, bt.A, bt.a_stride, bt.lda, bt.rank, bt.piv,
                     bt.piv_stride, Dinv, nblk, bt.mask);
  FFC_LAUNCH_CHECK("k_diag_inv");
  if (regs) {
    // Up to 2048 wavefronts (two per SIMD) the launch cannot hide its load
    // latency with other wavefronts: load whole blocks' operands at once.
    const bool small = (int64_t)batch * ((bt.n_max + MB - 1) / MB) <= 2048;
    hipLaunchKernelGGL(small ? k_id_solve_regs<kRegSolveRank / MB - 1> : k_id_solve_regs<2>,
                       dim3(batch, (bt.n_max + MB - 1) / MB), dim3(64), lds, st, bt.A, bt.a_stride, bt.lda, bt.n_arr,
                       bt.n_uniform, bt.n_max, bt.rank, bt.piv, bt.piv_stride, Dinv, nblk, bt.P, bt.p_stride, bt.p_ld,
                       r_max, bt.mask);
    FFC_LAUNCH_CHECK("k_id_solve_regs");
  } else {
    hipLaunchKernelGGL(k_id_solve_mfma, dim3(batch, (bt.n_max + MB - 1) / MB), dim3(64), lds, st, bt.A,
                       bt.a_stride, bt.lda, bt.n_arr, bt.n_uniform, bt.n_max, bt.rank, bt.piv, bt.piv_stride, Dinv,
                       nblk, bt.P, bt.p_stride, bt.p_ld, r_max, bt.mask);
    FFC_LAUNCH_CHECK("k_id_solve_mfma");
  }
  return FFC_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: the first factorization of each shape (s_max, n_max, batch,
// rank cap) times every variant that can hold the blocks on a scratch copy
// of the real blocks (best of two runs, HIP events) and keeps the fastest.
// Disabled by FFC_AUTOTUNE=0 and while the stream is being captured into a
// graph (then the first valid variant runs).
// ---------------------------------------------------------------------------
using QrLaunch = ffc_status (*)(const IdBatch&, int, QrScratch, hipStream_t, bool&);
using QrBytes = size_t (*)(const IdBatch&, int);
struct Variant {
  int R, CS, threads, LG;
  QrLaunch fn;
  QrBytes bytes;
  int rows() const { return R * LG; }   // the most rows a block may have
  // 32-lane groups only for blocks that 16-lane groups cannot hold: the two
  // sum rows in different orders, and every variant that a shape may use
  // gives the same bits.
  bool holds(int s_max) const { return s_max <= rows() && (LG == 16 || s_max > 16 * 32); }
};
#define FFC_VARIANT(R, CS, T, LG) {R, CS, T, LG, &launch_qr<R, CS, T, LG>, &qr_scratch_bytes<R, CS, T, LG>}
const Variant kVariants[] = {
    FFC_VARIANT(32, 2, 512, 16), FFC_VARIANT(32, 2, 256, 16), FFC_VARIANT(32, 1, 512, 16),
    FFC_VARIANT(32, 1, 256, 16), FFC_VARIANT(32, 1, 128, 16), FFC_VARIANT(16, 1, 512, 16),
    FFC_VARIANT(16, 1, 128, 16), FFC_VARIANT(32, 2, 512, 32), FFC_VARIANT(32, 1, 512, 32),
    FFC_VARIANT(32, 2, 256, 32), FFC_VARIANT(32, 1, 256, 32),
};
#undef FFC_VARIANT
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

struct TuneEntry {
  int s_max, n_max, batch, max_rank;
  int choice;
  float best_us, first_us;
  bool from_cache;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

bool autotune_enabled() {
  const char* e = std::getenv("FFC_AUTOTUNE");
  return !(e && e[0] == '0');
}

// Persistent choices: with FFC_TUNE_CACHE=<file>, choices are read from the
// file on first use and every new one is appended, so later processes on the
// same kind of device skip the timing. One line per choice: device key
// (architecture name and compute-unit count), s_max, n_max, batch, rank cap,
// the most rows the variant holds, columns per lane group, threads, best us. Lines for other
// devices or unknown variants are ignored.
std::string device_key() {
  int dev = 0, cus = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  std::string arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ' ' || c == ':') c = '_';
  return arch + "-" + std::to_string(cus);
}

bool g_cache_loaded = false;

int variant_index(int rows, int CS, int threads) {
  for (int v = 0; v < kNumVariants; ++v)
    if (kVariants[v].rows() == rows && kVariants[v].CS == CS && kVariants[v].threads == threads) return v;
  return -1;
}

// Called with g_tune_mu held.
void load_tune_cache() {
  if (g_cache_loaded) return;
  g_cache_loaded = true;
  const char* path = std::getenv("FFC_TUNE_CACHE");
  if (!path || !path[0]) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  const std::string key = device_key();
  char dk[128];
  TuneEntry te{};
  int R = 0, CS = 0, T = 0;
  float best = 0.f;
  while (std::fscanf(f, "%127s %d %d %d %d %d %d %d %f", dk, &te.s_max, &te.n_max, &te.batch, &te.max_rank, &R, &CS,
                     &T, &best) == 9) {
    const int v = variant_index(R, CS, T);
    if (key != dk || v < 0) continue;
    te.choice = v;
    te.best_us = te.first_us = best;
    te.from_cache = true;
    g_tune.push_back(te);
  }
  std::fclose(f);
}

void append_tune_cache(const TuneEntry& te) {
  const char* path = std::getenv("FFC_TUNE_CACHE");
  if (!path || !path[0]) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  const Variant& v = kVariants[te.choice];
  std::fprintf(f, "%s %d %d %d %d %d %d %d %.1f\n", device_key().c_str(), te.s_max, te.n_max, te.batch, te.max_rank,
               v.rows(), v.CS, v.threads, te.best_us);
  std::fclose(f);
}

ffc_status tune(const IdBatch& bt, int batch, QrScratch scratch, hipStream_t st, const std::vector<int>& cand,
                TuneEntry& te) {
  DevBuf<double> copy;
  const size_t words = (size_t)batch * bt.a_stride;
  FFC_TRY(copy.alloc(words));
  IdBatch tb = bt;
  tb.A = copy.ptr;
  hipEvent_t e0, e1;
  FFC_HIP_TRY(hipEventCreate(&e0));
  FFC_HIP_TRY(hipEventCreate(&e1));
  te.choice = -1;
  te.best_us = te.first_us = 0.f;
  ffc_status status = FFC_OK;
  for (int v : cand) {
    float best = -1.f;
    for (int rep = 0; rep < 2 && status == FFC_OK; ++rep) {
      bool fits = false;
      hipError_t he = hipMemcpyAsync(copy.ptr, bt.A, words * sizeof(double), hipMemcpyDeviceToDevice, st);
      if (he == hipSuccess) he = hipEventRecord(e0, st);
      if (he != hipSuccess) {
        set_error(std::string("copy of the blocks or start event: ") + hipGetErrorString(he));
        status = FFC_ERR_HIP;
        break;
      }
      status = kVariants[v].fn(tb, batch, scratch, st, fits);
      if (status != FFC_OK || !fits) break;
      float ms = 0.f;
      he = hipEventRecord(e1, st);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he != hipSuccess) {
        set_error(std::string("timing of variant ") + std::to_string(v) + ": " + hipGetErrorString(he));
        status = FFC_ERR_HIP;
        break;
      }
      best = best < 0.f ? ms : std::min(best, ms);
    }
    if (status != FFC_OK) break;
    if (best < 0.f) continue;   // does not fit
    if (te.first_us == 0.f) te.first_us = best * 1e3f;
    if (te.choice < 0 || best * 1e3f < te.best_us) {
      te.choice = v;
      te.best_us = best * 1e3f;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);   // the copy is freed below
  if (status != FFC_OK) set_error(std::string("autotuning of the QR kernel failed: ") + ffc_last_error());
  return status;
}

}  // namespace

// The autotuner's earlier choice for this shape (or FFC_QR_VARIANT), -1 if none.
int tuned_choice(const IdBatch& bt, int batch) {
  int choice = -1;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    load_tune_cache();
    for (const TuneEntry& te : g_tune)
      if (te.s_max == bt.s_max && te.n_max == bt.n_max && te.batch == batch && te.max_rank == bt.max_rank)
        choice = te.choice;
  }
  // FFC_QR_VARIANT=i forces variant i when it can hold the blocks (tests run
  // every variant this way; the variants give the same bits).
  if (const char* fv = std::getenv("FFC_QR_VARIANT")) {
    const int v = std::atoi(fv);
    if (v >= 0 && v < kNumVariants && kVariants[v].holds(bt.s_max)) choice = v;
  }
  return choice;
}

ffc_status launch_interp_decomp_coop(const IdBatch& bt, int batch, DevBuf<unsigned char>& scratch_buf, hipStream_t st,
                                     bool& used) {
  QrScratch scratch;
  scratch.buf = &scratch_buf;
  used = false;
  if (batch <= 0) return FFC_OK;
  if (mfma_solve_lds_bytes(solve_rank_bound(bt), bt.n_max) > 150 * 1024) return FFC_OK;
  std::vector<int> cand;
  for (int v = 0; v < kNumVariants; ++v)
    if (kVariants[v].holds(bt.s_max)) cand.push_back(v);
  if (cand.empty()) return FFC_OK;
  int choice = tuned_choice(bt, batch);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  FFC_HIP_TRY(hipStreamIsCapturing(st, &cs));
  if (choice < 0 && cand.size() > 1 && autotune_enabled() && cs == hipStreamCaptureStatusNone) {
    TuneEntry te{bt.s_max, bt.n_max, batch, bt.max_rank, -1, 0.f, 0.f, false};
    FFC_TRY(tune(bt, batch, scratch, st, cand, te));
    if (te.choice >= 0) {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      g_tune.push_back(te);
      append_tune_cache(te);
      choice = te.choice;
    }
  }
  // The chosen variant first, then the others in order (one that fits is used).
  std::vector<int> order;
  if (choice >= 0) order.push_back(choice);
  for (int v : cand)
    if (v != choice) order.push_back(v);
  for (int v : order) {
    bool fits = false;
    FFC_TRY(kVariants[v].fn(bt, batch, scratch, st, fits));
    if (fits) {
      FFC_TRY(launch_solve(bt, batch, scratch, st));
      used = true;
      return FFC_OK;
    }
  }
  return FFC_OK;
}

ffc_status launch_interp_decomp_fixed(const IdBatch& bt, int batch, unsigned char* fixed, size_t fixed_bytes,
                                      hipStream_t st) {
  if (batch <= 0) return FFC_OK;
  if (mfma_solve_lds_bytes(solve_rank_bound(bt), bt.n_max) > 150 * 1024) {
    set_error("the interpolation solve of these blocks does not fit in LDS");
    return FFC_ERR_INVALID_ARG;
  }
  const int choice = tuned_choice(bt, batch);
  g_coop_refused = false;
  std::vector<int> order;
  if (choice >= 0) order.push_back(choice);
  for (int v = 0; v < kNumVariants; ++v)
    if (v != choice && kVariants[v].holds(bt.s_max)) order.push_back(v);
  QrScratch scratch;
  scratch.fixed = fixed;
  scratch.fixed_bytes = fixed_bytes;
  for (int v : order) {
    if (kVariants[v].bytes(bt, batch) > fixed_bytes) continue;
    bool fits = false;
    FFC_TRY(kVariants[v].fn(bt, batch, scratch, st, fits));
    if (fits) return launch_solve(bt, batch, scratch, st);
  }
  if (g_coop_refused) {
    set_error("the cooperative QR launch was refused: another process on this device holds its cooperative-launch "
              "resource");
    return FFC_ERR_STATE;
  }
  set_error("no register-resident QR variant holds these blocks within the fixed scratch (rows above 512, or "
            "too many blocks)");
  return FFC_ERR_INVALID_ARG;
}

void autotune_reset() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
  g_cache_loaded = false;
}

int autotune_entries(int32_t* out, int cap) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  load_tune_cache();
  const int n = (int)g_tune.size();
  for (int e = 0; e < n && e < cap; ++e) {
    const TuneEntry& te = g_tune[e];
    int32_t* o = out + 8 * e;
    o[0] = te.s_max;
    o[1] = te.n_max;
    o[2] = te.batch;
    o[3] = te.max_rank;
    o[4] = kVariants[te.choice].rows() * 100 + kVariants[te.choice].CS;
    o[5] = kVariants[te.choice].threads;
    o[6] = (int32_t)te.best_us;
    o[7] = te.from_cache ? -1 : (int32_t)te.first_us;
  }
  return n;
}

}  // namespace ffc
