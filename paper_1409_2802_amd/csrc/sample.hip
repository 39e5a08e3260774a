// Uniform target-row sampling and per-level column lists.
//
// Rows are drawn uniformly without replacement from the points outside the
// node (Section 4.1.3, uniform sampling; Theorem thm_column_sampling_approx2).
// The draw is Floyd's algorithm (Bentley & Floyd, CACM 1987) fed by a
// counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the value for
// counter j is the first SplitMix64 output from state seed ^ (node << 32) ^ j,
// and a uniform integer in [0, j] is the high 64 bits of u64 * (j + 1).
// Candidate t maps to tree position t (t < begin) or t + node size. With
// separation the candidates are the node's separated points in ascending tree
// order (a bitmap per node with a prefix count per 64-bit word): candidate t is
// the t-th set bit, found by a binary search over the word prefixes.
//
// Two kernels implement the same draw. The bitmap kernel (used whenever the
// bitmap of the complement fits the LDS budget) keeps the chosen set as bits;
// the general kernel keeps it as a list scanned by one wavefront with a
// ballot, then sorts it with an LDS bitonic network.
#include <climits>

#include "ffc_internal.h"

namespace ffc {
namespace {

__device__ inline uint64_t splitmix_first(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Candidates of a draw: the separated points of the node when it has any
// (bitmap words and their prefix counts), else the range or its complement.
struct Candidates {
  const uint64_t* bits = nullptr;   // non-null: separated candidates
  const int32_t* pre = nullptr;
  int words = 0;
  int lo = 0, shift = 0;
  __device__ inline int operator()(int t) const {
    if (!bits) return t < lo ? t : t + shift;
    int a = 0, z = words - 1;       // the last word whose prefix is <= t holds candidate t
    while (a < z) {
      const int mid = (a + z + 1) >> 1;
      if (pre[mid] <= t) a = mid;
      else z = mid - 1;
    }
    uint64_t w = bits[a];
    for (int r = t - pre[a]; r > 0; --r) w &= w - 1;
    return a * 64 + __ffsll((unsigned long long)w) - 1;
  }
};

__device__ inline Candidates candidates(const SepView& sv, int node, int b, int e, int64_t N, bool inside,
                                        int64_t& M) {
  Candidates c;
  c.lo = inside ? 0 : b;
  c.shift = inside ? b : e - b;
  M = inside ? (e - b) : N - (e - b);
  if (sv.bits && !inside) {
    const int32_t* pre = sv.pre + (int64_t)node * (sv.words + 1);
    const int m = pre[sv.words];
    if (m > 0) {
      c.bits = sv.bits + (int64_t)node * sv.words;
      c.pre = pre;
      c.words = sv.words;
      M = m;
    }
  }
  return c;
}

__global__ void k_sample_rows(const int32_t* __restrict__ nb, const int32_t* __restrict__ ne, int64_t N, int first,
                              int s, int s_cap, int sort_n, uint64_t seed, uint32_t stream_or, int inside,
                              const unsigned char* __restrict__ mask, SepView sv, int32_t* __restrict__ rows,
                              int32_t* __restrict__ nrows) {
  extern __shared__ int set[];   // sort_n ints (power of two >= s)
  const int node = first + blockIdx.x;
  const int lane = threadIdx.x;
  if (mask && !mask[node]) return;
  const int b = nb[node], e = ne[node];
  int64_t M;
  const Candidates cand = candidates(sv, node, b, e, N, inside != 0, M);
  int32_t* out = rows + (int64_t)node * s_cap;
  if (s >= M) {
    for (int64_t i = lane; i < M; i += 64) out[i] = (int32_t)cand((int)i);
    if (lane == 0) nrows[node] = (int32_t)M;
    return;
  }
  const uint64_t stream = (uint64_t)((uint32_t)node | stream_or) << 32;
  int cnt = 0;
  for (int64_t j = M - s; j < M; ++j) {
    const uint64_t u = splitmix_first(seed ^ stream ^ (uint64_t)j);
    const int t = (int)__umul64hi(u, (uint64_t)(j + 1));
    bool hit = false;
    for (int i = lane; i < cnt; i += 64) hit |= (set[i] == t);
    const bool any = __ballot(hit) != 0ull;
    if (lane == 0) set[cnt] = any ? (int)j : t;
    ++cnt;
    __syncthreads();
  }
  for (int i = cnt + lane; i < sort_n; i += 64) set[i] = INT_MAX;
  __syncthreads();
  for (int k = 2; k <= sort_n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = lane; t < sort_n / 2; t += 64) {
        const int i = (t / j) * 2 * j + (t % j);
        const bool asc = (i & k) == 0;
        const int x = set[i], y = set[i + j];
        if ((y < x) == asc) { set[i] = y; set[i + j] = x; }
      }
      __syncthreads();
    }
  }
  for (int i = lane; i < s; i += 64) out[i] = cand(set[i]);
  if (lane == 0) nrows[node] = s;
}

// Bitmap variant (complement size M up to 32 * kMaxBitmapWords): the chosen
// set lives as a bitmap of {0..M-1} in LDS, so membership is one bit test and
// the ascending order falls out of a prefix count over the words. The Floyd
// values t_j are produced in parallel; the sequential insert rule (j replaces
// t_j when t_j is already taken) is applied 64 steps at a time.
constexpr int kMaxBitmapWords = 12288;   // 48 KB of LDS -> M <= 393216
constexpr int kBitmapThreads = 256;

__global__ void __launch_bounds__(kBitmapThreads)
k_sample_rows_bitmap(const int32_t* __restrict__ nb, const int32_t* __restrict__ ne, int64_t N, int first, int s,
                     int s_cap, uint64_t seed, uint32_t stream_or, int inside,
                     const unsigned char* __restrict__ mask, SepView sv, int32_t* __restrict__ rows,
                     int32_t* __restrict__ nrows) {
  // LDS: with separation the node's word prefixes (sv.words + 1 ints, read by
  // every candidate lookup's binary search), then nwords bitmap words, then s
  // ints of t values.
  extern __shared__ unsigned int lds_words[];
  const int pre_len = sv.bits ? sv.words + 1 : 0;
  unsigned int* bits = lds_words + pre_len;
  __shared__ int wsum[kBitmapThreads / 64];
  const int node = first + blockIdx.x;
  const int tid = threadIdx.x;
  if (mask && !mask[node]) return;
  const int b = nb[node], e = ne[node];
  int64_t M64;
  Candidates cand = candidates(sv, node, b, e, N, inside != 0, M64);
  const int M = (int)M64;
  if (cand.bits) {
    int32_t* spre = reinterpret_cast<int32_t*>(lds_words);
    for (int w = tid; w <= cand.words; w += kBitmapThreads) spre[w] = cand.pre[w];
    cand.pre = spre;
    __syncthreads();
  }
  int32_t* out = rows + (int64_t)node * s_cap;
  if (s >= M) {
    for (int i = tid; i < M; i += kBitmapThreads) out[i] = cand(i);
    if (tid == 0) nrows[node] = M;
    return;
  }
  const int nwords = (M + 31) / 32;
  int* tv = reinterpret_cast<int*>(bits + nwords);
  for (int w = tid; w < nwords; w += kBitmapThreads) bits[w] = 0u;
  const uint64_t stream = (uint64_t)((uint32_t)node | stream_or) << 32;
  for (int q = tid; q < s; q += kBitmapThreads) {
    const int64_t j = (int64_t)(M - s) + q;
    const uint64_t u = splitmix_first(seed ^ stream ^ (uint64_t)j);
    tv[q] = (int)__umul64hi(u, (uint64_t)(j + 1));
  }
  __syncthreads();
  // The insert rule, 64 steps at a time on wave 0. Against the set as it
  // stood before the chunk, step q's choice c_q is j_q when t_q is taken and
  // t_q otherwise. Every c_q is absent from that set (earlier values are all
  // below j_q), so the chunk's choices agree with the sequential rule exactly
  // when they are pairwise distinct: a lane that finds its bit already set by
  // the atomic OR reveals a repeat, the chunk's bits are cleared again and
  // lane 0 replays those 64 steps one by one.
  if (tid < 64) {
    for (int q0 = 0; q0 < s; q0 += 64) {
      const int q = q0 + tid;
      const bool act = q < s;
      int c = 0;
      unsigned int bit = 0u;
      if (act) {
        const int t = tv[q];
        c = (bits[t >> 5] >> (t & 31)) & 1u ? M - s + q : t;
        bit = 1u << (c & 31);
      }
      const unsigned int old = act ? atomicOr(&bits[c >> 5], bit) : 0u;
      if (__ballot(act && (old & bit)) != 0ull) {
        if (act) atomicAnd(&bits[c >> 5], ~bit);
        if (tid == 0) {
          for (int p = q0; p < min(s, q0 + 64); ++p) {
            int t = tv[p];
            if ((bits[t >> 5] >> (t & 31)) & 1u) t = M - s + p;
            bits[t >> 5] |= 1u << (t & 31);
          }
        }
      }
    }
  }
  __syncthreads();
  // Ascending extraction: each thread owns a contiguous range of words.
  const int per = (nwords + kBitmapThreads - 1) / kBitmapThreads;
  const int w0 = tid * per, w1 = min(nwords, w0 + per);
  int cnt = 0;
  for (int w = w0; w < w1; ++w) cnt += __popc(bits[w]);
  // Block-wide exclusive prefix of the counts: a shuffle scan per wave, then
  // the totals of the waves before this one.
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
    unsigned int word = bits[w];
    while (word) {
      const int bit = __ffs(word) - 1;
      word &= word - 1;
      out[pos++] = cand(w * 32 + bit);
    }
  }
  if (tid == 0) nrows[node] = s;
}

__global__ void k_level_columns(const int32_t* __restrict__ nb, const int32_t* __restrict__ ne, int first,
                                int leaves, int n_cap, int r_cap, const int32_t* __restrict__ rank,
                                const int32_t* __restrict__ skel, int32_t* __restrict__ cols,
                                int32_t* __restrict__ ncols, const unsigned char* __restrict__ mask) {
  const int node = first + blockIdx.x;
  if (mask && !mask[node]) return;
  int32_t* out = cols + (int64_t)node * n_cap;
  if (leaves) {
    const int b = nb[node], n = ne[node] - b;
    for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = b + i;
    if (threadIdx.x == 0) ncols[node] = n;
    return;
  }
  const int l = 2 * node + 1, r = 2 * node + 2;
  const int rl = rank[l], rr = rank[r];
  for (int i = threadIdx.x; i < rl; i += blockDim.x) out[i] = skel[(int64_t)l * r_cap + i];
  for (int i = threadIdx.x; i < rr; i += blockDim.x) out[rl + i] = skel[(int64_t)r * r_cap + i];
  if (threadIdx.x == 0) ncols[node] = rl + rr;
}

}  // namespace

namespace {
ffc_status draw(const int32_t* nb, const int32_t* ne, int64_t N, bool inside, int32_t* rows, int32_t* nrows, int cap,
                int first, int count, int s, uint64_t seed, uint32_t stream_or, const unsigned char* mask,
                const SepView& sv, hipStream_t st) {
  if (count <= 0) return FFC_OK;
  if (s > cap) {
    set_error("row sample larger than its buffer");
    return FFC_ERR_INVALID_ARG;
  }
  const int64_t nwords = (N + 31) / 32;
  const size_t lds = (size_t)nwords * sizeof(unsigned int) + (size_t)s * sizeof(int) +
                     (sv.bits ? (size_t)(sv.words + 1) * sizeof(int32_t) : 0);
  if (nwords <= kMaxBitmapWords && lds <= 64 * 1024) {
    hipLaunchKernelGGL(k_sample_rows_bitmap, dim3(count), dim3(kBitmapThreads), lds, st, nb, ne, N, first, s, cap,
                       seed, stream_or, inside ? 1 : 0, mask, sv, rows, nrows);
    FFC_LAUNCH_CHECK("k_sample_rows_bitmap");
    return FFC_OK;
  }
  int sort_n = 1;
  while (sort_n < s) sort_n <<= 1;
  if ((size_t)sort_n * sizeof(int) > 64 * 1024) {
    set_error("row sample too large for the sampling kernel");
    return FFC_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_sample_rows, dim3(count), dim3(64), (size_t)sort_n * sizeof(int), st, nb, ne, N, first, s, cap,
                     sort_n, seed, stream_or, inside ? 1 : 0, mask, sv, rows, nrows);
  FFC_LAUNCH_CHECK("k_sample_rows");
  return FFC_OK;
}
}  // namespace

ffc_status launch_draw(const int32_t* nb, const int32_t* ne, int64_t N, bool inside, int32_t* rows, int32_t* nrows,
                       int cap, int first, int count, int s, uint64_t seed, uint32_t stream_or,
                       const unsigned char* mask, hipStream_t st) {
  return draw(nb, ne, N, inside, rows, nrows, cap, first, count, s, seed, stream_or, mask, SepView{}, st);
}

ffc_status launch_sample_rows_sep(const ffc_tree* t, ffc_skel* sk, int first, int count, int s, uint64_t seed,
                                  hipStream_t st, const unsigned char* mask) {
  if (!sk->sep_bits.ptr) {
    set_error("separation bitmaps are missing");
    return FFC_ERR_STATE;
  }
  const SepView sv{sk->sep_bits.ptr, sk->sep_pre.ptr, sk->sep_words};
  return draw(t->begin.ptr, t->end.ptr, t->N, false, sk->rows.ptr, sk->nrows.ptr, sk->s_cap, first, count, s, seed,
              0u, mask, sv, st);
}

ffc_status launch_sample_rows_into(const ffc_tree* t, int32_t* rows, int32_t* nrows, int cap, int first, int count,
                                   int s, uint64_t seed, uint32_t stream_or, const unsigned char* mask,
                                   hipStream_t st) {
  return launch_draw(t->begin.ptr, t->end.ptr, t->N, false, rows, nrows, cap, first, count, s, seed, stream_or, mask,
                     st);
}

ffc_status launch_sample_rows(const ffc_tree* t, ffc_skel* sk, int first, int count, int s, uint64_t seed,
                              hipStream_t st, const unsigned char* mask) {
  return launch_sample_rows_into(t, sk->rows.ptr, sk->nrows.ptr, sk->s_cap, first, count, s, seed, 0u, mask, st);
}

ffc_status launch_level_columns(const ffc_tree* t, ffc_skel* sk, int first, int count, bool leaves,
                                hipStream_t st, const unsigned char* mask) {
  hipLaunchKernelGGL(k_level_columns, dim3(count), dim3(256), 0, st, t->begin.ptr, t->end.ptr, first,
                     leaves ? 1 : 0, sk->n_cap, sk->r_cap, sk->rank.ptr, sk->skel.ptr, sk->cols.ptr,
                     sk->ncols.ptr, mask);
  FFC_LAUNCH_CHECK("k_level_columns");
  return FFC_OK;
}

}  // namespace ffc
