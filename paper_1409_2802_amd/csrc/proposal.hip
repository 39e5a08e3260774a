// Learned row proposal: features, the 16-64-64-1 network (inference,
// gradients, Adam) and importance selection of target rows.
//
// Leverage-score sampling is the paper's gold standard for choosing rows but
// needs the whole block (Section 3, importance sampling); the cheap geometric
// heuristics of Section 3.2 motivate learning the map from per-target
// geometry to leverage. Definitions (shared with the CPU reference):
//  * column geometry of a node: centroid c and radius rho of its column
//    points, a 256-point subsample S (Floyd draw, stream node | 2^30, ascending)
//    and up to 7 anchors of S by farthest-point selection from c;
//  * 16 features of a target: |y-c|/rho, its log, the 4 smallest |y-x|/rho
//    over S, their mean over S, log of the smallest, the projections of y - c
//    on the 7 anchor directions over rho, and a constant 1;
//  * scores from the network on standardized features; weights 0.9 softmax
//    + 0.1 uniform over a pool of c s uniform candidates; Efraimidis-Spirakis
//    keys -ln(U)/w select s rows without replacement.
#include <climits>

#include "ffc_internal.h"

namespace ffc {
namespace {

constexpr int NF = 16, NH = 64;   // features per target, hidden width
constexpr int NPARAM = NF * NH + NH + NH * NH + NH + NH + 1;   // 5313
constexpr int OFF_W1 = 0, OFF_B1 = NF * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH,
              OFF_B3 = OFF_W3 + NH;
constexpr int SUB = 256;   // column subsample size
constexpr int kMaxGeomCols = 16384;   // column-set capacity (the indices are held in 64 KiB of LDS)
constexpr int NANCH = 7;    // anchor directions
constexpr uint64_t STREAM_SUBSAMPLE = 1ull << 30, STREAM_KEYS = 3ull << 30;

__device__ inline uint64_t splitmix_first(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ inline uint64_t counter_u64(uint64_t seed, uint64_t stream, uint64_t j) {
  return splitmix_first(seed ^ (stream << 32) ^ j);
}

// ---------------------------------------------------------------------------
// Column geometry: one 256-thread workgroup per node. The node's column
// indices go to LDS first, so that every coordinate load is a single hop; for
// d <= kGeomStageD the subsample's coordinates are then staged in LDS as well
// (rows padded to d + 1 doubles) and the anchor search and directions read
// them there. Every sum keeps one fixed order: the centroid's as described
// below, the squared distances sequential over the coordinates.
// ---------------------------------------------------------------------------
constexpr int kGeomStageD = 64;

// Dynamic LDS of k_geometry: the centroid (d doubles), then the column indices
// and the radius pass's four transposition tiles or, once they are no longer
// needed, the staged subsample.
size_t geometry_lds(int d, int64_t col_stride) {
  const size_t idx = (size_t)((col_stride + 1) & ~1ll) * sizeof(int32_t) + 4 * 16 * 65 * sizeof(double);
  const size_t sub = d <= kGeomStageD ? (size_t)SUB * (d + 1) * sizeof(double) : 0;
  return (size_t)d * sizeof(double) + (idx > sub ? idx : sub);
}

// Max of v over the workgroup (exact in any order): shuffles, then the 4 waves.
__device__ inline double block_max(double v, double* wred) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = v;
  __syncthreads();
  return fmax(fmax(wred[0], wred[1]), fmax(wred[2], wred[3]));
}

__global__ void __launch_bounds__(256) k_geometry(const double* __restrict__ Xt, int d, GeomArgs ga) {
  extern __shared__ double geo_dyn[];
  double* scen = geo_dyn;                                   // [d]
  int32_t* scol = reinterpret_cast<int32_t*>(geo_dyn + d);  // [n] column indices
  double* sx = geo_dyn + d;                                  // [SUB][d + 1] staged subsample (after scol)
  __shared__ __align__(16) int sval[SUB];
  __shared__ int sidx[SUB];
  __shared__ int srej[SUB];
  __shared__ double sd2[SUB], mind[SUB];
  __shared__ double red[256];
  __shared__ double wred[4], snrm[NANCH];
  __shared__ int s_changed, anchors[NANCH];
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63;
  const int n = ga.ncols[b];
  const int32_t* cols = ga.cols + (int64_t)b * ga.col_stride;
  double* cen = ga.cen + (int64_t)b * d;
  const uint64_t node = (uint64_t)ga.node_ids[b];
  // (Eight passes' loads at a time, issued before their stores.)
  for (int j0 = 0; j0 < n; j0 += 256 * 8) {
    int cv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) cv[u] = cols[min(j0 + 256 * u + tid, n - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (j0 + 256 * u + tid < n) scol[j0 + 256 * u + tid] = cv[u];
  }
  __syncthreads();
  // Centroid: dimension k is summed in P interleaved column parts (part p
  // takes columns p, p + P, ...), each with two alternating accumulators, and
  // the parts are added in order (a fixed summation order).
  {
    const int P = d >= 256 ? 1 : min(16, 256 / d);
    for (int e = tid; e < d * P; e += 256) {
      const int k = e % d, part = e / d;
      double s0 = 0.0, s1 = 0.0;
      int j = part;
      // (Unrolled so that many columns' coordinate loads are in flight at
      // once; the two sums keep their order.)
#pragma unroll 16
      for (; j + P < n; j += 2 * P) {
        s0 += Xt[(int64_t)scol[j] * d + k];
        s1 += Xt[(int64_t)scol[j + P] * d + k];
      }
      if (j < n) s0 += Xt[(int64_t)scol[j] * d + k];
      if (P == 1) {
        const double c = n > 0 ? (s0 + s1) / n : 0.0;
        cen[k] = c;
        scen[k] = c;
      } else {
        red[e] = s0 + s1;
      }
    }
    __syncthreads();
    if (P > 1) {
      for (int k = tid; k < d; k += 256) {
        double s = 0.0;
        for (int part = 0; part < P; ++part) s += red[part * d + k];
        const double c = n > 0 ? s / n : 0.0;
        cen[k] = c;
        scen[k] = c;
      }
      __syncthreads();
    }
  }
  // Radius. Each wave takes 64 columns at a time, one per lane; their
  // coordinates arrive in chunks of 16, loaded coalesced (16 lanes per
  // column segment, the next chunk in flight) and transposed through the
  // wave's own LDS tile, from which each lane sums its column's squared
  // differences in order.
  double mx = 0.0;
  {
    const int wv = tid >> 6;
    double* tw = reinterpret_cast<double*>(scol + ((ga.col_stride + 1) & ~1ll)) + wv * (16 * 65);   // [16][65]
    const int nchunk = (d + 15) / 16, ngroup = (n + 255 - wv * 64) / 256;  // this wave's 64-column groups
    const int steps = ngroup * nchunk;
    int ci[16];
    double r[16];
    auto load = [&](int st) {
      const int g = st / nchunk, ch = st - g * nchunk, c0 = wv * 64 + g * 256, k = ch * 16 + (lane & 15);
      if (ch == 0)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int cc = c0 + 4 * i + (lane >> 4);
          ci[i] = cc < n ? scol[cc] : -1;
        }
#pragma unroll
      for (int i = 0; i < 16; ++i) r[i] = ci[i] >= 0 && k < d ? Xt[(int64_t)ci[i] * d + k] : 0.0;
    };
    double sq = 0.0;
    if (steps > 0) load(0);
    for (int st = 0; st < steps; ++st) {
      const int g = st / nchunk, ch = st - g * nchunk;
#pragma unroll
      for (int i = 0; i < 16; ++i) tw[(lane & 15) * 65 + 4 * i + (lane >> 4)] = r[i];
      __builtin_amdgcn_wave_barrier();
      if (st + 1 < steps) load(st + 1);
      const int kc = min(16, d - ch * 16);
#pragma unroll 16
      for (int kk = 0; kk < kc; ++kk) {
        const double df = tw[kk * 65 + lane] - scen[ch * 16 + kk];
        sq = fma(df, df, sq);
      }
      __builtin_amdgcn_wave_barrier();
      if (ch == nchunk - 1) {
        if (wv * 64 + g * 256 + lane < n) mx = fmax(mx, sq);
        sq = 0.0;
      }
    }
  }
  mx = block_max(mx, wred);
  if (tid == 0) {
    const double r = sqrt(mx);
    ga.rho[b] = r > 0.0 ? r : 1.0;
  }
  // Subsample: Floyd's algorithm over {0..n-1}. Step q draws t_q in
  // [0, n - SUB + q] and takes t_q unless it is already taken, else
  // n - SUB + q. t_q is taken before step q exactly when an earlier draw
  // equals it, or when t_q = n - SUB + p for an earlier step p that was
  // itself refused; the refusals are resolved from the first rule by
  // propagating the second to a fixed point. The taken values are then put in
  // ascending order by counting.
  const int ns = min(n, SUB);
  if (n > SUB) {
    int t = 0;
    if (tid < SUB) {
      const int j = n - SUB + tid;
      t = (int)__umul64hi(counter_u64(ga.seed, node | STREAM_SUBSAMPLE, (uint64_t)j), (uint64_t)(j + 1));
      sval[tid] = t;
    }
    __syncthreads();
    if (tid < SUB) {
      int dup = 0;
      const int4* s4 = reinterpret_cast<const int4*>(sval);
      for (int p = 0; p < (tid + 3) / 4; ++p) {
        const int4 w = s4[p];
        dup |= (w.x == t) | ((4 * p + 1 < tid) & (w.y == t)) | ((4 * p + 2 < tid) & (w.z == t)) |
               ((4 * p + 3 < tid) & (w.w == t));
      }
      srej[tid] = dup;
    }
    const int pq = t - (n - SUB);   // the earlier step whose fallback value equals t_q, if 0 <= pq < q
    for (;;) {
      if (tid == 0) s_changed = 0;
      __syncthreads();
      if (tid < SUB && !srej[tid] && pq >= 0 && pq < tid && srej[pq]) {
        srej[tid] = 1;
        s_changed = 1;
      }
      __syncthreads();
      const int more = s_changed;
      __syncthreads();
      if (!more) break;
    }
    const int v = srej[tid < SUB ? tid : 0] ? n - SUB + tid : t;
    if (tid < SUB) sval[tid] = v;
    __syncthreads();
    if (tid < SUB) {
      int rank = 0;
      const int4* s4 = reinterpret_cast<const int4*>(sval);
#pragma unroll 8
      for (int p = 0; p < SUB / 4; ++p) {
        const int4 w = s4[p];
        rank += (w.x < v) + (w.y < v) + (w.z < v) + (w.w < v);
      }
      sidx[rank] = v;
    }
  } else if (tid < ns) {
    sidx[tid] = tid;
  }
  __syncthreads();
  if (tid < ns) sval[tid] = scol[sidx[tid]];   // tree positions of the subsample
  int32_t* S_out = ga.sub + (int64_t)b * SUB;
  if (tid < SUB) S_out[tid] = tid < ns ? scol[sidx[tid]] : -1;
  if (tid == 0) ga.nsub[b] = ns;
  __syncthreads();
  // Stage the subsample (the column indices are dead from here on).
  const bool staged = d <= kGeomStageD;
  if (staged) {
    const int wv = tid >> 6;
    if (lane < d)
#pragma unroll 8
      for (int q = wv; q < ns; q += 4) sx[q * (d + 1) + lane] = Xt[(int64_t)sval[q] * d + lane];
    __syncthreads();
  }
  // The anchor search and directions, instantiated for LDS rows and for
  // global rows (so that the LDS instance compiles to LDS loads).
  __shared__ int wbi[4];
  const int na = min(NANCH, ns);
  auto search = [&](auto xrow) {
    // Anchors: farthest-point selection, starting from the point farthest from
    // c. (The squared norms of the subsample points are formed on the way.)
    if (tid < SUB) {
      double sq = -1.0, nx = 0.0;
      if (tid < ns) {
        const double* x = xrow(tid);
        sq = 0.0;
#pragma unroll 16
        for (int k = 0; k < d; ++k) {
          const double df = x[k] - scen[k];
          sq = fma(df, df, sq);
          nx = fma(x[k], x[k], nx);
        }
      }
      sd2[tid] = sq;
      ga.subn2[(int64_t)b * SUB + tid] = nx;
    }
    __syncthreads();
    for (int a = 0; a < na; ++a) {
      // Arg-max of the key over the subsample, ties to the smaller index: per
      // wavefront by shuffles, then over the four wavefronts.
      const double* key = a == 0 ? sd2 : mind;
      double bv = tid < ns ? key[tid] : -INFINITY;
      int bi = tid < ns ? tid : INT_MAX;
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        wred[tid >> 6] = bv;
        wbi[tid >> 6] = bi;
      }
      __syncthreads();
      double v = wred[0];
      int i = wbi[0];
      for (int q = 1; q < 4; ++q)
        if (wred[q] > v || (wred[q] == v && wbi[q] < i)) {
          v = wred[q];
          i = wbi[q];
        }
      if (tid == 0) anchors[a] = i;
      if (tid < ns) {
        const double* x = xrow(tid);
        const double* y = xrow(i);
        double sq = 0.0;
#pragma unroll 16
        for (int k = 0; k < d; ++k) {
          const double df = x[k] - y[k];
          sq = fma(df, df, sq);
        }
        mind[tid] = a == 0 ? sq : fmin(mind[tid], sq);
      }
      __syncthreads();
    }
    // Anchor directions: the norms one thread each, then the unit vectors.
    if (tid < na) {
      const double* y = xrow(anchors[tid]);
      double nrm2 = 0.0;
#pragma unroll 16
      for (int k = 0; k < d; ++k) {
        const double df = y[k] - scen[k];
        nrm2 = fma(df, df, nrm2);
      }
      snrm[tid] = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
    }
    __syncthreads();
    double* U = ga.U + (int64_t)b * NANCH * d;
    for (int a = 0; a < NANCH; ++a) {
      const double* y = a < na ? xrow(anchors[a]) : nullptr;
      for (int k = tid; k < d; k += 256) U[(int64_t)a * d + k] = a < na ? (y[k] - scen[k]) * snrm[a] : 0.0;
    }
  };
  if (staged)
    search([&](int q) -> const double* { return sx + q * (d + 1); });
  else
    search([&](int q) -> const double* { return Xt + (int64_t)sval[q] * d; });
}

// ---------------------------------------------------------------------------
// Features on the FP64 matrix cores. One 256-thread workgroup per 64 targets
// of a block; wave w owns targets 16 w .. 16 w + 15. The subsample is taken in
// rounds of 64 points, each swept over the coordinates in chunks of 16 that
// pass through a double-buffered LDS stage (targets and points row-major, the
// next chunk's loads in flight, the subsample's positions read from LDS so
// that the loads do not wait on one another). Per chunk a wave issues 4 x 4
// v_mfma_f64_16x16x4f64 for the inner products of its 16 targets with the
// round's 64 points; step u of a chunk takes coordinates 4 g + u from lane
// group g = lane / 16, so that a lane reads its 4 values of a row with two
// 16-byte LDS loads (rows padded to 18 doubles, which spreads the 16 rows of a
// read over all banks). Operand layouts of the instruction: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[4 v + l / 16][l % 16]
// for v = 0..3.
//
// Squared distances are taken in Gram form |y|^2 + |x|^2 - 2 y.x; a pair whose
// Gram value is below 2^-10 (|y|^2 + |x|^2), where the form could have lost
// more than 10 bits, is recomputed from explicit coordinate differences. Lane
// l holds targets 16 w + 4 v + l / 16 (v < 4) against points l % 16 + 16 c
// (c < 4) of each round, keeps per target the 4 smallest squared distances
// and the sum of the distances, and the 16 lanes of a target group merge
// them at the end in a fixed order (four DPP exchange steps).
// The target norms, the distance to the centroid and the anchor projections
// are summed in order over the coordinates from the first round's stages.
// ---------------------------------------------------------------------------
// Keep the 4 smallest values, ascending (a branch-free insertion).
__device__ inline void insert4(double (&b)[4], double v) {
  b[3] = fmin(b[3], v);
#pragma unroll
  for (int a = 3; a > 0; --a) {
    const double lo = fmin(b[a - 1], b[a]), hi = fmax(b[a - 1], b[a]);
    b[a - 1] = lo;
    b[a] = hi;
  }
}

// sqrt(g) for g >= 0 to about 2^-45 relative: the hardware reciprocal square
// root refined by one Newton step on h^2 = g (g is raised to 2^-900 first, so
// a zero distance adds 2^-450). Used only for the sum of the distances, a
// float feature.
__device__ inline double sqrt_sum(double g) {
  g = fmax(g, 0x1p-900);
  const double r = __builtin_amdgcn_rsq(g), h = g * r;
  return fma(fma(-h, h, g), 0.5 * r, h);
}

// x of the DPP partner lane (CTRL: a DPP row control: quad permutation or
// mirror).
template <int CTRL>
__device__ inline double dpp_partner(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One exchange step of the 4-smallest lists and sums of 4 targets.
template <int CTRL>
__device__ inline void merge_step(double (&best)[4][4], double (&sum)[4]) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    sum[v] += dpp_partner<CTRL>(sum[v]);
    double c[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = fmin(best[v][i], dpp_partner<CTRL>(best[v][3 - i]));
    // c is bitonic; sort it.
    const double a0 = fmin(c[0], c[2]), a2 = fmax(c[0], c[2]), a1 = fmin(c[1], c[3]), a3 = fmax(c[1], c[3]);
    best[v][0] = fmin(a0, a1);
    best[v][1] = fmax(a0, a1);
    best[v][2] = fmin(a2, a3);
    best[v][3] = fmax(a2, a3);
  }
}

typedef double fdbl4 __attribute__((ext_vector_type(4)));
constexpr int FT = 64, FR = 64, FK = 16, FKP = FK + 2;   // targets, points per round, chunk, LDS row
constexpr int FSR = 256 / FK, FNI = FT / FSR, FNP = FR / FSR;   // stage rows per pass; passes for targets, points
constexpr int FCT = FR / 16;                                      // column tiles per round
struct FeatSmem {
  double ys[2][FT][FKP];
  double xs[2][FR][FKP];
  double cu[2][1 + NANCH][FK + 1];   // centroid and anchor directions, first round
  double ny[FT];
  double subn[SUB];                  // and their squared norms
  int sub[SUB];                      // the subsample's tree positions
};

// (At most 168 registers, three workgroups per compute unit: the extra
// resident waves hide the stage loads better than larger rounds would.)
__global__ void __launch_bounds__(256, 3) k_features(const double* __restrict__ Xt, int d, GeomArgs ga,
                                                  const int32_t* __restrict__ tgt, int tgt_stride,
                                                  const int32_t* __restrict__ ntgt, int tiles,
                                                  float* __restrict__ feat, int64_t feat_stride) {
  __shared__ __align__(16) FeatSmem sm;
  const int b = blockIdx.x / tiles, t0 = (blockIdx.x % tiles) * FT;
  const int nt = ntgt[b];
  if (t0 >= nt) return;
  const int ns = ga.nsub[b];
  const double rho = ga.rho[b];
  const int32_t* S = ga.sub + (int64_t)b * SUB;
  const double* nxg = ga.subn2 + (int64_t)b * SUB;
  const double* cen = ga.cen + (int64_t)b * d;
  const double* U = ga.U + (int64_t)b * NANCH * d;
  const int32_t* tg = tgt + (int64_t)b * tgt_stride + t0;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lg = lane >> 4;
  const int nrow = min(FT, nt - t0);
  // Stage map: element tid + 256 it of a 64 x FK stage is row tid / FK + FSR it,
  // coordinate tid % FK.
  const int sr = tid / FK, sk = tid % FK;
  int yrow[FNI];
#pragma unroll
  for (int it = 0; it < FNI; ++it) yrow[it] = sr + FSR * it < nrow ? tg[sr + FSR * it] : -1;
  const int nchunk = (d + FK - 1) / FK, nround = max(1, (ns + FR - 1) / FR), total = nround * nchunk;
  double ry[FNI], rx[FNP], rc = 0.0;
  auto load = [&](int st) {
    const int r = st / nchunk, k = (st - r * nchunk) * FK + sk;
#pragma unroll
    for (int it = 0; it < FNI; ++it) ry[it] = yrow[it] >= 0 && k < d ? Xt[(int64_t)yrow[it] * d + k] : 0.0;
#pragma unroll
    for (int it = 0; it < FNP; ++it) {
      const int p = r * FR + sr + FSR * it;
      rx[it] = p < ns && k < d ? Xt[(int64_t)sm.sub[p] * d + k] : 0.0;
    }
    if (r == 0 && tid < (1 + NANCH) * FK) {
      const int a = tid / FK;
      rc = k < d ? (a == 0 ? cen[k] : U[(int64_t)(a - 1) * d + k]) : 0.0;
    }
  };
  auto store = [&](int st, int buf) {
#pragma unroll
    for (int it = 0; it < FNI; ++it) sm.ys[buf][sr + FSR * it][sk] = ry[it];
#pragma unroll
    for (int it = 0; it < FNP; ++it) sm.xs[buf][sr + FSR * it][sk] = rx[it];
    if (st < nchunk && tid < (1 + NANCH) * FK) sm.cu[buf][tid / FK][sk] = rc;
  };
  fdbl4 acc[FCT];
  double best[4][4], sum[4];
#pragma unroll
  for (int c = 0; c < FCT; ++c) acc[c] = fdbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    sum[v] = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) best[v][i] = INFINITY;
  }
  // First-round sums of target tid / 4: its squared norm, and dot products
  // 2 (tid % 4), 2 (tid % 4) + 1 (0: |y - c|^2, a > 0: (y - c) . u_a).
  double nyv = 0.0, dp0 = 0.0, dp1 = 0.0;
  const int drow = tid >> 2, da = 2 * (tid & 3);
  // The subsample's positions go to LDS first: a coordinate load then waits
  // on an LDS read, not on an earlier global load (which would serialize the
  // stage's loads). Their norms too, which each round's distances read.
  for (int q = tid; q < SUB; q += 256) {
    sm.sub[q] = q < ns ? S[q] : 0;
    sm.subn[q] = q < ns ? nxg[q] : 0.0;
  }
  __syncthreads();
  load(0);
  store(0, 0);
  __syncthreads();
  for (int st = 0; st < total; ++st) {
    const int buf = st & 1, r = st / nchunk, ch = st - r * nchunk;
    if (st + 1 < total) load(st + 1);
#pragma unroll
    for (int h = 0; h < FK / 16; ++h) {
      const double2* ya = reinterpret_cast<const double2*>(&sm.ys[buf][16 * w + li][16 * h + 4 * lg]);
      const double2 a01 = ya[0], a23 = ya[1];
#pragma unroll
      for (int c = 0; c < FCT; ++c) {
        const double2* xb = reinterpret_cast<const double2*>(&sm.xs[buf][16 * c + li][16 * h + 4 * lg]);
        const double2 b01 = xb[0], b23 = xb[1];
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a01.x, b01.x, acc[c], 0, 0, 0);
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a01.y, b01.y, acc[c], 0, 0, 0);
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a23.x, b23.x, acc[c], 0, 0, 0);
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a23.y, b23.y, acc[c], 0, 0, 0);
      }
    }
    if (r == 0) {
#pragma unroll 4
      for (int kk = 0; kk < FK; ++kk) {
        const double y = sm.ys[buf][drow][kk], df = y - sm.cu[buf][0][kk], u0 = sm.cu[buf][da][kk];
        dp0 = fma(df, da == 0 ? df : u0, dp0);
        dp1 = fma(df, sm.cu[buf][da + 1][kk], dp1);
        nyv = fma(y, y, nyv);
      }
    }
    if (ch == nchunk - 1) {   // the round is complete
      if (r == 0) {
        if ((tid & 3) == 0) sm.ny[drow] = nyv;
        __syncthreads();
      }
      double nyr[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) nyr[v] = sm.ny[16 * w + 4 * v + lg];
#pragma unroll
      for (int c = 0; c < FCT; ++c) {
        const int p = r * FR + 16 * c + li;
        if (p < ns) {
          const double nx = sm.subn[p];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 16 * w + 4 * v + lg;
            const double n2 = nyr[v] + nx;
            double g = fma(-2.0, acc[c][v], n2);
            if (!(g >= 0x1p-10 * n2) && row < nrow) {   // explicit differences
              const double* y = Xt + (int64_t)tg[row] * d;
              const double* x = Xt + (int64_t)sm.sub[p] * d;
              g = 0.0;
              for (int k = 0; k < d; ++k) {
                const double df = y[k] - x[k];
                g = fma(df, df, g);
              }
            }
            // (g >= 0 here for every real target: a smaller Gram value took
            // the explicit differences.)
            sum[v] += sqrt_sum(g);
            insert4(best[v], g);
          }
        }
        acc[c] = fdbl4{0.0, 0.0, 0.0, 0.0};
      }
    }
    if (st + 1 < total) store(st + 1, buf ^ 1);
    __syncthreads();
  }
  // Merge the 16 lanes of a target group in four exchange steps (partners by
  // DPP: lane ^ 1, lane ^ 2, then mirrored within 8 and within 16 lanes, so
  // that every lane ends with the whole group): the sums add (both partners
  // get the same value), the two sorted 4-lists merge bitonically.
  merge_step<0xB1>(best, sum);
  merge_step<0x4E>(best, sum);
  merge_step<0x141>(best, sum);
  merge_step<0x140>(best, sum);
  // The first-round dot products go through LDS (the stage buffers are free).
  double* dots = &sm.ys[0][0][0];   // [64 targets][1 + NANCH]
  dots[drow * (1 + NANCH) + da] = dp0;
  dots[drow * (1 + NANCH) + da + 1] = dp1;
  __syncthreads();
  if (li != 0) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = 16 * w + 4 * v + lg;
    if (row >= nrow) continue;
    const double* dr = dots + row * (1 + NANCH);
    double b4[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) b4[i] = sqrt(best[v][i]) / rho;
    const double dc = sqrt(dr[0]) / rho;
    float* f = feat + (int64_t)b * feat_stride + (int64_t)(t0 + row) * NF;
    f[0] = (float)dc;
    f[1] = (float)log(dc + 1e-12);
    for (int i = 0; i < 4; ++i) f[2 + i] = (float)(i < ns ? b4[i] : b4[max(ns - 1, 0)]);
    f[6] = (float)(ns > 0 ? sum[v] / rho / ns : 0.0);
    f[7] = (float)log(b4[0] + 1e-12);
    for (int a = 0; a < NANCH; ++a) f[8 + a] = (float)(dr[1 + a] / rho);
    f[15] = 1.0f;
  }
}

// ---------------------------------------------------------------------------
// Network inference on the matrix cores (v_mfma_f32_16x16x4f32, FP32
// operands and accumulation). Each wavefront takes 16 samples at a time (a
// grid-stride loop) with the layers transposed, so that the samples run
// along the instruction's N dimension: H1^T = W1^T Z^T, then H2^T = W2^T
// relu(H1^T + b1), then y = b3 + w3 . relu(H2^T + b2) by lane sums. Operand
// layouts: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and
// receives D[kMlpRow(l / 16, v)][l % 16], v = 0..3. The K index of step v
// of a 16-row block is kMlpRow(g, v) for lane group g = l / 16, so a lane's
// outputs of one layer are its operands for the next; for the first layer,
// step v takes feature 4 g + v, so a lane reads its 4 features at once. The
// weights stay in registers for the whole loop.
// ---------------------------------------------------------------------------
typedef float ff4 __attribute__((ext_vector_type(4)));
__device__ constexpr int kMlpRow(int g, int v) { return 4 * g + v; }

__global__ void __launch_bounds__(256) k_mlp_score(const float* __restrict__ theta, const float* __restrict__ mu,
                                                   const float* __restrict__ sdv, const float* __restrict__ feat,
                                                   int64_t count, float* __restrict__ score) {
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int64_t ntile = (count + 15) / 16;
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  if (wave0 >= ntile) return;
  float a1[4][4], a2[4][16], b1[4][4], b2[4][4], w3[4][4], zm[4], zs[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int out = 16 * m + li, row = 16 * m + kMlpRow(g, v);   // (A row, and the hidden unit this lane holds)
      a1[m][v] = theta[OFF_W1 + (4 * g + v) * NH + out];
      b1[m][v] = theta[OFF_B1 + row];
      b2[m][v] = theta[OFF_B2 + row];
      w3[m][v] = theta[OFF_W3 + row];
    }
#pragma unroll
    for (int m1 = 0; m1 < 4; ++m1)
#pragma unroll
      for (int v = 0; v < 4; ++v) a2[m][4 * m1 + v] = theta[OFF_W2 + (16 * m1 + kMlpRow(g, v)) * NH + 16 * m + li];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    zm[v] = mu[4 * g + v];
    zs[v] = sdv[4 * g + v];
  }
  const float b3 = theta[OFF_B3];
  for (int64_t t = wave0; t < ntile; t += nwaves) {
    const int64_t smp = 16 * t + li;
    float z[4];
    if (smp < count) {
      const float4 f = *reinterpret_cast<const float4*>(feat + smp * NF + 4 * g);
      z[0] = f.x;
      z[1] = f.y;
      z[2] = f.z;
      z[3] = f.w;
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) z[v] = 0.f;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) z[v] = (4 * g + v == NF - 1) ? 1.f : (z[v] - zm[v]) / zs[v];
    ff4 h1[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      h1[m] = ff4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) h1[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[m][v], z[v], h1[m], 0, 0, 0);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) h1[m][v] = fmaxf(h1[m][v] + b1[m][v], 0.f);
    float y = 0.f;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      ff4 h2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int m1 = 0; m1 < 4; ++m1)
#pragma unroll
        for (int v = 0; v < 4; ++v) h2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[m][4 * m1 + v], h1[m1][v], h2, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) y = fmaf(fmaxf(h2[v] + b2[m][v], 0.f), w3[m][v], y);
    }
    y += __shfl_xor(y, 16, 64);
    y += __shfl_xor(y, 32, 64);
    if (g == 0 && smp < count) score[smp] = y + b3;
  }
}

// ---------------------------------------------------------------------------
// Gradients of the mean squared error over sub-batches of 64 samples; one
// workgroup writes the sum of its samples' contributions (scaled by 1/total).
// Sample positions p map to rows (p * stride_mul) mod count (a fixed shuffle).
// ---------------------------------------------------------------------------
constexpr int GB = 64;

struct GradSmem {
  float w[NPARAM];
  float smu[NF], ssd[NF];
  float Z[GB][NF];
  float A1[GB][NH];   // pre-activations, later dA1
  float A2[GB][NH];   // pre-activations, later dA2
  float dy[GB];
  float loss[GB];
};

__global__ void __launch_bounds__(256) k_mlp_grad(const float* __restrict__ theta, const float* __restrict__ mu,
                                                  const float* __restrict__ sdv, const float* __restrict__ feat,
                                                  const float* __restrict__ target, int64_t count, int64_t p0,
                                                  int64_t stride_mul, int64_t total, float* __restrict__ grads) {
  extern __shared__ float gsm_raw[];
  GradSmem& sm = *reinterpret_cast<GradSmem*>(gsm_raw);
  const int tid = threadIdx.x;
  for (int p = tid; p < NPARAM; p += 256) sm.w[p] = theta[p];
  for (int p = tid; p < NF; p += 256) { sm.smu[p] = mu[p]; sm.ssd[p] = sdv[p]; }
  const int64_t base = p0 + (int64_t)blockIdx.x * GB;
  __syncthreads();
  const int s = tid >> 2, qd = tid & 3;   // sample, quarter of the hidden units
  const int64_t pos = base + s;
  const bool valid = pos < p0 + total;
  const int64_t row = valid ? (int64_t)(((unsigned __int128)pos * (unsigned __int128)stride_mul) % (unsigned __int128)count) : 0;
  if (qd == 0) {
    for (int q = 0; q < NF; ++q) sm.Z[s][q] = valid ? (feat[row * NF + q] - sm.smu[q]) / sm.ssd[q] : 0.f;
    sm.Z[s][NF - 1] = valid ? 1.f : 0.f;
  }
  __syncthreads();
  for (int j = qd * 16; j < qd * 16 + 16; ++j) {
    float a = sm.w[OFF_B1 + j];
    for (int q = 0; q < NF; ++q) a = fmaf(sm.Z[s][q], sm.w[OFF_W1 + q * NH + j], a);
    sm.A1[s][j] = a;
  }
  __syncthreads();
  float ypart = 0.f;
  for (int j = qd * 16; j < qd * 16 + 16; ++j) {
    float a = sm.w[OFF_B2 + j];
    for (int q = 0; q < NH; ++q) a = fmaf(fmaxf(sm.A1[s][q], 0.f), sm.w[OFF_W2 + q * NH + j], a);
    sm.A2[s][j] = a;
    ypart = fmaf(fmaxf(a, 0.f), sm.w[OFF_W3 + j], ypart);
  }
  // y = b3 + sum over the four quarters (lanes 4s..4s+3 are adjacent).
  ypart += __shfl_xor(ypart, 1, 64);
  ypart += __shfl_xor(ypart, 2, 64);
  if (qd == 0) {
    const float y = ypart + sm.w[OFF_B3];
    const float r = valid ? y - target[row] : 0.f;
    sm.dy[s] = 2.f * r / (float)total;
    sm.loss[s] = r * r;
  }
  __syncthreads();
  float* g = grads + (int64_t)blockIdx.x * (NPARAM + 1);
  // Output layer.
  if (tid < NH) {
    float a = 0.f;
    for (int q = 0; q < GB; ++q) a = fmaf(sm.dy[q], fmaxf(sm.A2[q][tid], 0.f), a);
    g[OFF_W3 + tid] = a;
  }
  if (tid == NH) {
    float a = 0.f, l = 0.f;
    for (int q = 0; q < GB; ++q) { a += sm.dy[q]; l += sm.loss[q]; }
    g[OFF_B3] = a;
    g[NPARAM] = l;
  }
  __syncthreads();
  // dA2 = dy w3 (A2 > 0), in place.
  for (int j = qd * 16; j < qd * 16 + 16; ++j) sm.A2[s][j] = sm.A2[s][j] > 0.f ? sm.dy[s] * sm.w[OFF_W3 + j] : 0.f;
  __syncthreads();
  // dW2 = H1^T dA2, db2 = sum dA2 (fixed sample order).
  for (int e = tid; e < NH * NH; e += 256) {
    const int i = e / NH, j = e % NH;
    float a = 0.f;
    for (int q = 0; q < GB; ++q) a = fmaf(fmaxf(sm.A1[q][i], 0.f), sm.A2[q][j], a);
    g[OFF_W2 + e] = a;
  }
  if (tid < NH) {
    float a = 0.f;
    for (int q = 0; q < GB; ++q) a += sm.A2[q][tid];
    g[OFF_B2 + tid] = a;
  }
  // dA1 = (dA2 W2^T) (A1 > 0): computed into registers, then stored over A1.
  float da1[16];
  for (int jj = 0; jj < 16; ++jj) {
    const int j = qd * 16 + jj;
    float a = 0.f;
    for (int q = 0; q < NH; ++q) a = fmaf(sm.A2[s][q], sm.w[OFF_W2 + j * NH + q], a);
    da1[jj] = sm.A1[s][j] > 0.f ? a : 0.f;
  }
  __syncthreads();
  for (int jj = 0; jj < 16; ++jj) sm.A1[s][qd * 16 + jj] = da1[jj];
  __syncthreads();
  for (int e = tid; e < NF * NH; e += 256) {
    const int i = e / NH, j = e % NH;
    float a = 0.f;
    for (int q = 0; q < GB; ++q) a = fmaf(sm.Z[q][i], sm.A1[q][j], a);
    g[OFF_W1 + e] = a;
  }
  if (tid < NH) {
    float a = 0.f;
    for (int q = 0; q < GB; ++q) a += sm.A1[q][tid];
    g[OFF_B1 + tid] = a;
  }
}

// Sum of the workgroup gradients (fixed order; rows of NPARAM + 1 floats, the
// last one the loss, read only when loss_out is set); optionally one Adam step.
__global__ void k_grad_reduce_adam(const float* __restrict__ grads, int nwg, float* __restrict__ theta,
                                   float* __restrict__ m1, float* __restrict__ m2, float* __restrict__ gsum,
                                   float* __restrict__ loss_out, int adam, float lr, float c1, float c2, int64_t total) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > NPARAM || (p == NPARAM && !loss_out)) return;
  float a = 0.f;
  for (int w = 0; w < nwg; ++w) a += grads[(int64_t)w * (NPARAM + 1) + p];
  if (p == NPARAM) {
    *loss_out = a / (float)total;
    return;
  }
  if (gsum) gsum[p] = a;
  if (adam) {
    const float mm = 0.9f * m1[p] + 0.1f * a;
    const float vv = 0.999f * m2[p] + 0.001f * a * a;
    m1[p] = mm;
    m2[p] = vv;
    theta[p] -= lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
  }
}

// Feature standardization statistics (mean and population std per feature),
// one workgroup per feature, fixed-order reduction in double.
__global__ void __launch_bounds__(256) k_feature_stats(const float* __restrict__ feat, int64_t count,
                                                       float* __restrict__ mu, float* __restrict__ sdv) {
  __shared__ double r1[256], r2[256];
  const int f = blockIdx.x;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) {
    const double v = feat[i * NF + f];
    s1 += v;
    s2 += v * v;
  }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) { r1[threadIdx.x] += r1[threadIdx.x + off]; r2[threadIdx.x] += r2[threadIdx.x + off]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = count ? r1[0] / count : 0.0;
    const double var = count ? fmax(r2[0] / count - m * m, 0.0) : 0.0;
    mu[f] = f == NF - 1 ? 0.f : (float)m;
    sdv[f] = f == NF - 1 ? 1.f : (float)fmax(sqrt(var), 1e-6);
  }
}

// ---------------------------------------------------------------------------
// Importance selection: one 512-thread workgroup per node; pool <= 8192
// candidates.
// mode 0 (learned): Efraimidis-Spirakis keys -ln(u) / w with w = 0.9 softmax(score) + 0.1 / P;
// mode 1 (distance): keys -ln(u) * max(v, 1e-12), i.e. weights proportional to 1 / v;
// mode 2 (nearest): keys v (deterministic). Value i of node b is score[b * score_stride + i * elem_stride].
// The s smallest keys, ties to the smaller index, are found by a radix select
// on order-preserving 64-bit images of the keys (8 passes of 8 bits over LDS
// histograms); the ties at the cut are taken in index order. Thread t holds
// candidates [t E, t E + E). The chosen rows are written in candidate order,
// which is ascending for an ascending pool; another pool's rows are sorted.
// ---------------------------------------------------------------------------
constexpr int SEL_T = 512, SEL_E = 16;   // threads, candidates per thread

// a < b exactly when image(a) < image(b) (-0 counts as +0).
__device__ inline uint64_t order_image(double kv) {
  const uint64_t u = (uint64_t)__double_as_longlong(kv == 0.0 ? 0.0 : kv);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Exclusive prefix sum of v over the 512 threads; `total` receives the sum.
// wsum: 8 ints of LDS. Synchronizes twice.
__device__ inline int block_exscan(int v, int* wsum, int& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  __syncthreads();
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int q = 0; q < SEL_T / 64; ++q) {
    const int t = wsum[q];
    before += q < wv ? t : 0;
    all += t;
  }
  total = all;
  return before + x - v;
}

__global__ void __launch_bounds__(512) k_select_rows(const float* __restrict__ score, int64_t score_stride,
                                                     int elem_stride, int mode,
                                                     const int32_t* __restrict__ pool, int pool_stride,
                                                     const int32_t* __restrict__ npool, int first, int s_req,
                                                     uint64_t seed, const int32_t* __restrict__ ncols,
                                                     const unsigned char* __restrict__ mask,
                                                     int32_t* __restrict__ rows, int s_cap, int32_t* __restrict__ nrows,
                                                     int sort_s) {
  extern __shared__ int sel_out[];   // sort_s chosen rows
  __shared__ double red[SEL_T];
  __shared__ int hist[256], wsum[SEL_T / 64], s_k;
  __shared__ uint64_t s_prefix;
  const int b = blockIdx.x, node = first + b, tid = threadIdx.x, lane = tid & 63;
  if (mask && !mask[node]) return;
  if (ncols[node] == 0) {   // empty column set: nothing to sample for
    if (tid == 0) nrows[node] = 0;
    return;
  }
  const int P = npool[b];
  const float* sc = score + (int64_t)b * score_stride;
  const int32_t* pl = pool + (int64_t)b * pool_stride;
  int32_t* out = rows + (int64_t)node * s_cap;
  if (s_req >= P) {   // every candidate is taken
    for (int i = tid; i < P; i += SEL_T) out[i] = pl[i];
    if (tid == 0) nrows[node] = P;
    return;
  }
  double mx = 0.0, se = 1.0;
  if (mode == 0) {
    // Softmax: the maximum, then the sum of exponentials (each thread sums
    // candidates tid, tid + 512, ... in order, then a pairwise tree: halves
    // 256, 128, 64 through LDS, the rest by shuffles in wave 0).
    float st[SEL_E];   // candidates tid + 512 j, loaded together
#pragma unroll
    for (int j = 0; j < SEL_E; ++j) st[j] = sc[(int64_t)min(tid + SEL_T * j, P - 1) * elem_stride];
    mx = -INFINITY;
#pragma unroll
    for (int j = 0; j < SEL_E; ++j)
      if (tid + SEL_T * j < P) mx = fmax(mx, (double)st[j]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) red[tid >> 6] = mx;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SEL_T / 64; ++q) mx = fmax(mx, red[q]);
    __syncthreads();
    se = 0.0;
#pragma unroll
    for (int j = 0; j < SEL_E; ++j)
      if (tid + SEL_T * j < P) se += exp((double)st[j] - mx);
    red[tid] = se;
    __syncthreads();
    for (int off = SEL_T / 2; off >= 64; off >>= 1) {
      if (tid < off) red[tid] += red[tid + off];
      __syncthreads();
    }
    if (tid < 64) {
      double x = red[tid];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double y = __shfl_down(x, off, 64);
        if (tid < off) x += y;
      }
      if (tid == 0) red[0] = x;
    }
    __syncthreads();
    se = red[0];
  }
  // Keys of this thread's candidates (padding sorts after every key).
  const int E = (P + SEL_T - 1) / SEL_T, i0 = tid * E;
  // (The scores are loaded first, all together, from clamped positions.)
  float sv[SEL_E];
#pragma unroll
  for (int j = 0; j < SEL_E; ++j) sv[j] = sc[(int64_t)min(i0 + j, P - 1) * elem_stride];
  uint64_t u[SEL_E];
#pragma unroll
  for (int j = 0; j < SEL_E; ++j) {
    const int i = i0 + j;
    u[j] = ~0ull;
    if (j < E && i < P) {
      const double v = (double)sv[j];
      double kv;
      if (mode == 2) {
        kv = v;
      } else {
        const double uu =
            ((double)(counter_u64(seed, (uint64_t)node | STREAM_KEYS, (uint64_t)i) >> 11) + 0.5) * 0x1.0p-53;
        kv = mode == 1 ? -log(uu) * fmax(v, 1e-12) : -log(uu) / (0.9 * exp(v - mx) / se + 0.1 / P);
      }
      u[j] = order_image(isfinite(kv) ? kv : INFINITY);   // a non-finite value is drawn last (by index)
    }
  }
  // Radix select of the image T of the s-th smallest key, and its rank k
  // among the keys equal to T.
  uint64_t prefix = 0;
  int k = s_req - 1;
  for (int shift = 56; shift >= 0; shift -= 8) {
    const uint64_t hmask = shift == 56 ? 0ull : ~0ull << (shift + 8);
    if (tid < 256) hist[tid] = 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SEL_E; ++j)
      if ((u[j] & hmask) == prefix) atomicAdd(&hist[(u[j] >> shift) & 255], 1);
    __syncthreads();
    if (tid < 64) {
      const int c0 = hist[4 * lane], c1 = hist[4 * lane + 1], c2 = hist[4 * lane + 2], c3 = hist[4 * lane + 3];
      const int part = c0 + c1 + c2 + c3;
      int incl = part;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
      }
      const int excl = incl - part;
      if (excl <= k && k < incl) {
        int kk = k - excl, dg = 4 * lane;
        if (kk >= c0) {
          kk -= c0;
          ++dg;
          if (kk >= c1) {
            kk -= c1;
            ++dg;
            if (kk >= c2) {
              kk -= c2;
              ++dg;
            }
          }
        }
        s_prefix = prefix | ((uint64_t)dg << shift);
        s_k = kk;
      }
    }
    __syncthreads();
    prefix = s_prefix;
    k = s_k;
  }
  // Candidates below T are chosen, and the first k + 1 equal to T by index.
  const uint64_t T = prefix;
  int neq = 0;
#pragma unroll
  for (int j = 0; j < SEL_E; ++j) neq += u[j] == T;
  int total = 0;
  int req = block_exscan(neq, wsum, total);
  unsigned int chosen = 0;
  int nsel = 0;
#pragma unroll
  for (int j = 0; j < SEL_E; ++j) {
    const bool eq = u[j] == T, take = u[j] < T || (eq && req <= k);
    req += eq;
    chosen |= (unsigned int)take << j;
    nsel += take;
  }
  int o = block_exscan(nsel, wsum, total);
  int pv[SEL_E + 1];   // this thread's pool rows and the next one (loaded together)
#pragma unroll
  for (int j = 0; j <= SEL_E; ++j) pv[j] = pl[min(i0 + j, P - 1)];
  bool descent = false;   // the pool is not ascending here
#pragma unroll
  for (int j = 0; j < SEL_E; ++j) {
    const int i = i0 + j;
    if (j < E && i + 1 < P) descent |= pv[j + 1] <= pv[j];
    if ((chosen >> j) & 1) sel_out[o++] = pv[j];
  }
  if (__syncthreads_or(descent)) {   // bitonic sort of the chosen rows
    for (int i = s_req + tid; i < sort_s; i += SEL_T) sel_out[i] = INT_MAX;
    __syncthreads();
    for (int kk = 2; kk <= sort_s; kk <<= 1)
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int t = tid; t < sort_s / 2; t += SEL_T) {
          const int i = (t / j) * 2 * j + (t % j);
          const int a0 = sel_out[i], a1 = sel_out[i + j];
          if ((a1 < a0) == ((i & kk) == 0)) {
            sel_out[i] = a1;
            sel_out[i + j] = a0;
          }
        }
        __syncthreads();
      }
  }
  for (int i = tid; i < s_req; i += SEL_T) out[i] = sel_out[i];
  if (tid == 0) nrows[node] = s_req;
}

// Held-out residual: err = ||K_h - K_h(:, piv[:r]) P|| / ||K_h|| per node, over
// the node's nh_arr[node] held-out rows (K_h column-major, leading dimension
// h_cap); sets the node's fallback mask when err > tol. One workgroup per node.
// One workgroup per node. The residual K_h - K_h(:, J) P vanishes exactly on
// the skeleton columns (P is the identity there), so only the other columns
// are formed: the skeleton columns of K_h (r x 32) are staged in LDS, each
// thread owns one column j with its 32 held-out rows in registers and
// accumulates K_h(:, J) P(:, j) over the rank (P read coalesced, the LDS reads
// broadcast). Fixed-order reduction of the squared norms.
constexpr int kHeldRows = 32;
__global__ void __launch_bounds__(256) k_heldout_check(const double* __restrict__ Kh, const int32_t* __restrict__ nh_arr,
                                                       int h_cap, int n_cap,
                                                       int r_cap, int first, const int32_t* __restrict__ rank,
                                                       const int32_t* __restrict__ ncols,
                                                       const int32_t* __restrict__ piv, const double* __restrict__ P,
                                                       double tol, unsigned char* __restrict__ mask,
                                                       unsigned int* __restrict__ fallbacks, HeldoutGrow grow) {
  extern __shared__ double kj[];                  // r_cap x kHeldRows, then the pivot bitmap
  unsigned int* isp = reinterpret_cast<unsigned int*>(kj + (size_t)r_cap * kHeldRows);
  __shared__ double r1[256], r2[256];
  const int b = blockIdx.x, node = first + b, tid = threadIdx.x;
  const int n = ncols[node], r = rank[node], nh = nh_arr[node];
  const double* K = Kh + (int64_t)b * h_cap * n_cap;   // column-major h_cap x n
  const int32_t* pv = piv + (int64_t)node * n_cap;
  const double* Pn = P + (int64_t)node * r_cap * n_cap;
  for (int w = tid; w < (n + 31) / 32; w += 256) isp[w] = 0u;
  for (int e = tid; e < r * kHeldRows; e += 256) {
    const int i = e / kHeldRows, h = e % kHeldRows;
    kj[e] = h < nh ? K[(int64_t)pv[i] * h_cap + h] : 0.0;
  }
  __syncthreads();
  for (int i = tid; i < r; i += 256) atomicOr(&isp[pv[i] >> 5], 1u << (pv[i] & 31));
  __syncthreads();
  double num = 0.0, den = 0.0;
  for (int j = tid; j < n; j += 256) {
    double acc[kHeldRows];
#pragma unroll
    for (int h = 0; h < kHeldRows; ++h) acc[h] = 0.0;
    if (!((isp[j >> 5] >> (j & 31)) & 1u)) {
      for (int i = 0; i < r; ++i) {
        const double p = Pn[(int64_t)i * n_cap + j];
#pragma unroll
        for (int h = 0; h < kHeldRows; ++h) acc[h] = fma(kj[i * kHeldRows + h], p, acc[h]);
      }
    } else {
#pragma unroll
      for (int h = 0; h < kHeldRows; ++h) acc[h] = h < nh ? K[(int64_t)j * h_cap + h] : 0.0;   // exact
    }
#pragma unroll
    for (int h = 0; h < kHeldRows; ++h) {
      if (h < nh) {
        const double kv = K[(int64_t)j * h_cap + h];
        const double res = kv - acc[h];
        num = fma(res, res, num);
        den = fma(kv, kv, den);
      }
    }
  }
  r1[tid] = num;
  r2[tid] = den;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) { r1[tid] += r1[tid + off]; r2[tid] += r2[tid + off]; }
    __syncthreads();
  }
  if (tid == 0) {
    const double err = r2[0] > 0.0 ? sqrt(r1[0] / r2[0]) : 0.0;
    bool fall = err > tol;
    if (fall && grow.nrows) {   // adaptive sample count: only nodes whose rows can still grow
      const int nr = grow.nrows[node];
      const int64_t M = grow.N - (grow.ne[node] - grow.nb[node]);
      fall = nr < grow.s_limit && nr < M;
    }
    mask[node] = fall ? 1 : 0;
    if (fall) atomicAdd(fallbacks, 1u);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
ffc_status launch_geometry(const double* Xt, int d, const GeomArgs& ga, int count, hipStream_t st) {
  if (count <= 0) return FFC_OK;
  if (ga.col_stride > kMaxGeomCols) {
    set_error("column sets above 16384 points are not supported by the proposal features");
    return FFC_ERR_INVALID_ARG;
  }
  const size_t lds = geometry_lds(d, ga.col_stride);
  if (lds > 144 * 1024) {
    set_error("the proposal geometry does not fit in LDS for this dimension");
    return FFC_ERR_INVALID_ARG;
  }
  static size_t lds_set = 64 * 1024;
  if (lds > lds_set) {
    FFC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_geometry),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    lds_set = lds;
  }
  hipLaunchKernelGGL(k_geometry, dim3(count), dim3(256), lds, st, Xt, d, ga);
  FFC_LAUNCH_CHECK("k_geometry");
  return FFC_OK;
}

ffc_status launch_features(const double* Xt, int d, const GeomArgs& ga, const int32_t* tgt, int tgt_stride,
                           const int32_t* ntgt, int count, float* feat, int64_t feat_stride, hipStream_t st) {
  const int tiles = (tgt_stride + FT - 1) / FT;
  const int64_t blocks = (int64_t)count * tiles;
  if (blocks <= 0) return FFC_OK;
  hipLaunchKernelGGL(k_features, dim3((unsigned)blocks), dim3(256), 0, st, Xt, d, ga, tgt, tgt_stride, ntgt, tiles,
                     feat, feat_stride);
  FFC_LAUNCH_CHECK("k_features");
  return FFC_OK;
}

ffc_status launch_mlp_score(const float* theta, const float* mu, const float* sdv, const float* feat, int64_t count,
                            float* score, hipStream_t st) {
  if (count <= 0) return FFC_OK;
  const int64_t waves = std::min<int64_t>((count + 15) / 16, 2048);
  hipLaunchKernelGGL(k_mlp_score, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, theta, mu, sdv, feat, count,
                     score);
  FFC_LAUNCH_CHECK("k_mlp_score");
  return FFC_OK;
}

ffc_status launch_mlp_grad(const float* theta, const float* mu, const float* sdv, const float* feat,
                           const float* target, int64_t count, int64_t p0, int64_t stride_mul, int64_t total,
                           float* grads, hipStream_t st) {
  const int nwg = (int)((total + GB - 1) / GB);
  const size_t lds = sizeof(GradSmem);
  static bool attr = false;
  if (!attr) {
    FFC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp_grad),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  hipLaunchKernelGGL(k_mlp_grad, dim3(nwg), dim3(256), lds, st, theta, mu, sdv, feat, target, count, p0, stride_mul,
                     total, grads);
  FFC_LAUNCH_CHECK("k_mlp_grad");
  return FFC_OK;
}

ffc_status launch_grad_reduce_adam(const float* grads, int nwg, float* theta, float* m1, float* m2, float* gsum,
                                   float* loss_out, bool adam, float lr, int step, int64_t total, hipStream_t st) {
  // Bias corrections 1 / (1 - beta^t), formed in double (1 - 0.999f alone is
  // off by 1.3e-5 relative).
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, step))), c2 = (float)(1.0 / (1.0 - std::pow(0.999, step)));
  hipLaunchKernelGGL(k_grad_reduce_adam, dim3((NPARAM + 1 + 255) / 256), dim3(256), 0, st, grads, nwg, theta, m1, m2,
                     gsum, loss_out, adam ? 1 : 0, lr, c1, c2, total);
  FFC_LAUNCH_CHECK("k_grad_reduce_adam");
  return FFC_OK;
}

ffc_status launch_feature_stats(const float* feat, int64_t count, float* mu, float* sdv, hipStream_t st) {
  hipLaunchKernelGGL(k_feature_stats, dim3(NF), dim3(256), 0, st, feat, count, mu, sdv);
  FFC_LAUNCH_CHECK("k_feature_stats");
  return FFC_OK;
}

ffc_status launch_select_rows(const float* score, int64_t score_stride, int elem_stride, int mode,
                              const int32_t* pool, int pool_stride, const int32_t* npool, int first, int count, int s,
                              uint64_t seed, const int32_t* ncols, const unsigned char* mask, int32_t* rows, int s_cap,
                              int32_t* nrows, hipStream_t st) {
  if (count <= 0) return FFC_OK;
  if (pool_stride > SEL_T * SEL_E) {
    set_error("candidate pool too large for the selection kernel");
    return FFC_ERR_INVALID_ARG;
  }
  int sort_s = 1;
  while (sort_s < s) sort_s <<= 1;
  const size_t lds = (size_t)sort_s * sizeof(int);
  if (lds > 64 * 1024) {
    set_error("too many rows requested for the selection kernel");
    return FFC_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_select_rows, dim3(count), dim3(SEL_T), lds, st, score, score_stride, elem_stride, mode, pool,
                     pool_stride, npool, first, s, seed, ncols, mask, rows, s_cap, nrows, sort_s);
  FFC_LAUNCH_CHECK("k_select_rows");
  return FFC_OK;
}

ffc_status launch_heldout_check(const double* Kh, const int32_t* nh, int h_cap, const ffc_skel* sk, int first,
                                int count, double tol, unsigned char* mask, unsigned int* fallbacks,
                                const HeldoutGrow& grow, hipStream_t st) {
  if (count <= 0) return FFC_OK;
  if (h_cap != kHeldRows) {
    set_error("held-out check: 32 held-out rows expected");
    return FFC_ERR_INVALID_ARG;
  }
  const size_t lds = (size_t)sk->r_cap * kHeldRows * sizeof(double) + ((size_t)sk->n_cap + 31) / 32 * sizeof(int);
  if (lds > 64 * 1024)
    FFC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_heldout_check),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_heldout_check, dim3(count), dim3(256), lds, st, Kh, nh, h_cap, sk->n_cap, sk->r_cap, first,
                     sk->rank.ptr, sk->ncols.ptr, sk->piv.ptr, sk->P.ptr, tol, mask, fallbacks, grow);
  FFC_LAUNCH_CHECK("k_heldout_check");
  return FFC_OK;
}

}  // namespace ffc
