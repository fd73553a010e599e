// Similarity-graph edge sampling through a KDE tree (Sec. "The MS
// Algorithm": every edge (i, j) is drawn with probability close to eq.
// (sampling_prob), the kernel sums coming from a KDE algorithm used as a
// black box; the black box here is the random-sampling estimator of Sec.
// "Kernel Density Estimation", evaluated per tree node).
//
// Tree: leaves are blocks of 32 consecutive rows (nb = ceil(n/32)); h =
// ceil(log2 nb); node (l, k) holds rows [k 32 2^(h-l), (k+1) 32 2^(h-l))
// clipped to [0, n).  No tree is stored: a node is its index range.
//
// est(i, node): P rows; P <= t: the exact sum of k_ij over its rows j != i;
// else (P/t) sum_{c<t} k_{i,j_c} [j_c != i], j_c = lo + floor(U_c P).
// Draw (i, r): at level l the children A, B get eA, eB from their own
// sample streams, u = U(i, r, l); go to A iff u (eA + eB) < eA, and if both
// are 0 to the child with more rows other than i (A on a tie).  At the leaf
// an inverse CDF over its rows' exact values (0 for j = i) on u = U(i, r, h);
// if they are all 0, the floor(u m)-th of its m rows other than i.
// Degrees: rest_i = est(i, root) with t_deg samples; deg = 1 + rest; the
// draw (i, j) gets weight 1/(s (1/rest_i + 1/rest_j)) (0 if one is 0).
//
// Randomness: SplitMix64 (Steele, Lea & Flood 2014) counter streams; output
// c of stream (seed, tag, a, b) is mix(S + (c+1) gamma) with S =
// mix(mix(mix(seed ^ tag) ^ a) ^ b).  Sample streams: tag "TREE", a = i,
// b = r << 16 | l << 1 | side; descent uniforms: tag "TRUN", a = i, b = r,
// c = l; degree samples: tag "TDEG", a = i, b = 0.  A uniform is the top 53
// bits times 2^-53 and an index is floor(u53 P / 2^53), exact in integers.
//
// Layout and work: one wave per draw (4 per block), x_i staged in LDS; at
// each level lanes 0-31 evaluate child A's samples (or rows), lanes 32-63
// child B's, one kernel value per lane from fp64 direct differences; each
// half sums its 32 values in a fixed butterfly order.  Work per draw: h
// levels x 2t kernel values + 32 at the leaf, each d fp64 operations on a
// gathered row.  Results are deterministic; against a sequential fp64 sum
// they differ by rounding only, which moves a decision only when its target
// lies within that rounding of a boundary.
#include <utility>

#include "runtime.h"
#include "sort.h"

namespace stag {
namespace {

constexpr uint64_t kTagTreeSamples = 0x54524545ULL;  // "TREE"
constexpr uint64_t kTagTreeUniform = 0x5452554EULL;  // "TRUN"
constexpr uint64_t kTagTreeDegree = 0x54444547ULL;   // "TDEG"
constexpr uint64_t kGammaTree = 0x9E3779B97F4A7C15ULL;
constexpr int kTreeLeaf = 32;
constexpr int kTreeWaves = 4;

__device__ inline uint64_t tmix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__device__ inline uint64_t tstream(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b) {
  return tmix(tmix(tmix(seed ^ tag) ^ a) ^ b);
}
__device__ inline uint64_t tout(uint64_t st, uint64_t c) { return tmix(st + (c + 1) * kGammaTree); }
__device__ inline double tuniform(uint64_t bits) { return (double)(bits >> 11) * 0x1.0p-53; }
__device__ inline int64_t tpick(uint64_t bits, int64_t P) {
  const uint64_t u = bits >> 11;
  const uint64_t hi = __umul64hi(u, (uint64_t)P), lo = u * (uint64_t)P;
  return (int64_t)((hi << 11) | (lo >> 53));
}

// exp(-a ||x_i - x_j||^2), squared distance by direct differences, each
// product and sum rounded separately (ascending coordinates).
__device__ inline double tkernel(const float* __restrict__ xi, const float* __restrict__ xj, int d, double a,
                                 bool vec4) {
  double D = 0.0;
  if (vec4) {
    const float4* x4 = reinterpret_cast<const float4*>(xj);
    auto piece = [&](const float4& v, int c) {
      double t = (double)xi[4 * c] - (double)v.x;
      D = __dadd_rn(D, __dmul_rn(t, t));
      t = (double)xi[4 * c + 1] - (double)v.y;
      D = __dadd_rn(D, __dmul_rn(t, t));
      t = (double)xi[4 * c + 2] - (double)v.z;
      D = __dadd_rn(D, __dmul_rn(t, t));
      t = (double)xi[4 * c + 3] - (double)v.w;
      D = __dadd_rn(D, __dmul_rn(t, t));
    };
    // eight 16-byte pieces' loads issued before their products (same order)
    const int d4 = d / 4;
    int c = 0;
    for (; c + 7 < d4; c += 8) {
      float4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = x4[c + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) piece(v[u], c + u);
    }
    for (; c < d4; ++c) piece(x4[c], c);
  } else {
    for (int c = 0; c < d; ++c) {
      const double t = (double)xi[c] - (double)xj[c];
      D = __dadd_rn(D, __dmul_rn(t, t));
    }
  }
  return exp(-a * D);
}

__device__ inline double half_sum(double v) {  // fixed butterfly within each 32-lane half
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// rest[i] = est(i, root) with t_deg samples; one wave per row i.
__global__ __launch_bounds__(256) void tree_degrees(const float* __restrict__ X, int64_t n, int d, double a,
                                                    int64_t t_deg, uint64_t seed, bool vec4,
                                                    double* __restrict__ rest, double* __restrict__ deg_out) {
  extern __shared__ float txi[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * kTreeWaves + wave;
  float* xi = txi + wave * d;
  if (i < n)
    for (int c = lane; c < d; c += 64) xi[c] = X[i * d + c];
  __syncthreads();
  if (i >= n) return;
  double s = 0.0;
  if (n <= t_deg) {
    for (int64_t j = lane; j < n; j += 64)
      if (j != i) s += tkernel(xi, X + j * d, d, a, vec4);
  } else {
    const uint64_t st = tstream(seed, kTagTreeDegree, (uint64_t)i, 0);
    for (int64_t c = lane; c < t_deg; c += 64) {
      const int64_t j = tpick(tout(st, (uint64_t)c), n);
      if (j != i) s += tkernel(xi, X + j * d, d, a, vec4);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (n > t_deg) s = s * ((double)n / (double)t_deg);
  if (lane == 0) {
    rest[i] = s;
    if (deg_out) deg_out[i] = 1.0 + s;
  }
}

// Draws run level by level: one launch per tree level, then the draws are
// sorted (stable radix sort) by the node they reached, so that the waves of
// a launch that work in the same node are neighbours; with the XCD-aware
// block order below each XCD takes a contiguous range of nodes, and from the
// level where a node's rows fit an XCD's L2 the gathers hit in L2.  The
// order changes only where a draw runs, not what it computes.
//
// Workgroups go round-robin to the 8 XCDs: block b works on logical block
// (b % 8) per + b / 8 (the grid is 8 per blocks), i.e. slots
// [4 L, 4 L + 4) of the sorted order.
__device__ inline int64_t tree_slot(int per) {
  const int b = blockIdx.x;
  const int64_t L = (int64_t)(b % 8) * per + b / 8;
  return L * kTreeWaves + (threadIdx.x >> 6);
}

// Stage x_i of the draw in slot `slot` (if any) into this wave's LDS row.
__device__ inline void stage_row(float* xi, const float* __restrict__ X, int64_t i, int d, bool active) {
  const int lane = threadIdx.x & 63;
  if (active)
    for (int c = lane; c < d; c += 64) xi[c] = X[i * d + c];
}

// perm[w] = w, node[w] = 0.
__global__ void tree_init(uint32_t* __restrict__ perm, uint32_t* __restrict__ node, int64_t total) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w < total) {
    perm[w] = (uint32_t)w;
    node[w] = 0;
  }
}

// One level l < h for the draw in each slot: node_in[slot] -> node_out[slot].
__global__ __launch_bounds__(256) void tree_level(const float* __restrict__ X, int64_t n, int d, double a, int s,
                                                  int t, int h, int l, uint64_t seed, bool vec4,
                                                  const uint32_t* __restrict__ perm,
                                                  const uint32_t* __restrict__ node_in, uint32_t* __restrict__ node_out,
                                                  int64_t total, int per) {
  extern __shared__ float txi[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t slot = tree_slot(per);
  const bool active = slot < total;
  const int64_t e = active ? (int64_t)perm[slot] : 0;
  const int64_t i = e / s, r = e % s;
  float* xi = txi + wave * d;
  stage_row(xi, X, i, d, active);
  __syncthreads();
  if (!active) return;
  const int side = lane >> 5, c = lane & 31;
  const int64_t k = node_in[slot];
  const int64_t span = (int64_t)kTreeLeaf << (h - l - 1);
  const int64_t lo = min(n, (2 * k + side) * span), hi = min(n, (2 * k + side + 1) * span);
  const int64_t P = hi - lo;
  double v = 0.0;
  if (P > 0 && P <= t) {
    const int64_t j = lo + c;
    if (c < P && j != i) v = tkernel(xi, X + j * d, d, a, vec4);
  } else if (P > t && c < t) {
    const uint64_t st =
        tstream(seed, kTagTreeSamples, (uint64_t)i, ((uint64_t)r << 16) | ((uint64_t)l << 1) | (uint64_t)side);
    const int64_t j = lo + tpick(tout(st, (uint64_t)c), P);
    if (j != i) v = tkernel(xi, X + j * d, d, a, vec4);
  }
  double est = half_sum(v);
  if (P > t) est = est * ((double)P / (double)t);
  const double eA = __shfl(est, 0), eB = __shfl(est, 32);
  const double u = tuniform(tout(tstream(seed, kTagTreeUniform, (uint64_t)i, (uint64_t)r), (uint64_t)l));
  const double tot = eA + eB;
  bool left;
  if (tot > 0.0) {
    left = u * tot < eA;
  } else {
    const int64_t aLo = min(n, 2 * k * span), aHi = min(n, (2 * k + 1) * span), bHi = min(n, (2 * k + 2) * span);
    const int64_t mA = (aHi - aLo) - ((i >= aLo && i < aHi) ? 1 : 0);
    const int64_t mB = (bHi - aHi) - ((i >= aHi && i < bHi) ? 1 : 0);
    left = mA >= mB;
  }
  if (lane == 0) node_out[slot] = (uint32_t)(left ? 2 * k : 2 * k + 1);
}

// The leaf (level h) of the draw in each slot: inverse CDF over its rows in
// row order; outputs at the draw's own index e = i s + r.
__global__ __launch_bounds__(256) void tree_leaf(const float* __restrict__ X, int64_t n, int d, double a, int s,
                                                 int h, uint64_t seed, bool vec4, const uint32_t* __restrict__ perm,
                                                 const uint32_t* __restrict__ node, const double* __restrict__ rest,
                                                 int64_t* __restrict__ src, int64_t* __restrict__ dst,
                                                 double* __restrict__ w, int64_t total, int per) {
  extern __shared__ float txi[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t slot = tree_slot(per);
  const bool active = slot < total;
  const int64_t e = active ? (int64_t)perm[slot] : 0;
  const int64_t i = e / s, r = e % s;
  float* xi = txi + wave * d;
  stage_row(xi, X, i, d, active);
  __syncthreads();
  if (!active) return;
  const int side = lane >> 5, c = lane & 31;
  const int64_t k = node[slot];
  const int64_t lo = min(n, k * kTreeLeaf), hi = min(n, (k + 1) * kTreeLeaf);
  const int64_t j = lo + c;
  double v = 0.0;
  if (side == 0 && j < hi && j != i) v = tkernel(xi, X + j * d, d, a, vec4);
  double incl = v;  // inclusive prefix over lanes 0-31 (lanes 32-63 hold 0)
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) {
    const double y = __shfl_up(incl, o);
    if (c >= o) incl += y;
  }
  const double T = __shfl(incl, 31);
  const double u = tuniform(tout(tstream(seed, kTagTreeUniform, (uint64_t)i, (uint64_t)r), (uint64_t)h));
  int64_t pick;
  if (T > 0.0) {
    const double target = u * T;
    // only a row with a positive value can take the draw (the butterfly
    // prefix need not be exactly monotone where a value is 0)
    const uint64_t pass = __ballot(side == 0 && v > 0.0 && incl > target);
    if (pass != 0) {
      pick = lo + __builtin_ctzll(pass);
    } else {  // rounding left the target above the total: the last positive value
      const uint64_t pos = __ballot(side == 0 && v > 0.0);
      pick = lo + 63 - __builtin_clzll(pos);
    }
  } else {
    const int64_t m = (hi - lo) - ((i >= lo && i < hi) ? 1 : 0);
    const int64_t idx = (int64_t)(u * (double)m);
    pick = lo + idx;
    if (i >= lo && i < hi && pick >= i) ++pick;
  }
  if (lane == 0) {
    src[e] = i;
    dst[e] = pick;
    const double ri = rest[i], rj = rest[pick];
    w[e] = (ri > 0.0 && rj > 0.0) ? 1.0 / ((double)s * (1.0 / ri + 1.0 / rj)) : 0.0;
  }
}

}  // namespace
}  // namespace stag

extern "C" stag_status stag_simgraph_sample_tree(const float* X, int64_t n, int32_t d, double a,
                                                 int32_t samples_per_node, int32_t est_samples,
                                                 int64_t degree_samples, uint64_t seed, int64_t* src_out,
                                                 int64_t* dst_out, double* w_out, double* deg_out,
                                                 hipStream_t stream) {
  using namespace stag;
  const char* fn = "stag_simgraph_sample_tree";
  if (!X || !src_out || !dst_out || !w_out) return fail(STAG_E_INVAL, "%s: NULL argument", fn);
  if (n < 2 || n > 2147483647LL || d < 1) return fail(STAG_E_INVAL, "%s: need 2 <= n < 2^31, d >= 1", fn);
  if (d > 1024) return fail(STAG_E_UNSUPPORTED, "%s: d = %d > 1024 is not supported", fn, d);
  if (!(a > 0.0) || !std::isfinite(a)) return fail(STAG_E_INVAL, "%s: a must be positive and finite", fn);
  if (samples_per_node < 0 || samples_per_node > 64)
    return fail(STAG_E_INVAL, "%s: samples_per_node must be in [0, 64]", fn);
  if (est_samples < 1 || est_samples > 32) return fail(STAG_E_INVAL, "%s: est_samples must be in [1, 32]", fn);
  if (degree_samples < 1) return fail(STAG_E_INVAL, "%s: degree_samples must be >= 1", fn);
  const int s = stag_simgraph_draws_per_node(n, samples_per_node);
  const int64_t draws = n * s;
  if (draws >= 2147483647LL) return fail(STAG_E_INVAL, "%s: n * samples_per_node must be < 2^31", fn);
  const int64_t nb = (n + kTreeLeaf - 1) / kTreeLeaf;
  int h = 0;
  while (((int64_t)1 << h) < nb) ++h;
  clear_error();
  Workspace ws(stream);
  double* rest = nullptr;
  STAG_TRY(ws.alloc(&rest, (size_t)n));
  const size_t lds = (size_t)kTreeWaves * d * sizeof(float);
  const bool vec4 = (d % 4) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;  // float4 row loads
  {
    ScopedTimer tm("tree_degrees", stream);
    hipLaunchKernelGGL(tree_degrees, dim3((unsigned)ceil_div(n, kTreeWaves)), dim3(256), lds, stream, X, n, (int)d,
                       a, degree_samples, seed, vec4, rest, deg_out);
    STAG_TRY(check_launch("tree_degrees"));
  }
  // draws level by level, sorted by node between levels
  const int per = (int)ceil_div(ceil_div(draws, kTreeWaves), 8);
  const dim3 grid((unsigned)(8 * per));
  uint32_t *perm = nullptr, *perm2 = nullptr, *node = nullptr, *node2 = nullptr;
  STAG_TRY(ws.alloc(&perm, (size_t)draws));
  STAG_TRY(ws.alloc(&perm2, (size_t)draws));
  STAG_TRY(ws.alloc(&node, (size_t)draws));
  STAG_TRY(ws.alloc(&node2, (size_t)draws));
  hipLaunchKernelGGL(tree_init, dim3((unsigned)ceil_div(draws, 256)), dim3(256), 0, stream, perm, node, draws);
  STAG_TRY(check_launch("tree_init"));
  for (int l = 0; l < h; ++l) {
    {
      ScopedTimer tm("tree_draws", stream);
      hipLaunchKernelGGL(tree_level, grid, dim3(256), lds, stream, X, n, (int)d, a, s, (int)est_samples, h, l, seed,
                         vec4, perm, node, node2, draws, per);
      STAG_TRY(check_launch("tree_level"));
    }
    ScopedTimer tm("tree_sort", stream);
    STAG_TRY(radix_sort_pairs_u32(node2, perm, node, perm2, draws, l + 1, ws, stream));
    std::swap(perm, perm2);
  }
  {
    ScopedTimer tm("tree_draws", stream);
    hipLaunchKernelGGL(tree_leaf, grid, dim3(256), lds, stream, X, n, (int)d, a, s, h, seed, vec4, perm, node, rest,
                       src_out, dst_out, w_out, draws, per);
    STAG_TRY(check_launch("tree_leaf"));
  }
  return STAG_OK;
}
