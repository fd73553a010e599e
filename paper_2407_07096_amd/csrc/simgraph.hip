// Similarity-graph edge sampling (Sec. "The MS Algorithm": sample edge (i,j)
// with probability proportional to w_F(i,j)/deg_F(i) + w_F(i,j)/deg_F(j), the
// degrees being kernel sums, so that the sampled graph keeps the cluster
// structure of the fully connected one with O~(n) edges).
//
// Mechanism (the paper leaves it open): every node i draws s neighbours
// j != i with probability k_ij / rest_i, rest_i = sum_{j != i} k_ij, and each
// draw carries weight 1 / (s (1/rest_i + 1/rest_j)), so the expected sampled
// weight of every pair is k_ij.  deg(i) = 1 + rest_i.
//
// Exact mode: one self-excluding pass of the exact tile kernel gives the
// per-chunk (4096 rows) fp64 sums and per-tile (32 rows) fp32 sums of every
// row of the kernel matrix (tile sums stored node-major, so one draw reads
// its chunk's 128 tile sums contiguously); a draw walks chunk sums, then tile sums, then
// recomputes the 32 kernel values of its tile in fp64 (direct differences,
// two lanes per row) and inverts the cumulative sum at each level, j
// ascending.  Between the tile and the row step the draws are sorted by tile
// so that draws gathering the same rows run together.
// LSH mode: the CKNS estimator's terms replace the kernel row (lsh.hip).
#include <cmath>

#include "kde_exact.h"
#include "lsh.h"
#include "runtime.h"
#include "sort.h"

namespace stag {
namespace {

constexpr uint64_t kGammaS = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t kTagDrawS = 0x44524157ULL;
// Rows up to this width draw in one fused kernel, wider ones through the
// tile sort (measured at n = 100,000, 17 draws per node: the fused draw is
// faster by 20% at d = 64 and by 5% at d = 256, the sorted one by 9% at
// d = 512 and, on sparse rows at n = 70,000, by 43% at d = 784).
constexpr int kDrawFusedMaxDim = 256;
constexpr int kChunkTiles = 128;  // 32-row tiles per 4096-row chunk
constexpr double kLog2eS = 1.4426950408889634074;

__device__ inline uint64_t mixs(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ inline double scan64(double v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  return v;
}

// rest_i (chunk order) and a node-major copy of the chunk sums, so that a
// draw reads its node's P sums from consecutive addresses.
// A row whose sum is below kRescueBelow sets flag[i] and the flag of its
// query tile of qtile_rows rows (underflow rescue).
__global__ void row_rest(const double* __restrict__ partial, int P, int64_t m_pad, int64_t n,
                         double* __restrict__ rest, double* __restrict__ deg, double* __restrict__ chunk_t,
                         int* __restrict__ flag, int* __restrict__ qtile_flag, int qtile_rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int p = 0; p < P; ++p) {
    const double v = partial[(int64_t)p * m_pad + i];
    chunk_t[i * P + p] = v;
    s += v;
  }
  rest[i] = s;
  if (deg) deg[i] = 1.0 + s;
  if (flag && s < kRescueBelow) {
    flag[i] = 1;
    qtile_flag[i / qtile_rows] = 1;
  }
}

// Rows of the rescue's second self pass: a flagged row takes its shifted
// chunk sums (the draws use them and the shifted total rest_draw), and its
// true total rest = rest_draw 2^{m_i} for the weights and degrees; other rows
// keep rest_draw = rest.
__global__ void rescue_rows(const double* __restrict__ partial, int P, int64_t m_pad, int64_t n,
                            const int* __restrict__ flag, const double* __restrict__ shift,
                            double* __restrict__ rest, double* __restrict__ rest_draw, double* __restrict__ deg,
                            double* __restrict__ chunk_t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!flag[i]) {
    rest_draw[i] = rest[i];
    return;
  }
  double s = 0.0;
  for (int p = 0; p < P; ++p) {
    const double v = partial[(int64_t)p * m_pad + i];
    chunk_t[i * P + p] = v;
    s += v;
  }
  rest_draw[i] = s;
  const double t = s * exp2(shift[i]);
  rest[i] = t;
  if (deg) deg[i] = 1.0 + t;
}

// Inverts a cumulative sum over `count` values v(k) (k ascending, fetched by
// the lane that owns k) for `target`; returns the index and the remainder
// below it.  Past the total (rounding), the last positive value is taken with
// an infinite remainder so that lower levels also take their last element.
template <class Fetch>
__device__ inline int invert_level(int count, double target, Fetch&& fetch, double* resid_out) {
  const int lane = threadIdx.x & 63;
  double running = 0.0;
  int last = -1;
  for (int k0 = 0; k0 < count; k0 += 64) {
    const int k = k0 + lane;
    const double v = k < count ? fetch(k) : 0.0;
    const double incl = scan64(v);
    const double btot = __shfl(incl, 63);
    const uint64_t pos = __ballot(v > 0.0);
    if (pos) last = k0 + 63 - __clzll((long long)pos);
    if (running + btot > target) {
      // only a positive value can be the crossing: past the block's last
      // positive value the tree scan may differ from it by a rounding, and a
      // crossing found there means the target lies beyond this block
      const uint64_t over = __ballot(running + incl > target) & pos;
      if (over) {
        const int kl = __ffsll((long long)over) - 1;
        *resid_out = target - (running + __shfl(incl - v, kl));
        return k0 + kl;
      }
    }
    running += btot;
  }
  *resid_out = INFINITY;
  return last;
}

// A draw of node i takes a chunk, then a 32-row tile within it, then a row
// within the tile, each by inversion of a cumulative sum.  The first two
// steps read only the chunk and tile sums; the last reads the 32 rows of the
// tile.  For wide rows they run as two kernels with the draws sorted by tile
// in between (stable radix sort): with the XCD-aware block order of
// `draw_row` each XCD takes a contiguous range of tiles, and the waves that
// gather the same tile run side by side and hit in that XCD's L2.  For
// narrow rows, whose tiles stay in cache anyway, one fused kernel does both.
// The order changes only where a draw runs, not what it computes.

// The uniform of draw r of node i.
__device__ inline double draw_uniform(uint64_t seed, int64_t i, int r) {
  uint64_t ds = mixs(mixs(mixs(seed ^ kTagDrawS) ^ (uint64_t)i) ^ 0ULL);
  return (double)(mixs(ds + (uint64_t)(r + 1) * kGammaS) >> 11) * 0x1.0p-53;
}

// Steps 1 and 2 of a draw (the whole wave): the tile (ntile when the draw
// finds none) and the remainder of the target below it.
__device__ inline int64_t draw_tile_of(int64_t i, double u, int P, int64_t ntile, int64_t tstride,
                                       const double* __restrict__ chunk_t, const float* __restrict__ tp,
                                       const double* __restrict__ rest, const double* __restrict__ rest_draw,
                                       double* resid2) {
  // rest_draw: the total in the scale of the chunk and tile sums (2^{-m_i}
  // times the true one for a row of the underflow rescue, else the same)
  const double tot = rest_draw[i];
  *resid2 = 0.0;
  if (!(rest[i] > 0.0 && tot > 0.0)) return ntile;
  double resid = 0.0;
  const int c = invert_level(P, u * tot, [&](int k) { return chunk_t[i * P + k]; }, &resid);
  if (c < 0) return ntile;
  const int64_t t0 = (int64_t)c * kChunkTiles;
  const int nt = (int)((ntile - t0) < kChunkTiles ? (ntile - t0) : kChunkTiles);
  const int tl = invert_level(nt, resid, [&](int k) { return (double)tp[i * tstride + t0 + k]; }, resid2);
  return tl >= 0 ? t0 + tl : ntile;
}

__device__ inline double sq_diff4(double D, const float4& p, const float4& q) {
  double t = (double)p.x - (double)q.x;
  D = __builtin_fma(t, t, D);
  t = (double)p.y - (double)q.y;
  D = __builtin_fma(t, t, D);
  t = (double)p.z - (double)q.z;
  D = __builtin_fma(t, t, D);
  t = (double)p.w - (double)q.w;
  return __builtin_fma(t, t, D);
}

// Copies x_i into this wave's LDS row xs (16-byte pieces when vec4).
__device__ inline void stage_xi(float* xs, const float* __restrict__ X, int64_t i, int d, int vec4, bool active) {
  const int lane = threadIdx.x & 63;
  if (!active) return;
  if (vec4) {
    const float4* src4 = reinterpret_cast<const float4*>(X + i * d);
    float4* xs4 = reinterpret_cast<float4*>(xs);
    for (int c = lane; c < (d >> 2); c += 64) xs4[c] = src4[c];
  } else {
    for (int c = lane; c < d; c += 64) xs[c] = X[i * d + c];
  }
}

// Step 3 (the whole wave): the row of tile T for remainder resid2, or -1;
// xi is node i's row staged in LDS.  Rows of the tile: lanes l and l + 32
// share row l % 32 and take alternate 16-byte pieces (or alternate
// elements) of it, summed in order; the loads of four pieces are issued
// before their products so that they overlap.
__device__ inline int64_t draw_row_of(const float* xi, const float* __restrict__ X, int64_t n, int d, double a,
                                      int64_t i, int64_t T, double resid2, double sh, int vec4) {
  const int lane = threadIdx.x & 63;
  const int64_t rb = T * 32;
  const int half = lane >> 5;
  const int64_t j = rb + (lane & 31);
  const bool live = j < n && j != i;
  double D = 0.0;
  if (live) {
    const float* xj = X + j * d;
    if (vec4) {
      const float4* a4 = reinterpret_cast<const float4*>(xi);
      const float4* b4 = reinterpret_cast<const float4*>(xj);
      const int n4 = d >> 2;
      int k4 = half;
      for (; k4 + 6 < n4; k4 += 8) {
        const float4 p0 = a4[k4], q0 = b4[k4], p1 = a4[k4 + 2], q1 = b4[k4 + 2];
        const float4 p2 = a4[k4 + 4], q2 = b4[k4 + 4], p3 = a4[k4 + 6], q3 = b4[k4 + 6];
        D = sq_diff4(D, p0, q0);
        D = sq_diff4(D, p1, q1);
        D = sq_diff4(D, p2, q2);
        D = sq_diff4(D, p3, q3);
      }
      for (; k4 < n4; k4 += 2) D = sq_diff4(D, a4[k4], b4[k4]);
    } else {
      for (int h = half; h < d; h += 2) {
        const double t = (double)xi[h] - (double)xj[h];
        D = __builtin_fma(t, t, D);
      }
    }
  }
  D += __shfl_xor(D, 32);
  // a shifted row's values are 2^{E - m_i} with E = -a log2(e) D in one
  // exponent (2^{-m_i} alone overflows for m_i < -1024, and exp(-a D) is
  // subnormal there)
  double kv = 0.0;
  if (lane < 32 && live) kv = sh == 0.0 ? exp(-a * D) : exp2(fma(-a * kLog2eS, D, -sh));
  double resid3 = 0.0;
  const int jl = invert_level(32, resid2, [&](int) { return kv; }, &resid3);  // lane k owns row k
  return jl >= 0 ? rb + jl : -1;
}

__device__ inline void draw_store(int64_t e, int64_t i, int64_t pick, int s, const double* __restrict__ rest,
                                  int64_t* __restrict__ src, int64_t* __restrict__ dst, double* __restrict__ w) {
  if ((threadIdx.x & 63) == 0) {
    src[e] = i;
    dst[e] = pick;
    w[e] = pick >= 0 ? 1.0 / ((double)s * (1.0 / rest[i] + 1.0 / rest[pick])) : 0.0;
  }
}

// Fused draw, one wave per draw e = (node i, draw r); dynamic LDS: one
// row of d floats per wave.
__global__ __launch_bounds__(256) void draw_exact(const float* __restrict__ X, int64_t n, int d, double a, int s,
                                                  uint64_t seed, int P, int64_t ntile, int64_t tstride,
                                                  const double* __restrict__ chunk_t, const float* __restrict__ tp,
                                                  const double* __restrict__ rest,
                                                  const double* __restrict__ rest_draw,
                                                  const double* __restrict__ shift, int vec4,
                                                  int64_t* __restrict__ src, int64_t* __restrict__ dst,
                                                  double* __restrict__ w) {
  extern __shared__ float4 dxs4[];
  float* xs = reinterpret_cast<float*>(dxs4) + (threadIdx.x >> 6) * d;
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const bool active = e < n * s;
  const int64_t i = active ? e / s : 0;
  stage_xi(xs, X, i, d, vec4, active);
  double resid2 = 0.0;
  int64_t T = ntile;
  if (active)
    T = draw_tile_of(i, draw_uniform(seed, i, (int)(e % s)), P, ntile, tstride, chunk_t, tp, rest, rest_draw,
                     &resid2);
  __syncthreads();
  if (!active) return;
  const int64_t pick = T < ntile ? draw_row_of(xs, X, n, d, a, i, T, resid2, shift[i], vec4) : -1;
  draw_store(e, i, pick, s, rest, src, dst, w);
}

// Split draw, step 1 (one wave per draw e): tile[e], order[e] = e and the
// remainder.
__global__ __launch_bounds__(256) void draw_tile(int64_t n, int s, uint64_t seed, int P, int64_t ntile,
                                                 int64_t tstride, const double* __restrict__ chunk_t,
                                                 const float* __restrict__ tp, const double* __restrict__ rest,
                                                 const double* __restrict__ rest_draw, uint32_t* __restrict__ tile,
                                                 uint32_t* __restrict__ order, double* __restrict__ resid_out) {
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= n * s) return;
  const int64_t i = e / s;
  double resid2 = 0.0;
  const int64_t T =
      draw_tile_of(i, draw_uniform(seed, i, (int)(e % s)), P, ntile, tstride, chunk_t, tp, rest, rest_draw, &resid2);
  if ((threadIdx.x & 63) == 0) {
    tile[e] = (uint32_t)T;
    order[e] = (uint32_t)e;
    resid_out[e] = resid2;
  }
}

// Split draw, step 2, one wave per draw in the order given by `order`
// (tile[k] is the tile of draw order[k]); dynamic LDS: one row of d floats
// per wave.  Workgroups go round-robin to the 8 XCDs: block b works on
// logical block (b % 8) per + b / 8 (the grid is 8 per blocks), i.e. slots
// [4 L, 4 L + 4).
__global__ __launch_bounds__(256) void draw_row(const float* __restrict__ X, int64_t n, int d, double a, int s,
                                                int64_t ntile, int per, const uint32_t* __restrict__ tile,
                                                const uint32_t* __restrict__ order,
                                                const double* __restrict__ resid_in,
                                                const double* __restrict__ rest, const double* __restrict__ shift,
                                                int vec4, int64_t* __restrict__ src, int64_t* __restrict__ dst,
                                                double* __restrict__ w) {
  extern __shared__ float4 dxs4[];
  float* xs = reinterpret_cast<float*>(dxs4) + (threadIdx.x >> 6) * d;
  const int b = blockIdx.x;
  const int64_t slot = ((int64_t)(b % 8) * per + b / 8) * 4 + (threadIdx.x >> 6);
  const bool active = slot < n * s;
  const int64_t e = active ? (int64_t)order[slot] : 0;
  const int64_t i = e / s;
  stage_xi(xs, X, i, d, vec4, active);
  __syncthreads();
  if (!active) return;
  const int64_t T = tile[slot];
  const int64_t pick = T < ntile ? draw_row_of(xs, X, n, d, a, i, T, resid_in[e], shift[i], vec4) : -1;
  draw_store(e, i, pick, s, rest, src, dst, w);
}

stag_status sample_exact(const float* X, int64_t n, int d, double a, int form, int s, uint64_t seed, int64_t* src,
                         int64_t* dst, double* w, double* deg_out, hipStream_t st) {
  Workspace ws(st);
  Operands xo, qo;
  STAG_TRY(prepare_operands(form, X, n, d, a, false, ws, &xo, st));
  STAG_TRY(prepare_operands(form, X, n, d, a, true, ws, &qo, st));
  const int P = (int)exact_chunks(xo.rows_pad);
  const int64_t ntile = xo.rows_pad / 32;
  const int64_t tstride = round_up(ntile, 16);
  double* partial = nullptr;
  float* tp = nullptr;
  double* rest = nullptr;
  double* chunk_t = nullptr;
  STAG_TRY(ws.alloc(&partial, (size_t)P * qo.rows_pad));
  STAG_TRY(ws.alloc(&chunk_t, (size_t)P * n));
  STAG_TRY(ws.alloc(&tp, (size_t)tstride * qo.rows_pad));
  STAG_TRY(ws.alloc(&rest, (size_t)n));
  TileExtra ex;
  ex.self = 1;
  ex.tp = tp;
  ex.ntile = tstride;
  STAG_TRY(launch_exact_tiles(xo, qo, partial, ex, st));
  // underflow rescue: rows whose sum is below kRescueBelow get their
  // exponents shifted by their maximum over the other rows and a second self
  // pass (over their 128-row tiles only; other workgroups return at once)
  const int64_t nqt = qo.rows_pad / query_tile_rows();
  int *flag = nullptr, *qflag = nullptr;
  double *rest_draw = nullptr, *shift = nullptr;
  float* off2 = nullptr;
  STAG_TRY(ws.alloc(&flag, (size_t)n));
  STAG_TRY(ws.alloc(&qflag, (size_t)nqt));
  STAG_TRY(ws.alloc(&rest_draw, (size_t)n));
  STAG_TRY(ws.alloc(&shift, (size_t)qo.rows_pad));
  STAG_TRY(ws.alloc(&off2, (size_t)qo.rows_pad));
  STAG_TRY(zero_async(flag, (size_t)n * sizeof(int), st));
  STAG_TRY(zero_async(qflag, (size_t)nqt * sizeof(int), st));
  hipLaunchKernelGGL(row_rest, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, partial, P, qo.rows_pad, n, rest,
                     deg_out, chunk_t, flag, qflag, (int)query_tile_rows());
  STAG_TRY(check_launch("row_rest"));
  STAG_TRY(rescue_offsets(xo, qo, P, a, 1, flag, qflag, off2, shift, ws, st));
  Operands q2 = qo;
  q2.off = off2;
  TileExtra exr = ex;
  exr.qtile_active = qflag;
  STAG_TRY(launch_exact_tiles(xo, q2, partial, exr, st));
  hipLaunchKernelGGL(rescue_rows, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, partial, P, qo.rows_pad, n,
                     flag, shift, rest, rest_draw, deg_out, chunk_t);
  STAG_TRY(check_launch("rescue_rows"));
  const int vec4 = (d % 4 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
  const int64_t nd = n * s;
  const size_t lds = (size_t)4 * d * sizeof(float);  // x_i of each of the 4 waves
  ScopedTimer tm("simgraph_draw_exact", st);
  if (d <= kDrawFusedMaxDim) {
    hipLaunchKernelGGL(draw_exact, dim3((unsigned)ceil_div(nd, 4)), dim3(256), lds, st, X, n, d, a, s, seed, P, ntile,
                       tstride, chunk_t, tp, rest, rest_draw, shift, vec4, src, dst, w);
    return check_launch("draw_exact");
  }
  // the sort carries draw indices in 32 bits (the n x n/32 tile sums above
  // bound n far below this in practice)
  if (nd >= ((int64_t)1 << 31)) return fail(STAG_E_UNSUPPORTED, "stag_simgraph_sample: n * s >= 2^31 draws");
  uint32_t *tile = nullptr, *order = nullptr, *tile_s = nullptr, *order_s = nullptr;
  double* resid = nullptr;
  STAG_TRY(ws.alloc(&tile, (size_t)nd));
  STAG_TRY(ws.alloc(&order, (size_t)nd));
  STAG_TRY(ws.alloc(&tile_s, (size_t)nd));
  STAG_TRY(ws.alloc(&order_s, (size_t)nd));
  STAG_TRY(ws.alloc(&resid, (size_t)nd));
  hipLaunchKernelGGL(draw_tile, dim3((unsigned)ceil_div(nd, 4)), dim3(256), 0, st, n, s, seed, P, ntile, tstride,
                     chunk_t, tp, rest, rest_draw, tile, order, resid);
  STAG_TRY(check_launch("draw_tile"));
  int bits = 1;
  while (((int64_t)1 << bits) <= ntile) ++bits;  // keys 0..ntile
  STAG_TRY(radix_sort_pairs_u32(tile, order, tile_s, order_s, nd, bits, ws, st));
  const int per = (int)ceil_div(ceil_div(nd, 4), 8);
  hipLaunchKernelGGL(draw_row, dim3((unsigned)(8 * per)), dim3(256), lds, st, X, n, d, a, s, ntile, per, tile_s,
                     order_s, resid, rest, shift, vec4, src, dst, w);
  return check_launch("draw_row");
}

}  // namespace
}  // namespace stag

extern "C" int32_t stag_simgraph_draws_per_node(int64_t n, int32_t samples_per_node) {
  if (n < 1 || samples_per_node < 0 || samples_per_node > 64) return -1;
  if (samples_per_node > 0) return samples_per_node;
  int s = 0;
  while (((int64_t)1 << s) < n) ++s;  // ceil(log2 n)
  return s < 1 ? 1 : s;
}

extern "C" stag_status stag_simgraph_sample(const float* X, int64_t n, int32_t d, double a, int32_t samples_per_node,
                                            int32_t kde_mode, int32_t form, double eps, const stag_lsh_params* lsh,
                                            uint64_t seed, int64_t* src_out, int64_t* dst_out, double* w_out,
                                            double* deg_out, hipStream_t stream) {
  using namespace stag;
  if (!X || !src_out || !dst_out || !w_out) return fail(STAG_E_INVAL, "stag_simgraph_sample: NULL argument");
  if (n < 2 || d < 1 || n > 2147483647LL) return fail(STAG_E_INVAL, "stag_simgraph_sample: need 2 <= n < 2^31, d >= 1");
  if (!(a > 0.0) || !std::isfinite(a)) return fail(STAG_E_INVAL, "stag_simgraph_sample: a must be positive and finite");
  if (samples_per_node < 0 || samples_per_node > 64)
    return fail(STAG_E_INVAL, "stag_simgraph_sample: samples_per_node must be in [0, 64]");
  const int s = stag_simgraph_draws_per_node(n, samples_per_node);
  clear_error();
  if (kde_mode == STAG_SIMGRAPH_EXACT) {
    if (form < STAG_FORM_FP32 || form > STAG_FORM_BF16_SPLIT3)
      return fail(STAG_E_INVAL, "stag_simgraph_sample: unknown form %d", form);
    if (exact_padded_dim(d) == 0 || (d > 256 && form == STAG_FORM_BF16_SPLIT3))
      return fail(STAG_E_UNSUPPORTED, "stag_simgraph_sample: d = %d not supported by this form", d);
    return sample_exact(X, n, d, a, form, s, seed, src_out, dst_out, w_out, deg_out, stream);
  }
  if (kde_mode == STAG_SIMGRAPH_LSH) {
    stag_lsh_index* idx = nullptr;
    STAG_TRY(stag_lsh_index_create(X, n, d, a, eps, lsh, &idx, stream));
    const stag_status st = lsh_sample_edges(idx, s, seed, src_out, dst_out, w_out, deg_out, stream);
    (void)hipStreamSynchronize(stream);
    stag_lsh_index_destroy(idx);
    return st;
  }
  return fail(STAG_E_INVAL, "stag_simgraph_sample: unknown kde_mode %d", kde_mode);
}
