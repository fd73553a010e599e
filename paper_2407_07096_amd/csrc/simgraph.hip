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
// ascending.
// LSH mode: the CKNS estimator's terms replace the kernel row (lsh.hip).
#include <cmath>

#include "kde_exact.h"
#include "lsh.h"
#include "runtime.h"

namespace stag {
namespace {

constexpr uint64_t kGammaS = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t kTagDrawS = 0x44524157ULL;
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

// One wave per draw (node i, draw r).
__global__ __launch_bounds__(256) void draw_exact(const float* __restrict__ X, int64_t n, int d, double a, int s,
                                                  uint64_t seed, int P, int64_t m_pad, int64_t ntile, int64_t tstride,
                                                  const double* __restrict__ chunk_t, const float* __restrict__ tp,
                                                  const double* __restrict__ rest,
                                                  const double* __restrict__ rest_draw,
                                                  const double* __restrict__ shift, int vec4,
                                                  int64_t* __restrict__ src, int64_t* __restrict__ dst,
                                                  double* __restrict__ w) {
  const int lane = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= n * s) return;
  const int64_t i = e / s;
  const int r = (int)(e % s);
  uint64_t ds = mixs(mixs(mixs(seed ^ kTagDrawS) ^ (uint64_t)i) ^ 0ULL);
  const double u = (double)(mixs(ds + (uint64_t)(r + 1) * kGammaS) >> 11) * 0x1.0p-53;
  // rest_draw: the total in the scale of the chunk and tile sums (2^{-m_i}
  // times the true one for a row of the underflow rescue, else the same)
  const double tot = rest_draw[i];
  const double sh = shift[i];  // 0 for rows without a shift
  int64_t pick = -1;
  if (rest[i] > 0.0 && tot > 0.0) {
    double resid = 0.0;
    const int c = invert_level(P, u * tot, [&](int k) { return chunk_t[i * P + k]; }, &resid);
    if (c >= 0) {
      const int64_t t0 = (int64_t)c * kChunkTiles;
      const int nt = (int)((ntile - t0) < kChunkTiles ? (ntile - t0) : kChunkTiles);
      double resid2 = 0.0;
      const int tl = invert_level(nt, resid, [&](int k) { return (double)tp[i * tstride + t0 + k]; }, &resid2);
      if (tl >= 0) {
        // rows of the tile: lanes l and l + 32 share row l % 32 and take
        // alternate 16-byte pieces (or alternate elements) of it
        const int64_t rb = (t0 + tl) * 32;
        const int half = lane >> 5;
        const int64_t j = rb + (lane & 31);
        const bool live = j < n && j != i;
        double D = 0.0;
        if (live) {
          const float* xi = X + i * d;
          const float* xj = X + j * d;
          if (vec4) {
            const float4* a4 = reinterpret_cast<const float4*>(xi);
            const float4* b4 = reinterpret_cast<const float4*>(xj);
            for (int k4 = half; k4 < (d >> 2); k4 += 2) {
              const float4 p = a4[k4], q = b4[k4];
              double t = (double)p.x - (double)q.x;
              D = __builtin_fma(t, t, D);
              t = (double)p.y - (double)q.y;
              D = __builtin_fma(t, t, D);
              t = (double)p.z - (double)q.z;
              D = __builtin_fma(t, t, D);
              t = (double)p.w - (double)q.w;
              D = __builtin_fma(t, t, D);
            }
          } else {
            for (int h = half; h < d; h += 2) {
              const double t = (double)xi[h] - (double)xj[h];
              D = __builtin_fma(t, t, D);
            }
          }
        }
        D += __shfl_xor(D, 32);
        // a shifted row's values are 2^{E - m_i} with E = -a log2(e) D in one
        // exponent (2^{-m_i} alone overflows for m_i < -1024, and exp(-a D)
        // is subnormal there)
        double kv = 0.0;
        if (lane < 32 && live) kv = sh == 0.0 ? exp(-a * D) : exp2(fma(-a * kLog2eS, D, -sh));
        double resid3 = 0.0;
        const int jl = invert_level(32, resid2, [&](int) { return kv; }, &resid3);  // lane k owns row k
        if (jl >= 0) pick = rb + jl;
      }
    }
  }
  if (lane == 0) {
    src[e] = i;
    dst[e] = pick;
    w[e] = pick >= 0 ? 1.0 / ((double)s * (1.0 / rest[i] + 1.0 / rest[pick])) : 0.0;
  }
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
  ScopedTimer tm("simgraph_draw_exact", st);
  hipLaunchKernelGGL(draw_exact, dim3((unsigned)ceil_div(n * s, 4)), dim3(256), 0, st, X, n, d, a, s, seed, P,
                     qo.rows_pad, ntile, tstride, chunk_t, tp, rest, rest_draw, shift, vec4, src, dst, w);
  return check_launch("draw_exact");
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
