// Exact kernel density on the gfx950 matrix cores: operand preparation, the
// cross-chunk reduction and the C ABI entry points.  The tiles themselves are
// in kde_tiles.h.
//
// S(q) = sum_i k(||q - x_i||)   (Sec. "Kernel Density Estimation": the density
// K(q) = S(q)/n; ExactGaussianKDE evaluates it naively in O(dmn)); k is the
// Gaussian exp(-a r^2), the exponential exp(-a r) or the logistic
// 4/(2 + e^{ar} + e^{-ar}) kernel.
//
// The squared distance is expanded, ||q-x||^2 = ||q||^2 + ||x||^2 - 2 q.x,
// and scaled into a base-2 exponent
//     E = -lambda ||q-x||^2 = alpha_q + beta_x + (s q).x,
// alpha = -lambda ||q||^2, beta = -lambda ||x||^2, s = 2 lambda, with
// lambda = a log2(e) for the Gaussian kernel and (a log2(e))^2 for the other
// two.  The matrix cores produce the cross term from the (split) operands on
// top of alpha + beta; the epilogue maps E to the kernel value and sums.
//
// Pipeline of one call:
//   prep_rows  (data)    fp64 norms, beta, operand copy/split, padding rows
//   prep_rows  (queries) fp64 norms, alpha, scaled operand copy/split
//   tile_*               grid = (query tile of 128) x (data chunk of 4096 rows);
//                        4 waves, each owns 32 queries held in registers as
//                        the B operand; 32-row data tiles are streamed
//                        through double-buffered LDS as the A operand; per
//                        tile each lane adds its 16 kernel values in fp32 and
//                        flushes them into an fp64 accumulator.
//   reduce               S(q) = sum over chunks in chunk order (fp64), bound.
// The value of a query depends only on its own row, X and a: chunking and
// tiling are functions of n alone, so results are identical whatever m is and
// whatever other queries share a launch.
#include <cstring>
#include <mutex>

#include "runtime.h"
#include "kde_exact.h"
#include "kde_tiles.h"

// Scratch of stag_kde_exact_noalloc: one array per device (the runtime gives
// each device its own copy of a __device__ variable), kept until the process
// ends.  Host code never passes `scratch` itself to a kernel (on the host it
// names a stand-in, not device memory): the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current.
static constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace stag {
namespace {

using namespace tiles;

template <int FORM>
__device__ inline void split_value(float v, unsigned short* p) {
  if constexpr (FORM == STAG_FORM_FP16_SPLIT) {
    if (!(fabsf(v) < 65504.0f)) {  // out of fp16 range: poison the result
      p[0] = 0x7E00; p[1] = 0;
      return;
    }
    p[0] = f16_rne(v);
    p[1] = f16_rne(v - f16_to_f32(p[0]));
  } else if constexpr (FORM == STAG_FORM_BF16_SPLIT) {
    p[0] = bf16_rne(v);
    p[1] = bf16_rne(v - bf16_to_f32(p[0]));
  } else {  // three bf16 parts
    p[0] = bf16_rne(v);
    float r = v - bf16_to_f32(p[0]);
    p[1] = bf16_rne(r);
    p[2] = bf16_rne(r - bf16_to_f32(p[1]));
  }
}

// One wave per row, 16 rows per wave, 64 rows per block.  `scale` multiplies
// the operand (1 for data, 2a log2 e for queries); off = -a log2(e) ||row||^2
// in fp32; aug = bf16 three-way parts of off laid out for the augmentation
// step (data: [o1,o2,o3,1,1,1,0,0], queries: [1,1,1,o1,o2,o3,0,0]).  Rows >= n
// are padding.  The block's largest norm goes to max_nrm_bits with one atomic.
// With map, row r is src row map[r] (-1: padding), n unused.
constexpr int kPrepRowsPerWave = 16;
constexpr int kPrepRowsPerBlock = 4 * kPrepRowsPerWave;

template <int FORM>
__global__ __launch_bounds__(256) void prep_rows(const float* __restrict__ src, int64_t n, int d, int dp,
                                                 int64_t rows_pad, double scale, double neg_a_log2e,
                                                 int is_query, void* __restrict__ part0, void* __restrict__ part1,
                                                 void* __restrict__ part2, float* __restrict__ off,
                                                 u16x8* __restrict__ aug, double* __restrict__ nrm,
                                                 unsigned long long* __restrict__ max_nrm_bits,
                                                 const int* __restrict__ map) {
  __shared__ double wmax[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double mx = 0.0;
  for (int rr = 0; rr < kPrepRowsPerWave; ++rr) {
    const int64_t row = (int64_t)blockIdx.x * kPrepRowsPerBlock + wave * kPrepRowsPerWave + rr;
    if (row >= rows_pad) break;
    const int64_t srow = map ? (int64_t)map[row] : row;
    const bool real = map ? srow >= 0 : row < n;
    double sq = 0.0;
    for (int j = lane; j < dp; j += 64) {
      float v = 0.0f;
      if (real && j < d) v = src[srow * d + j];
      sq += (double)v * (double)v;
      const float w = (float)((double)v * scale);
      const int64_t o = row * dp + j;
      if constexpr (FORM == STAG_FORM_FP32) {
        static_cast<float*>(part0)[o] = w;
      } else {
        unsigned short p[3] = {0, 0, 0};
        split_value<FORM>(w, p);
        static_cast<unsigned short*>(part0)[o] = p[0];
        static_cast<unsigned short*>(part1)[o] = p[1];
        if constexpr (FORM == STAG_FORM_BF16_SPLIT3) static_cast<unsigned short*>(part2)[o] = p[2];
      }
    }
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
    if (real) mx = fmax(mx, sq);
    if (lane == 0) {
      const float ov = real ? (float)(neg_a_log2e * sq) : (is_query ? 0.0f : kPadOffset);
      off[row] = ov;
      if (aug) {
        unsigned short p[3];
        p[0] = bf16_rne(ov);
        const float r = ov - bf16_to_f32(p[0]);
        p[1] = bf16_rne(r);
        p[2] = bf16_rne(r - bf16_to_f32(p[1]));
        u16x8 v;
        if (is_query) v = u16x8{kBf16One, kBf16One, kBf16One, p[0], p[1], p[2], 0, 0};
        else v = u16x8{p[0], p[1], p[2], kBf16One, kBf16One, kBf16One, 0, 0};
        aug[row] = v;
      }
      if (real && nrm) nrm[row] = sq;
    }
  }
  if (max_nrm_bits) {
    if (lane == 0) wmax[wave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      const double b = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
      atomicMax(max_nrm_bits, (unsigned long long)__double_as_longlong(b));
    }
  }
}

// S(q) = sum of chunk partials in chunk order; optional 1/n; a-priori bound.
// With flag: a sum below kRescueBelow sets flag[q] and its 128-query tile's
// flag (both zeroed beforehand).
__global__ void reduce_partials(const double* __restrict__ partial, int P, int64_t m_pad, int64_t m, double scale,
                                const double* __restrict__ qnrm, const unsigned long long* __restrict__ max_xnrm_bits,
                                BoundModel bm, const int* __restrict__ near_over, double* __restrict__ S_out,
                                double* __restrict__ bound_out, int* __restrict__ flag, int* __restrict__ qtile_flag) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const double s = chunk_sum(partial + q, P, m_pad);
  if (flag && s < kRescueBelow) {
    flag[q] = 1;
    qtile_flag[q / kBQ] = 1;
  }
  S_out[q] = s * scale;
  if (bound_out) {
    const double xm = __longlong_as_double((long long)*max_xnrm_bits);
    if (near_over && near_over[q]) bm.near_y2 = 0.0;  // near pairs left in the tile sums
    bound_out[q] = relative_bound(bm, qnrm[q], xm);
  }
}

// Centred fp32 data: S(q) = sum of chunk partials in chunk order; the
// bound is (sum of the chunks' bound numerators) / S, plus its square and
// c_tail (the numerators come from computed tile sums: first-order slack),
// and infinite for S = 0.  Flags as in reduce_partials.
__global__ void reduce_centred(const double* __restrict__ partial, const double* __restrict__ bpart, int P,
                               int64_t m_pad, int64_t m, double scale, double c_tail, double* __restrict__ S_out,
                               double* __restrict__ bound_out, int* __restrict__ flag, int* __restrict__ qtile_flag) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const double s = chunk_sum(partial + q, P, m_pad);
  const double b = chunk_sum(bpart + q, P, m_pad);
  if (flag && s < kRescueBelow) {
    flag[q] = 1;
    qtile_flag[q / kBQ] = 1;
  }
  S_out[q] = s * scale;
  if (bound_out) {
    const double r = b / s;
    bound_out[q] = s > 0.0 ? r + r * r + c_tail : HUGE_VAL;
  }
}

// Adaptive form, per (sorted) query: the first pass's sum S1 over its P
// chunk partials, and the threshold T below which its chunks keep their
// first-pass values.  With budget = share * S1, T is the largest of the
// candidates 4^-j budget (j = 0 .. kBudgetSteps - 1) for which the chunk
// bound numerators below it add up to at most 0.999 budget (each candidate's
// sum kept in a register, in units of the budget); the chunks left to the
// first pass then carry at most share * S1 of bound numerator between them,
// and the recomputed ones are those with the largest numerators.  T = 0 where
// the budget is 0 (S1 = 0) or outside the range its reciprocal needs, on the
// rows past m and outside qmask (where S1 is not needed and not written).
constexpr int kBudgetSteps = 16;
__global__ void adaptive_budget(const double* __restrict__ partial, const double* __restrict__ bpart, int P,
                                int64_t m_pad, int64_t m, double share, const int* __restrict__ qmask,
                                double* __restrict__ S1, double* __restrict__ T) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m_pad) return;
  if (q >= m || (qmask && qmask[q / kBQ] == 0)) {
    T[q] = 0.0;
    return;
  }
  const double s = chunk_sum(partial + q, P, m_pad);
  S1[q] = s;
  const double budget = share * s;
  const double inv = 1.0 / budget;
  if (!(budget > 0.0) || !(inv < HUGE_VAL)) {
    T[q] = 0.0;
    return;
  }
  float acc[kBudgetSteps];
#pragma unroll
  for (int j = 0; j < kBudgetSteps; ++j) acc[j] = 0.0f;
  auto count = [&](double v) {
    if (!(v < budget)) return;  // recomputed whatever the others hold (NaN as well)
    const float r = (float)(v * inv);
    // every chunk with v < 4^-j budget is counted under candidate j (the
    // margin covers the roundings of r)
    float c = 1.000001f;
#pragma unroll
    for (int j = 0; j < kBudgetSteps; ++j) {
      acc[j] += r <= c ? r : 0.0f;
      c *= 0.25f;
    }
  };
  int p = 0;
  for (; p + 8 <= P; p += 8) {  // loads eight at a time, counted in order
    double v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = bpart[(int64_t)(p + i) * m_pad + q];
#pragma unroll
    for (int i = 0; i < 8; ++i) count(v[i]);
  }
  for (; p < P; ++p) count(bpart[(int64_t)p * m_pad + q]);
  double t = 0.0, c = 1.0;
#pragma unroll
  for (int j = 0; j < kBudgetSteps; ++j) {
    if (t == 0.0 && acc[j] <= 0.999f) t = c;
    c *= 0.25;
  }
  T[q] = t * budget;
}

// Adaptive form: a (chunk, 256-query tile) pair is recomputed in the split
// form when some query's bound numerator v of that chunk from the single-
// product pass is positive and not below the query's threshold T (cflag
// starts at zero; every writer stores 1).  Grid: (query blocks, chunks).
__global__ void adaptive_flags(const double* __restrict__ bpart, const double* __restrict__ T, int64_t m_pad,
                               int64_t m, int n_qt256, const int* __restrict__ qmask, uint8_t* __restrict__ cflag) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (q >= m || (qmask && qmask[q / kBQ] == 0)) return;
  const double v = bpart[c * m_pad + q];
  if (v > 0.0 && !(v < T[q])) cflag[c * n_qt256 + q / 256] = 1;
}

// Adaptive form, the estimate: every stride-th 128-query tile is sampled.
__global__ void mark_sample(int* __restrict__ qsample, int n_qt128, int stride) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_qt128) qsample[t] = t % stride == 0 ? 1 : 0;
}

// counts[0] += selected and counts[1] += all (chunk, 256-query tile) pairs
// of the tiles that hold a sampled 128-query tile.  Grid: (tiles, chunks).
__global__ void count_selected(const uint8_t* __restrict__ cflag, int n_qt256, const int* __restrict__ qsample,
                               int n_qt128, unsigned int* __restrict__ counts) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (t >= n_qt256) return;
  const bool sampled = qsample[2 * t] != 0 || (2 * t + 1 < n_qt128 && qsample[2 * t + 1] != 0);
  if (!sampled) return;
  atomicAdd(counts, cflag[c * n_qt256 + t] ? 1u : 0u);
  atomicAdd(counts + 1, 1u);
}

__global__ void fill_ones(uint8_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 1;
}

// Adaptive form: S(q) = sum of the chunk partials in chunk order (first
// pass, or the split form where the chunk was recomputed); the bound's
// numerator adds the first pass's bound numerator of a kept chunk and
// partial x the split form's a-priori relative bound of a recomputed one;
// bound = r + r^2 + c_tail with r = numerator / S.  Results in sorted order;
// rescue flags as in reduce_partials.
__global__ void reduce_adaptive(const double* __restrict__ partial, const double* __restrict__ bpart,
                                const uint8_t* __restrict__ cflag, int P, int64_t m_pad, int64_t m, int n_qt256,
                                double scale, const double* __restrict__ qnrm,
                                const unsigned long long* __restrict__ max_xnrm_bits, BoundModel bm, double c_tail,
                                double* __restrict__ S_s, double* __restrict__ B_s, int* __restrict__ flag,
                                int* __restrict__ qtile_flag) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const double xm = __longlong_as_double((long long)*max_xnrm_bits);
  const double rs = relative_bound(bm, qnrm[q], xm);
  double s = 0.0, b = 0.0;
  auto add = [&](double v, uint8_t f, double w) {
    s += v;
    b += f ? v * rs : w;
  };
  const int64_t t = q / 256;
  int p = 0;
  for (; p + 8 <= P; p += 8) {  // loads eight at a time, added in order
    double v[8], w[8];
    uint8_t f[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      v[i] = partial[(int64_t)(p + i) * m_pad + q];
      w[i] = bpart[(int64_t)(p + i) * m_pad + q];
      f[i] = cflag[(int64_t)(p + i) * n_qt256 + t];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) add(v[i], f[i], w[i]);
  }
  for (; p < P; ++p)
    add(partial[(int64_t)p * m_pad + q], cflag[(int64_t)p * n_qt256 + t], bpart[(int64_t)p * m_pad + q]);
  if (s < kRescueBelow) {
    flag[q] = 1;
    qtile_flag[q / kBQ] = 1;
  }
  S_s[q] = s * scale;
  const double r = b / s;
  B_s[q] = s > 0.0 ? r + r * r + c_tail : HUGE_VAL;
}

// Sorted results back to the queries' rows.
__global__ void scatter_results(const double* __restrict__ S_s, const double* __restrict__ B_s,
                                const int* __restrict__ perm, int64_t m_pad, double* __restrict__ S_out,
                                double* __restrict__ bound_out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m_pad) return;
  const int i = perm[q];
  if (i < 0) return;
  S_out[i] = S_s[q];
  if (bound_out) bound_out[i] = B_s[q];
}

template <int FORM>
stag_status launch_prep(const float* src, int64_t n, int d, int dp, int64_t rows_pad, double scale, double neg_a_l2e,
                        int is_query, void* const* parts, float* off, u16x8* aug, double* nrm,
                        unsigned long long* maxbits, hipStream_t st, const int* map) {
  ScopedTimer tm("kde_prep", st);
  hipLaunchKernelGGL(prep_rows<FORM>, dim3((unsigned)ceil_div(rows_pad, kPrepRowsPerBlock)), dim3(256), 0, st, src,
                     n, d, dp, rows_pad, scale, neg_a_l2e, is_query, parts[0], parts[1], parts[2], off, aug, nrm,
                     maxbits, map);
  return check_launch("prep_rows");
}

stag_status prep_any(int form, const float* src, int64_t n, int d, int dp, int64_t rows_pad, double scale,
                     double neg_a_l2e, int is_query, void* const* parts, float* off, u16x8* aug, double* nrm,
                     unsigned long long* maxbits, hipStream_t st, const int* map = nullptr) {
  switch (form) {
    case STAG_FORM_FP32:
      return launch_prep<STAG_FORM_FP32>(src, n, d, dp, rows_pad, scale, neg_a_l2e, is_query, parts, off, aug, nrm,
                                         maxbits, st, map);
    case STAG_FORM_BF16_SPLIT:
      return launch_prep<STAG_FORM_BF16_SPLIT>(src, n, d, dp, rows_pad, scale, neg_a_l2e, is_query, parts, off, aug,
                                               nrm, maxbits, st, map);
    case STAG_FORM_FP16_SPLIT:
      return launch_prep<STAG_FORM_FP16_SPLIT>(src, n, d, dp, rows_pad, scale, neg_a_l2e, is_query, parts, off, aug,
                                               nrm, maxbits, st, map);
    default:
      return launch_prep<STAG_FORM_BF16_SPLIT3>(src, n, d, dp, rows_pad, scale, neg_a_l2e, is_query, parts, off, aug,
                                                nrm, maxbits, st, map);
  }
}

// Statistics of an input for the form choice and the finiteness check: the
// largest squared row norm (fp64 bits), the largest |element| (fp32 bits) and
// whether any element is not finite.  One wave per row, 16 rows per wave.
__global__ __launch_bounds__(256) void scan_rows(const float* __restrict__ src, int64_t rows, int d,
                                                 unsigned long long* __restrict__ max_nrm_bits,
                                                 unsigned int* __restrict__ max_abs_bits, int* __restrict__ bad) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double mx = 0.0;
  float amax = 0.0f;
  int nonfinite = 0;
  for (int rr = 0; rr < kPrepRowsPerWave; ++rr) {
    const int64_t row = (int64_t)blockIdx.x * kPrepRowsPerBlock + wave * kPrepRowsPerWave + rr;
    if (row >= rows) break;
    double sq = 0.0;
    for (int j = lane; j < d; j += 64) {
      const float v = src[row * d + j];
      if (!(fabsf(v) <= 3.402823466e38f)) nonfinite = 1;
      else amax = fmaxf(amax, fabsf(v));
      sq += (double)v * (double)v;
    }
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
    if (sq == sq) mx = fmax(mx, sq);
  }
  for (int o = 32; o > 0; o >>= 1) {
    amax = fmaxf(amax, __shfl_xor(amax, o));
    nonfinite |= __shfl_xor(nonfinite, o);
  }
  if (lane == 0) {
    if (mx > 0.0) atomicMax(max_nrm_bits, (unsigned long long)__double_as_longlong(mx));
    if (amax > 0.0f) atomicMax(max_abs_bits, __float_as_uint(amax));
    if (nonfinite) atomicOr(bad, 1);
  }
}

}  // namespace

int exact_padded_dim(int d) {
  static const int dims[] = {16, 32, 64, 96, 128, 160, 192, 224, 256};
  for (int v : dims)
    if (d <= v) return v;
  if (d <= kWideMaxDim) return (int)round_up(d, 64);
  return 0;
}

size_t form_element_bytes(int form) { return form == STAG_FORM_FP32 ? 4 : 2; }
int form_parts(int form) {
  return form == STAG_FORM_FP32 ? 1 : (form == STAG_FORM_BF16_SPLIT3 ? 3 : 2);
}

stag_status alloc_operands(int form, int64_t rows, int d, bool is_query, Workspace& ws, Operands* out) {
  const int dp = exact_padded_dim(d);
  const int64_t rows_pad = round_up(rows, is_query ? kBQ : kTileRows);
  out->form = form;
  out->rows = rows;
  out->rows_pad = rows_pad;
  out->d = d;
  out->dp = dp;
  for (int p = 0; p < 3; ++p) out->part[p] = nullptr;
  for (int p = 0; p < form_parts(form); ++p)
    STAG_TRY(ws.alloc_bytes(&out->part[p], (size_t)rows_pad * dp * form_element_bytes(form)));
  STAG_TRY(ws.alloc(&out->off, (size_t)rows_pad));
  out->aug = nullptr;  // the tiles take the offsets directly
  STAG_TRY(ws.alloc(&out->nrm, (size_t)rows));
  out->max_nrm_bits = nullptr;
  if (!is_query) STAG_TRY(ws.alloc(&out->max_nrm_bits, 1));
  return STAG_OK;
}

stag_status prep_operands(const float* src, double a, bool is_query, const Operands& o, hipStream_t st) {
  if (o.max_nrm_bits) STAG_TRY(zero_async(o.max_nrm_bits, sizeof(unsigned long long), st));
  const double scale = is_query ? 2.0 * a * kLog2e : 1.0;
  return prep_any(o.form, src, o.rows, o.d, o.dp, o.rows_pad, scale, -a * kLog2e, is_query ? 1 : 0, o.part, o.off,
                  static_cast<u16x8*>(o.aug), o.nrm, o.max_nrm_bits, st);
}

stag_status prepare_operands(int form, const float* src, int64_t rows, int d, double a, bool is_query,
                             Workspace& ws, Operands* out, hipStream_t st) {
  STAG_TRY(alloc_operands(form, rows, d, is_query, ws, out));
  return prep_operands(src, a, is_query, *out, st);
}

int64_t exact_chunks(int64_t n_pad) { return ceil_div(n_pad, kChunkRows); }

stag_status prep_query_into(int form, const float* src, int64_t rows, int d, double a, const Operands& batch,
                            int64_t row0, hipStream_t st, bool centred) {
  const int dp = batch.dp;
  const int64_t rows_pad = round_up(rows, kBQ);
  const size_t eb = form_element_bytes(form);
  void* parts[3] = {nullptr, nullptr, nullptr};
  for (int p = 0; p < form_parts(form); ++p)
    parts[p] = static_cast<char*>(batch.part[p]) + (size_t)row0 * dp * eb;
  u16x8* aug = batch.aug ? static_cast<u16x8*>(batch.aug) + row0 : nullptr;
  // queries of centred data are kept unscaled with offset 0 (the tile adds
  // -a log2(e) ||q - c_T||^2 itself)
  return prep_any(form, src, rows, d, dp, rows_pad, centred ? 1.0 : 2.0 * a * kLog2e, centred ? 0.0 : -a * kLog2e, 1,
                  parts, batch.off + row0, aug, batch.nrm ? batch.nrm + row0 : nullptr, nullptr, st);
}

stag_status row_stats_async(const float* A, int64_t rows, int d, unsigned long long* nrm_bits, unsigned int* abs_bits,
                            int* bad, hipStream_t st) {
  STAG_TRY(zero_async(nrm_bits, sizeof(unsigned long long), st));
  STAG_TRY(zero_async(abs_bits, sizeof(unsigned int), st));
  STAG_TRY(zero_async(bad, sizeof(int), st));
  hipLaunchKernelGGL(scan_rows, dim3((unsigned)ceil_div(rows, kPrepRowsPerBlock)), dim3(256), 0, st, A, rows, d,
                     nrm_bits, abs_bits, bad);
  return check_launch("scan_rows");
}

int choose_resident_form(uint32_t resident, int d, double a, double eps, double max_nrm_q, double max_nrm_x,
                         float max_abs_q, float max_abs_x) {
  const double qscale = 2.0 * a * kLog2e;
  const bool fp16_ok = (double)max_abs_x < 65504.0 && (double)max_abs_q * qscale < 65504.0;
  const int order[3] = {STAG_FORM_FP16_SPLIT, STAG_FORM_BF16_SPLIT, STAG_FORM_BF16_SPLIT3};
  int best = -1;
  double best_b = HUGE_VAL;
  for (int f : order) {
    if (!(resident & (1u << f)) || d > 256 || (f == STAG_FORM_FP16_SPLIT && !fp16_ok)) continue;
    const double b = relative_bound(make_bound_model(f, d, a, STAG_KERNEL_GAUSSIAN), max_nrm_q, max_nrm_x);
    if (b <= eps) return f;
    if (b < best_b) {
      best_b = b;
      best = f;
    }
  }
  if (resident & (1u << STAG_FORM_FP32)) return STAG_FORM_FP32;
  return best;
}

int64_t query_tile_rows() { return kBQ; }

stag_status launch_exact_tiles(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                               hipStream_t st) {
  if (ex.kernel != STAG_KERNEL_GAUSSIAN && (ex.self || ex.tp))
    return fail(STAG_E_UNSUPPORTED, "tile extras need the Gaussian kernel");
  switch (tiles::tile_mode(ex)) {
    case tiles::kModeMax: return launch_tiles_max(xo, qo, partial, ex, st);
    case tiles::kModeGaussRescue: return launch_tiles_gauss_rescue(xo, qo, partial, ex, st);
    case tiles::kModeGaussExtraRescue: return launch_tiles_gauss_extra_rescue(xo, qo, partial, ex, st);
    case tiles::kModeExpShift: return launch_tiles_exp_shift(xo, qo, partial, ex, st);
    case tiles::kModeLogShift: return launch_tiles_log_shift(xo, qo, partial, ex, st);
    case tiles::kModeGauss: return launch_tiles_gauss(xo, qo, partial, ex, st);
    case tiles::kModeGaussExtra: return launch_tiles_gauss_extra(xo, qo, partial, ex, st);
    case tiles::kModeExponential: return launch_tiles_exponential(xo, qo, partial, ex, st);
    default: return launch_tiles_logistic(xo, qo, partial, ex, st);
  }
}

stag_status launch_reduce(const double* partial, int P, const Operands& qo, const Operands& xo, double scale,
                          const BoundModel& bm, double* S_out, double* bound_out, hipStream_t st,
                          const int* near_over, int* flag, int* qtile_flag) {
  const int64_t m = qo.rows;
  ScopedTimer tm("kde_reduce", st);
  hipLaunchKernelGGL(reduce_partials, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, partial, P, qo.rows_pad, m,
                     scale, qo.nrm, xo.max_nrm_bits, bm, near_over, S_out, bound_out, flag, qtile_flag);
  return check_launch("reduce_partials");
}

double kernel_tile_a(int kernel, double a) { return kernel == STAG_KERNEL_GAUSSIAN ? a : a * a * kLog2e; }

BoundModel make_bound_model(int form, int d, double a_tile, int kernel) {
  BoundModel bm;
  const double u = 0x1.0p-24;
  bm.la = a_tile * kLog2e;
  bm.kern = kernel;
  // fp32 accumulation of the d cross products and the six offset parts,
  // probabilistic model with lambda = 6 (Higham & Mary 2019)
  bm.c_acc = 6.0 * std::sqrt((double)d + 6.0) * u;
  double c_split;
  switch (form) {
    case STAG_FORM_FP32: c_split = u; break;                          // rounding of s*q to fp32
    case STAG_FORM_FP16_SPLIT: c_split = 3.0 * 0x1.0p-22 + u; break;  // dropped lo*lo, part rounding
    case STAG_FORM_BF16_SPLIT: c_split = 3.0 * 0x1.0p-16 + u; break;
    default: c_split = 4.0 * 0x1.0p-24 + u; break;
  }
  bm.c_split = c_split;
  bm.c_off = 3.0 * u;                   // alpha, beta rounded to fp32
  bm.c_tail = 0x1.0p-22 + 16.0 * u;     // exp2 and the 16-term fp32 tile sums
  // centred fp32 tile (per term, times M_T): the MFMA accumulation and the
  // fp32 sum of the d squared differences (c_acc each), the roundings of
  // q - c, its scaling and x - c in the cross term (3u), beta, the final
  // exponent add and the offset (3u), with 2u to spare
  bm.c_cent = 2.0 * bm.c_acc + 8.0 * u;
  if (kernel == STAG_KERNEL_EXPONENTIAL) bm.near_y2 = kNearY2;
  return bm;
}

}  // namespace stag

namespace stag {

namespace {

// Underflow rescue of the Gaussian exact sum.  For a flagged query (sum
// below kRescueBelow), m_q = the largest exponent E over the data (max pass
// of the tiles); its offset becomes fl32(-a log2(e) ||q||^2 - m_q) (one
// rounding from binary64), so that its largest term is about 2^0, and the
// tiles run again on the flagged query tiles; S = (sum) 2^{m_q}.
__global__ void rescue_shift(const double* __restrict__ pmax, int P, int64_t m_pad, int64_t m,
                             const int* __restrict__ flag, const double* __restrict__ qnrm, double neg_a_l2e,
                             const float* __restrict__ off, float* __restrict__ off2, double* __restrict__ shift) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m_pad) return;
  double mq = 0.0;
  float o = off[q];
  if (q < m && flag[q]) {
    mq = -HUGE_VAL;
    for (int p = 0; p < P; ++p) mq = fmax(mq, pmax[(int64_t)p * m_pad + q]);
    o = (float)(neg_a_l2e * qnrm[q] - mq);
  }
  off2[q] = o;
  shift[q] = mq;
}

__global__ void rescue_reduce(const double* __restrict__ partial, int P, int64_t m_pad, int64_t m,
                              const int* __restrict__ flag, const double* __restrict__ shift, double scale,
                              const double* __restrict__ qnrm, const unsigned long long* __restrict__ max_xnrm_bits,
                              BoundModel bm, double* __restrict__ S_out, double* __restrict__ bound_out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m || !flag[q]) return;
  const double s = chunk_sum(partial + q, P, m_pad);
  S_out[q] = s * exp2(shift[q]) * scale;
  if (bound_out) {
    const double xm = __longlong_as_double((long long)*max_xnrm_bits);
    bound_out[q] = relative_bound(bm, qnrm[q], xm, fabs(shift[q]));
  }
}

// Centred data: a flagged query's offset becomes fl32(-m_q) (the tile adds it
// to alpha'), others keep theirs (0).
__global__ void rescue_shift_centred(const double* __restrict__ pmax, int P, int64_t m_pad, int64_t m,
                                     const int* __restrict__ flag, const float* __restrict__ off,
                                     float* __restrict__ off2, double* __restrict__ shift) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m_pad) return;
  double mq = 0.0;
  float o = off[q];
  if (q < m && flag[q]) {
    mq = -HUGE_VAL;
    for (int p = 0; p < P; ++p) mq = fmax(mq, pmax[(int64_t)p * m_pad + q]);
    o = (float)(-mq);
  }
  off2[q] = o;
  shift[q] = mq;
}

__global__ void rescue_reduce_centred(const double* __restrict__ partial, const double* __restrict__ bpart, int P,
                                      int64_t m_pad, int64_t m, const int* __restrict__ flag,
                                      const double* __restrict__ shift, double scale, double c_tail,
                                      double* __restrict__ S_out, double* __restrict__ bound_out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m || !flag[q]) return;
  double s = 0.0, b = 0.0;
  for (int p = 0; p < P; ++p) {
    s += partial[(int64_t)p * m_pad + q];
    b += bpart[(int64_t)p * m_pad + q];
  }
  S_out[q] = s * exp2(shift[q]) * scale;
  if (bound_out) {
    const double r = b / s;
    bound_out[q] = s > 0.0 ? r + r * r + c_tail : HUGE_VAL;
  }
}

stag_status rescue_underflow(const Operands& xo, const Operands& qo, int P, double a_tile, double scale,
                             const BoundModel& bm, const RescueBuffers& rb, double* S_out, double* bound_out,
                             hipStream_t st) {
  const int64_t m_pad = qo.rows_pad, m = qo.rows;
  STAG_TRY(rescue_offsets_into(xo, qo, P, a_tile, 0, rb.flag, rb.qflag, rb.pmax, rb.off2, rb.shift, st));
  Operands q2 = qo;
  q2.off = rb.off2;
  TileExtra exs;
  exs.qtile_active = rb.qflag;
  STAG_TRY(launch_exact_tiles(xo, q2, rb.p2, exs, st));
  hipLaunchKernelGGL(rescue_reduce, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, rb.p2, P, m_pad, m, rb.flag,
                     rb.shift, scale, qo.nrm, xo.max_nrm_bits, bm, S_out, bound_out);
  return check_launch("rescue_reduce");
}

// Exponential and logistic kernels: ys = sqrt(-max E) of each flagged
// query (its smallest y), 0 otherwise.
__global__ void rescue_yshift(const double* __restrict__ pmax, int P, int64_t m_pad, int64_t m,
                              const int* __restrict__ flag, float* __restrict__ yshift) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m_pad) return;
  float ys = 0.0f;
  if (q < m && flag[q]) {
    double mq = -HUGE_VAL;
    for (int p = 0; p < P; ++p) mq = fmax(mq, pmax[(int64_t)p * m_pad + q]);
    ys = (float)sqrt(fmax(-mq, 0.0));
  }
  yshift[q] = ys;
}

__global__ void rescue_reduce_y(const double* __restrict__ partial, int P, int64_t m_pad, int64_t m,
                                const int* __restrict__ flag, const float* __restrict__ yshift, double scale,
                                const double* __restrict__ qnrm, const unsigned long long* __restrict__ max_xnrm_bits,
                                BoundModel bm, double* __restrict__ S_out, double* __restrict__ bound_out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m || !flag[q]) return;
  const double s = chunk_sum(partial + q, P, m_pad);
  const double ys = (double)yshift[q];
  S_out[q] = s * exp2(-ys) * scale;
  if (bound_out) {
    const double xm = __longlong_as_double((long long)*max_xnrm_bits);
    bound_out[q] = relative_bound(bm, qnrm[q], xm, ys);
  }
}

}  // namespace

stag_status rescue_offsets_into(const Operands& xo, const Operands& qo, int P, double a_tile, int self,
                                const int* flag, const int* qtile_flag, double* pmax, float* off2, double* shift,
                                hipStream_t st) {
  const int64_t m_pad = qo.rows_pad, m = qo.rows;
  TileExtra exm;
  exm.max_pass = 1;
  exm.self = self;
  exm.qtile_active = qtile_flag;
  STAG_TRY(launch_exact_tiles(xo, qo, pmax, exm, st));
  hipLaunchKernelGGL(rescue_shift, dim3((unsigned)ceil_div(m_pad, 256)), dim3(256), 0, st, pmax, P, m_pad, m, flag,
                     qo.nrm, -a_tile * kLog2e, qo.off, off2, shift);
  return check_launch("rescue_shift");
}

stag_status rescue_offsets(const Operands& xo, const Operands& qo, int P, double a_tile, int self, const int* flag,
                           const int* qtile_flag, float* off2, double* shift, Workspace& ws, hipStream_t st) {
  double* pmax = nullptr;
  STAG_TRY(ws.alloc(&pmax, (size_t)P * qo.rows_pad));
  return rescue_offsets_into(xo, qo, P, a_tile, self, flag, qtile_flag, pmax, off2, shift, st);
}

stag_status alloc_rescue(int kernel, int P, const Operands& qo, Workspace& ws, RescueBuffers* rb) {
  const int64_t m = qo.rows, m_pad = qo.rows_pad;
  *rb = RescueBuffers();
  STAG_TRY(ws.alloc(&rb->flag, (size_t)m));
  STAG_TRY(ws.alloc(&rb->qflag, (size_t)(m_pad / kBQ)));
  STAG_TRY(ws.alloc(&rb->pmax, (size_t)P * m_pad));
  STAG_TRY(ws.alloc(&rb->p2, (size_t)P * m_pad));
  if (kernel == STAG_KERNEL_GAUSSIAN) {
    STAG_TRY(ws.alloc(&rb->shift, (size_t)m_pad));
    STAG_TRY(ws.alloc(&rb->off2, (size_t)m_pad));
  } else {
    STAG_TRY(ws.alloc(&rb->yshift, (size_t)m_pad));
  }
  return STAG_OK;
}

// launch_reduce for the exponential and logistic kernels with the underflow
// rescue: a flagged query's terms are recomputed as 2^{ys - y}, ys its
// smallest y (from the max pass), and S = (sum) 2^{-ys}.
stag_status reduce_with_rescue_y(const double* partial, int P, const Operands& qo, const Operands& xo, int kernel,
                                 double scale, const BoundModel& bm, const int* near_over, const RescueBuffers& rb,
                                 double* S_out, double* bound_out, hipStream_t st) {
  const int64_t m = qo.rows, m_pad = qo.rows_pad;
  STAG_TRY(zero_async(rb.flag, (size_t)m * sizeof(int), st));
  STAG_TRY(zero_async(rb.qflag, (size_t)(m_pad / kBQ) * sizeof(int), st));
  STAG_TRY(launch_reduce(partial, P, qo, xo, scale, bm, S_out, bound_out, st, near_over, rb.flag, rb.qflag));
  TileExtra exm;
  exm.max_pass = 1;
  exm.qtile_active = rb.qflag;
  STAG_TRY(launch_exact_tiles(xo, qo, rb.pmax, exm, st));
  hipLaunchKernelGGL(rescue_yshift, dim3((unsigned)ceil_div(m_pad, 256)), dim3(256), 0, st, rb.pmax, P, m_pad, m,
                     rb.flag, rb.yshift);
  STAG_TRY(check_launch("rescue_yshift"));
  TileExtra exs;
  exs.kernel = kernel;
  exs.qtile_active = rb.qflag;
  exs.yshift = rb.yshift;
  STAG_TRY(launch_exact_tiles(xo, qo, rb.p2, exs, st));
  hipLaunchKernelGGL(rescue_reduce_y, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, rb.p2, P, m_pad, m, rb.flag,
                     rb.yshift, scale, qo.nrm, xo.max_nrm_bits, bm, S_out, bound_out);
  return check_launch("rescue_reduce_y");
}

stag_status reduce_with_rescue_into(const double* partial, int P, const Operands& qo, const Operands& xo,
                                    double a_tile, double scale, const BoundModel& bm, const RescueBuffers& rb,
                                    double* S_out, double* bound_out, hipStream_t st) {
  STAG_TRY(zero_async(rb.flag, (size_t)qo.rows * sizeof(int), st));
  STAG_TRY(zero_async(rb.qflag, (size_t)(qo.rows_pad / kBQ) * sizeof(int), st));
  STAG_TRY(launch_reduce(partial, P, qo, xo, scale, bm, S_out, bound_out, st, nullptr, rb.flag, rb.qflag));
  return rescue_underflow(xo, qo, P, a_tile, scale, bm, rb, S_out, bound_out, st);
}

stag_status reduce_with_rescue(const double* partial, int P, const Operands& qo, const Operands& xo, double a_tile,
                               double scale, const BoundModel& bm, double* S_out, double* bound_out, Workspace& ws,
                               hipStream_t st) {
  RescueBuffers rb;
  STAG_TRY(alloc_rescue(STAG_KERNEL_GAUSSIAN, P, qo, ws, &rb));
  return reduce_with_rescue_into(partial, P, qo, xo, a_tile, scale, bm, rb, S_out, bound_out, st);
}

namespace {

struct InputStats {
  double max_nrm_x, max_nrm_q;
  float max_abs_x, max_abs_q;
  bool nonfinite;
};

stag_status input_stats(const float* X, int64_t n, const float* Q, int64_t m, int d, Workspace& ws,
                        InputStats* out, hipStream_t st) {
  unsigned long long* nb = nullptr;
  unsigned int* ab = nullptr;
  int* bad = nullptr;
  STAG_TRY(ws.alloc(&nb, 2));
  STAG_TRY(ws.alloc(&ab, 2));
  STAG_TRY(ws.alloc(&bad, 1));
  STAG_HIP(hipMemsetAsync(nb, 0, 2 * sizeof(unsigned long long), st));
  STAG_HIP(hipMemsetAsync(ab, 0, 2 * sizeof(unsigned int), st));
  STAG_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
  hipLaunchKernelGGL(scan_rows, dim3((unsigned)ceil_div(n, kPrepRowsPerBlock)), dim3(256), 0, st, X, n, d, nb, ab,
                     bad);
  STAG_TRY(check_launch("scan_rows"));
  hipLaunchKernelGGL(scan_rows, dim3((unsigned)ceil_div(m, kPrepRowsPerBlock)), dim3(256), 0, st, Q, m, d, nb + 1,
                     ab + 1, bad);
  STAG_TRY(check_launch("scan_rows"));
  unsigned long long hn[2];
  unsigned int ha[2];
  int hb = 0;
  STAG_HIP(hipMemcpyAsync(hn, nb, sizeof(hn), hipMemcpyDeviceToHost, st));
  STAG_HIP(hipMemcpyAsync(ha, ab, sizeof(ha), hipMemcpyDeviceToHost, st));
  STAG_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  STAG_HIP(hipStreamSynchronize(st));
  std::memcpy(&out->max_nrm_x, &hn[0], sizeof(double));
  std::memcpy(&out->max_nrm_q, &hn[1], sizeof(double));
  std::memcpy(&out->max_abs_x, &ha[0], sizeof(float));
  std::memcpy(&out->max_abs_q, &ha[1], sizeof(float));
  out->nonfinite = hb != 0;
  return STAG_OK;
}

// The cheapest form whose a-priori bound at the largest query norm is <= eps
// (the bound grows with ||q||), FP32 if none is.
int choose_form(int d, double a_tile, int kernel, double eps, const InputStats& is) {
  const double qscale = 2.0 * a_tile * kLog2e;  // the split query operand is q * qscale
  const bool fp16_ok = (double)is.max_abs_x < 65504.0 && (double)is.max_abs_q * qscale < 65504.0;
  const int order[3] = {STAG_FORM_FP16_SPLIT, STAG_FORM_BF16_SPLIT, STAG_FORM_BF16_SPLIT3};
  if (d <= 256)
    for (int f : order) {
      if (f == STAG_FORM_FP16_SPLIT && !fp16_ok) continue;
      if (relative_bound(make_bound_model(f, d, a_tile, kernel), is.max_nrm_q, is.max_nrm_x) <= eps) return f;
    }
  return STAG_FORM_FP32;
}

stag_status check_exact_args(const char* fn, const float* X, int64_t n, const float* Q, int64_t m, int32_t d,
                             int32_t kernel, double a, double eps, int32_t form, uint32_t flags, double* S_out) {
  if (!X || !Q || !S_out) return fail(STAG_E_INVAL, "%s: NULL pointer argument", fn);
  if (n < 1 || m < 1 || d < 1) return fail(STAG_E_INVAL, "%s: n, m, d must be >= 1", fn);
  if (!(a > 0.0) || !std::isfinite(a)) return fail(STAG_E_INVAL, "%s: a must be positive and finite", fn);
  if (kernel < STAG_KERNEL_GAUSSIAN || kernel > STAG_KERNEL_LOGISTIC)
    return fail(STAG_E_INVAL, "%s: unknown kernel %d", fn, kernel);
  if (form < STAG_FORM_FP32 || form > STAG_FORM_FP16_ADAPTIVE)
    return fail(STAG_E_INVAL, "%s: unknown form %d", fn, form);
  if ((form == STAG_FORM_FP16_CENTRED || form == STAG_FORM_FP16_ADAPTIVE) && kernel != STAG_KERNEL_GAUSSIAN)
    return fail(STAG_E_UNSUPPORTED, "%s: the fp16 centred forms compute Gaussian sums only", fn);
  if (form == STAG_FORM_AUTO && !(eps > 0.0))
    return fail(STAG_E_INVAL, "%s: STAG_FORM_AUTO needs a target eps > 0", fn);
  if (flags & ~(STAG_NORMALIZE | STAG_CHECK_FINITE)) return fail(STAG_E_INVAL, "%s: unknown flags 0x%x", fn, flags);
  if (d > 1024) return fail(STAG_E_UNSUPPORTED, "%s: d = %d > 1024 is not supported", fn, d);
  if (d > 256 && form != STAG_FORM_FP32 && form != STAG_FORM_AUTO && form != STAG_FORM_FP16_SPLIT &&
      form != STAG_FORM_BF16_SPLIT)
    return fail(STAG_E_UNSUPPORTED, "%s: d = %d > 256 is supported by the fp32, fp16 split and bf16 split forms only",
                fn, d);
  if ((double)n * d >= 2147483648.0 || (double)m * d >= 2147483648.0)
    return fail(STAG_E_INVAL, "%s: n*d and m*d must be < 2^31", fn);
  const double at = kernel_tile_a(kernel, a);
  if (!std::isfinite(at) || !(at > 0.0)) return fail(STAG_E_INVAL, "%s: a out of range for this kernel", fn);
  return STAG_OK;
}

// Every device buffer of one exact call, taken from one Workspace before
// any launch (so that a counting Workspace gives the call's exact need).
struct ExactBuffers {
  Operands xo, qo;
  int P = 0;
  double* partial = nullptr;
  int* near_over = nullptr;  // exponential kernel
  RescueBuffers rb;
  // centred data (fp32 or fp16 centred form, Gaussian kernel, d <= 256)
  bool centred = false;
  CentreTemp ct;
  double *bpart = nullptr, *bp2 = nullptr;
  // adaptive form: the split operands (data in the grouped order, queries
  // sorted), the query order, the first pass's sums, the chunk selection
  // and the sorted results
  bool adaptive = false;
  Operands xs, qsp;
  QuerySort qs;
  double *S1 = nullptr, *T = nullptr, *Ss = nullptr, *Bs = nullptr;
  uint8_t* cflag = nullptr;
  int* qsample = nullptr;
  unsigned int* counts = nullptr;
};

// The fp32 form of the Gaussian sum centres the data tile by tile (the wide
// tile of d > 256 does not); the fp16 centred form centres it group by group.
bool use_centred(int form, int kernel, int d) {
  return (form == STAG_FORM_FP32 || form == STAG_FORM_FP16_CENTRED) && kernel == STAG_KERNEL_GAUSSIAN &&
         exact_padded_dim(d) <= 256;
}

stag_status alloc_exact(int form, int kernel, int64_t n, int64_t m, int d, Workspace& ws, ExactBuffers* b) {
  if (form == STAG_FORM_FP16_ADAPTIVE) {
    b->centred = true;
    b->adaptive = true;
    STAG_TRY(alloc_centred_h_operands(n, d, ws, &b->xo));
    STAG_TRY(alloc_centre_temp(b->xo, ws, &b->ct));
    STAG_TRY(alloc_operands(STAG_FORM_FP32, m, d, true, ws, &b->qo));
    STAG_TRY(alloc_operands(STAG_FORM_FP16_SPLIT, b->xo.rows_pad, d, false, ws, &b->xs));
    STAG_TRY(alloc_operands(STAG_FORM_FP16_SPLIT, m, d, true, ws, &b->qsp));
    STAG_TRY(alloc_query_sort(m, b->qo.rows_pad, b->ct.K, ws, &b->qs));
    b->P = (int)exact_chunks(b->xo.rows_pad);
    const int64_t m_pad = b->qo.rows_pad;
    STAG_TRY(ws.alloc(&b->partial, (size_t)b->P * m_pad));
    STAG_TRY(ws.alloc(&b->bpart, (size_t)b->P * m_pad));
    STAG_TRY(ws.alloc(&b->S1, (size_t)m_pad));
    STAG_TRY(ws.alloc(&b->T, (size_t)m_pad));
    STAG_TRY(ws.alloc(&b->Ss, (size_t)m_pad));
    STAG_TRY(ws.alloc(&b->Bs, (size_t)m_pad));
    STAG_TRY(ws.alloc(&b->cflag, (size_t)b->P * ceil_div(m_pad, 256)));
    STAG_TRY(ws.alloc(&b->qsample, (size_t)(m_pad / kBQ)));
    STAG_TRY(ws.alloc(&b->counts, 2));
    return alloc_rescue(kernel, b->P, b->qsp, ws, &b->rb);
  }
  if (use_centred(form, kernel, d)) {
    b->centred = true;
    if (form == STAG_FORM_FP16_CENTRED)
      STAG_TRY(alloc_centred_h_operands(n, d, ws, &b->xo));
    else
      STAG_TRY(alloc_centred_operands(n, d, ws, &b->xo));
    STAG_TRY(alloc_centre_temp(b->xo, ws, &b->ct));
    STAG_TRY(alloc_operands(STAG_FORM_FP32, m, d, true, ws, &b->qo));
    b->P = (int)exact_chunks(b->xo.rows_pad);
    STAG_TRY(ws.alloc(&b->partial, (size_t)b->P * b->qo.rows_pad));
    STAG_TRY(ws.alloc(&b->bpart, (size_t)b->P * b->qo.rows_pad));
    STAG_TRY(ws.alloc(&b->bp2, (size_t)b->P * b->qo.rows_pad));
    return alloc_rescue(kernel, b->P, b->qo, ws, &b->rb);
  }
  STAG_TRY(alloc_operands(form, n, d, false, ws, &b->xo));
  STAG_TRY(alloc_operands(form, m, d, true, ws, &b->qo));
  b->P = (int)exact_chunks(b->xo.rows_pad);
  STAG_TRY(ws.alloc(&b->partial, (size_t)b->P * b->qo.rows_pad));
  if (kernel == STAG_KERNEL_EXPONENTIAL) STAG_TRY(ws.alloc(&b->near_over, (size_t)m));
  return alloc_rescue(kernel, b->P, b->qo, ws, &b->rb);
}

// Centred Gaussian sum (fp32, or the fp16 centred form): grouping and
// centring of X, the unscaled query copy, the centred tiles with their bound
// numerators, the reduction, and the underflow rescue (max pass, offsets
// -m_q, second pass) on the same tiles.
stag_status run_centred(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, double a, uint32_t flags,
                        double* S_out, double* bound_out, const ExactBuffers& b, hipStream_t st) {
  const Operands& xo = b.xo;
  const Operands& qo = b.qo;
  const RescueBuffers& rb = b.rb;
  if (xo.form == STAG_FORM_FP16_CENTRED)
    STAG_TRY(prep_centred_h_operands(X, a, xo, b.ct, st));
  else
    STAG_TRY(prep_centred_operands(X, a, xo, b.ct, st));
  STAG_TRY(prep_any(STAG_FORM_FP32, Q, m, d, qo.dp, qo.rows_pad, 1.0, 0.0, 1, qo.part, qo.off, nullptr, qo.nrm,
                    nullptr, st));
  const BoundModel bm = make_bound_model(STAG_FORM_FP32, d, a, STAG_KERNEL_GAUSSIAN);
  TileExtra ex;
  ex.a = a;
  ex.bpart = b.bpart;
  ex.c_cent = (float)bm.c_cent;
  STAG_TRY(launch_exact_tiles(xo, qo, b.partial, ex, st));
  const double scale = (flags & STAG_NORMALIZE) ? 1.0 / (double)n : 1.0;
  const int64_t m_pad = qo.rows_pad;
  STAG_TRY(zero_async(rb.flag, (size_t)m * sizeof(int), st));
  STAG_TRY(zero_async(rb.qflag, (size_t)(m_pad / kBQ) * sizeof(int), st));
  {
    ScopedTimer tm("kde_reduce", st);
    hipLaunchKernelGGL(reduce_centred, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, b.partial, b.bpart, b.P,
                       m_pad, m, scale, bm.c_tail, S_out, bound_out, rb.flag, rb.qflag);
    STAG_TRY(check_launch("reduce_centred"));
  }
  TileExtra exm;
  exm.max_pass = 1;
  exm.qtile_active = rb.qflag;
  exm.a = a;
  STAG_TRY(launch_exact_tiles(xo, qo, rb.pmax, exm, st));
  hipLaunchKernelGGL(rescue_shift_centred, dim3((unsigned)ceil_div(m_pad, 256)), dim3(256), 0, st, rb.pmax, b.P,
                     m_pad, m, rb.flag, qo.off, rb.off2, rb.shift);
  STAG_TRY(check_launch("rescue_shift_centred"));
  Operands q2 = qo;
  q2.off = rb.off2;
  TileExtra exs = ex;
  exs.qtile_active = rb.qflag;
  exs.bpart = b.bp2;
  STAG_TRY(launch_exact_tiles(xo, q2, rb.p2, exs, st));
  hipLaunchKernelGGL(rescue_reduce_centred, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, rb.p2, b.bp2, b.P,
                     m_pad, m, rb.flag, rb.shift, scale, bm.c_tail, S_out, bound_out);
  return check_launch("rescue_reduce_centred");
}

// Adaptive fp16 form: the single-product centred pass over all pairs with
// the queries in group order, then the fp16 split form over the (chunk,
// 256-query tile) pairs where some query's first-pass bound numerator lies
// above the part of its budget, kAdaptiveShare of its sum, that its smaller
// numerators fill (adaptive_budget), the reduction in sorted order with the
// underflow rescue in the split form, and the results back to the query rows.
// First an estimate: the single-product pass and the selection on every
// stride-th 128-query tile (about kAdaptiveSamples of them), read back with
// one synchronisation; when more than kAdaptiveMaxShare of the sampled pairs
// are selected (wide kernels: every chunk matters), the single-product pass
// is skipped and every pair runs in the split form.
constexpr double kAdaptiveShare = 1.0e-5;
constexpr int kAdaptiveSamples = 8;
constexpr double kAdaptiveMaxShare = 0.5;

stag_status run_adaptive(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, double a, uint32_t flags,
                         double* S_out, double* bound_out, const ExactBuffers& b, hipStream_t st) {
  const Operands& xo = b.xo;
  const Operands& qo = b.qo;
  const int64_t m_pad = qo.rows_pad;
  const int n_qt256 = (int)ceil_div(m_pad, 256);
  STAG_TRY(prep_centred_h_operands(X, a, xo, b.ct, st));
  STAG_TRY(sort_queries(Q, m, m_pad, d, xo.dp, b.ct, b.qs, st));
  STAG_TRY(prep_any(STAG_FORM_FP32, Q, m, d, qo.dp, m_pad, 1.0, 0.0, 1, qo.part, qo.off, nullptr, qo.nrm, nullptr,
                    st, b.qs.perm));
  STAG_TRY(zero_async(b.xs.max_nrm_bits, sizeof(unsigned long long), st));
  STAG_TRY(prep_any(STAG_FORM_FP16_SPLIT, X, b.xs.rows, d, b.xs.dp, b.xs.rows_pad, 1.0, -a * kLog2e, 0, b.xs.part,
                    b.xs.off, nullptr, b.xs.nrm, b.xs.max_nrm_bits, st, b.ct.map));
  STAG_TRY(prep_any(STAG_FORM_FP16_SPLIT, Q, m, d, b.qsp.dp, b.qsp.rows_pad, 2.0 * a * kLog2e, -a * kLog2e, 1,
                    b.qsp.part, b.qsp.off, nullptr, b.qsp.nrm, nullptr, st, b.qs.perm));
  // first pass: one fp16 product per pair, with the bound numerators, then
  // the selection of the pairs to recompute (on the sampled tiles: qmask)
  const BoundModel bm1 = make_bound_model(STAG_FORM_FP32, d, a, STAG_KERNEL_GAUSSIAN);
  TileExtra ex1;
  ex1.a = a;
  ex1.bpart = b.bpart;
  ex1.c_cent = (float)bm1.c_cent;
  const int n_qt128 = (int)(m_pad / kBQ);
  const int stride = std::max(1, n_qt128 / kAdaptiveSamples);
  auto first_pass = [&](const int* qmask) -> stag_status {
    TileExtra e = ex1;
    e.qtile_active = qmask;
    e.sample = qmask ? 1 : 0;
    e.fold_alpha = 1;
    if (qmask && ceil_div(n_qt128, stride) <= TileExtra::kMaxSel) {
      // the sampled tiles (those mark_sample flags), launched alone
      for (int t = 0; t < n_qt128; t += stride) e.qsel[e.qsel_n++] = t;
    }
    STAG_TRY(launch_exact_tiles(xo, qo, b.partial, e, st));
    ScopedTimer tm("kde_adaptive_select", st);
    hipLaunchKernelGGL(adaptive_budget, dim3((unsigned)ceil_div(m_pad, 256)), dim3(256), 0, st, b.partial, b.bpart,
                       b.P, m_pad, m, kAdaptiveShare, qmask, b.S1, b.T);
    STAG_TRY(check_launch("adaptive_budget"));
    STAG_TRY(zero_async(b.cflag, (size_t)b.P * n_qt256, st));
    hipLaunchKernelGGL(adaptive_flags, dim3((unsigned)ceil_div(m, 256), (unsigned)b.P), dim3(256), 0, st, b.bpart,
                       b.T, m_pad, m, n_qt256, qmask, b.cflag);
    return check_launch("adaptive_flags");
  };
  hipLaunchKernelGGL(mark_sample, dim3((unsigned)ceil_div(n_qt128, 256)), dim3(256), 0, st, b.qsample, n_qt128,
                     stride);
  STAG_TRY(check_launch("mark_sample"));
  STAG_TRY(first_pass(stride > 1 ? b.qsample : nullptr));
  unsigned int hc[2] = {0u, 0u};
  {
    ScopedTimer tm("kde_adaptive_select", st);
    STAG_TRY(zero_async(b.counts, 2 * sizeof(unsigned int), st));
    hipLaunchKernelGGL(count_selected, dim3((unsigned)ceil_div(n_qt256, 256), (unsigned)b.P), dim3(256), 0, st,
                       b.cflag, n_qt256, b.qsample, n_qt128, b.counts);
    STAG_TRY(check_launch("count_selected"));
    STAG_HIP(hipMemcpyAsync(hc, b.counts, sizeof(hc), hipMemcpyDeviceToHost, st));
    STAG_HIP(hipStreamSynchronize(st));
  }
  if (hc[1] > 0 && (double)hc[0] > kAdaptiveMaxShare * (double)hc[1]) {
    // every pair in the split form (the partials of the sampled pass are overwritten)
    hipLaunchKernelGGL(fill_ones, dim3((unsigned)ceil_div((int64_t)b.P * n_qt256, 256)), dim3(256), 0, st, b.cflag,
                       (int64_t)b.P * n_qt256);
    STAG_TRY(check_launch("fill_ones"));
  } else if (stride > 1) {
    STAG_TRY(first_pass(nullptr));
  }
  // second pass: the split form on the selected pairs (overwrites their partials)
  TileExtra ex2;
  ex2.cflag = b.cflag;
  STAG_TRY(launch_exact_tiles(b.xs, b.qsp, b.partial, ex2, st));
  const BoundModel bm2 = make_bound_model(STAG_FORM_FP16_SPLIT, d, a, STAG_KERNEL_GAUSSIAN);
  const double scale = (flags & STAG_NORMALIZE) ? 1.0 / (double)n : 1.0;
  STAG_TRY(zero_async(b.rb.flag, (size_t)m * sizeof(int), st));
  STAG_TRY(zero_async(b.rb.qflag, (size_t)(m_pad / kBQ) * sizeof(int), st));
  {
    ScopedTimer tm("kde_reduce", st);
    hipLaunchKernelGGL(reduce_adaptive, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, b.partial, b.bpart,
                       b.cflag, b.P, m_pad, m, n_qt256, scale, b.qsp.nrm, b.xs.max_nrm_bits, bm2, bm1.c_tail, b.Ss,
                       b.Bs, b.rb.flag, b.rb.qflag);
    STAG_TRY(check_launch("reduce_adaptive"));
  }
  // queries whose sum lies below the fp32 terms' range: recomputed in the split form
  STAG_TRY(rescue_underflow(b.xs, b.qsp, b.P, a, scale, bm2, b.rb, b.Ss, b.Bs, st));
  hipLaunchKernelGGL(scatter_results, dim3((unsigned)ceil_div(m_pad, 256)), dim3(256), 0, st, b.Ss, b.Bs, b.qs.perm,
                     m_pad, S_out, bound_out);
  return check_launch("scatter_results");
}

// The launches of one exact call into buffers from alloc_exact.
stag_status run_exact(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, int32_t kernel, double a,
                      int32_t form, uint32_t flags, double* S_out, double* bound_out, const ExactBuffers& b,
                      hipStream_t stream) {
  if (b.adaptive) return run_adaptive(X, n, Q, m, d, a, flags, S_out, bound_out, b, stream);
  if (b.centred) return run_centred(X, n, Q, m, d, a, flags, S_out, bound_out, b, stream);
  const double at = kernel_tile_a(kernel, a);
  STAG_TRY(prep_operands(X, at, false, b.xo, stream));
  STAG_TRY(prep_operands(Q, at, true, b.qo, stream));
  TileExtra ex;
  ex.kernel = kernel;
  if (kernel == STAG_KERNEL_EXPONENTIAL) {
    ex.near_x = X;
    ex.near_q = Q;
    ex.d = d;
    ex.near_e = (float)kNearY2;
    ex.a = a;
    ex.m_rows = m;
    ex.near_over = b.near_over;
    STAG_TRY(zero_async(ex.near_over, (size_t)m * sizeof(int), stream));
  }
  STAG_TRY(launch_exact_tiles(b.xo, b.qo, b.partial, ex, stream));
  const double scale = (flags & STAG_NORMALIZE) ? 1.0 / (double)n : 1.0;
  const BoundModel bm = make_bound_model(form, d, at, kernel);
  // Gaussian: sums below kRescueBelow are recomputed with shifted exponents
  if (kernel == STAG_KERNEL_GAUSSIAN)
    return reduce_with_rescue_into(b.partial, b.P, b.qo, b.xo, at, scale, bm, b.rb, S_out, bound_out, stream);
  return reduce_with_rescue_y(b.partial, b.P, b.qo, b.xo, kernel, scale, bm, ex.near_over, b.rb, S_out, bound_out,
                              stream);
}

stag_status exact_kernel_impl(const char* fn, const float* X, int64_t n, const float* Q, int64_t m, int32_t d,
                              int32_t kernel, double a, double eps, int32_t form, uint32_t flags, double* S_out,
                              double* bound_out, hipStream_t stream) {
  STAG_TRY(check_exact_args(fn, X, n, Q, m, d, kernel, a, eps, form, flags, S_out));
  clear_error();
  Workspace ws(stream);
  if (form == STAG_FORM_AUTO || (flags & STAG_CHECK_FINITE)) {
    InputStats is;
    STAG_TRY(input_stats(X, n, Q, m, d, ws, &is, stream));
    if ((flags & STAG_CHECK_FINITE) && is.nonfinite) return fail(STAG_E_INVAL, "%s: X or Q holds NaN or Inf", fn);
    if (form == STAG_FORM_AUTO) form = choose_form(d, kernel_tile_a(kernel, a), kernel, eps, is);
  }
  ExactBuffers b;
  STAG_TRY(alloc_exact(form, kernel, n, m, d, ws, &b));
  return run_exact(X, n, Q, m, d, kernel, a, form, flags, S_out, bound_out, b, stream);
}

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

stag_status scratch_on_current_device(void** out) {
  int dev = 0;
  STAG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(STAG_E_UNSUPPORTED, "device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    STAG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(STAG_E_DEVICE, "hipGetSymbolAddress gave a null scratch address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return STAG_OK;
}

}  // namespace
}  // namespace stag

extern "C" stag_status stag_kde_exact_noalloc(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, double a,
                                              int32_t form, uint32_t flags, double* S_out, double* bound_out,
                                              hipStream_t stream) {
  using namespace stag;
  const char* fn = "stag_kde_exact_noalloc";
  if (form == STAG_FORM_AUTO) return fail(STAG_E_UNSUPPORTED, "%s: STAG_FORM_AUTO is not available here", fn);
  if (flags & STAG_CHECK_FINITE) return fail(STAG_E_UNSUPPORTED, "%s: STAG_CHECK_FINITE is not available here", fn);
  STAG_TRY(check_exact_args(fn, X, n, Q, m, d, STAG_KERNEL_GAUSSIAN, a, 0.0, form, flags, S_out));
  ExactBuffers need;
  Workspace counter{Workspace::CountTag{}};
  STAG_TRY(alloc_exact(form, STAG_KERNEL_GAUSSIAN, n, m, d, counter, &need));
  if (counter.used() > kScratchBytes)
    return fail(STAG_E_INVAL, "%s: this call needs %zu bytes of scratch, more than the %zu available", fn,
                counter.used(), kScratchBytes);
  clear_error();
  void* base = nullptr;
  STAG_TRY(scratch_on_current_device(&base));
  Workspace arena(stream, base, kScratchBytes);
  ExactBuffers b;
  STAG_TRY(alloc_exact(form, STAG_KERNEL_GAUSSIAN, n, m, d, arena, &b));
  return run_exact(X, n, Q, m, d, STAG_KERNEL_GAUSSIAN, a, form, flags, S_out, bound_out, b, stream);
}

extern "C" stag_status stag_kde_exact(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, double a,
                                      double eps, int32_t form, uint32_t flags, double* S_out, double* bound_out,
                                      hipStream_t stream) {
  return stag::exact_kernel_impl("stag_kde_exact", X, n, Q, m, d, STAG_KERNEL_GAUSSIAN, a, eps, form, flags, S_out,
                                 bound_out, stream);
}

extern "C" stag_status stag_kde_exact_kernel(const float* X, int64_t n, const float* Q, int64_t m, int32_t d,
                                             int32_t kernel, double a, double eps, int32_t form, uint32_t flags,
                                             double* S_out, double* bound_out, hipStream_t stream) {
  return stag::exact_kernel_impl("stag_kde_exact_kernel", X, n, Q, m, d, kernel, a, eps, form, flags, S_out,
                                 bound_out, stream);
}
