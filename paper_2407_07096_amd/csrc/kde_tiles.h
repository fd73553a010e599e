// Matrix-core tiles of the exact kernel density (internal; included by the
// per-mode translation units kde_tiles_*.hip and, for the shared constants
// and conversions, by kde_exact.hip).  Each epilogue mode is instantiated in
// a translation unit of its own so that the four compile in parallel.
//
// A tile accumulates E = alpha_q + beta_x + (s q).x (base-2 exponent of the
// Gaussian, or -lambda D for the other kernels) for 32 data rows x 32 queries
// per wave; the epilogue turns the 16 values a lane holds into kernel values
// and an fp32 tree sum, flushed into a per-lane fp64 accumulator.
#pragma once

#include "runtime.h"
#include "kde_exact.h"

namespace stag {
namespace tiles {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
// Word 3 of a raw buffer resource on gfx9-family GPUs (gfx950 included):
// 32-bit data format, no swizzle; loads past num_records return 0.
constexpr int kBufferWord3 = 0x00020000;

constexpr double kLog2e = 1.4426950408889634074;
constexpr int kTileRows = 32;
constexpr int kWaves = 4;
constexpr int kBQ = 32 * kWaves;      // queries per workgroup
constexpr int kChunkRows = 4096;      // data rows per partial sum
constexpr float kPadOffset = -1.0e30f;  // exponent offset of padding rows: exp2 -> 0
constexpr unsigned short kBf16One = 0x3F80;
constexpr int kWideMaxDim = 1024;     // largest d of the wide fp32 tile

__device__ inline unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return (unsigned short)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }
__device__ inline unsigned short f16_rne(float f) { return __builtin_bit_cast(unsigned short, (_Float16)f); }
__device__ inline float f16_to_f32(unsigned short h) { return (float)__builtin_bit_cast(_Float16, h); }

// Epilogue modes of the tiles.  The accumulators hold E = -lambda D (base 2)
// with lambda = a log2(e) for the Gaussian kernel and (a log2(e))^2 for the
// other two, so that for those sqrt(-E) = a log2(e) r:
//   Gaussian       k = 2^E
//   exponential    k = 2^-y,             y = sqrt(max(-E, 0)) = a r log2(e)
//   logistic       k = 4t / (1 + t)^2,   t = 2^-y = e^{-a r}
// (4t/(1+t)^2 = 4/(2 + e^{ar} + e^{-ar})).  The clamp keeps a NaN exponent NaN.
// kModeGaussExtra is the Gaussian with the TileExtra outputs.
constexpr int kModeGauss = 0;
constexpr int kModeGaussExtra = 1;
constexpr int kModeExponential = 2;
constexpr int kModeLogistic = 3;
// kModeMax: no kernel values; each partial is the largest exponent E of its
// (chunk, query), the shift of the underflow rescue of the Gaussian sum.
constexpr int kModeMax = 4;
// kModeGaussRescue: the Gaussian sum of the rescue's second pass (the same
// arithmetic as kModeGauss, a kernel of its own so that traces and timers
// tell it apart from the tiles it repeats).
constexpr int kModeGaussRescue = 5;
// kModeGaussExtraRescue: kModeGaussExtra (diagonal drop, tile sums) in the
// rescue's second pass of the edge sampler's self pass, a kernel of its own.
constexpr int kModeGaussExtraRescue = 6;
// modes with the TileExtra outputs (self, tp), and modes that need the true
// row and column bases of a tile in the epilogue
template <int MODE>
constexpr bool kExtraMode = MODE == kModeGaussExtra || MODE == kModeGaussExtraRescue;
template <int MODE>
constexpr bool kBasedMode = kExtraMode<MODE> || MODE == kModeMax;
// kModeExpShift, kModeLogShift: the exponential and logistic kernels in the
// rescue's second pass, with each query's terms scaled by 2^{ys}, ys = the
// smallest y = sqrt(-E) of the query (TileExtra::yshift): the largest term
// becomes about 1 and the sum is multiplied by 2^{-ys} afterwards.
constexpr int kModeExpShift = 7;
constexpr int kModeLogShift = 8;
template <int MODE>
constexpr bool kShiftMode = MODE == kModeExpShift || MODE == kModeLogShift;

// Per-lane accumulation across tiles: fp64 sum, or the maximum in kModeMax.
template <int MODE>
__device__ inline double acc_init() {
  return MODE == kModeMax ? -HUGE_VAL : 0.0;
}
template <int MODE>
__device__ inline double acc_add(double acc, double v) {
  if constexpr (MODE == kModeMax) return fmax(acc, v);
  else return acc + v;
}

template <int MODE>
__device__ inline float kernel_value(float e, float ys = 0.0f) {
  if constexpr (MODE == kModeGauss || MODE == kModeGaussExtra || MODE == kModeGaussRescue ||
                MODE == kModeGaussExtraRescue) {
    return __builtin_amdgcn_exp2f(e);
  } else if constexpr (kShiftMode<MODE>) {
    const float ne = -e;
    const float y = __builtin_amdgcn_sqrtf(ne < 0.0f ? 0.0f : ne);
    const float ts = __builtin_amdgcn_exp2f(ys - y);  // 2^{ys} t
    if constexpr (MODE == kModeExpShift) {
      return ts;
    } else {
      const float u = 1.0f + __builtin_amdgcn_exp2f(-y);
      return 4.0f * ts * __builtin_amdgcn_rcpf(u * u);
    }
  } else {
    const float ne = -e;
    const float t = __builtin_amdgcn_exp2f(-__builtin_amdgcn_sqrtf(ne < 0.0f ? 0.0f : ne));
    if constexpr (MODE == kModeExponential) {
      return t;
    } else {
      const float u = 1.0f + t;
      return 4.0f * t * __builtin_amdgcn_rcpf(u * u);
    }
  }
}

// Kernel values of one 32x32 accumulator tile held by a lane (16 exponents),
// summed as a balanced tree in fp32.
template <int MODE>
__device__ inline float kernel_tile_sum(const float* c, float ys = 0.0f) {
  float k[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) k[i] = kernel_value<MODE>(c[i], ys);
#pragma unroll
  for (int w = 8; w > 0; w >>= 1)
#pragma unroll
    for (int i = 0; i < w; ++i) k[i] = k[i] + k[i + w];
  return k[0];
}

// Tile sums of a group of 16 consecutive data tiles (global tile indices
// 16g .. 16g+15) for one query: lane half h buffers tiles 16g + 8h .. +7, and
// once the group is complete (or the chunk ends) both halves store their 32
// bytes in the same instructions, so each query's 64-byte segment of tp is
// written whole.  The row stride of tp is a multiple of 16 tiles; slots past
// the last data tile receive stale values and are never read.
struct TileSums8 {
  float v[8];
};

// Near pairs of the exponential kernel.  The epilogue only records them: per
// lane and chunk up to kNearSlots tiles that hold some, each as (chunk-relative
// tile index << 16 | 16-bit mask of the lane's values), in the workgroup's LDS
// (slot k of thread tid at k * 256 + tid), in tile order.  After the tile
// loop each lane adds their exact values, exp(-a ||q - x||) from fp64
// differences of the input rows, in row order; a lane with near pairs in more
// tiles than slots leaves the rest in its tile sums and flags its query in
// ex.near_over (the bound of that query then takes no credit for the
// refinement).  The slow path stays outside the tile loop.
constexpr int kNearSlots = 8;

struct NearRec {
  uint32_t* slots;  // LDS, kNearSlots * 256
  int n;
  bool over;
};

template <int MODE>
using near_lds_t = uint32_t[MODE == kModeExponential ? kNearSlots * 256 : 1];

// End of a chunk for one lane (column qi, half h; value i of tile t is row
// 32 t + 8(i/4) + 4h + i%4 of the chunk starting at row0): exact near terms
// and the overflow flag.
__device__ inline double near_finish(const TileExtra& ex, const NearRec& nr, int64_t qi, int h, int64_t row0,
                                     int tid) {
  if (nr.over) ex.near_over[qi] = 1;
  double s = 0.0;
  if (nr.n > 0) {
    const float* qr = ex.near_q + qi * ex.d;
    for (int k = 0; k < nr.n; ++k) {
      const uint32_t e = nr.slots[k * 256 + tid];
      const int64_t rb = row0 + (int64_t)(e >> 16) * kTileRows + 4 * h;
      for (uint32_t b = e & 0xFFFFu; b != 0; b &= b - 1) {
        const int i = __builtin_ctz(b);
        const float* xr = ex.near_x + (rb + 8 * (i >> 2) + (i & 3)) * ex.d;
        double r2 = 0.0;
        for (int j = 0; j < ex.d; ++j) {
          const double t = (double)qr[j] - (double)xr[j];
          r2 = fma(t, t, r2);
        }
        s += exp(-ex.a * sqrt(r2));
      }
    }
  }
  return s;
}

// Epilogue of one finished 32x32 tile held by a lane (column qi, half h):
// kernel values and fp32 tree sum; in kModeGaussExtra, optionally drops the diagonal element
// (data row == query index, for a data set queried against itself) and
// records the tile's 32-row partial sum (both halves, fixed order), through
// the group buffer `grp` when the caller walks tiles in order (`last` marks
// the chunk's final tile), else with a direct store.  In kModeExponential
// with near pairs on (ex.near_x), values whose computed -E is below
// ex.near_e leave the fp32 sum and are recorded in *nr (tile_rel: the tile's
// index in its chunk).
template <int MODE>
__device__ inline float tile_epilogue(const f32x16& c, int64_t row_base, int64_t col_base, int r32, int h,
                                      int64_t qi, const TileExtra& ex, TileSums8* grp = nullptr,
                                      bool last = false, NearRec* nr = nullptr, int tile_rel = 0,
                                      float ys = 0.0f) {
  constexpr bool EXTRA = kExtraMode<MODE>;
  float cp[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) cp[i] = c[i];
  if constexpr (MODE == kModeMax) {
    if (ex.self && row_base == col_base) {  // a data set against itself: leave out the diagonal
      const int idg = 4 * (r32 >> 3) + (r32 & 3);
      const bool mine = h == ((r32 & 7) >> 2);
#pragma unroll
      for (int i = 0; i < 16; ++i) cp[i] = (mine && i == idg) ? kPadOffset : cp[i];
    }
    float mx = cp[0];
#pragma unroll
    for (int i = 1; i < 16; ++i) mx = fmaxf(mx, cp[i]);
    return mx;
  }
  if constexpr (EXTRA) {
    if (ex.self && row_base == col_base) {
      // lane (column r32, half h) holds rows 8(i/4) + 4h + i%4
      const int idg = 4 * (r32 >> 3) + (r32 & 3);
      const bool mine = h == ((r32 & 7) >> 2);
#pragma unroll
      for (int i = 0; i < 16; ++i) cp[i] = (mine && i == idg) ? kPadOffset : cp[i];
    }
  }
  if constexpr (MODE == kModeExponential) {
    if (ex.near_x) {
      // Near a data point -E = y^2 is the difference of large terms and y =
      // sqrt(-E) magnifies its error; such terms (kernel above 2^-sqrt(near_e))
      // are rare and are evaluated from the input rows instead.
      float mx = cp[0];
#pragma unroll
      for (int i = 1; i < 16; ++i) mx = fmaxf(mx, cp[i]);
      if (-mx < ex.near_e && qi < ex.m_rows) {
        uint32_t nm = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) nm |= (-cp[i] < ex.near_e) ? (1u << i) : 0u;
        const bool room = nr->n < kNearSlots;
        if (room) nr->slots[nr->n * 256 + threadIdx.x] = ((uint32_t)tile_rel << 16) | nm;
        nr->n += room ? 1 : 0;
        nr->over |= !room;
        const uint32_t took = room ? nm : 0u;
#pragma unroll
        for (int i = 0; i < 16; ++i) cp[i] = ((took >> i) & 1u) ? kPadOffset : cp[i];
      }
    }
  }
  const float s = kernel_tile_sum<MODE>(cp, ys);
  if constexpr (EXTRA) {
    if (ex.tp) {
      const float o = __shfl_xor(s, 32);
      const float tot = h == 0 ? s + o : o + s;
      const int64_t tile = row_base / kTileRows;
      if (grp == nullptr) {
        if (h == 0) ex.tp[qi * ex.ntile + tile] = tot;
      } else {
        const int k16 = (int)(tile & 15);
        const int k = k16 - 8 * h;  // this half's slot, if in [0, 8)
#pragma unroll
        for (int e = 0; e < 8; ++e) grp->v[e] = e == k ? tot : grp->v[e];
        if (k16 == 15 || last) {
          f32x4* dst = reinterpret_cast<f32x4*>(ex.tp + qi * ex.ntile + (tile & ~(int64_t)15) + 8 * h);
          // streamed once and read by the draws much later: non-temporal, so
          // that the tile sums do not evict the data tiles that the
          // workgroups share in L2
          __builtin_nontemporal_store(f32x4{grp->v[0], grp->v[1], grp->v[2], grp->v[3]}, dst);
          __builtin_nontemporal_store(f32x4{grp->v[4], grp->v[5], grp->v[6], grp->v[7]}, dst + 1);
        }
      }
    }
  }
  return s;
}

// ---------------------------------------------------------------------------
// Tile loop shared by both forms.  Each step t (one 32-row data tile):
//   barrier (tile t is in LDS buffer t&1, buffer (t+1)&1 is free)
//   epilogue of tile t-1: exp2 of its 16 accumulators, fp32 tree sum, fp64 add
//   matrix-core chain of tile t (independent of the epilogue, so the two are
//   interleaved in one basic block)
//   store tile t+1 (loaded into registers one step earlier) to LDS and load
//   tile t+2 into registers.
// Staging is branch-free: indices past the end are clamped, so the redundant
// copies write identical values.  Two steps per loop iteration swap the roles
// of the two accumulator sets without register copies.
// ---------------------------------------------------------------------------

// FP32 form: v_mfma_f32_32x32x2_f32.  Lane l supplies A[l%32][k] and
// B[k][l%32] for the k-slot k = l/32; with the k ordering chosen here, lane
// half h covers dimensions [h*DP/2, (h+1)*DP/2) of every row.
template <int DP, int MODE>
__global__ __launch_bounds__(256, 2) void tile_f32(const float* __restrict__ Xp, const float* __restrict__ beta,
                                                   const float* __restrict__ Qs, const float* __restrict__ alpha,
                                                   int64_t n_pad, int n_qtiles, int64_t m_pad,
                                                   double* __restrict__ partial, TileExtra ex) {
  constexpr int H = DP / 2;
  constexpr int LD = DP + 4;  // LDS row stride (floats): 16-byte aligned, rows 4 banks apart
  constexpr int F4_ROW = DP / 4;
  constexpr int NV = kTileRows * F4_ROW;
  constexpr int NLD = (NV + 255) / 256;
  constexpr int NMMA = H;
  __shared__ __attribute__((aligned(16))) float tile[2][kTileRows * LD];
  __shared__ __attribute__((aligned(16))) float tbeta[2][kTileRows];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r32 = lane & 31, h = lane >> 5;
  const int qtile = blockIdx.x % n_qtiles;
  const int chunk = blockIdx.x / n_qtiles;
  const int64_t col_base = (int64_t)qtile * kBQ + wave * 32;
  const int64_t qi = col_base + r32;
  if (ex.qtile_active && ex.qtile_active[qtile] == 0) return;  // whole block: no query of its tile is active

  float bq[H];
  {
    const f32x4* qrow = reinterpret_cast<const f32x4*>(Qs + qi * DP + h * H);
#pragma unroll
    for (int s = 0; s < H / 4; ++s) {
      f32x4 v = qrow[s];
      bq[4 * s] = v.x; bq[4 * s + 1] = v.y; bq[4 * s + 2] = v.z; bq[4 * s + 3] = v.w;
    }
  }
  const float aq = alpha[qi];
  const float ys = kShiftMode<MODE> ? ex.yshift[qi] : 0.0f;

  const int64_t row0 = (int64_t)chunk * kChunkRows;
  const int64_t rem = (n_pad - row0) / kTileRows;
  const int ntiles = (int)(rem < kChunkRows / kTileRows ? rem : kChunkRows / kTileRows);

  f32x4 stage[NLD];
  float sbeta;
  auto gload = [&](int t) {
    const f32x4* srcp = reinterpret_cast<const f32x4*>(Xp + (row0 + (int64_t)t * kTileRows) * DP);
#pragma unroll
    for (int k = 0; k < NLD; ++k) stage[k] = srcp[min(tid + 256 * k, NV - 1)];
    sbeta = beta[row0 + (int64_t)t * kTileRows + (tid & 31)];
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int idx = min(tid + 256 * k, NV - 1);
      const int r = idx / F4_ROW, c4 = idx % F4_ROW;
      *reinterpret_cast<f32x4*>(&tile[buf][r * LD + c4 * 4]) = stage[k];
    }
    tbeta[buf][tid & 31] = sbeta;
  };

  double acc = acc_init<MODE>();
  TileSums8 grp = {};
  __shared__ near_lds_t<MODE> near_lds;
  NearRec nr = {near_lds, 0, false};
  auto step = [&](int t, const f32x16& cdone, f32x16& cnew) {
    const int buf = t & 1;
    __syncthreads();
    if constexpr (kBasedMode<MODE>) {
      if (t > 0)
        acc = acc_add<MODE>(acc, (double)tile_epilogue<MODE>(cdone, row0 + (int64_t)(t - 1) * kTileRows, col_base, r32, h, qi, ex, &grp));
    } else if constexpr (MODE == kModeExponential) {
      acc = acc_add<MODE>(acc, (double)tile_epilogue<MODE>(cdone, 0, 0, r32, h, qi, ex, nullptr, false, &nr, t - 1));
    } else {
      acc = acc_add<MODE>(acc, (double)tile_epilogue<MODE>(cdone, 0, 0, r32, h, qi, ex, nullptr, false, nullptr, 0, ys));
    }
    const float* arow = &tile[buf][r32 * LD + h * H];
    // the accumulators start from the offsets alpha_q + beta_x of their pairs
    f32x16 c;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const f32x4 bv = *reinterpret_cast<const f32x4*>(&tbeta[buf][8 * g + 4 * h]);
      c[4 * g] = aq + bv.x;
      c[4 * g + 1] = aq + bv.y;
      c[4 * g + 2] = aq + bv.z;
      c[4 * g + 3] = aq + bv.w;
    }
#pragma unroll
    for (int s = 0; s < H; s += 4) {
      const f32x4 a4 = *reinterpret_cast<const f32x4*>(arow + s);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, bq[s], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, bq[s + 1], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, bq[s + 2], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, bq[s + 3], c, 0, 0, 0);
    }
    cnew = c;
    lstore(buf ^ 1);
    gload(min(t + 2, ntiles - 1));
#pragma unroll
    for (int i = 0; i < NMMA; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, (40 + NMMA - 1) / NMMA, 0);
    }
  };

  gload(0);
  lstore(0);
  gload(min(1, ntiles - 1));
  f32x16 ca, cb;
#pragma unroll
  for (int i = 0; i < 16; ++i) ca[i] = kPadOffset;  // kernel value 0: neutral first epilogue
  int t = 0;
  for (; t + 1 < ntiles; t += 2) {
    step(t, ca, cb);
    step(t + 1, cb, ca);
  }
  if (t < ntiles) {
    step(t, ca, cb);
    ca = cb;
  }
  acc = acc_add<MODE>(acc, (double)tile_epilogue<MODE>(ca, row0 + (int64_t)(ntiles - 1) * kTileRows, col_base, r32, h, qi, ex, &grp,
                                    true, &nr, ntiles - 1, ys));
  if constexpr (MODE == kModeExponential) acc += near_finish(ex, nr, qi, h, row0, tid);
  const double other = __shfl_down(acc, 32);
  if (h == 0) partial[(int64_t)chunk * m_pad + qi] = acc_add<MODE>(acc, other);
}

// Centred fp32 form: the data rows are grouped into compact 32-row tiles,
// each stored as fl32(x - c_T) with beta = -a log2(e) ||x - c_T||^2 and its
// centre c_T and radius R_T (kde_centre.hip).  As tile_f32, but the queries
// (unscaled fp32) are re-centred on every tile: the B operand of dimension k
// is b = fl(s fl(q_k - c_k)), s = 2 a log2(e), the accumulators start from
// beta, and alpha' = -a log2(e) ||q - c_T||^2 (fp32 sum of the squared
// differences of both lane halves) plus the query's offset off[q] (0, or the
// shift -m_q of the underflow rescue) is added to the 16 exponents before
// the epilogue.  For the bound, each lane adds the tile's kernel sum times
// 2^{c_cent M_T} - 1, M_T = la (||q - c_T|| + R_T)^2 + |off[q]|, to a second
// fp64 accumulator (every term of the tile has an exponent error of at most
// c_cent M_T), written to ex.bpart.  The padded row count is read from the
// device (*n_pad); chunks past it write the neutral partial.
__device__ inline float centred_bound_factor(float sqt, float R, float qoff, float la, float c_cent) {
  const float r = __builtin_amdgcn_sqrtf(sqt) + R;
  const float M = (la * r * r + fabsf(qoff)) * 1.000001f;
  const float x = c_cent * M * 0.6931472f;
  // e^x - 1 <= x (1 + x) on [0, 1]; beyond, 2^{c M} - 1 itself (kept finite
  // so that a zero tile sum times it stays 0)
  const float e = x <= 1.0f ? x * (1.0f + x) : __builtin_amdgcn_exp2f(c_cent * M) - 1.0f;
  return fminf(e, 3.0e38f);
}

template <int DP, int MODE>
__global__ __launch_bounds__(256, 2) void tile_f32c(const float* __restrict__ Xp, const float* __restrict__ beta,
                                                    const float* __restrict__ cen, const float* __restrict__ rad,
                                                    const int64_t* __restrict__ n_pad_dev, const float* __restrict__ Qu,
                                                    const float* __restrict__ qoff, float la, int n_qtiles,
                                                    int64_t m_pad, double* __restrict__ partial, TileExtra ex) {
  constexpr int H = DP / 2;
  constexpr int LD = DP + 4;
  constexpr int F4_ROW = DP / 4;
  constexpr int NV = kTileRows * F4_ROW;
  constexpr int NLD = (NV + 255) / 256;
  constexpr int NMMA = H;
  __shared__ __attribute__((aligned(16))) float tile[2][kTileRows * LD];
  __shared__ __attribute__((aligned(16))) float tbeta[2][kTileRows];
  __shared__ __attribute__((aligned(16))) float tcen[2][DP];
  __shared__ float trad[2];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r32 = lane & 31, h = lane >> 5;
  const int qtile = blockIdx.x % n_qtiles;
  const int chunk = blockIdx.x / n_qtiles;
  const int64_t col_base = (int64_t)qtile * kBQ + wave * 32;
  const int64_t qi = col_base + r32;
  if (ex.qtile_active && ex.qtile_active[qtile] == 0) return;  // whole block: no query of its tile is active
  const int64_t n_pad = *n_pad_dev;
  const int64_t row0 = (int64_t)chunk * kChunkRows;
  if (row0 >= n_pad) {
    if (h == 0) {
      partial[(int64_t)chunk * m_pad + qi] = acc_init<MODE>();
      if (ex.bpart) ex.bpart[(int64_t)chunk * m_pad + qi] = 0.0;
    }
    return;
  }
  const float s2 = 2.0f * la;
  const float c_cent = ex.c_cent;
  float bq[H];
  {
    const f32x4* qrow = reinterpret_cast<const f32x4*>(Qu + qi * DP + h * H);
#pragma unroll
    for (int s = 0; s < H / 4; ++s) {
      f32x4 v = qrow[s];
      bq[4 * s] = v.x; bq[4 * s + 1] = v.y; bq[4 * s + 2] = v.z; bq[4 * s + 3] = v.w;
    }
  }
  const float qo = qoff[qi];

  const int64_t rem = (n_pad - row0) / kTileRows;
  const int ntiles = (int)(rem < kChunkRows / kTileRows ? rem : kChunkRows / kTileRows);
  const int64_t tile0 = row0 / kTileRows;

  f32x4 stage[NLD];
  float sbeta;
  f32x4 scen = {0.0f, 0.0f, 0.0f, 0.0f};
  float srad = 0.0f;
  auto gload = [&](int t) {
    const f32x4* srcp = reinterpret_cast<const f32x4*>(Xp + (row0 + (int64_t)t * kTileRows) * DP);
#pragma unroll
    for (int k = 0; k < NLD; ++k) stage[k] = srcp[min(tid + 256 * k, NV - 1)];
    sbeta = beta[row0 + (int64_t)t * kTileRows + (tid & 31)];
    const int64_t tg = tile0 + t;
    if (tid < F4_ROW) scen = reinterpret_cast<const f32x4*>(cen + tg * DP)[tid];
    srad = rad[tg];
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int idx = min(tid + 256 * k, NV - 1);
      const int r = idx / F4_ROW, c4 = idx % F4_ROW;
      *reinterpret_cast<f32x4*>(&tile[buf][r * LD + c4 * 4]) = stage[k];
    }
    tbeta[buf][tid & 31] = sbeta;
    if (tid < F4_ROW) *reinterpret_cast<f32x4*>(&tcen[buf][4 * tid]) = scen;
    if (tid == 0) trad[buf] = srad;
  };

  double acc = acc_init<MODE>();
  double bacc = 0.0;
  auto epilogue = [&](const f32x16& cdone, float adone, float edone) {
    float e[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) e[i] = cdone[i] + adone;
    if constexpr (MODE == kModeMax) {
      float mx = e[0];
#pragma unroll
      for (int i = 1; i < 16; ++i) mx = fmaxf(mx, e[i]);
      acc = acc_add<MODE>(acc, (double)mx);
    } else {
      const float sum = kernel_tile_sum<MODE>(e);
      acc += (double)sum;
      bacc += (double)(sum * edone);
    }
  };
  auto step = [&](int t, const f32x16& cdone, float adone, float edone, f32x16& cnew, float& anew, float& enew) {
    const int buf = t & 1;
    __syncthreads();
    epilogue(cdone, adone, edone);
    const float* arow = &tile[buf][r32 * LD + h * H];
    const float* crow = &tcen[buf][h * H];
    f32x16 c;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const f32x4 bv = *reinterpret_cast<const f32x4*>(&tbeta[buf][8 * g + 4 * h]);
      c[4 * g] = bv.x;
      c[4 * g + 1] = bv.y;
      c[4 * g + 2] = bv.z;
      c[4 * g + 3] = bv.w;
    }
    float sq = 0.0f;
#pragma unroll
    for (int s = 0; s < H; s += 4) {
      const f32x4 a4 = *reinterpret_cast<const f32x4*>(arow + s);
      const f32x4 c4 = *reinterpret_cast<const f32x4*>(crow + s);
      const float d0 = bq[s] - c4.x, d1 = bq[s + 1] - c4.y, d2 = bq[s + 2] - c4.z, d3 = bq[s + 3] - c4.w;
      sq = fmaf(d0, d0, sq);
      sq = fmaf(d1, d1, sq);
      sq = fmaf(d2, d2, sq);
      sq = fmaf(d3, d3, sq);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, d0 * s2, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, d1 * s2, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, d2 * s2, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, d3 * s2, c, 0, 0, 0);
    }
    const float sqt = sq + __shfl_xor(sq, 32);
    cnew = c;
    anew = -la * sqt + qo;
    enew = MODE == kModeMax ? 0.0f : centred_bound_factor(sqt, trad[buf], qo, la, c_cent);
    lstore(buf ^ 1);
    gload(min(t + 2, ntiles - 1));
#pragma unroll
    for (int i = 0; i < NMMA; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, (40 + 3 * H + NMMA - 1) / NMMA, 0);
    }
  };

  gload(0);
  lstore(0);
  gload(min(1, ntiles - 1));
  f32x16 ca, cb;
#pragma unroll
  for (int i = 0; i < 16; ++i) ca[i] = kPadOffset;  // kernel value 0: neutral first epilogue
  float aa = 0.0f, ab = 0.0f, ea = 0.0f, eb = 0.0f;
  int t = 0;
  for (; t + 1 < ntiles; t += 2) {
    step(t, ca, aa, ea, cb, ab, eb);
    step(t + 1, cb, ab, eb, ca, aa, ea);
  }
  if (t < ntiles) {
    step(t, ca, aa, ea, cb, ab, eb);
    ca = cb;
    aa = ab;
    ea = eb;
  }
  epilogue(ca, aa, ea);
  const double other = __shfl_down(acc, 32);
  const double bother = __shfl_down(bacc, 32);
  if (h == 0) {
    partial[(int64_t)chunk * m_pad + qi] = acc_add<MODE>(acc, other);
    if (ex.bpart) ex.bpart[(int64_t)chunk * m_pad + qi] = bacc + bother;
  }
}

// Split forms: v_mfma_f32_32x32x16_{f16,bf16}.  Lane l supplies 8 consecutive
// k values of row/column l%32; lane half h covers dimensions
// [16 s + 8 h, 16 s + 8 h + 8) of k-step s.
template <int FORM>
__device__ inline f32x16 mma16(u16x8 a, u16x8 b, f32x16 c) {
  if constexpr (FORM == STAG_FORM_FP16_SPLIT)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                  0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

__device__ inline f32x16 mma16_bf16(u16x8 a, u16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

template <int FORM, int DP, int MODE>
__global__ __launch_bounds__(256, 2) void tile_split(
    const unsigned short* __restrict__ X0, const unsigned short* __restrict__ X1,
    const unsigned short* __restrict__ X2, const float* __restrict__ Xoff, const unsigned short* __restrict__ Q0,
    const unsigned short* __restrict__ Q1, const unsigned short* __restrict__ Q2, const float* __restrict__ Qoff,
    int64_t n_pad, int n_qtiles, int64_t m_pad, double* __restrict__ partial, TileExtra ex) {
  constexpr int NP = FORM == STAG_FORM_BF16_SPLIT3 ? 3 : 2;
  constexpr int KS = DP / 16;
  constexpr int LD = DP + 8;     // LDS row stride (halves): 16-byte aligned
  constexpr int V_ROW = DP / 8;  // 16-byte vectors per row
  constexpr int NV = kTileRows * V_ROW;
  constexpr int NLD = (NV + 255) / 256;
  constexpr int NMMA = KS * (NP == 3 ? 6 : 3);
  __shared__ __attribute__((aligned(16))) unsigned short tile[2][NP][kTileRows * LD];
  __shared__ __attribute__((aligned(16))) float tbeta[2][kTileRows];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r32 = lane & 31, h = lane >> 5;
  const int qtile = blockIdx.x % n_qtiles;
  const int chunk = blockIdx.x / n_qtiles;
  const int64_t col_base = (int64_t)qtile * kBQ + wave * 32;
  const int64_t qi = col_base + r32;
  if (ex.qtile_active && ex.qtile_active[qtile] == 0) return;  // whole block: no query of its tile is active
  if (ex.cflag && ex.cflag[(int64_t)chunk * ((m_pad + 255) / 256) + qtile / 2] == 0) return;  // not selected

  const unsigned short* Qp[3] = {Q0, Q1, Q2};
  const unsigned short* Xpp[3] = {X0, X1, X2};
  u16x8 bq[NP][KS];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int s = 0; s < KS; ++s)
      bq[p][s] = *reinterpret_cast<const u16x8*>(Qp[p] + qi * DP + s * 16 + h * 8);
  const float alpha = Qoff[qi];
  const float ys = kShiftMode<MODE> ? ex.yshift[qi] : 0.0f;

  const int64_t row0 = (int64_t)chunk * kChunkRows;
  const int64_t rem = (n_pad - row0) / kTileRows;
  const int ntiles = (int)(rem < kChunkRows / kTileRows ? rem : kChunkRows / kTileRows);

  // the chunk's rows and offsets through buffer resources based at the chunk
  // (as in the centred tile: no per-tile address arithmetic)
  const int64_t rows_left = min((int64_t)kChunkRows, n_pad - row0);
  __amdgpu_buffer_rsrc_t xr[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p)
    xr[p] = __builtin_amdgcn_make_buffer_rsrc((void*)(Xpp[p] + row0 * DP), (short)0, (int)(rows_left * DP * 2),
                                              kBufferWord3);
  const __amdgpu_buffer_rsrc_t br =
      __builtin_amdgcn_make_buffer_rsrc((void*)(Xoff + row0), (short)0, (int)(rows_left * 4), kBufferWord3);
  int voff[NLD];
#pragma unroll
  for (int k = 0; k < NLD; ++k) voff[k] = min(tid + 256 * k, NV - 1) * 16;
  const int boff = (tid & 31) * 4;
  u16x8 stage[NP][NLD];
  float sbeta;
  auto gload = [&](int t) {
    const int so = t * kTileRows * DP * 2;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int k = 0; k < NLD; ++k)
        stage[p][k] = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(xr[p], voff[k], so, 0));
    sbeta = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(br, boff, t * kTileRows * 4, 0));
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int k = 0; k < NLD; ++k) {
        const int idx = min(tid + 256 * k, NV - 1);
        const int r = idx / V_ROW, c8 = idx % V_ROW;
        *reinterpret_cast<u16x8*>(&tile[buf][p][r * LD + c8 * 8]) = stage[p][k];
      }
    tbeta[buf][tid & 31] = sbeta;
  };

  double acc = acc_init<MODE>();
  TileSums8 grp = {};
  __shared__ near_lds_t<MODE> near_lds;
  NearRec nr = {near_lds, 0, false};
  auto step = [&](int t, const f32x16& cdone, f32x16& cnew) {
    const int buf = t & 1;
    __syncthreads();
    if constexpr (kBasedMode<MODE>) {
      if (t > 0)
        acc = acc_add<MODE>(acc, (double)tile_epilogue<MODE>(cdone, row0 + (int64_t)(t - 1) * kTileRows, col_base, r32, h, qi, ex, &grp));
    } else if constexpr (MODE == kModeExponential) {
      acc = acc_add<MODE>(acc, (double)tile_epilogue<MODE>(cdone, 0, 0, r32, h, qi, ex, nullptr, false, &nr, t - 1));
    } else {
      acc = acc_add<MODE>(acc, (double)tile_epilogue<MODE>(cdone, 0, 0, r32, h, qi, ex, nullptr, false, nullptr, 0, ys));
    }
    // the accumulators start from the offsets alpha_q + beta_x of their pairs
    f32x16 c;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const f32x4 bv = *reinterpret_cast<const f32x4*>(&tbeta[buf][8 * g + 4 * h]);
      c[4 * g] = alpha + bv.x;
      c[4 * g + 1] = alpha + bv.y;
      c[4 * g + 2] = alpha + bv.z;
      c[4 * g + 3] = alpha + bv.w;
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      u16x8 a[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p)
        a[p] = *reinterpret_cast<const u16x8*>(&tile[buf][p][r32 * LD + s * 16 + h * 8]);
      // small corrections first, then the leading product
      if constexpr (NP == 3) {
        c = mma16<FORM>(a[2], bq[0][s], c);
        c = mma16<FORM>(a[1], bq[1][s], c);
        c = mma16<FORM>(a[0], bq[2][s], c);
      }
      c = mma16<FORM>(a[1], bq[0][s], c);
      c = mma16<FORM>(a[0], bq[1][s], c);
      c = mma16<FORM>(a[0], bq[0][s], c);
    }
    cnew = c;
    lstore(buf ^ 1);
    gload(min(t + 2, ntiles - 1));
#pragma unroll
    for (int i = 0; i < NMMA; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, (40 + NMMA - 1) / NMMA, 0);
    }
  };

  gload(0);
  lstore(0);
  gload(min(1, ntiles - 1));
  f32x16 ca, cb;
#pragma unroll
  for (int i = 0; i < 16; ++i) ca[i] = kPadOffset;  // kernel value 0: neutral first epilogue
  int t = 0;
  for (; t + 1 < ntiles; t += 2) {
    step(t, ca, cb);
    step(t + 1, cb, ca);
  }
  if (t < ntiles) {
    step(t, ca, cb);
    ca = cb;
  }
  acc = acc_add<MODE>(acc, (double)tile_epilogue<MODE>(ca, row0 + (int64_t)(ntiles - 1) * kTileRows, col_base, r32, h, qi, ex, &grp,
                                    true, &nr, ntiles - 1, ys));
  if constexpr (MODE == kModeExponential) acc += near_finish(ex, nr, qi, h, row0, tid);
  const double other = __shfl_down(acc, 32);
  if (h == 0) partial[(int64_t)chunk * m_pad + qi] = acc_add<MODE>(acc, other);
}

// Split forms (hi + lo), 64 queries per wave.  Every wave holds two 32-query
// column blocks as B operands and uses each A operand it reads from LDS for
// both, which halves the LDS reads per matrix-core product: in tile_split
// the four waves of a workgroup each read the whole data tile from LDS for
// their 32 queries, and at d = 128 those reads (with the staging writes)
// kept the matrix cores waiting.  Four waves cover 256 queries; when m_pad
// is an odd multiple of 128 the last workgroup's waves 2 and 3 have no
// queries and only stage tiles.  The products per block come in the same k
// order, from the same accumulator seeds, as in tile_split, so every result
// is bitwise the same.  Gaussian sums only (kModeGauss).
template <int FORM, int DP, int MODE>
__global__ __launch_bounds__(256, 2) void tile_split_w64(
    const unsigned short* __restrict__ X0, const unsigned short* __restrict__ X1, const float* __restrict__ Xoff,
    const unsigned short* __restrict__ Q0, const unsigned short* __restrict__ Q1, const float* __restrict__ Qoff,
    int64_t n_pad, int n_qt256, int64_t m_pad, double* __restrict__ partial, TileExtra ex) {
  static_assert(MODE == kModeGauss, "Gaussian sums only");
  constexpr int NP = 2;
  constexpr int KS = DP / 16;
  constexpr int LD = DP + 8;
  constexpr int V_ROW = DP / 8;
  constexpr int NV = kTileRows * V_ROW;
  constexpr int NLD = (NV + 255) / 256;
  constexpr int NMMA = KS * 6;
  __shared__ __attribute__((aligned(16))) unsigned short tile[2][NP][kTileRows * LD];
  __shared__ __attribute__((aligned(16))) float tbeta[2][kTileRows];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r32 = lane & 31, h = lane >> 5;
  const int qtile = blockIdx.x % n_qt256;
  const int chunk = blockIdx.x / n_qt256;
  if (ex.cflag && ex.cflag[(int64_t)chunk * n_qt256 + qtile] == 0) return;  // whole block: not selected
  const int64_t col0 = (int64_t)qtile * 256 + wave * 64;
  const bool live = col0 < m_pad;  // wave-uniform
  const int64_t q0 = col0 + r32, q1 = q0 + 32;

  u16x8 b0[NP][KS], b1[NP][KS];
  float alpha0 = 0.0f, alpha1 = 0.0f;
  {
    const unsigned short* Qp[2] = {Q0, Q1};
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        b0[p][s] = live ? *reinterpret_cast<const u16x8*>(Qp[p] + q0 * DP + s * 16 + h * 8) : u16x8{};
        b1[p][s] = live ? *reinterpret_cast<const u16x8*>(Qp[p] + q1 * DP + s * 16 + h * 8) : u16x8{};
      }
    if (live) {
      alpha0 = Qoff[q0];
      alpha1 = Qoff[q1];
    }
  }

  const int64_t row0 = (int64_t)chunk * kChunkRows;
  const int64_t rem = (n_pad - row0) / kTileRows;
  const int ntiles = (int)(rem < kChunkRows / kTileRows ? rem : kChunkRows / kTileRows);

  const unsigned short* Xpp[2] = {X0, X1};
  // the chunk's rows and offsets through buffer resources based at the chunk
  // (as in the centred tile: no per-tile address arithmetic)
  const int64_t rows_left = min((int64_t)kChunkRows, n_pad - row0);
  __amdgpu_buffer_rsrc_t xr[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p)
    xr[p] = __builtin_amdgcn_make_buffer_rsrc((void*)(Xpp[p] + row0 * DP), (short)0, (int)(rows_left * DP * 2),
                                              kBufferWord3);
  const __amdgpu_buffer_rsrc_t br =
      __builtin_amdgcn_make_buffer_rsrc((void*)(Xoff + row0), (short)0, (int)(rows_left * 4), kBufferWord3);
  int voff[NLD];
#pragma unroll
  for (int k = 0; k < NLD; ++k) voff[k] = min(tid + 256 * k, NV - 1) * 16;
  const int boff = (tid & 31) * 4;
  u16x8 stage[NP][NLD];
  float sbeta;
  auto gload = [&](int t) {
    const int so = t * kTileRows * DP * 2;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int k = 0; k < NLD; ++k)
        stage[p][k] = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(xr[p], voff[k], so, 0));
    sbeta = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(br, boff, t * kTileRows * 4, 0));
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int k = 0; k < NLD; ++k) {
        const int idx = min(tid + 256 * k, NV - 1);
        const int r = idx / V_ROW, c8 = idx % V_ROW;
        *reinterpret_cast<u16x8*>(&tile[buf][p][r * LD + c8 * 8]) = stage[p][k];
      }
    tbeta[buf][tid & 31] = sbeta;
  };

  double acc0 = 0.0, acc1 = 0.0;
  auto step = [&](int t, const f32x16& d0, const f32x16& d1, f32x16& n0, f32x16& n1) {
    const int buf = t & 1;
    __syncthreads();
    if (live) {
      float e0[16], e1[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        e0[i] = d0[i];
        e1[i] = d1[i];
      }
      acc0 += (double)kernel_tile_sum<MODE>(e0);
      acc1 += (double)kernel_tile_sum<MODE>(e1);
      // the accumulators start from the offsets alpha_q + beta_x of their pairs
      f32x16 c0, c1;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const f32x4 bv = *reinterpret_cast<const f32x4*>(&tbeta[buf][8 * g + 4 * h]);
        c0[4 * g] = alpha0 + bv.x;
        c0[4 * g + 1] = alpha0 + bv.y;
        c0[4 * g + 2] = alpha0 + bv.z;
        c0[4 * g + 3] = alpha0 + bv.w;
        c1[4 * g] = alpha1 + bv.x;
        c1[4 * g + 1] = alpha1 + bv.y;
        c1[4 * g + 2] = alpha1 + bv.z;
        c1[4 * g + 3] = alpha1 + bv.w;
      }
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const u16x8 ahi = *reinterpret_cast<const u16x8*>(&tile[buf][0][r32 * LD + s * 16 + h * 8]);
        const u16x8 alo = *reinterpret_cast<const u16x8*>(&tile[buf][1][r32 * LD + s * 16 + h * 8]);
        // small corrections first, then the leading product (tile_split's order)
        c0 = mma16<FORM>(alo, b0[0][s], c0);
        c1 = mma16<FORM>(alo, b1[0][s], c1);
        c0 = mma16<FORM>(ahi, b0[1][s], c0);
        c1 = mma16<FORM>(ahi, b1[1][s], c1);
        c0 = mma16<FORM>(ahi, b0[0][s], c0);
        c1 = mma16<FORM>(ahi, b1[0][s], c1);
      }
      n0 = c0;
      n1 = c1;
    }
    lstore(buf ^ 1);
    gload(min(t + 2, ntiles - 1));
#pragma unroll
    for (int i = 0; i < NMMA; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, (80 + NMMA - 1) / NMMA, 0);
    }
  };

  gload(0);
  lstore(0);
  gload(min(1, ntiles - 1));
  f32x16 ca0, ca1, cb0, cb1;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    ca0[i] = kPadOffset;  // kernel value 0: neutral first epilogue
    ca1[i] = kPadOffset;
    cb0[i] = kPadOffset;
    cb1[i] = kPadOffset;
  }
  int t = 0;
  for (; t + 1 < ntiles; t += 2) {
    step(t, ca0, ca1, cb0, cb1);
    step(t + 1, cb0, cb1, ca0, ca1);
  }
  if (t < ntiles) {
    step(t, ca0, ca1, cb0, cb1);
    ca0 = cb0;
    ca1 = cb1;
  }
  if (live) {
    float e0[16], e1[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      e0[i] = ca0[i];
      e1[i] = ca1[i];
    }
    acc0 += (double)kernel_tile_sum<MODE>(e0);
    acc1 += (double)kernel_tile_sum<MODE>(e1);
  }
  const double o0 = __shfl_down(acc0, 32);
  const double o1 = __shfl_down(acc1, 32);
  if (live && h == 0) {
    partial[(int64_t)chunk * m_pad + q0] = acc0 + o0;
    partial[(int64_t)chunk * m_pad + q1] = acc1 + o1;
  }
}

// Centred fp16 form (STAG_FORM_FP16_CENTRED): one fp16 product per pair.
// The data rows come grouped around centres c_g (each group a run of whole
// 32-row tiles, tgroup[tile] = g), stored once as fl16(x - c_g) with
// beta = fl32(-la ||x - c_g||^2).  Whenever the group of the data tile
// changes, every wave forms its queries' operand fl16(2 la fl32(q - c_g))
// and alpha = fl32(-la ||q - c_g||^2) + qoff from the fp32 query rows, so
//   E = alpha + beta + fl16(2 la (q - c_g)) . fl16(x - c_g),
// and, per query and group, the bound factor 2^{M} - 1 of
// h1c_bound_factor; bpart collects the group's sums times that factor.
// Up to d = 128, 64 queries per wave as in tile_split_w64 (each A operand
// read from LDS feeds two 32-query blocks), 256 per workgroup; above, 32 per
// wave (the query operands alone take 4 d / 16 registers per block).  With
// qtile_active, a workgroup whose 128-query tiles are all inactive returns at
// once and a wave whose tile is inactive only stages.  A query element with
// |2 la (q_j - c_j)| >= 65520 (fp16 infinity) makes alpha NaN for the group.
// Gaussian sums with ex.fold_alpha: where every alpha of the wave lies in
// [-60, 0] for the group, the accumulators start from beta alone (the first
// product reads the beta registers as its accumulator input: no seeding
// instructions) and the group's sum is multiplied by fl32(2^alpha) instead,
// so that a term is 2^(beta + cross) 2^alpha with 2^(beta + cross) <= 2^-alpha
// <= 2^60; the bound factor of such a group adds 2^-21 for the rounding of
// fl32(2^alpha).  A query's result then depends on the other queries of its
// wave.

// Exponent error bound M (base 2) of every term of a (query, group):
//   fp32 part as in the centred fp32 tile: c_cent (la (|q - c| + R)^2 + |qoff|)
//   two fp16 roundings (and the fp32 roundings before them) of each product:
//     2 la |q - c| R 2^-10 (1 + 2^-10) by Cauchy-Schwarz
//   fp16 subnormal spacing 2^-24 (at most 2^-25 per rounding) on either
//   operand: 2^-25 sqrt(dp) (2 la |q - c| + R) (1 + 2^-6), and dp 2^-50 < 1e-12
// and the relative error of the terms' sum is at most 2^M - 1.
__device__ inline float h1c_bound_factor(float sqt, float R, float qoff, float la, float c_cent, float rdp) {
  const float dq = __builtin_amdgcn_sqrtf(sqt);
  const float s2 = 2.0f * la;
  const float r = dq + R;
  const float M = (c_cent * (la * r * r + fabsf(qoff)) + s2 * dq * R * 0x1.004p-10f +
                   0x1.04p-25f * rdp * (s2 * dq + R) + 1.0e-12f) *
                  1.00001f;
  const float x = M * 0.6931472f;
  // e^x - 1 <= x (1 + x) on [0, 1]; beyond, 2^M - 1 itself (kept finite so
  // that a zero tile sum times it stays 0)
  const float e = x <= 1.0f ? x * (1.0f + x) : __builtin_amdgcn_exp2f(M) - 1.0f;
  return fminf(e, 3.0e38f);
}

template <int DP>
constexpr int kH1cBlocks = DP <= 128 ? 2 : 1;  // 32-query blocks per wave

// XCD-aware order of the (query tile, chunk) workgroups of the centred fp16
// tile.  Workgroup b runs on XCD b % 8 (the dispatcher deals workgroups to
// the 8 XCDs in turn); XCD x owns the query tiles [x Qx, (x+1) Qx), Qx =
// ceil(nq / 8), and takes them in windows of kWinQ tiles, each window over
// all P chunks with the window's tiles innermost: the window's query rows
// (kWinQ x 256 x d_pad x 4 bytes, 2 MB at d = 128) stay in that XCD's L2
// while the chunks stream past, instead of every workgroup fetching its
// query rows again; the data (fp16, one part) are fetched once per window.
// (The split tiles keep the chunk-major order: their data are twice the
// bytes, and fetching them once per window cost more L2 misses than the
// query rows saved.)  Grid = 8 Qx P; every (tile, chunk) pair has exactly
// one workgroup, and those past the last tile (qtile >= nq) return at once.
constexpr int kWinQ = 16;
__device__ inline void xcd_tile(int64_t b, int nq, int P, int* qtile, int* chunk) {
  const int Qx = (nq + 7) / 8;
  const int x = (int)(b % 8);
  const int64_t j = b / 8;  // < Qx P
  const int64_t per = (int64_t)kWinQ * P;
  const int w = (int)(j / per);
  const int64_t r = j - (int64_t)w * per;
  const int wq = min(kWinQ, Qx - w * kWinQ);  // the window's width (the last may be narrower)
  *chunk = (int)(r / wq);
  *qtile = x * Qx + w * kWinQ + (int)(r % wq);
}

template <int DP, int MODE>
__global__ __launch_bounds__(256, 2) void tile_h1c(const unsigned short* __restrict__ Xh,
                                                   const float* __restrict__ beta, const int* __restrict__ tgroup,
                                                   const float* __restrict__ cen, const float* __restrict__ grad,
                                                   const int64_t* __restrict__ n_pad_dev,
                                                   const float* __restrict__ Qu, const float* __restrict__ qoff,
                                                   float la, int n_qtw, int64_t m_pad,
                                                   double* __restrict__ partial, TileExtra ex) {
  static_assert(MODE == kModeGauss || MODE == kModeGaussRescue || MODE == kModeMax, "Gaussian sums and maxima");
  constexpr int NB = kH1cBlocks<DP>;
  constexpr int QW = 32 * NB;  // queries per wave
  constexpr int KS = DP / 16;
  constexpr int LD = DP + 8;
  constexpr int V_ROW = DP / 8;
  constexpr int NV = kTileRows * V_ROW;
  constexpr int NLD = (NV + 255) / 256;
  constexpr int NMMA = KS * NB;
  __shared__ __attribute__((aligned(16))) unsigned short tile[2][kTileRows * LD];
  __shared__ __attribute__((aligned(16))) float tbeta[2][kTileRows];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r32 = lane & 31, h = lane >> 5;
  // with a tile list (qsel holds workgroup tiles here), blockIdx.x runs over
  // (list entry, chunk); else the XCD-aware order of xcd_tile
  int qtile, chunk;
  if (ex.qsel_n > 0) {
    qtile = ex.qsel[blockIdx.x % ex.qsel_n];
    chunk = blockIdx.x / ex.qsel_n;
  } else {
    xcd_tile(blockIdx.x, n_qtw, (int)ex.h1c_chunks, &qtile, &chunk);
    if (qtile >= n_qtw) return;
  }
  const int64_t col0 = (int64_t)qtile * (4 * QW) + wave * QW;
  if (ex.qtile_active) {
    // the workgroup's 128-query tiles (NB of them)
    bool any = false;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int64_t tq = (int64_t)qtile * NB + b;
      any = any || (tq * kBQ < m_pad && ex.qtile_active[tq] != 0);
    }
    if (!any) return;
  }
  bool live = col0 < m_pad;  // wave-uniform
  if (live && ex.qtile_active) live = ex.qtile_active[col0 / kBQ] != 0;
  int64_t qi[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) qi[b] = col0 + 32 * b + r32;
  const int64_t n_pad = *n_pad_dev;
  const int64_t row0 = (int64_t)chunk * kChunkRows;
  if (row0 >= n_pad) {
    if (live && h == 0)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        partial[(int64_t)chunk * m_pad + qi[b]] = acc_init<MODE>();
        if (ex.bpart) ex.bpart[(int64_t)chunk * m_pad + qi[b]] = 0.0;
      }
    return;
  }
  const int64_t rem = (n_pad - row0) / kTileRows;
  const int ntiles = (int)(rem < kChunkRows / kTileRows ? rem : kChunkRows / kTileRows);
  const int64_t tile0 = row0 / kTileRows;
  const float s2 = 2.0f * la;
  const float c_cent = ex.c_cent;
  const float rdp = __builtin_amdgcn_sqrtf((float)DP);
  float qo[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) qo[b] = live ? qoff[qi[b]] : 0.0f;

  // the queries' operands, offsets and bound factors for group g
  u16x8 bq[NB][KS];
  float alpha[NB], eg[NB], scl[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    alpha[b] = 0.0f;
    eg[b] = 0.0f;
    scl[b] = 1.0f;
  }
  bool noseed = false;  // wave-uniform
  int cur = -1;
  auto form_queries = [&](int g) {
    const float* cg = cen + (int64_t)g * DP;
    float sq[NB], mx[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      sq[b] = 0.0f;
      mx[b] = 0.0f;
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k0 = s * 16 + h * 8;
      const f32x4 c4[2] = {*reinterpret_cast<const f32x4*>(cg + k0), *reinterpret_cast<const f32x4*>(cg + k0 + 4)};
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const f32x4 u4[2] = {*reinterpret_cast<const f32x4*>(Qu + qi[b] * DP + k0),
                             *reinterpret_cast<const f32x4*>(Qu + qi[b] * DP + k0 + 4)};
        u16x8 o;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float e = u4[i >> 2][i & 3] - c4[i >> 2][i & 3];
          sq[b] = fmaf(e, e, sq[b]);
          const float w = e * s2;
          mx[b] = fmaxf(mx[b], fabsf(w));
          o[i] = f16_rne(w);
        }
        bq[b][s] = o;
      }
      // keeps the loads of the next k-step behind this one (register use)
      __builtin_amdgcn_sched_barrier(0);
    }
    const float R = grad[g];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const float t = sq[b] + __shfl_xor(sq[b], 32);
      const float m = fmaxf(mx[b], __shfl_xor(mx[b], 32));
      // a NaN element fails the comparison as well
      alpha[b] = m < 65520.0f ? fmaf(-la, t, qo[b]) : __builtin_nanf("");
      if constexpr (MODE != kModeMax) eg[b] = h1c_bound_factor(t, R, qo[b], la, c_cent, rdp);
    }
    if constexpr (MODE == kModeGauss) {
      bool ok = ex.fold_alpha != 0;
#pragma unroll
      for (int b = 0; b < NB; ++b) ok = ok && alpha[b] >= -60.0f && alpha[b] <= 0.0f;  // NaN fails
      noseed = __all(ok) != 0;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        scl[b] = noseed ? __builtin_amdgcn_exp2f(alpha[b]) : 1.0f;
        if (noseed) eg[b] += 0x1p-21f;
      }
    }
  };

  // The chunk's rows and offsets through buffer resources based at the
  // chunk (range-checked loads; the lane's byte offsets are fixed, the
  // tile's is a scalar, so that staging a tile takes no address arithmetic)
  const int64_t rows_left = min((int64_t)kChunkRows, n_pad - row0);
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(Xh + row0 * DP), (short)0, (int)(rows_left * DP * 2), kBufferWord3);
  const __amdgpu_buffer_rsrc_t br =
      __builtin_amdgcn_make_buffer_rsrc((void*)(beta + row0), (short)0, (int)(rows_left * 4), kBufferWord3);
  int voff[NLD];
#pragma unroll
  for (int k = 0; k < NLD; ++k) voff[k] = min(tid + 256 * k, NV - 1) * 16;
  const int boff = (tid & 31) * 4;
  u16x8 stage[NLD];
  float sbeta;
  auto gload = [&](int t) {
    const int so = t * kTileRows * DP * 2;
#pragma unroll
    for (int k = 0; k < NLD; ++k)
      stage[k] = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(xr, voff[k], so, 0));
    sbeta = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(br, boff, t * kTileRows * 4, 0));
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int idx = min(tid + 256 * k, NV - 1);
      const int r = idx / V_ROW, c8 = idx % V_ROW;
      *reinterpret_cast<u16x8*>(&tile[buf][r * LD + c8 * 8]) = stage[k];
    }
    tbeta[buf][tid & 31] = sbeta;
  };

  // Sums: a group's tiles add their tile sums into aseg (fp64); once the
  // group's last tile is in (one step after the group changed, so that the
  // epilogue stays beside the next tile's products), aseg times the group's
  // scale goes to acc and times scale and bound factor to bacc.
  double acc[NB], bacc[NB], aseg[NB];
  float psc[NB], peg[NB];  // the closed group's scale and bound factor
  bool pend = false;       // wave-uniform: a closed group awaits its flush
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    acc[b] = acc_init<MODE>();
    bacc[b] = 0.0;
    aseg[b] = 0.0;
  }
  auto epilogue = [&](const f32x16 (&d)[NB]) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if constexpr (MODE == kModeMax) {
        float mv = d[b][0];
#pragma unroll
        for (int i = 1; i < 16; ++i) mv = fmaxf(mv, d[b][i]);
        acc[b] = acc_add<MODE>(acc[b], (double)mv);
      } else {
        float e[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) e[i] = d[b][i];
        aseg[b] += (double)kernel_tile_sum<MODE>(e);
      }
    }
  };
  auto flush = [&](const float (&fs)[NB], const float (&fe)[NB]) {
    if constexpr (MODE != kModeMax) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const double sc = (double)fs[b];
        acc[b] = fma(aseg[b], sc, acc[b]);
        bacc[b] = fma(aseg[b], sc * (double)fe[b], bacc[b]);
        aseg[b] = 0.0;
      }
    }
  };
  int gnext = tgroup[tile0];  // the next tile's group, loaded a step ahead
  auto step = [&](int t, const f32x16 (&d)[NB], f32x16 (&nc)[NB]) {
    const int buf = t & 1;
    __syncthreads();
    const int g = gnext;
    gnext = tgroup[tile0 + min(t + 1, ntiles - 1)];
    if (live) {
      if (pend) {
        // aseg holds the closed group's tiles (the last one added a step ago)
        flush(psc, peg);
        pend = false;
      }
      if (g != cur) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          psc[b] = scl[b];
          peg[b] = eg[b];
        }
        pend = true;
        form_queries(g);
        cur = g;
      }
      epilogue(d);
      // the accumulators start from the offsets alpha_q + beta_x of their
      // pairs, or from beta_x alone (alpha applied to the group's sums)
      f32x16 bvec;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 bv = *reinterpret_cast<const f32x4*>(&tbeta[buf][8 * q + 4 * h]);
#pragma unroll
        for (int i = 0; i < 4; ++i) bvec[4 * q + i] = bv[i];
      }
      f32x16 c[NB];
      const u16x8 a0 = *reinterpret_cast<const u16x8*>(&tile[buf][r32 * LD + h * 8]);
      if (noseed) {
#pragma unroll
        for (int b = 0; b < NB; ++b) c[b] = mma16<STAG_FORM_FP16_SPLIT>(a0, bq[b][0], bvec);
      } else {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          f32x16 c0;
#pragma unroll
          for (int i = 0; i < 16; ++i) c0[i] = alpha[b] + bvec[i];
          c[b] = mma16<STAG_FORM_FP16_SPLIT>(a0, bq[b][0], c0);
        }
      }
#pragma unroll
      for (int s = 1; s < KS; ++s) {
        const u16x8 a = *reinterpret_cast<const u16x8*>(&tile[buf][r32 * LD + s * 16 + h * 8]);
#pragma unroll
        for (int b = 0; b < NB; ++b) c[b] = mma16<STAG_FORM_FP16_SPLIT>(a, bq[b][s], c[b]);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) nc[b] = c[b];
    }
    lstore(buf ^ 1);
    gload(min(t + 2, ntiles - 1));
    // the products after the first k-step, each with its share of the epilogue
    constexpr int NM2 = NMMA - NB;
#pragma unroll
    for (int i = 0; i < NM2; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, (40 * NB + NM2 - 1) / (NM2 > 0 ? NM2 : 1), 0);
    }
  };

  gload(0);
  lstore(0);
  gload(min(1, ntiles - 1));
  f32x16 ca[NB], cb[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      ca[b][i] = kPadOffset;  // kernel value 0: neutral first epilogue
      cb[b][i] = kPadOffset;
    }
  }
  int t = 0;
  for (; t + 1 < ntiles; t += 2) {
    step(t, ca, cb);
    step(t + 1, cb, ca);
  }
  if (t < ntiles) {
    step(t, ca, cb);
#pragma unroll
    for (int b = 0; b < NB; ++b) ca[b] = cb[b];
  }
  if (live) {
    if (pend) flush(psc, peg);
    epilogue(ca);
    flush(scl, eg);
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const double o = __shfl_down(acc[b], 32);
    const double ob = __shfl_down(bacc[b], 32);
    if (live && h == 0) {
      partial[(int64_t)chunk * m_pad + qi[b]] = acc_add<MODE>(acc[b], o);
      if (ex.bpart) ex.bpart[(int64_t)chunk * m_pad + qi[b]] = bacc[b] + ob;
    }
  }
}

// ---------------------------------------------------------------------------
// Wide rows (256 < d <= 1024), fp32 form.  The 32 queries of a workgroup sit
// in LDS as the B operand ([32][DP+4] floats, loaded once); each of the 4
// waves takes every 4th 32-row data tile of the chunk and streams its A
// operand straight from global memory in blocks of 32 coordinates (register
// double-buffered).  Per-wave fp64 sums are combined in wave order.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void tile_f32_wide(const float* __restrict__ Xp, const float* __restrict__ beta,
                                                     const float* __restrict__ Qs, const float* __restrict__ alpha,
                                                     int DP, int64_t n_pad, int n_qt32, int64_t m_pad,
                                                     double* __restrict__ partial, TileExtra ex) {
  extern __shared__ __attribute__((aligned(16))) float qlds[];
  __shared__ double wsum[4][32];
  const int H = DP / 2, LD = DP + 4;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r32 = lane & 31, h = lane >> 5;
  const int qtile = blockIdx.x % n_qt32;
  const int chunk = blockIdx.x / n_qt32;
  const int64_t col_base = (int64_t)qtile * 32;
  const int64_t qi = col_base + r32;
  if (ex.qtile_active && ex.qtile_active[col_base / kBQ] == 0) return;  // whole block
  // B operand into LDS
  {
    const f32x4* src = reinterpret_cast<const f32x4*>(Qs + col_base * DP);
    const int nv = 32 * DP / 4;
    for (int v = tid; v < nv; v += 256) {
      const int r = (v * 4) / DP, c = (v * 4) % DP;
      *reinterpret_cast<f32x4*>(&qlds[r * LD + c]) = src[v];
    }
  }
  __syncthreads();
  const float baug = h == 0 ? alpha[qi] : 1.0f;
  const float ys = kShiftMode<MODE> ? ex.yshift[qi] : 0.0f;
  const int64_t row0 = (int64_t)chunk * kChunkRows;
  const int64_t rem = (n_pad - row0) / kTileRows;
  const int ntiles = (int)(rem < kChunkRows / kTileRows ? rem : kChunkRows / kTileRows);
  const float* brow = &qlds[r32 * LD + h * H];
  double acc = acc_init<MODE>();
  __shared__ near_lds_t<MODE> near_lds;
  NearRec nr = {near_lds, 0, false};
  for (int t = wave; t < ntiles; t += 4) {
    const int64_t rb = row0 + (int64_t)t * kTileRows;
    const f32x4* arow = reinterpret_cast<const f32x4*>(Xp + (rb + r32) * DP + h * H);
    f32x16 c = {0};
    f32x4 a_cur[8], a_nxt[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a_cur[k] = arow[k];
    for (int kb = 0; kb < H; kb += 32) {
      const bool more = kb + 32 < H;
#pragma unroll
      for (int k = 0; k < 8; ++k) a_nxt[k] = more ? arow[(kb + 32) / 4 + k] : a_cur[k];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const f32x4 b4 = *reinterpret_cast<const f32x4*>(brow + kb + 4 * k);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a_cur[k].x, b4.x, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a_cur[k].y, b4.y, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a_cur[k].z, b4.z, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a_cur[k].w, b4.w, c, 0, 0, 0);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) a_cur[k] = a_nxt[k];
    }
    const float tb = beta[rb + r32];
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(h == 0 ? 1.0f : tb, baug, c, 0, 0, 0);
    acc = acc_add<MODE>(acc, (double)tile_epilogue<MODE>(c, rb, col_base, r32, h, qi, ex, nullptr, false, &nr, t, ys));
  }
  if constexpr (MODE == kModeExponential) acc += near_finish(ex, nr, qi, h, row0, tid);
  const double other = __shfl_down(acc, 32);
  if (h == 0) wsum[wave][r32] = acc_add<MODE>(acc, other);
  __syncthreads();
  if (tid < 32) {
    const double tot =
        acc_add<MODE>(acc_add<MODE>(acc_add<MODE>(wsum[0][tid], wsum[1][tid]), wsum[2][tid]), wsum[3][tid]);
    partial[(int64_t)chunk * m_pad + col_base + tid] = tot;
  }
}

// ---------------------------------------------------------------------------
// Wide rows (256 < d <= 1024), split forms (fp16 or bf16 hi + lo: three
// products per pair).  The 32 queries of a workgroup sit in LDS as hi and lo
// B operands ([2][32][DP+8] halfs, loaded once); each of the 4 waves takes
// every 4th 32-row data tile of the chunk and streams its hi and lo A
// operands from global memory, four k-steps of 16 at a time (register double
// buffered); the accumulators start from the offsets alpha_q + beta_x.  The
// epilogue is tile_epilogue in every mode, as in tile_f32_wide; per-wave fp64
// sums are combined in wave order.  DP is a multiple of 64 (so of 4 k-steps).
// ---------------------------------------------------------------------------
template <int FORM, int MODE>
__global__ __launch_bounds__(256) void tile_split_wide(const unsigned short* __restrict__ X0,
                                                       const unsigned short* __restrict__ X1,
                                                       const float* __restrict__ Xoff,
                                                       const unsigned short* __restrict__ Q0,
                                                       const unsigned short* __restrict__ Q1,
                                                       const float* __restrict__ Qoff, int DP, int64_t n_pad,
                                                       int n_qt32, int64_t m_pad, double* __restrict__ partial,
                                                       TileExtra ex) {
  static_assert(FORM == STAG_FORM_FP16_SPLIT || FORM == STAG_FORM_BF16_SPLIT, "hi + lo split forms");
  extern __shared__ __attribute__((aligned(16))) unsigned short qsh[];
  __shared__ double wsum[4][32];
  const int LD = DP + 8;
  const int KS = DP / 16;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r32 = lane & 31, h = lane >> 5;
  const int qtile = blockIdx.x % n_qt32;
  const int chunk = blockIdx.x / n_qt32;
  const int64_t col_base = (int64_t)qtile * 32;
  const int64_t qi = col_base + r32;
  if (ex.qtile_active && ex.qtile_active[col_base / kBQ] == 0) return;  // whole block
  // B operands (hi, lo) into LDS
  {
    const int nv = 32 * DP / 8;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const u16x8* src = reinterpret_cast<const u16x8*>((p == 0 ? Q0 : Q1) + col_base * DP);
      for (int v = tid; v < nv; v += 256) {
        const int r = (v * 8) / DP, c = (v * 8) % DP;
        *reinterpret_cast<u16x8*>(&qsh[(p * 32 + r) * LD + c]) = src[v];
      }
    }
  }
  __syncthreads();
  const float alpha = Qoff[qi];
  const float ys = kShiftMode<MODE> ? ex.yshift[qi] : 0.0f;
  const int64_t row0 = (int64_t)chunk * kChunkRows;
  const int64_t rem = (n_pad - row0) / kTileRows;
  const int ntiles = (int)(rem < kChunkRows / kTileRows ? rem : kChunkRows / kTileRows);
  const unsigned short* bh = &qsh[r32 * LD + h * 8];
  const unsigned short* bl = &qsh[(32 + r32) * LD + h * 8];
  double acc = acc_init<MODE>();
  __shared__ near_lds_t<MODE> near_lds;
  NearRec nr = {near_lds, 0, false};
  for (int t = wave; t < ntiles; t += 4) {
    const int64_t rb = row0 + (int64_t)t * kTileRows;
    // k-step s of row rb + r32, lane half h: dimensions [16 s + 8 h, +8)
    const u16x8* ah = reinterpret_cast<const u16x8*>(X0 + (rb + r32) * DP) + h;
    const u16x8* al = reinterpret_cast<const u16x8*>(X1 + (rb + r32) * DP) + h;
    f32x16 c;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 bv = *reinterpret_cast<const f32x4*>(Xoff + rb + 8 * q + 4 * h);
#pragma unroll
      for (int i = 0; i < 4; ++i) c[4 * q + i] = alpha + bv[i];
    }
    // blocks of four k-steps in three rotating register buffers: a block's
    // loads are issued two blocks before its products
    u16x8 bufh[3][4], bufl[3][4];
    auto load = [&](int j, int kb) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        bufh[j][k] = ah[2 * (kb + k)];
        bufl[j][k] = al[2 * (kb + k)];
      }
    };
    auto products = [&](int j, int kb) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int s16 = (kb + k) * 16;
        const u16x8 b_h = *reinterpret_cast<const u16x8*>(bh + s16);
        const u16x8 b_l = *reinterpret_cast<const u16x8*>(bl + s16);
        c = mma16<FORM>(bufh[j][k], b_h, c);
        c = mma16<FORM>(bufh[j][k], b_l, c);
        c = mma16<FORM>(bufl[j][k], b_h, c);
      }
    };
    load(0, 0);
    if (4 < KS) load(1, 4);
    if (8 < KS) load(2, 8);
    for (int kb = 0; kb < KS; kb += 12) {
      products(0, kb);
      if (kb + 12 < KS) load(0, kb + 12);
      if (kb + 4 < KS) {
        products(1, kb + 4);
        if (kb + 16 < KS) load(1, kb + 16);
      }
      if (kb + 8 < KS) {
        products(2, kb + 8);
        if (kb + 20 < KS) load(2, kb + 20);
      }
    }
    acc = acc_add<MODE>(acc, (double)tile_epilogue<MODE>(c, rb, col_base, r32, h, qi, ex, nullptr, false, &nr, t, ys));
  }
  if constexpr (MODE == kModeExponential) acc += near_finish(ex, nr, qi, h, row0, tid);
  const double other = __shfl_down(acc, 32);
  if (h == 0) wsum[wave][r32] = acc_add<MODE>(acc, other);
  __syncthreads();
  if (tid < 32) {
    const double tot =
        acc_add<MODE>(acc_add<MODE>(acc_add<MODE>(wsum[0][tid], wsum[1][tid]), wsum[2][tid]), wsum[3][tid]);
    partial[(int64_t)chunk * m_pad + col_base + tid] = tot;
  }
}

// Timer name of a launch: the underflow rescue's passes are timed apart from
// the tiles they repeat.
inline const char* rescue_timer(const TileExtra& ex, const char* name) {
  if (ex.sample) return "kde_adaptive_sample";
  return ex.max_pass ? "kde_rescue_max" : (ex.qtile_active ? "kde_rescue_sum" : name);
}

// Epilogue mode of a launch (kernel function, TileExtra outputs).
inline int tile_mode(const TileExtra& ex) {
  if (ex.max_pass) return kModeMax;
  if (ex.qtile_active) {
    if (ex.kernel == STAG_KERNEL_EXPONENTIAL) return kModeExpShift;
    if (ex.kernel == STAG_KERNEL_LOGISTIC) return kModeLogShift;
    return (ex.self || ex.tp) ? kModeGaussExtraRescue : kModeGaussRescue;
  }
  if (ex.kernel == STAG_KERNEL_EXPONENTIAL) return kModeExponential;
  if (ex.kernel == STAG_KERNEL_LOGISTIC) return kModeLogistic;
  return (ex.self || ex.tp) ? kModeGaussExtra : kModeGauss;
}

template <int DP, int MODE>
stag_status launch_tile_f32(const float* Xp, const float* beta, const float* Qs, const float* alpha, int64_t n_pad,
                            int n_qtiles, int64_t m_pad, int P, double* partial, const TileExtra& ex,
                            hipStream_t st) {
  ScopedTimer tm(rescue_timer(ex, "kde_tile_f32"), st);
  hipLaunchKernelGGL((tile_f32<DP, MODE>), dim3((unsigned)((int64_t)n_qtiles * P)), dim3(256), 0, st, Xp, beta, Qs,
                     alpha, n_pad, n_qtiles, m_pad, partial, ex);
  return check_launch("tile_f32");
}

template <int FORM, int DP, int MODE>
stag_status launch_tile_split(void* const* xp, const float* xaug, void* const* qp, const float* qaug, int64_t n_pad,
                              int n_qtiles, int64_t m_pad, int P, double* partial, const TileExtra& ex,
                              hipStream_t st) {
  using U = const unsigned short*;
  if constexpr (MODE == kModeGauss && FORM != STAG_FORM_BF16_SPLIT3 && DP >= 64 && DP <= 128) {
    // 64 queries per wave (the same results, fewer LDS reads per product)
    ScopedTimer tm(FORM == STAG_FORM_FP16_SPLIT ? "kde_tile_fp16x3" : "kde_tile_bf16x3", st);
    const int n_qt256 = (int)ceil_div(m_pad, 256);
    hipLaunchKernelGGL((tile_split_w64<FORM, DP, MODE>), dim3((unsigned)((int64_t)n_qt256 * P)), dim3(256), 0, st,
                       (U)xp[0], (U)xp[1], xaug, (U)qp[0], (U)qp[1], qaug, n_pad, n_qt256, m_pad, partial, ex);
    (void)n_qtiles;
    return check_launch("tile_split_w64");
  }
  ScopedTimer tm(rescue_timer(ex, FORM == STAG_FORM_FP16_SPLIT
                                     ? "kde_tile_fp16x3"
                                     : (FORM == STAG_FORM_BF16_SPLIT ? "kde_tile_bf16x3" : "kde_tile_bf16x6")),
                 st);
  hipLaunchKernelGGL((tile_split<FORM, DP, MODE>), dim3((unsigned)((int64_t)n_qtiles * P)), dim3(256), 0, st,
                     (U)xp[0], (U)xp[1], (U)xp[2], xaug, (U)qp[0], (U)qp[1], (U)qp[2], qaug, n_pad, n_qtiles, m_pad,
                     partial, ex);
  return check_launch("tile_split");
}

template <int FORM, int MODE>
stag_status dispatch_split(int dp, void* const* xp, const float* xaug, void* const* qp, const float* qaug,
                           int64_t n_pad, int n_qtiles, int64_t m_pad, int P, double* partial, const TileExtra& ex,
                           hipStream_t st) {
  switch (dp) {
    case 16: return launch_tile_split<FORM, 16, MODE>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 32: return launch_tile_split<FORM, 32, MODE>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 64: return launch_tile_split<FORM, 64, MODE>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 96: return launch_tile_split<FORM, 96, MODE>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 128: return launch_tile_split<FORM, 128, MODE>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 160: return launch_tile_split<FORM, 160, MODE>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 192: return launch_tile_split<FORM, 192, MODE>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 224: return launch_tile_split<FORM, 224, MODE>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 256: return launch_tile_split<FORM, 256, MODE>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
  }
  return fail(STAG_E_UNSUPPORTED, "padded dimension %d not instantiated", dp);
}

template <int MODE>
stag_status dispatch_f32(int dp, const float* Xp, const float* beta, const float* Qs, const float* alpha,
                         int64_t n_pad, int n_qtiles, int64_t m_pad, int P, double* partial, const TileExtra& ex,
                         hipStream_t st) {
  switch (dp) {
    case 16: return launch_tile_f32<16, MODE>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 32: return launch_tile_f32<32, MODE>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 64: return launch_tile_f32<64, MODE>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 96: return launch_tile_f32<96, MODE>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 128: return launch_tile_f32<128, MODE>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 160: return launch_tile_f32<160, MODE>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 192: return launch_tile_f32<192, MODE>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 224: return launch_tile_f32<224, MODE>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 256: return launch_tile_f32<256, MODE>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
  }
  return fail(STAG_E_UNSUPPORTED, "padded dimension %d not instantiated", dp);
}
template <int DP, int MODE>
stag_status launch_tile_f32c(const Operands& xo, const Operands& qo, float la, int n_qtiles, int P, double* partial,
                             const TileExtra& ex, hipStream_t st) {
  ScopedTimer tm(rescue_timer(ex, "kde_tile_f32c"), st);
  hipLaunchKernelGGL((tile_f32c<DP, MODE>), dim3((unsigned)((int64_t)n_qtiles * P)), dim3(256), 0, st,
                     (const float*)xo.part[0], xo.off, xo.centre, xo.radius, xo.n_pad_dev, (const float*)qo.part[0],
                     qo.off, la, n_qtiles, qo.rows_pad, partial, ex);
  return check_launch("tile_f32c");
}

template <int MODE>
stag_status dispatch_f32c(const Operands& xo, const Operands& qo, float la, int n_qtiles, int P, double* partial,
                          const TileExtra& ex, hipStream_t st) {
  switch (xo.dp) {
    case 16: return launch_tile_f32c<16, MODE>(xo, qo, la, n_qtiles, P, partial, ex, st);
    case 32: return launch_tile_f32c<32, MODE>(xo, qo, la, n_qtiles, P, partial, ex, st);
    case 64: return launch_tile_f32c<64, MODE>(xo, qo, la, n_qtiles, P, partial, ex, st);
    case 96: return launch_tile_f32c<96, MODE>(xo, qo, la, n_qtiles, P, partial, ex, st);
    case 128: return launch_tile_f32c<128, MODE>(xo, qo, la, n_qtiles, P, partial, ex, st);
    case 160: return launch_tile_f32c<160, MODE>(xo, qo, la, n_qtiles, P, partial, ex, st);
    case 192: return launch_tile_f32c<192, MODE>(xo, qo, la, n_qtiles, P, partial, ex, st);
    case 224: return launch_tile_f32c<224, MODE>(xo, qo, la, n_qtiles, P, partial, ex, st);
    case 256: return launch_tile_f32c<256, MODE>(xo, qo, la, n_qtiles, P, partial, ex, st);
  }
  return fail(STAG_E_UNSUPPORTED, "padded dimension %d not instantiated", xo.dp);
}

template <int DP, int MODE>
stag_status launch_tile_h1c(const Operands& xo, const Operands& qo, float la, int P, double* partial,
                            const TileExtra& ex, hipStream_t st) {
  ScopedTimer tm(rescue_timer(ex, "kde_tile_fp16c"), st);
  const int n_qtw = (int)ceil_div(qo.rows_pad, 128 * kH1cBlocks<DP>);
  // a list of 128-query tiles becomes the list of the workgroup tiles that
  // hold them (ascending, each once); the mask still marks the active ones
  TileExtra e = ex;
  int nw = n_qtw;
  if (ex.qsel_n > 0) {
    int n = 0;
    for (int i = 0; i < ex.qsel_n; ++i) {
      const int w = ex.qsel[i] / kH1cBlocks<DP>;
      if (w < n_qtw && (n == 0 || e.qsel[n - 1] < w)) e.qsel[n++] = w;
    }
    e.qsel_n = n;
    nw = n;
  }
  if (nw == 0) return STAG_OK;
  // the full grid in the XCD-aware order: 8 ceil(n_qtw / 8) P workgroups
  if (ex.qsel_n == 0) nw = 8 * (int)ceil_div(n_qtw, 8);
  e.h1c_chunks = P;
  hipLaunchKernelGGL((tile_h1c<DP, MODE>), dim3((unsigned)((int64_t)nw * P)), dim3(256), 0, st,
                     static_cast<const unsigned short*>(xo.part[0]), xo.off, xo.tgroup, xo.centre, xo.radius,
                     xo.n_pad_dev, (const float*)qo.part[0], qo.off, la, n_qtw, qo.rows_pad, partial, e);
  return check_launch("tile_h1c");
}

template <int MODE>
stag_status dispatch_h1c(const Operands& xo, const Operands& qo, float la, int P, double* partial,
                         const TileExtra& ex, hipStream_t st) {
  switch (xo.dp) {
    case 16: return launch_tile_h1c<16, MODE>(xo, qo, la, P, partial, ex, st);
    case 32: return launch_tile_h1c<32, MODE>(xo, qo, la, P, partial, ex, st);
    case 64: return launch_tile_h1c<64, MODE>(xo, qo, la, P, partial, ex, st);
    case 96: return launch_tile_h1c<96, MODE>(xo, qo, la, P, partial, ex, st);
    case 128: return launch_tile_h1c<128, MODE>(xo, qo, la, P, partial, ex, st);
    case 160: return launch_tile_h1c<160, MODE>(xo, qo, la, P, partial, ex, st);
    case 192: return launch_tile_h1c<192, MODE>(xo, qo, la, P, partial, ex, st);
    case 224: return launch_tile_h1c<224, MODE>(xo, qo, la, P, partial, ex, st);
    case 256: return launch_tile_h1c<256, MODE>(xo, qo, la, P, partial, ex, st);
  }
  return fail(STAG_E_UNSUPPORTED, "padded dimension %d not instantiated", xo.dp);
}

// All tiles of one launch in epilogue mode MODE: wide fp32 rows, the fp32
// tile, the centred fp32 tile or a split form, by padded dimension.
template <int MODE>
stag_status launch_tiles(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                         hipStream_t st) {
  const int P = (int)exact_chunks(xo.rows_pad);
  const int n_qtiles = (int)(qo.rows_pad / kBQ);
  if (xo.centred) {
    if constexpr (MODE == kModeGauss || MODE == kModeGaussRescue || MODE == kModeMax) {
      if (xo.form == STAG_FORM_FP16_CENTRED)
        return dispatch_h1c<MODE>(xo, qo, (float)(ex.a * kLog2e), P, partial, ex, st);
      return dispatch_f32c<MODE>(xo, qo, (float)(ex.a * kLog2e), n_qtiles, P, partial, ex, st);
    } else {
      return fail(STAG_E_UNSUPPORTED, "centred data: Gaussian sums only");
    }
  }
  if (xo.dp > 256 && (xo.form == STAG_FORM_FP16_SPLIT || xo.form == STAG_FORM_BF16_SPLIT)) {
    const int n_qt32 = (int)(qo.rows_pad / 32);
    const size_t lds = (size_t)2 * 32 * (xo.dp + 8) * sizeof(unsigned short);
    using U = const unsigned short*;
    if (xo.form == STAG_FORM_FP16_SPLIT) {
      STAG_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tile_split_wide<STAG_FORM_FP16_SPLIT, MODE>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      ScopedTimer tm(rescue_timer(ex, "kde_tile_fp16x3_wide"), st);
      hipLaunchKernelGGL((tile_split_wide<STAG_FORM_FP16_SPLIT, MODE>), dim3((unsigned)((int64_t)n_qt32 * P)),
                         dim3(256), lds, st, (U)xo.part[0], (U)xo.part[1], xo.off, (U)qo.part[0], (U)qo.part[1],
                         qo.off, xo.dp, xo.rows_pad, n_qt32, qo.rows_pad, partial, ex);
    } else {
      STAG_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tile_split_wide<STAG_FORM_BF16_SPLIT, MODE>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      ScopedTimer tm(rescue_timer(ex, "kde_tile_bf16x3_wide"), st);
      hipLaunchKernelGGL((tile_split_wide<STAG_FORM_BF16_SPLIT, MODE>), dim3((unsigned)((int64_t)n_qt32 * P)),
                         dim3(256), lds, st, (U)xo.part[0], (U)xo.part[1], xo.off, (U)qo.part[0], (U)qo.part[1],
                         qo.off, xo.dp, xo.rows_pad, n_qt32, qo.rows_pad, partial, ex);
    }
    return check_launch("tile_split_wide");
  }
  if (xo.dp > 256) {
    if (xo.form != STAG_FORM_FP32) return fail(STAG_E_UNSUPPORTED, "d > 256 needs the fp32, fp16 split or bf16 split form");
    const int n_qt32 = (int)(qo.rows_pad / 32);
    const size_t lds = (size_t)32 * (xo.dp + 4) * sizeof(float);
    STAG_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tile_f32_wide<MODE>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    ScopedTimer tm(rescue_timer(ex, "kde_tile_f32_wide"), st);
    hipLaunchKernelGGL(tile_f32_wide<MODE>, dim3((unsigned)((int64_t)n_qt32 * P)), dim3(256), lds, st,
                       (const float*)xo.part[0], xo.off, (const float*)qo.part[0], qo.off, xo.dp, xo.rows_pad,
                       n_qt32, qo.rows_pad, partial, ex);
    return check_launch("tile_f32_wide");
  }
  if (xo.form == STAG_FORM_FP32)
    return dispatch_f32<MODE>(xo.dp, (const float*)xo.part[0], xo.off, (const float*)qo.part[0], qo.off,
                              xo.rows_pad, n_qtiles, qo.rows_pad, P, partial, ex, st);
  switch (xo.form) {
    case STAG_FORM_BF16_SPLIT:
      return dispatch_split<STAG_FORM_BF16_SPLIT, MODE>(xo.dp, xo.part, xo.off, qo.part, qo.off, xo.rows_pad,
                                                        n_qtiles, qo.rows_pad, P, partial, ex, st);
    case STAG_FORM_FP16_SPLIT:
      return dispatch_split<STAG_FORM_FP16_SPLIT, MODE>(xo.dp, xo.part, xo.off, qo.part, qo.off, xo.rows_pad,
                                                        n_qtiles, qo.rows_pad, P, partial, ex, st);
    default:
      return dispatch_split<STAG_FORM_BF16_SPLIT3, MODE>(xo.dp, xo.part, xo.off, qo.part, qo.off, xo.rows_pad,
                                                         n_qtiles, qo.rows_pad, P, partial, ex, st);
  }
}

}  // namespace tiles

// Per-mode entry points (one translation unit each).
stag_status launch_tiles_gauss(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                               hipStream_t st);
stag_status launch_tiles_gauss_extra(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                                     hipStream_t st);
stag_status launch_tiles_exponential(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                                     hipStream_t st);
stag_status launch_tiles_logistic(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                                  hipStream_t st);
stag_status launch_tiles_max(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                             hipStream_t st);
stag_status launch_tiles_gauss_rescue(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                                      hipStream_t st);
stag_status launch_tiles_gauss_extra_rescue(const Operands& xo, const Operands& qo, double* partial,
                                            const TileExtra& ex, hipStream_t st);
stag_status launch_tiles_exp_shift(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                                   hipStream_t st);
stag_status launch_tiles_log_shift(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                                   hipStream_t st);

}  // namespace stag
