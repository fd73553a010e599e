// Exact Gaussian kernel density on the gfx950 matrix cores.
//
// S(q) = sum_i exp(-a ||q - x_i||^2)   (Sec. "Kernel Density Estimation": the
// density K(q) = S(q)/n; ExactGaussianKDE evaluates it naively in O(dmn)).
//
// The squared distance is expanded, ||q-x||^2 = ||q||^2 + ||x||^2 - 2 q.x,
// and the whole exponent in base 2,
//     E = log2(e) * (-a ||q||^2 - a ||x||^2 + 2a q.x) = alpha_q + beta_x + (s q).x,
// s = 2a log2(e), is produced by the matrix cores: the cross term from the
// (split) operands, alpha and beta through one extra augmentation step whose
// operands pair each of them with 1.0.  The epilogue is then just
// k = exp2(E) and a row sum, per lane, with no cross-lane traffic per tile.
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
#include "runtime.h"
#include "kde_exact.h"

namespace stag {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

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

// Kernel values of one 32x32 accumulator tile held by a lane (16 exponents),
// summed as a balanced tree in fp32.
__device__ inline float exp2_tile_sum(const float* c) {
  float k[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) k[i] = __builtin_amdgcn_exp2f(c[i]);
#pragma unroll
  for (int w = 8; w > 0; w >>= 1)
#pragma unroll
    for (int i = 0; i < w; ++i) k[i] = k[i] + k[i + w];
  return k[0];
}

// A lane's tile sums of 8 consecutive data tiles (global tile indices
// 8g .. 8g+7), written to tp as two 16-byte stores once the group is complete
// (or the chunk ends): the row stride of tp is a multiple of 8 tiles.
struct TileSums8 {
  float v[8];
};

// Epilogue of one finished 32x32 tile held by a lane (column qi, half h):
// exp2 and fp32 tree sum; with EXTRA, optionally drops the diagonal element
// (data row == query index, for a data set queried against itself) and
// records the tile's 32-row partial sum (both halves, fixed order), through
// the group buffer `grp` when the caller walks tiles in order (`last` marks
// the chunk's final tile), else with a direct store.
template <bool EXTRA>
__device__ inline float tile_epilogue(const f32x16& c, int64_t row_base, int64_t col_base, int r32, int h,
                                      int64_t qi, const TileExtra& ex, TileSums8* grp = nullptr,
                                      bool last = false) {
  float cp[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) cp[i] = c[i];
  if constexpr (EXTRA) {
    if (ex.self && row_base == col_base) {
      // lane (column r32, half h) holds rows 8(i/4) + 4h + i%4
      const int idg = 4 * (r32 >> 3) + (r32 & 3);
      const bool mine = h == ((r32 & 7) >> 2);
#pragma unroll
      for (int i = 0; i < 16; ++i) cp[i] = (mine && i == idg) ? kPadOffset : cp[i];
    }
  }
  const float s = exp2_tile_sum(cp);
  if constexpr (EXTRA) {
    if (ex.tp) {
      const float o = __shfl_xor(s, 32);
      const float tot = h == 0 ? s + o : o + s;
      const int64_t tile = row_base / kTileRows;
      if (grp == nullptr) {
        if (h == 0) ex.tp[qi * ex.ntile + tile] = tot;
      } else {
        const int k = (int)(tile & 7);
#pragma unroll
        for (int e = 0; e < 8; ++e) grp->v[e] = e == k ? tot : grp->v[e];
        if ((k == 7 || last) && h == 0) {
          f32x4* dst = reinterpret_cast<f32x4*>(ex.tp + qi * ex.ntile + (tile & ~(int64_t)7));
          dst[0] = f32x4{grp->v[0], grp->v[1], grp->v[2], grp->v[3]};
          dst[1] = f32x4{grp->v[4], grp->v[5], grp->v[6], grp->v[7]};
        }
      }
    }
  }
  return s;
}

// Split v into parts of the form's element type: v ~= p0 + p1 (+ p2); each
// remainder is exact in fp32 (Sterbenz), so only the last part is rounded.
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
constexpr int kPrepRowsPerWave = 16;
constexpr int kPrepRowsPerBlock = 4 * kPrepRowsPerWave;

template <int FORM>
__global__ __launch_bounds__(256) void prep_rows(const float* __restrict__ src, int64_t n, int d, int dp,
                                                 int64_t rows_pad, double scale, double neg_a_log2e,
                                                 int is_query, void* __restrict__ part0, void* __restrict__ part1,
                                                 void* __restrict__ part2, float* __restrict__ off,
                                                 u16x8* __restrict__ aug, double* __restrict__ nrm,
                                                 unsigned long long* __restrict__ max_nrm_bits) {
  __shared__ double wmax[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double mx = 0.0;
  for (int rr = 0; rr < kPrepRowsPerWave; ++rr) {
    const int64_t row = (int64_t)blockIdx.x * kPrepRowsPerBlock + wave * kPrepRowsPerWave + rr;
    if (row >= rows_pad) break;
    const bool real = row < n;
    double sq = 0.0;
    for (int j = lane; j < dp; j += 64) {
      float v = 0.0f;
      if (real && j < d) v = src[row * d + j];
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
template <int DP, bool EXTRA>
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

  double acc = 0.0;
  TileSums8 grp = {};
  auto step = [&](int t, const f32x16& cdone, f32x16& cnew) {
    const int buf = t & 1;
    __syncthreads();
    if constexpr (EXTRA) {
      if (t > 0)
        acc += (double)tile_epilogue<true>(cdone, row0 + (int64_t)(t - 1) * kTileRows, col_base, r32, h, qi, ex, &grp);
    } else {
      acc += (double)tile_epilogue<false>(cdone, 0, 0, r32, h, qi, ex);
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
  for (int i = 0; i < 16; ++i) ca[i] = kPadOffset;  // exp2 -> 0: neutral first epilogue
  int t = 0;
  for (; t + 1 < ntiles; t += 2) {
    step(t, ca, cb);
    step(t + 1, cb, ca);
  }
  if (t < ntiles) {
    step(t, ca, cb);
    ca = cb;
  }
  acc += (double)tile_epilogue<EXTRA>(ca, row0 + (int64_t)(ntiles - 1) * kTileRows, col_base, r32, h, qi, ex, &grp,
                                     true);
  const double other = __shfl_down(acc, 32);
  if (h == 0) partial[(int64_t)chunk * m_pad + qi] = acc + other;
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

template <int FORM, int DP, bool EXTRA>
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

  const unsigned short* Qp[3] = {Q0, Q1, Q2};
  const unsigned short* Xpp[3] = {X0, X1, X2};
  u16x8 bq[NP][KS];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int s = 0; s < KS; ++s)
      bq[p][s] = *reinterpret_cast<const u16x8*>(Qp[p] + qi * DP + s * 16 + h * 8);
  const float alpha = Qoff[qi];

  const int64_t row0 = (int64_t)chunk * kChunkRows;
  const int64_t rem = (n_pad - row0) / kTileRows;
  const int ntiles = (int)(rem < kChunkRows / kTileRows ? rem : kChunkRows / kTileRows);

  u16x8 stage[NP][NLD];
  float sbeta;
  auto gload = [&](int t) {
    const int64_t base = (row0 + (int64_t)t * kTileRows) * DP;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int k = 0; k < NLD; ++k)
        stage[p][k] = reinterpret_cast<const u16x8*>(Xpp[p] + base)[min(tid + 256 * k, NV - 1)];
    sbeta = Xoff[row0 + (int64_t)t * kTileRows + (tid & 31)];
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

  double acc = 0.0;
  TileSums8 grp = {};
  auto step = [&](int t, const f32x16& cdone, f32x16& cnew) {
    const int buf = t & 1;
    __syncthreads();
    if constexpr (EXTRA) {
      if (t > 0)
        acc += (double)tile_epilogue<true>(cdone, row0 + (int64_t)(t - 1) * kTileRows, col_base, r32, h, qi, ex, &grp);
    } else {
      acc += (double)tile_epilogue<false>(cdone, 0, 0, r32, h, qi, ex);
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
  for (int i = 0; i < 16; ++i) ca[i] = kPadOffset;  // exp2 -> 0: neutral first epilogue
  int t = 0;
  for (; t + 1 < ntiles; t += 2) {
    step(t, ca, cb);
    step(t + 1, cb, ca);
  }
  if (t < ntiles) {
    step(t, ca, cb);
    ca = cb;
  }
  acc += (double)tile_epilogue<EXTRA>(ca, row0 + (int64_t)(ntiles - 1) * kTileRows, col_base, r32, h, qi, ex, &grp,
                                     true);
  const double other = __shfl_down(acc, 32);
  if (h == 0) partial[(int64_t)chunk * m_pad + qi] = acc + other;
}

// ---------------------------------------------------------------------------
// Wide rows (256 < d <= 1024), fp32 form.  The 32 queries of a workgroup sit
// in LDS as the B operand ([32][DP+4] floats, loaded once); each of the 4
// waves takes every 4th 32-row data tile of the chunk and streams its A
// operand straight from global memory in blocks of 32 coordinates (register
// double-buffered).  Per-wave fp64 sums are combined in wave order.
// ---------------------------------------------------------------------------
template <bool EXTRA>
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
  const int64_t row0 = (int64_t)chunk * kChunkRows;
  const int64_t rem = (n_pad - row0) / kTileRows;
  const int ntiles = (int)(rem < kChunkRows / kTileRows ? rem : kChunkRows / kTileRows);
  const float* brow = &qlds[r32 * LD + h * H];
  double acc = 0.0;
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
    acc += (double)tile_epilogue<EXTRA>(c, rb, col_base, r32, h, qi, ex);
  }
  const double other = __shfl_down(acc, 32);
  if (h == 0) wsum[wave][r32] = acc + other;
  __syncthreads();
  if (tid < 32) {
    const double tot = ((wsum[0][tid] + wsum[1][tid]) + wsum[2][tid]) + wsum[3][tid];
    partial[(int64_t)chunk * m_pad + col_base + tid] = tot;
  }
}

// S(q) = sum of chunk partials in chunk order; optional 1/n; a-priori bound.
__global__ void reduce_partials(const double* __restrict__ partial, int P, int64_t m_pad, int64_t m, double scale,
                                const double* __restrict__ qnrm, const unsigned long long* __restrict__ max_xnrm_bits,
                                BoundModel bm, double* __restrict__ S_out, double* __restrict__ bound_out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  double s = 0.0;
  for (int p = 0; p < P; ++p) s += partial[(int64_t)p * m_pad + q];
  S_out[q] = s * scale;
  if (bound_out) {
    const double xm = __longlong_as_double((long long)*max_xnrm_bits);
    bound_out[q] = relative_bound(bm, qnrm[q], xm);
  }
}

template <int DP>
stag_status launch_tile_f32(const float* Xp, const float* beta, const float* Qs, const float* alpha, int64_t n_pad,
                            int n_qtiles, int64_t m_pad, int P, double* partial, const TileExtra& ex,
                            hipStream_t st) {
  ScopedTimer tm("kde_tile_f32", st);
  if (ex.self || ex.tp)
    hipLaunchKernelGGL((tile_f32<DP, true>), dim3((unsigned)((int64_t)n_qtiles * P)), dim3(256), 0, st, Xp, beta, Qs,
                       alpha, n_pad, n_qtiles, m_pad, partial, ex);
  else
    hipLaunchKernelGGL((tile_f32<DP, false>), dim3((unsigned)((int64_t)n_qtiles * P)), dim3(256), 0, st, Xp, beta,
                       Qs, alpha, n_pad, n_qtiles, m_pad, partial, ex);
  return check_launch("tile_f32");
}

template <int FORM, int DP>
stag_status launch_tile_split(void* const* xp, const float* xaug, void* const* qp, const float* qaug, int64_t n_pad,
                              int n_qtiles, int64_t m_pad, int P, double* partial, const TileExtra& ex,
                              hipStream_t st) {
  using U = const unsigned short*;
  ScopedTimer tm(FORM == STAG_FORM_FP16_SPLIT ? "kde_tile_fp16x3" : (FORM == STAG_FORM_BF16_SPLIT ? "kde_tile_bf16x3" : "kde_tile_bf16x6"), st);
  if (ex.self || ex.tp)
    hipLaunchKernelGGL((tile_split<FORM, DP, true>), dim3((unsigned)((int64_t)n_qtiles * P)), dim3(256), 0, st,
                       (U)xp[0], (U)xp[1], (U)xp[2], xaug, (U)qp[0], (U)qp[1], (U)qp[2], qaug, n_pad, n_qtiles, m_pad,
                       partial, ex);
  else
    hipLaunchKernelGGL((tile_split<FORM, DP, false>), dim3((unsigned)((int64_t)n_qtiles * P)), dim3(256), 0, st,
                       (U)xp[0], (U)xp[1], (U)xp[2], xaug, (U)qp[0], (U)qp[1], (U)qp[2], qaug, n_pad, n_qtiles, m_pad,
                       partial, ex);
  return check_launch("tile_split");
}

template <int FORM>
stag_status dispatch_split(int dp, void* const* xp, const float* xaug, void* const* qp, const float* qaug,
                           int64_t n_pad, int n_qtiles, int64_t m_pad, int P, double* partial, const TileExtra& ex,
                           hipStream_t st) {
  switch (dp) {
    case 16: return launch_tile_split<FORM, 16>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 32: return launch_tile_split<FORM, 32>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 64: return launch_tile_split<FORM, 64>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 96: return launch_tile_split<FORM, 96>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 128: return launch_tile_split<FORM, 128>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 160: return launch_tile_split<FORM, 160>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 192: return launch_tile_split<FORM, 192>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 224: return launch_tile_split<FORM, 224>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 256: return launch_tile_split<FORM, 256>(xp, xaug, qp, qaug, n_pad, n_qtiles, m_pad, P, partial, ex, st);
  }
  return fail(STAG_E_UNSUPPORTED, "padded dimension %d not instantiated", dp);
}

stag_status dispatch_f32(int dp, const float* Xp, const float* beta, const float* Qs, const float* alpha,
                         int64_t n_pad, int n_qtiles, int64_t m_pad, int P, double* partial, const TileExtra& ex,
                         hipStream_t st) {
  switch (dp) {
    case 16: return launch_tile_f32<16>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 32: return launch_tile_f32<32>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 64: return launch_tile_f32<64>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 96: return launch_tile_f32<96>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 128: return launch_tile_f32<128>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 160: return launch_tile_f32<160>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 192: return launch_tile_f32<192>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 224: return launch_tile_f32<224>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
    case 256: return launch_tile_f32<256>(Xp, beta, Qs, alpha, n_pad, n_qtiles, m_pad, P, partial, ex, st);
  }
  return fail(STAG_E_UNSUPPORTED, "padded dimension %d not instantiated", dp);
}

template <int FORM>
stag_status launch_prep(const float* src, int64_t n, int d, int dp, int64_t rows_pad, double scale, double neg_a_l2e,
                        int is_query, void* const* parts, float* off, u16x8* aug, double* nrm,
                        unsigned long long* maxbits, hipStream_t st) {
  ScopedTimer tm("kde_prep", st);
  hipLaunchKernelGGL(prep_rows<FORM>, dim3((unsigned)ceil_div(rows_pad, kPrepRowsPerBlock)), dim3(256), 0, st, src,
                     n, d, dp,
                     rows_pad, scale, neg_a_l2e, is_query, parts[0], parts[1], parts[2], off, aug, nrm, maxbits);
  return check_launch("prep_rows");
}

stag_status prep_any(int form, const float* src, int64_t n, int d, int dp, int64_t rows_pad, double scale,
                     double neg_a_l2e, int is_query, void* const* parts, float* off, u16x8* aug, double* nrm,
                     unsigned long long* maxbits, hipStream_t st) {
  switch (form) {
    case STAG_FORM_FP32:
      return launch_prep<STAG_FORM_FP32>(src, n, d, dp, rows_pad, scale, neg_a_l2e, is_query, parts, off, aug, nrm,
                                         maxbits, st);
    case STAG_FORM_BF16_SPLIT:
      return launch_prep<STAG_FORM_BF16_SPLIT>(src, n, d, dp, rows_pad, scale, neg_a_l2e, is_query, parts, off, aug,
                                               nrm, maxbits, st);
    case STAG_FORM_FP16_SPLIT:
      return launch_prep<STAG_FORM_FP16_SPLIT>(src, n, d, dp, rows_pad, scale, neg_a_l2e, is_query, parts, off, aug,
                                               nrm, maxbits, st);
    default:
      return launch_prep<STAG_FORM_BF16_SPLIT3>(src, n, d, dp, rows_pad, scale, neg_a_l2e, is_query, parts, off, aug,
                                                nrm, maxbits, st);
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

stag_status prepare_operands(int form, const float* src, int64_t rows, int d, double a, bool is_query,
                             Workspace& ws, Operands* out, hipStream_t st) {
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
  if (!is_query) {
    STAG_TRY(ws.alloc(&out->max_nrm_bits, 1));
    STAG_HIP(hipMemsetAsync(out->max_nrm_bits, 0, sizeof(unsigned long long), st));
  }
  const double scale = is_query ? 2.0 * a * kLog2e : 1.0;
  return prep_any(form, src, rows, d, dp, rows_pad, scale, -a * kLog2e, is_query ? 1 : 0, out->part, out->off,
                  static_cast<u16x8*>(out->aug), out->nrm, out->max_nrm_bits, st);
}

int64_t exact_chunks(int64_t n_pad) { return ceil_div(n_pad, kChunkRows); }

stag_status prep_query_into(int form, const float* src, int64_t rows, int d, double a, const Operands& batch,
                            int64_t row0, hipStream_t st) {
  const int dp = batch.dp;
  const int64_t rows_pad = round_up(rows, kBQ);
  const size_t eb = form_element_bytes(form);
  void* parts[3] = {nullptr, nullptr, nullptr};
  for (int p = 0; p < form_parts(form); ++p)
    parts[p] = static_cast<char*>(batch.part[p]) + (size_t)row0 * dp * eb;
  u16x8* aug = batch.aug ? static_cast<u16x8*>(batch.aug) + row0 : nullptr;
  return prep_any(form, src, rows, d, dp, rows_pad, 2.0 * a * kLog2e, -a * kLog2e, 1, parts, batch.off + row0, aug,
                  batch.nrm ? batch.nrm + row0 : nullptr, nullptr, st);
}

int64_t query_tile_rows() { return kBQ; }

stag_status launch_exact_tiles(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                               hipStream_t st) {
  const int P = (int)exact_chunks(xo.rows_pad);
  const int n_qtiles = (int)(qo.rows_pad / kBQ);
  if (xo.dp > 256) {
    if (xo.form != STAG_FORM_FP32) return fail(STAG_E_UNSUPPORTED, "d > 256 needs the fp32 form");
    const int n_qt32 = (int)(qo.rows_pad / 32);
    const size_t lds = (size_t)32 * (xo.dp + 4) * sizeof(float);
    STAG_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tile_f32_wide<true>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    STAG_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tile_f32_wide<false>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    ScopedTimer tm("kde_tile_f32_wide", st);
    if (ex.self || ex.tp)
      hipLaunchKernelGGL(tile_f32_wide<true>, dim3((unsigned)((int64_t)n_qt32 * P)), dim3(256), lds, st,
                         (const float*)xo.part[0], xo.off, (const float*)qo.part[0], qo.off, xo.dp, xo.rows_pad,
                         n_qt32, qo.rows_pad, partial, ex);
    else
      hipLaunchKernelGGL(tile_f32_wide<false>, dim3((unsigned)((int64_t)n_qt32 * P)), dim3(256), lds, st,
                         (const float*)xo.part[0], xo.off, (const float*)qo.part[0], qo.off, xo.dp, xo.rows_pad,
                         n_qt32, qo.rows_pad, partial, ex);
    return check_launch("tile_f32_wide");
  }
  if (xo.form == STAG_FORM_FP32)
    return dispatch_f32(xo.dp, (const float*)xo.part[0], xo.off, (const float*)qo.part[0], qo.off, xo.rows_pad,
                        n_qtiles, qo.rows_pad, P, partial, ex, st);
  const float* xaug = xo.off;
  const float* qaug = qo.off;
  switch (xo.form) {
    case STAG_FORM_BF16_SPLIT:
      return dispatch_split<STAG_FORM_BF16_SPLIT>(xo.dp, xo.part, xaug, qo.part, qaug, xo.rows_pad, n_qtiles,
                                                  qo.rows_pad, P, partial, ex, st);
    case STAG_FORM_FP16_SPLIT:
      return dispatch_split<STAG_FORM_FP16_SPLIT>(xo.dp, xo.part, xaug, qo.part, qaug, xo.rows_pad, n_qtiles,
                                                  qo.rows_pad, P, partial, ex, st);
    default:
      return dispatch_split<STAG_FORM_BF16_SPLIT3>(xo.dp, xo.part, xaug, qo.part, qaug, xo.rows_pad, n_qtiles,
                                                   qo.rows_pad, P, partial, ex, st);
  }
}

stag_status launch_reduce(const double* partial, int P, const Operands& qo, const Operands& xo, double scale,
                          const BoundModel& bm, double* S_out, double* bound_out, hipStream_t st) {
  const int64_t m = qo.rows;
  ScopedTimer tm("kde_reduce", st);
  hipLaunchKernelGGL(reduce_partials, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, partial, P, qo.rows_pad, m,
                     scale, qo.nrm, xo.max_nrm_bits, bm, S_out, bound_out);
  return check_launch("reduce_partials");
}

BoundModel make_bound_model(int form, int d, double a) {
  BoundModel bm;
  const double u = 0x1.0p-24;
  bm.la = a * kLog2e;
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
  return bm;
}

}  // namespace stag

extern "C" stag_status stag_kde_exact(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, double a,
                                      double eps, int32_t form, uint32_t flags, double* S_out, double* bound_out,
                                      hipStream_t stream) {
  using namespace stag;
  (void)eps;
  if (!X || !Q || !S_out) return fail(STAG_E_INVAL, "stag_kde_exact: NULL pointer argument");
  if (n < 1 || m < 1 || d < 1) return fail(STAG_E_INVAL, "stag_kde_exact: n, m, d must be >= 1");
  if (!(a > 0.0) || !std::isfinite(a)) return fail(STAG_E_INVAL, "stag_kde_exact: a must be positive and finite");
  if (form < STAG_FORM_FP32 || form > STAG_FORM_BF16_SPLIT3)
    return fail(STAG_E_INVAL, "stag_kde_exact: unknown form %d", form);
  if (flags & ~STAG_NORMALIZE) return fail(STAG_E_INVAL, "stag_kde_exact: unknown flags 0x%x", flags);
  if (d > 1024) return fail(STAG_E_UNSUPPORTED, "stag_kde_exact: d = %d > 1024 is not supported", d);
  if (d > 256 && form != STAG_FORM_FP32)
    return fail(STAG_E_UNSUPPORTED, "stag_kde_exact: d = %d > 256 is supported by the fp32 form only", d);
  if ((double)n * d >= 2147483648.0 || (double)m * d >= 2147483648.0)
    return fail(STAG_E_INVAL, "stag_kde_exact: n*d and m*d must be < 2^31");
  clear_error();
  Workspace ws(stream);
  Operands xo, qo;
  STAG_TRY(prepare_operands(form, X, n, d, a, false, ws, &xo, stream));
  STAG_TRY(prepare_operands(form, Q, m, d, a, true, ws, &qo, stream));
  const int P = (int)exact_chunks(xo.rows_pad);
  double* partial = nullptr;
  STAG_TRY(ws.alloc(&partial, (size_t)P * qo.rows_pad));
  STAG_TRY(launch_exact_tiles(xo, qo, partial, TileExtra{}, stream));
  const double scale = (flags & STAG_NORMALIZE) ? 1.0 / (double)n : 1.0;
  STAG_TRY(launch_reduce(partial, P, qo, xo, scale, make_bound_model(form, d, a), S_out, bound_out, stream));
  return STAG_OK;
}
