// Centring of the data for the fp32 and fp16 centred exact tiles (operand
// preparation: the reorder of the rows into groups and their centres).
//
// The exact tile expands ||q - x||^2 around a centre.  Around the origin the
// accumulators carry a(||q||^2 + ||x||^2), which for clustered data far from
// the origin is much larger than the exponent a||q - x||^2 of the terms that
// make up the sum, and fp32 rounding at that magnitude limits the accuracy.
// Here the data rows are grouped into spatially compact 32-row tiles and
// every tile is expanded around its own centre c_T:
//     ||q - x||^2 = ||q - c_T||^2 + ||x - c_T||^2 - 2 (q - c_T).(x - c_T),
// so that the magnitudes the tile carries are those of q - c_T and x - c_T.
//
// Grouping (deterministic; no host synchronisation):
//   pick_seeds        K seed rows x_{j_k}, j_k = floor(U_k n) from a
//                     SplitMix64 counter stream (tag "CNTR"), taken relative
//                     to seed 0's row r
//   assign_seeds      every row's nearest seed (largest (x - r).(s - r) -
//                     ||s - r||^2/2, the product in fp16 on the matrix
//                     cores, ties to the lower seed)
//   label_hist        per 1024-row block, the rows of each seed
//   scan_labels       per seed, the exclusive sum over blocks
//   group_offsets     group k starts at sum_{k' < k} ceil32(count_k'), so
//                     every group fills whole tiles; the padded row count
//                     goes to device memory (the tiles read it there)
//   scatter_labels    row i goes to its group in ascending i (ballot ranks)
//   build_tiles       per 32-row tile: centre c_T = fl32(mean of its rows),
//                     rows fl32(x - c_T), beta = fl32(-a log2(e) ||x - c_T||^2)
//                     (binary64 from the exact fp64 differences), radius
//                     R_T = max ||x - c_T|| rounded up; padding rows beta = -1e30
// The centred fp16 form uses one centre per group instead (the query operand
// then changes only where the group does, not at every tile):
//   tile_sums         fp64 coordinate sums per tile
//   group_centres     c_g = fl32(group sum / group count), sums in tile order
//   build_tiles_h     rows fl16(x - c_g), beta = fl32(-a log2(e) ||x - c_g||^2),
//                     the group of every tile, R_g = max ||x - c_g|| rounded up
// The result S(q) does not depend on the grouping beyond rounding; the
// grouping depends only on X, so results stay deterministic and independent
// of the queries.
#include "e2lsh.h"
#include "kde_exact.h"
#include "kde_tiles.h"
#include "runtime.h"

namespace stag {
namespace {

using namespace tiles;

constexpr uint64_t kSeedTag = 0x434E5452ULL;  // "CNTR"
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;
constexpr int kHistBlock = 1024;  // rows per histogram block

// Row floor(U_k n) of the seed stream.
__device__ inline int64_t seed_row(int k, int64_t n) {
  const uint64_t s = mix64(mix64(mix64(kSeedTag)));
  const uint64_t u53 = mix64(s + (uint64_t)(k + 1) * kGamma) >> 11;
  // floor(U n) with U = u53 2^-53, taken exactly in integers
  const uint64_t hi = __umul64hi(u53, (uint64_t)n), lo = u53 * (uint64_t)n;
  return (int64_t)((hi << 11) | (lo >> 53));
}

// Seed k < K: row floor(U_k n) minus the reference point r (seed 0's row, so
// that the distances below do not carry the data's offset from the origin)
// into seeds [K_pad][DP] (zero padded), with hn[k] = -||s - r||^2 / 2;
// padding seeds k >= K get hn = -inf; ref [DP] = r.  One wave per seed.
__global__ __launch_bounds__(256) void pick_seeds(const float* __restrict__ X, int64_t n, int d, int dp, int K,
                                                  int K_pad, float* __restrict__ seeds, float* __restrict__ hn,
                                                  float* __restrict__ ref) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= K_pad) return;
  if (k >= K) {
    for (int j = lane; j < dp; j += 64) seeds[(int64_t)k * dp + j] = 0.0f;
    if (lane == 0) hn[k] = -HUGE_VALF;
    return;
  }
  const int64_t r0 = seed_row(0, n), row = seed_row(k, n);
  double sq = 0.0;
  for (int j = lane; j < dp; j += 64) {
    const float rj = j < d ? X[r0 * d + j] : 0.0f;
    const float v = j < d ? X[row * d + j] - rj : 0.0f;
    seeds[(int64_t)k * dp + j] = v;
    if (k == 0) ref[j] = rj;
    sq += (double)v * (double)v;
  }
  for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
  if (lane == 0) hn[k] = (float)(-0.5 * sq);
}

// Nearest seed of every row: the largest x.s - ||s||^2/2 over the seeds
// (one v_mfma_f32_32x32x16_f16 product of fl16(x - r) and fl16(s - r) per
// 16 dimensions, accumulators seeded with -||s||^2/2; 32 seeds as the A
// operand staged in LDS, each wave's 32 rows as the B operand in registers),
// ties to the lower seed.  The fp16 roundings can send a row whose two
// nearest seeds lie within about 2^-10 ||x - r|| ||s - r|| of each other to
// the farther one: any assignment is valid (the centres and radii are
// measured on the groups as formed), and this one is deterministic.
template <int DP>
__global__ __launch_bounds__(256) void assign_seeds(const float* __restrict__ X, int64_t n, int d,
                                                    const float* __restrict__ seeds, const float* __restrict__ hn,
                                                    const float* __restrict__ ref, int K_pad,
                                                    uint8_t* __restrict__ label) {
  constexpr int KS = DP / 16;
  constexpr int LD = DP + 8;
  __shared__ __attribute__((aligned(16))) unsigned short st[32 * LD];
  __shared__ float shn[32];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r32 = lane & 31, h = lane >> 5;
  const int64_t row = (int64_t)blockIdx.x * 128 + wave * 32 + r32;
  u16x8 bq[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    u16x8 o;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int j = s * 16 + h * 8 + i;
      o[i] = f16_rne((row < n && j < d) ? X[row * d + j] - ref[j] : 0.0f);
    }
    bq[s] = o;
  }
  float best = -HUGE_VALF;
  int bests = 0;
  for (int g = 0; g < K_pad / 32; ++g) {
    __syncthreads();
    for (int v = tid; v < 32 * DP / 8; v += 256) {
      const int r = (v * 8) / DP, c = (v * 8) % DP;
      const float* src = &seeds[((int64_t)g * 32 + r) * DP + c];
      const f32x4 lo = *reinterpret_cast<const f32x4*>(src), hi = *reinterpret_cast<const f32x4*>(src + 4);
      u16x8 o;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        o[i] = f16_rne(lo[i]);
        o[4 + i] = f16_rne(hi[i]);
      }
      *reinterpret_cast<u16x8*>(&st[r * LD + c]) = o;
    }
    if (tid < 32) shn[tid] = hn[g * 32 + tid];
    __syncthreads();
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = shn[8 * (i >> 2) + 4 * h + (i & 3)];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const u16x8 a = *reinterpret_cast<const u16x8*>(&st[r32 * LD + s * 16 + h * 8]);
      acc = mma16<STAG_FORM_FP16_SPLIT>(a, bq[s], acc);
    }
    // the lane's 16 seeds come in increasing order: strict > keeps the lower
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int s = g * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
      if (acc[i] > best) {
        best = acc[i];
        bests = s;
      }
    }
  }
  const float ob = __shfl_xor(best, 32);
  const int os = __shfl_xor(bests, 32);
  if (ob > best || (ob == best && os < bests)) bests = os;
  if (h == 0 && row < n) label[row] = (uint8_t)bests;
}

// hist[k * nblk + b] = rows of block b (kHistBlock rows) with label k.
__global__ __launch_bounds__(256) void label_hist(const uint8_t* __restrict__ label, int64_t n, int K, int64_t nblk,
                                                  uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kHistBlock;
  for (int r = 0; r < kHistBlock / 256; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    if (i < n) atomicAdd(&cnt[label[i]], 1u);
  }
  __syncthreads();
  if ((int)threadIdx.x < K) hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// One workgroup per label k: exclusive sum of hist[k][0..nblk) in place;
// count[k] = the total.
__global__ __launch_bounds__(256) void scan_labels(uint32_t* __restrict__ hist, int64_t nblk,
                                                   uint32_t* __restrict__ count) {
  __shared__ uint32_t part[256];
  uint32_t* h = hist + (int64_t)blockIdx.x * nblk;
  const int64_t per = (nblk + 255) / 256;
  const int64_t b0 = (int64_t)threadIdx.x * per;
  uint32_t s = 0;
  for (int64_t b = b0; b < b0 + per && b < nblk; ++b) s += h[b];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int t = 0; t < 256; ++t) {
      const uint32_t v = part[t];
      part[t] = run;
      run += v;
    }
    count[blockIdx.x] = run;
  }
  __syncthreads();
  uint32_t run = part[threadIdx.x];
  for (int64_t b = b0; b < b0 + per && b < nblk; ++b) {
    const uint32_t v = h[b];
    h[b] = run;
    run += v;
  }
}

// goff[k] = sum_{k' < k} count[k'] rounded up to a multiple of align_mask + 1
// (32 for data: whole tiles; 1 for queries); n_pad = goff[K].  One thread.
__global__ void group_offsets(const uint32_t* __restrict__ count, int K, uint32_t align_mask,
                              uint32_t* __restrict__ goff, int64_t* __restrict__ n_pad) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t run = 0;
  for (int k = 0; k < K; ++k) {
    goff[k] = run;
    run += (count[k] + align_mask) & ~align_mask;
  }
  goff[K] = run;
  *n_pad = (int64_t)run;
}

// map[goff[k] + (rank of row i among the rows of label k)] = i, rows in
// ascending order within a label: the block's base from the scanned
// histogram, then 256 rows per round ranked with 8 ballots per wave.
__global__ __launch_bounds__(256) void scatter_labels(const uint8_t* __restrict__ label, int64_t n, int64_t nblk,
                                                      const uint32_t* __restrict__ hist,
                                                      const uint32_t* __restrict__ goff, int* __restrict__ map) {
  __shared__ uint32_t running[256];
  __shared__ uint32_t wcount[4][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  running[tid] = 0;
  for (int w = 0; w < 4; ++w) wcount[w][tid] = 0;
  __syncthreads();
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kHistBlock;
  for (int r = 0; r < kHistBlock / 256; ++r) {
    const int64_t i = base + r * 256 + tid;
    const bool valid = i < n;
    const uint32_t key = valid ? label[i] : 0u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (key >> b) & 1u;
      const uint64_t ones = __ballot(bit);
      peers &= bit ? ones : ~ones;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    if (valid && rank == 0) wcount[wave][key] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t before = running[key];
      for (int w = 0; w < wave; ++w) before += wcount[w][key];
      map[goff[key] + hist[(int64_t)key * nblk + blockIdx.x] + before + rank] = (int)i;
    }
    __syncthreads();
    running[tid] += wcount[0][tid] + wcount[1][tid] + wcount[2][tid] + wcount[3][tid];
    for (int w = 0; w < 4; ++w) wcount[w][tid] = 0;
    __syncthreads();
  }
}

__global__ void fill_minus_one(int* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = -1;
}

// One wave per 32-row tile below the padded row count (4 tiles per block).
// Lanes hold coordinates j = lane + 64 c.
template <int DP>
__global__ __launch_bounds__(256) void build_tiles(const float* __restrict__ X, int d, const int* __restrict__ map,
                                                   const int64_t* __restrict__ n_pad, double neg_a_log2e,
                                                   float* __restrict__ Xc, float* __restrict__ beta,
                                                   float* __restrict__ centre, float* __restrict__ radius) {
  constexpr int NC = (DP + 63) / 64;
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t * kTileRows >= *n_pad) return;
  double sum[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) sum[c] = 0.0;
  int cnt = 0;
  for (int r = 0; r < kTileRows; ++r) {
    const int src = map[t * kTileRows + r];
    if (src < 0) continue;
    ++cnt;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = lane + 64 * c;
      if (j < d) sum[c] += (double)X[(int64_t)src * d + j];
    }
  }
  float cen[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int j = lane + 64 * c;
    cen[c] = (j < d && cnt > 0) ? (float)(sum[c] / (double)cnt) : 0.0f;
    if (j < DP) centre[t * DP + j] = cen[c];
  }
  double rmax = 0.0;
  for (int r = 0; r < kTileRows; ++r) {
    const int64_t row = t * kTileRows + r;
    const int src = map[row];
    double sq = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = lane + 64 * c;
      float v = 0.0f;
      if (src >= 0 && j < d) {
        const double e = (double)X[(int64_t)src * d + j] - (double)cen[c];  // exact in binary64
        v = (float)e;
        sq = fma(e, e, sq);
      }
      if (j < DP) Xc[row * DP + j] = v;
    }
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
    if (src >= 0) rmax = fmax(rmax, sq);
    if (lane == 0) beta[row] = src >= 0 ? (float)(neg_a_log2e * sq) : kPadOffset;
  }
  if (lane == 0) {
    const float rf = (float)sqrt(rmax);
    radius[t] = (double)rf < sqrt(rmax) ? nextafterf(rf, HUGE_VALF) : rf;
  }
}

// Centred fp16 form: coordinate sums of each 32-row tile below the padded
// row count, fp64 (one wave per tile; lanes hold coordinates j = lane + 64 c).
template <int DP>
__global__ __launch_bounds__(256) void tile_sums(const float* __restrict__ X, int d, const int* __restrict__ map,
                                                 const int64_t* __restrict__ n_pad, double* __restrict__ tsum) {
  constexpr int NC = (DP + 63) / 64;
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t * kTileRows >= *n_pad) return;
  double sum[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) sum[c] = 0.0;
  for (int r = 0; r < kTileRows; ++r) {
    const int src = map[t * kTileRows + r];
    if (src < 0) continue;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = lane + 64 * c;
      if (j < d) sum[c] += (double)X[(int64_t)src * d + j];
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int j = lane + 64 * c;
    if (j < DP) tsum[t * DP + j] = sum[c];
  }
}

// One workgroup per group g < K_pad: c_g = fl32(sum of its tiles' sums, in
// tile order, / its row count) (zero for an empty or padding group), and
// radius[g] = 0 (build_tiles_h raises it).
template <int DP>
__global__ __launch_bounds__(256) void group_centres(const double* __restrict__ tsum,
                                                     const uint32_t* __restrict__ count,
                                                     const uint32_t* __restrict__ goff, int K,
                                                     float* __restrict__ centre, float* __restrict__ radius) {
  const int g = blockIdx.x;
  for (int j = threadIdx.x; j < DP; j += 256) {
    float c = 0.0f;
    if (g < K && count[g] > 0) {
      double s = 0.0;
      for (uint32_t t = goff[g] / kTileRows; t < goff[g + 1] / kTileRows; ++t) s += tsum[(int64_t)t * DP + j];
      c = (float)(s / (double)count[g]);
    }
    centre[(int64_t)g * DP + j] = c;
  }
  if (threadIdx.x == 0) radius[g] = 0.0f;
}

// One wave per 32-row tile below the padded row count: tgroup[t] = the group
// of its rows (its first row is never padding), rows fl16(x - c_g) (the
// difference exact in binary64, rounded to fp32, then to fp16), beta =
// fl32(-a log2(e) ||x - c_g||^2) from the exact differences (NaN if some
// |x_j - c_j| rounds to fp16 infinity), padding rows 0 with beta = -1e30;
// radius[g] = max over the group of ||x - c_g|| (fp32 rounded up; positive
// floats order as their bit patterns, so the atomic maximum is exact and
// does not depend on the order).
template <int DP>
__global__ __launch_bounds__(256) void build_tiles_h(const float* __restrict__ X, int d, const int* __restrict__ map,
                                                     const uint8_t* __restrict__ label,
                                                     const int64_t* __restrict__ n_pad, double neg_a_log2e,
                                                     const float* __restrict__ centre,
                                                     unsigned short* __restrict__ Xh, float* __restrict__ beta,
                                                     int* __restrict__ tgroup, float* __restrict__ radius) {
  constexpr int NC = (DP + 63) / 64;
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t * kTileRows >= *n_pad) return;
  const int g = label[map[t * kTileRows]];
  if (lane == 0) tgroup[t] = g;
  float cen[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int j = lane + 64 * c;
    cen[c] = j < DP ? centre[(int64_t)g * DP + j] : 0.0f;
  }
  double rmax = 0.0;
  for (int r = 0; r < kTileRows; ++r) {
    const int64_t row = t * kTileRows + r;
    const int src = map[row];
    double sq = 0.0;
    bool over = false;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = lane + 64 * c;
      unsigned short v = 0;
      if (src >= 0 && j < d) {
        const double e = (double)X[(int64_t)src * d + j] - (double)cen[c];  // exact in binary64
        v = f16_rne((float)e);
        over = over || (v & 0x7FFFu) == 0x7C00u;
        sq = fma(e, e, sq);
      }
      if (j < DP) Xh[row * DP + j] = v;
    }
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
    const bool any_over = __ballot(over) != 0ull;
    if (src >= 0) rmax = fmax(rmax, sq);
    if (lane == 0) beta[row] = src < 0 ? kPadOffset : (any_over ? __builtin_nanf("") : (float)(neg_a_log2e * sq));
  }
  if (lane == 0) {
    const float rf = (float)sqrt(rmax);
    const float ru = (double)rf < sqrt(rmax) ? nextafterf(rf, HUGE_VALF) : rf;
    atomicMax(reinterpret_cast<unsigned int*>(radius) + g, __float_as_uint(ru));
  }
}

template <int DP>
stag_status launch_assign(const float* X, int64_t n, int d, const CentreTemp& t, hipStream_t st) {
  hipLaunchKernelGGL(assign_seeds<DP>, dim3((unsigned)ceil_div(n, 128)), dim3(256), 0, st, X, n, d, t.seeds, t.hn,
                     t.ref, t.K_pad, t.label);
  return check_launch("assign_seeds");
}

template <int DP>
stag_status launch_build(const float* X, int d, const int* map, const int64_t* n_pad, double neg_a_log2e, float* Xc,
                         float* beta, float* centre, float* radius, int64_t tiles_max, hipStream_t st) {
  hipLaunchKernelGGL(build_tiles<DP>, dim3((unsigned)ceil_div(tiles_max, 4)), dim3(256), 0, st, X, d, map, n_pad,
                     neg_a_log2e, Xc, beta, centre, radius);
  return check_launch("build_tiles");
}

template <int DP>
stag_status launch_build_h(const float* X, int d, const Operands& o, const CentreTemp& t, double neg_a_log2e,
                           hipStream_t st) {
  const int64_t tiles_max = o.rows_pad / kTileRows;
  hipLaunchKernelGGL(tile_sums<DP>, dim3((unsigned)ceil_div(tiles_max, 4)), dim3(256), 0, st, X, d, t.map,
                     o.n_pad_dev, t.tsum);
  STAG_TRY(check_launch("tile_sums"));
  hipLaunchKernelGGL(group_centres<DP>, dim3((unsigned)t.K_pad), dim3(256), 0, st, t.tsum, t.count, t.goff, t.K,
                     o.centre, o.radius);
  STAG_TRY(check_launch("group_centres"));
  hipLaunchKernelGGL(build_tiles_h<DP>, dim3((unsigned)ceil_div(tiles_max, 4)), dim3(256), 0, st, X, d, t.map,
                     t.label, o.n_pad_dev, neg_a_log2e, o.centre, static_cast<unsigned short*>(o.part[0]), o.off,
                     o.tgroup, o.radius);
  return check_launch("build_tiles_h");
}

int seed_count(int64_t n) {
  const double k = std::floor(std::sqrt((double)n / 4.0) + 0.5);
  return (int)std::min(256.0, std::max(1.0, k));
}

}  // namespace

int64_t centred_rows_max(int64_t n) { return round_up(n, kTileRows) + (int64_t)kTileRows * seed_count(n); }

stag_status alloc_centre_temp(const Operands& o, Workspace& ws, CentreTemp* t) {
  const int64_t n = o.rows;
  t->K = seed_count(n);
  t->K_pad = (int)round_up(t->K, 32);
  t->nblk = ceil_div(n, kHistBlock);
  STAG_TRY(ws.alloc(&t->seeds, (size_t)t->K_pad * o.dp));
  STAG_TRY(ws.alloc(&t->hn, (size_t)t->K_pad));
  STAG_TRY(ws.alloc(&t->ref, (size_t)o.dp));
  STAG_TRY(ws.alloc(&t->label, (size_t)n));
  STAG_TRY(ws.alloc(&t->hist, (size_t)t->K * t->nblk));
  STAG_TRY(ws.alloc(&t->count, (size_t)t->K));
  STAG_TRY(ws.alloc(&t->goff, (size_t)t->K + 1));
  STAG_TRY(ws.alloc(&t->map, (size_t)o.rows_pad));
  t->tsum = nullptr;
  if (o.form == STAG_FORM_FP16_CENTRED) STAG_TRY(ws.alloc(&t->tsum, (size_t)(o.rows_pad / kTileRows) * o.dp));
  return STAG_OK;
}

stag_status alloc_centred_operands(int64_t n, int d, Workspace& ws, Operands* out) {
  const int dp = exact_padded_dim(d);
  if (dp == 0 || dp > 256) return fail(STAG_E_UNSUPPORTED, "centred operands need d <= 256");
  const int64_t rows_max = centred_rows_max(n);
  out->form = STAG_FORM_FP32;
  out->rows = n;
  out->rows_pad = rows_max;
  out->d = d;
  out->dp = dp;
  for (int p = 0; p < 3; ++p) out->part[p] = nullptr;
  STAG_TRY(ws.alloc_bytes(&out->part[0], (size_t)rows_max * dp * sizeof(float)));
  STAG_TRY(ws.alloc(&out->off, (size_t)rows_max));
  out->aug = nullptr;
  out->nrm = nullptr;
  out->max_nrm_bits = nullptr;
  out->centred = true;
  STAG_TRY(ws.alloc(&out->centre, (size_t)(rows_max / kTileRows) * dp));
  STAG_TRY(ws.alloc(&out->radius, (size_t)(rows_max / kTileRows)));
  STAG_TRY(ws.alloc(&out->n_pad_dev, 1));
  return STAG_OK;
}

// The grouping shared by both centred forms: seeds, nearest seed of every
// row, per-label counts and offsets (n_pad), and the row map.
static stag_status group_rows(const float* X, const Operands& o, const CentreTemp& t, hipStream_t st) {
  const int64_t n = o.rows;
  const int d = o.d, dp = o.dp;
  hipLaunchKernelGGL(pick_seeds, dim3((unsigned)ceil_div(t.K_pad, 4)), dim3(256), 0, st, X, n, d, dp, t.K, t.K_pad,
                     t.seeds, t.hn, t.ref);
  STAG_TRY(check_launch("pick_seeds"));
  switch (dp) {
    case 16: STAG_TRY(launch_assign<16>(X, n, d, t, st)); break;
    case 32: STAG_TRY(launch_assign<32>(X, n, d, t, st)); break;
    case 64: STAG_TRY(launch_assign<64>(X, n, d, t, st)); break;
    case 96: STAG_TRY(launch_assign<96>(X, n, d, t, st)); break;
    case 128: STAG_TRY(launch_assign<128>(X, n, d, t, st)); break;
    case 160: STAG_TRY(launch_assign<160>(X, n, d, t, st)); break;
    case 192: STAG_TRY(launch_assign<192>(X, n, d, t, st)); break;
    case 224: STAG_TRY(launch_assign<224>(X, n, d, t, st)); break;
    case 256: STAG_TRY(launch_assign<256>(X, n, d, t, st)); break;
    default: return fail(STAG_E_UNSUPPORTED, "centred operands: padded dimension %d", dp);
  }
  hipLaunchKernelGGL(label_hist, dim3((unsigned)t.nblk), dim3(256), 0, st, t.label, n, t.K, t.nblk, t.hist);
  STAG_TRY(check_launch("label_hist"));
  hipLaunchKernelGGL(scan_labels, dim3((unsigned)t.K), dim3(256), 0, st, t.hist, t.nblk, t.count);
  STAG_TRY(check_launch("scan_labels"));
  hipLaunchKernelGGL(group_offsets, dim3(1), dim3(64), 0, st, t.count, t.K, 31u, t.goff, o.n_pad_dev);
  STAG_TRY(check_launch("group_offsets"));
  hipLaunchKernelGGL(fill_minus_one, dim3((unsigned)ceil_div(o.rows_pad, 256)), dim3(256), 0, st, t.map, o.rows_pad);
  STAG_TRY(check_launch("fill_minus_one"));
  hipLaunchKernelGGL(scatter_labels, dim3((unsigned)t.nblk), dim3(256), 0, st, t.label, n, t.nblk, t.hist, t.goff,
                     t.map);
  STAG_TRY(check_launch("scatter_labels"));
  return STAG_OK;
}

stag_status prep_centred_operands(const float* X, double a_tile, const Operands& o, const CentreTemp& t,
                                  hipStream_t st) {
  ScopedTimer tm("kde_centre", st);
  const int d = o.d, dp = o.dp;
  STAG_TRY(group_rows(X, o, t, st));
  const double nl = -a_tile * kLog2e;
  const int64_t tiles_max = o.rows_pad / kTileRows;
  float* Xc = static_cast<float*>(o.part[0]);
  switch (dp) {
    case 16: return launch_build<16>(X, d, t.map, o.n_pad_dev, nl, Xc, o.off, o.centre, o.radius, tiles_max, st);
    case 32: return launch_build<32>(X, d, t.map, o.n_pad_dev, nl, Xc, o.off, o.centre, o.radius, tiles_max, st);
    case 64: return launch_build<64>(X, d, t.map, o.n_pad_dev, nl, Xc, o.off, o.centre, o.radius, tiles_max, st);
    case 96: return launch_build<96>(X, d, t.map, o.n_pad_dev, nl, Xc, o.off, o.centre, o.radius, tiles_max, st);
    case 128: return launch_build<128>(X, d, t.map, o.n_pad_dev, nl, Xc, o.off, o.centre, o.radius, tiles_max, st);
    case 160: return launch_build<160>(X, d, t.map, o.n_pad_dev, nl, Xc, o.off, o.centre, o.radius, tiles_max, st);
    case 192: return launch_build<192>(X, d, t.map, o.n_pad_dev, nl, Xc, o.off, o.centre, o.radius, tiles_max, st);
    case 224: return launch_build<224>(X, d, t.map, o.n_pad_dev, nl, Xc, o.off, o.centre, o.radius, tiles_max, st);
    default: return launch_build<256>(X, d, t.map, o.n_pad_dev, nl, Xc, o.off, o.centre, o.radius, tiles_max, st);
  }
}

stag_status alloc_centred_h_operands(int64_t n, int d, Workspace& ws, Operands* out) {
  const int dp = exact_padded_dim(d);
  if (dp == 0 || dp > 256) return fail(STAG_E_UNSUPPORTED, "centred operands need d <= 256");
  const int64_t rows_max = centred_rows_max(n);
  const int K_pad = (int)round_up(seed_count(n), 32);
  out->form = STAG_FORM_FP16_CENTRED;
  out->rows = n;
  out->rows_pad = rows_max;
  out->d = d;
  out->dp = dp;
  for (int p = 0; p < 3; ++p) out->part[p] = nullptr;
  STAG_TRY(ws.alloc_bytes(&out->part[0], (size_t)rows_max * dp * sizeof(unsigned short)));
  STAG_TRY(ws.alloc(&out->off, (size_t)rows_max));
  out->aug = nullptr;
  out->nrm = nullptr;
  out->max_nrm_bits = nullptr;
  out->centred = true;
  STAG_TRY(ws.alloc(&out->centre, (size_t)K_pad * dp));
  STAG_TRY(ws.alloc(&out->radius, (size_t)K_pad));
  STAG_TRY(ws.alloc(&out->tgroup, (size_t)(rows_max / kTileRows)));
  STAG_TRY(ws.alloc(&out->n_pad_dev, 1));
  return STAG_OK;
}

stag_status prep_centred_h_operands(const float* X, double a_tile, const Operands& o, const CentreTemp& t,
                                    hipStream_t st) {
  ScopedTimer tm("kde_centre", st);
  if (o.form != STAG_FORM_FP16_CENTRED || !t.tsum) return fail(STAG_E_INVAL, "centred fp16 operands: bad set-up");
  const int d = o.d;
  STAG_TRY(group_rows(X, o, t, st));
  const double nl = -a_tile * kLog2e;
  switch (o.dp) {
    case 16: return launch_build_h<16>(X, d, o, t, nl, st);
    case 32: return launch_build_h<32>(X, d, o, t, nl, st);
    case 64: return launch_build_h<64>(X, d, o, t, nl, st);
    case 96: return launch_build_h<96>(X, d, o, t, nl, st);
    case 128: return launch_build_h<128>(X, d, o, t, nl, st);
    case 160: return launch_build_h<160>(X, d, o, t, nl, st);
    case 192: return launch_build_h<192>(X, d, o, t, nl, st);
    case 224: return launch_build_h<224>(X, d, o, t, nl, st);
    case 256: return launch_build_h<256>(X, d, o, t, nl, st);
  }
  return fail(STAG_E_UNSUPPORTED, "centred operands: padded dimension %d", o.dp);
}

stag_status alloc_query_sort(int64_t m, int64_t m_pad, int K, Workspace& ws, QuerySort* qs) {
  qs->nblk = ceil_div(m, kHistBlock);
  STAG_TRY(ws.alloc(&qs->label, (size_t)m));
  STAG_TRY(ws.alloc(&qs->hist, (size_t)K * qs->nblk));
  STAG_TRY(ws.alloc(&qs->count, (size_t)K));
  STAG_TRY(ws.alloc(&qs->goff, (size_t)K + 1));
  STAG_TRY(ws.alloc(&qs->total, 1));
  STAG_TRY(ws.alloc(&qs->perm, (size_t)m_pad));
  return STAG_OK;
}

stag_status sort_queries(const float* Q, int64_t m, int64_t m_pad, int d, int dp, const CentreTemp& t,
                         const QuerySort& qs, hipStream_t st) {
  ScopedTimer tm("kde_query_sort", st);
  CentreTemp tq = t;  // the data's seeds, the queries' labels
  tq.label = qs.label;
  switch (dp) {
    case 16: STAG_TRY(launch_assign<16>(Q, m, d, tq, st)); break;
    case 32: STAG_TRY(launch_assign<32>(Q, m, d, tq, st)); break;
    case 64: STAG_TRY(launch_assign<64>(Q, m, d, tq, st)); break;
    case 96: STAG_TRY(launch_assign<96>(Q, m, d, tq, st)); break;
    case 128: STAG_TRY(launch_assign<128>(Q, m, d, tq, st)); break;
    case 160: STAG_TRY(launch_assign<160>(Q, m, d, tq, st)); break;
    case 192: STAG_TRY(launch_assign<192>(Q, m, d, tq, st)); break;
    case 224: STAG_TRY(launch_assign<224>(Q, m, d, tq, st)); break;
    case 256: STAG_TRY(launch_assign<256>(Q, m, d, tq, st)); break;
    default: return fail(STAG_E_UNSUPPORTED, "query sort: padded dimension %d", dp);
  }
  hipLaunchKernelGGL(label_hist, dim3((unsigned)qs.nblk), dim3(256), 0, st, qs.label, m, t.K, qs.nblk, qs.hist);
  STAG_TRY(check_launch("label_hist"));
  hipLaunchKernelGGL(scan_labels, dim3((unsigned)t.K), dim3(256), 0, st, qs.hist, qs.nblk, qs.count);
  STAG_TRY(check_launch("scan_labels"));
  hipLaunchKernelGGL(group_offsets, dim3(1), dim3(64), 0, st, qs.count, t.K, 0u, qs.goff, qs.total);
  STAG_TRY(check_launch("group_offsets"));
  hipLaunchKernelGGL(fill_minus_one, dim3((unsigned)ceil_div(m_pad, 256)), dim3(256), 0, st, qs.perm, m_pad);
  STAG_TRY(check_launch("fill_minus_one"));
  hipLaunchKernelGGL(scatter_labels, dim3((unsigned)qs.nblk), dim3(256), 0, st, qs.label, m, qs.nblk, qs.hist,
                     qs.goff, qs.perm);
  return check_launch("scatter_labels");
}

}  // namespace stag
