// CKNS kernel density estimator on E2LSH tables (Sec. "The CKNS Algorithm":
// levels L_i of points whose kernel value lies in (2^-i, 2^-i+1], log n
// subsamples drawn with probability 2^-i, one E2LSH table set per subsample
// to recover L_i, the importance-weighted sum, independent repetitions;
// constructor parameters eps, min_mu, K1, K2_constant, p_offset of
// CKNSGaussianKDE).
//
// Readings taken where the paper is silent (same as the library docs):
//   J = ceil(log2(1/mu_min)) levels, T_i = i ln2 / a, level i holds
//   T_{i-1} <= D < T_i; p_i = min(1, 2^-i/(n mu_min)) 2^-p_offset; L =
//   ceil(K2_constant) tables per level (default ceil(log2 n)); K the largest
//   with 1-(1-p(1)^K)^L >= 1 - eps/4; K1 = ceil(log2(n)/eps^2) copies; level i
//   hashes the space scaled by r_i = sqrt(T_i); a point found in several tables
//   of one level counts once (first table); each accepted term is reweighted
//   by 1/(p_i R_i) with R_i the recovery probability at its scaled distance
//   (1/p_i alone with STAG_LSH_LITERAL); copies are averaged.
//
// Device layout of an index (M = total sampled points over all copies/levels,
// segment s = t*J + (i-1), table group g = s*L + l):
//   X          [n][dx]       fp32 copy of the data (dx = d rounded up to 4)
//   G8         [K1 J L][nch][dg][8] binary64 level-scaled projections
//   B          [K1 J L][K]   offsets
//   seg_off    [K1 J + 1]    start of each segment in members/mkeys
//   members    [M]           point index, ascending within a segment
//   mkeys      [M][L]        bucket key of each member in each table
//   tab_*      per group an open-addressing table (capacity cap_s, a power of
//              two >= 2 |segment|): key, start and count of its bucket
//   csr        [M][L]        per group, member positions grouped by bucket,
//              ascending within a bucket (deterministic construction)
#include <algorithm>
#include <cmath>
#include <vector>

#include "e2lsh.h"
#include "lsh.h"
#include "runtime.h"
#include "scan.h"
#include "sort.h"

namespace stag {
namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t kTagMask = 0x4D41534BULL;
constexpr uint64_t kTagDraw = 0x44524157ULL;
constexpr uint64_t kTagProj = 0x50524F4AULL;
constexpr uint64_t kTagOffs = 0x4F464653ULL;
constexpr uint64_t kEmpty = 0xFFFFFFFFFFFFFFFFULL;
constexpr int kMaskBlock = 1024;  // points per counting block (4 per thread)

// State of the SplitMix64 stream (seed, tag, a, b); output c of it is
// mix64(state + (c + 1) gamma).
__host__ __device__ inline uint64_t mix64_hd(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t stream_state(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b) {
  return mix64_hd(mix64_hd(mix64_hd(seed ^ tag) ^ a) ^ b);
}

// ---------------------------------------------------------------------------
// randomness and projections
// ---------------------------------------------------------------------------

// Default randomness when the caller passes none: g ~ N(0,1) by Box-Muller on
// two counter uniforms, b = 4 U.
__global__ void gen_randomness(uint64_t seed, int64_t nproj, int d, float* __restrict__ G0,
                               double* __restrict__ B) {
  const int64_t total = nproj * d;
  const uint64_t sp = stream_state(seed, kTagProj, 0, 0);
  const uint64_t so = stream_state(seed, kTagOffs, 0, 0);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const double u1 = (double)((mix64_hd(sp + (uint64_t)(2 * e + 1) * kGamma) >> 11) + 1) * 0x1.0p-53;  // (0,1]
    const double u2 = (double)(mix64_hd(sp + (uint64_t)(2 * e + 2) * kGamma) >> 11) * 0x1.0p-53;
    G0[e] = (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586477 * u2));
    if (e < nproj) B[e] = 4.0 * (double)(mix64_hd(so + (uint64_t)(e + 1) * kGamma) >> 11) * 0x1.0p-53;
  }
}

// G8[tab][c][j][e] = fp32(G0[tab][8c+e][j] / r_i) as binary64 (0 beyond K, d).
__global__ void scale_projections(const float* __restrict__ G0, int64_t ntab, int J, int L, int K, int d, int dg,
                                  int nch, const double* __restrict__ rlev, double* __restrict__ G8) {
  const int64_t total = ntab * nch * dg * 8;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(idx & 7);
    const int64_t r = idx >> 3;
    const int j = (int)(r % dg);
    const int64_t tc = r / dg;
    const int c = (int)(tc % nch);
    const int64_t tab = tc / nch;
    const int k = 8 * c + e;
    const int i = (int)((tab / L) % J) + 1;
    double v = 0.0;
    if (k < K && j < d) v = (double)(float)((double)G0[(tab * K + k) * d + j] / rlev[i]);
    G8[idx] = v;
  }
}

// ---------------------------------------------------------------------------
// subsampling: count per (segment, block of points), then scatter in order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mask_count(uint64_t seed, int J, int64_t n, int nblk,
                                                  const uint64_t* __restrict__ thr, uint32_t* __restrict__ cnt) {
  const int seg = blockIdx.y;
  const int t = seg / J, i = seg % J + 1;
  const uint64_t st = stream_state(seed, kTagMask, (uint64_t)t, (uint64_t)i);
  const uint64_t th = thr[i];
  const int64_t j0 = (int64_t)blockIdx.x * kMaskBlock + threadIdx.x * 4;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t j = j0 + k;
    if (j < n && (mix64_hd(st + (uint64_t)(j + 1) * kGamma) >> 11) < th) ++c;
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  __shared__ uint32_t ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) cnt[(int64_t)seg * nblk + blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(256) void mask_scatter(uint64_t seed, int J, int64_t n, int nblk,
                                                    const uint64_t* __restrict__ thr,
                                                    const uint64_t* __restrict__ off, int32_t* __restrict__ members) {
  const int seg = blockIdx.y;
  const int t = seg / J, i = seg % J + 1;
  const uint64_t st = stream_state(seed, kTagMask, (uint64_t)t, (uint64_t)i);
  const uint64_t th = thr[i];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ uint32_t ws[4];
  // four passes of 256 consecutive points keep the output in ascending order
  uint64_t base = off[(int64_t)seg * nblk + blockIdx.x];
  for (int k = 0; k < 4; ++k) {
    const int64_t j = (int64_t)blockIdx.x * kMaskBlock + k * 256 + threadIdx.x;
    const bool keep = j < n && (mix64_hd(st + (uint64_t)(j + 1) * kGamma) >> 11) < th;
    const uint64_t bal = __ballot(keep);
    const uint32_t before = __popcll(bal & ((1ULL << lane) - 1ULL));
    if (lane == 0) ws[wave] = __popcll(bal);
    __syncthreads();
    uint32_t wbase = 0;
    for (int w = 0; w < wave; ++w) wbase += ws[w];
    if (keep) members[base + wbase + before] = (int32_t)j;
    base += ws[0] + ws[1] + ws[2] + ws[3];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// hashing of the sampled points: one lane per member, waves over tables
// ---------------------------------------------------------------------------
struct MemberBlock {
  int32_t seg;
  int32_t u0;
};

template <int DREG>
__global__ __launch_bounds__(256) void hash_members(const float* __restrict__ X, int dx, int d, int dg,
                                                    const MemberBlock* __restrict__ blocks,
                                                    const uint64_t* __restrict__ seg_off,
                                                    const int32_t* __restrict__ members, const double* __restrict__ G8,
                                                    const double* __restrict__ B, int K, int L, int nch,
                                                    uint64_t* __restrict__ mkeys) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const MemberBlock blk = blocks[blockIdx.x];
  const int64_t s0 = (int64_t)seg_off[blk.seg];
  const int64_t cnt = (int64_t)seg_off[blk.seg + 1] - s0;
  const int64_t u = blk.u0 + lane;
  const bool live = u < cnt;
  const int32_t j = members[s0 + (live ? u : 0)];
  const float* xrow = X + (int64_t)j * dx;
  double xr[DREG > 0 ? DREG : 1];
  load_point<DREG>(xr, xrow, d);
  for (int l = wave; l < L; l += 4) {
    const int64_t tab = (int64_t)blk.seg * L + l;
    const uint64_t key =
        table_key<DREG>(l, xr, xrow, d, dg, G8 + tab * nch * dg * 8, B + tab * K, K, nch, nullptr);
    if (live) mkeys[(s0 + u) * L + l] = key;
  }
}

// ---------------------------------------------------------------------------
// bucket tables: open addressing over each (segment, table), capacity a
// power of two >= 2 x members; every (table, member) pair is inserted at
// once, then the pairs are sorted stably by their bucket's global slot, which
// lays out the CSR with each bucket's members in ascending order
// ---------------------------------------------------------------------------
__device__ inline uint32_t probe_insert(uint64_t* __restrict__ keys, uint32_t mask, uint64_t key) {
  uint32_t s = (uint32_t)key & mask;
  while (true) {
    const unsigned long long prev =
        atomicCAS(reinterpret_cast<unsigned long long*>(keys + s), (unsigned long long)kEmpty,
                  (unsigned long long)key);
    if (prev == kEmpty || prev == key) return s;
    s = (s + 1) & mask;
  }
}

__device__ inline uint32_t lookup_present(const uint64_t* __restrict__ keys, uint32_t mask, uint64_t key) {
  uint32_t s = (uint32_t)key & mask;
  while (keys[s] != key) s = (s + 1) & mask;
  return s;
}

// Bucket tables of every (segment, table) pair at once.  The pairs
// (segment, table l, member u) are numbered table-major, [seg][l][u], which
// is also the CSR layout; pair p of segment seg starts at seg_off[seg] * L.
__device__ inline int upper_seg(const uint64_t* __restrict__ off, int count, uint64_t scale, uint64_t v) {
  // largest k in [0, count) with off[k] * scale <= v
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] * scale <= v) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct PairPos {
  int seg, l;
  int64_t u, s0, cnt, tb;
  uint32_t mask;
};

__device__ inline PairPos pair_pos(int64_t p, int L, int nseg, const uint64_t* __restrict__ seg_off,
                                   const uint64_t* __restrict__ tab_seg_off, const uint32_t* __restrict__ seg_cap) {
  PairPos q;
  q.seg = upper_seg(seg_off, nseg, (uint64_t)L, (uint64_t)p);
  q.s0 = (int64_t)seg_off[q.seg];
  q.cnt = (int64_t)seg_off[q.seg + 1] - q.s0;
  const int64_t r = p - q.s0 * L;
  q.l = (int)(r / q.cnt);
  q.u = r - (int64_t)q.l * q.cnt;
  const uint32_t cap = seg_cap[q.seg];
  q.mask = cap - 1;
  q.tb = (int64_t)tab_seg_off[q.seg] + (int64_t)q.l * cap;
  return q;
}

__global__ void table_clear(uint64_t* __restrict__ tab_key, uint32_t* __restrict__ tab_cnt, int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  tab_key[g] = kEmpty;
  tab_cnt[g] = 0;
}

__global__ void table_insert(int L, int nseg, int64_t npairs, const uint64_t* __restrict__ seg_off,
                             const uint64_t* __restrict__ tab_seg_off, const uint32_t* __restrict__ seg_cap,
                             const uint64_t* __restrict__ mkeys, uint64_t* __restrict__ tab_key,
                             uint32_t* __restrict__ tab_cnt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const PairPos q = pair_pos(p, L, nseg, seg_off, tab_seg_off, seg_cap);
  const uint32_t s = probe_insert(tab_key + q.tb, q.mask, mkeys[(q.s0 + q.u) * L + q.l]);
  atomicAdd(tab_cnt + q.tb + s, 1u);
}

// Sort key of a pair: its bucket's global slot; value: the member index.
__global__ void table_pairs(int L, int nseg, int64_t npairs, const uint64_t* __restrict__ seg_off,
                            const uint64_t* __restrict__ tab_seg_off, const uint32_t* __restrict__ seg_cap,
                            const uint64_t* __restrict__ mkeys, const uint64_t* __restrict__ tab_key,
                            uint32_t* __restrict__ skey, uint32_t* __restrict__ sval) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const PairPos q = pair_pos(p, L, nseg, seg_off, tab_seg_off, seg_cap);
  const uint32_t s = lookup_present(tab_key + q.tb, q.mask, mkeys[(q.s0 + q.u) * L + q.l]);
  skey[p] = (uint32_t)(q.tb + s);
  sval[p] = (uint32_t)q.u;
}

// Start of a slot's bucket relative to its table: the global scan of the
// slot counts at the slot minus at the table's first slot.
__global__ void table_starts(int L, int nseg, int64_t total, const uint64_t* __restrict__ tab_seg_off,
                             const uint32_t* __restrict__ seg_cap, const uint64_t* __restrict__ scan,
                             uint32_t* __restrict__ tab_start) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int seg = upper_seg(tab_seg_off, nseg, 1, (uint64_t)g);
  const uint32_t cap = seg_cap[seg];
  const int64_t first = (int64_t)tab_seg_off[seg] + ((g - (int64_t)tab_seg_off[seg]) / cap) * cap;
  tab_start[g] = (uint32_t)(scan[g] - scan[first]);
}

// Builds tab_key / tab_cnt / tab_start and the CSR of every (segment, table)
// pair: npairs = members x L pairs, total_slots slots (both known on the host).
stag_status build_tables_sorted(int L, int nseg, int64_t npairs, int64_t total_slots, const uint64_t* seg_off,
                                const uint64_t* tab_seg_off, const uint32_t* seg_cap, const uint64_t* mkeys,
                                uint64_t* tab_key, uint32_t* tab_start, uint32_t* tab_cnt, int32_t* csr, Workspace& ws,
                                hipStream_t st) {
  if (total_slots <= 0 || npairs <= 0) return STAG_OK;
  if (npairs >= ((int64_t)1 << 31) || total_slots >= ((int64_t)1 << 32))
    return fail(STAG_E_UNSUPPORTED, "bucket tables: %lld pairs / %lld slots exceed the 32-bit build",
                (long long)npairs, (long long)total_slots);
  uint32_t *skey = nullptr, *sval = nullptr, *skey2 = nullptr;
  uint64_t* scan = nullptr;
  STAG_TRY(ws.alloc(&skey, (size_t)npairs));
  STAG_TRY(ws.alloc(&sval, (size_t)npairs));
  STAG_TRY(ws.alloc(&skey2, (size_t)npairs));
  STAG_TRY(ws.alloc(&scan, (size_t)total_slots + 1));
  hipLaunchKernelGGL(table_clear, dim3((unsigned)ceil_div(total_slots, 256)), dim3(256), 0, st, tab_key, tab_cnt,
                     total_slots);
  STAG_TRY(check_launch("table_clear"));
  hipLaunchKernelGGL(table_insert, dim3((unsigned)ceil_div(npairs, 256)), dim3(256), 0, st, L, nseg, npairs, seg_off,
                     tab_seg_off, seg_cap, mkeys, tab_key, tab_cnt);
  STAG_TRY(check_launch("table_insert"));
  hipLaunchKernelGGL(table_pairs, dim3((unsigned)ceil_div(npairs, 256)), dim3(256), 0, st, L, nseg, npairs, seg_off,
                     tab_seg_off, seg_cap, mkeys, tab_key, skey, sval);
  STAG_TRY(check_launch("table_pairs"));
  int bits = 1;
  while (bits < 32 && ((uint64_t)(total_slots - 1) >> bits) != 0) ++bits;
  STAG_TRY(radix_sort_pairs_u32(skey, sval, skey2, reinterpret_cast<uint32_t*>(csr), npairs, bits, ws, st));
  STAG_TRY(exclusive_scan_u32(tab_cnt, scan, total_slots, ws, st));
  hipLaunchKernelGGL(table_starts, dim3((unsigned)ceil_div(total_slots, 256)), dim3(256), 0, st, L, nseg,
                     total_slots, tab_seg_off, seg_cap, scan, tab_start);
  return check_launch("table_starts");
}

// ---------------------------------------------------------------------------
// queries
// ---------------------------------------------------------------------------
// One lane per query; the 4 waves of a block take 256 consecutive queries
// through the same tpw tables, so that the projections a block reads (scalar
// loads) are shared by all its waves.
template <int DREG>
__global__ __launch_bounds__(256) void hash_queries(const float* __restrict__ Q, int ldq, int64_t q0, int64_t mb,
                                                    int d, int dg, const double* __restrict__ G8,
                                                    const double* __restrict__ B, int K, int L, int nch,
                                                    int64_t ntab, int tpw, uint64_t* __restrict__ qkeys) {
  const int64_t ql = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = ql < mb;
  const float* xrow = Q + (q0 + (live ? ql : 0)) * ldq;
  double xr[DREG > 0 ? DREG : 1];
  load_point<DREG>(xr, xrow, d);
  const int64_t t0 = (int64_t)blockIdx.y * tpw;
  for (int64_t tab = t0; tab < t0 + tpw && tab < ntab; ++tab) {
    const int l = (int)(tab % L);
    const uint64_t key =
        table_key<DREG>(l, xr, xrow, d, dg, G8 + tab * nch * dg * 8, B + tab * K, K, nch, nullptr);
    if (live) qkeys[tab * mb + ql] = key;
  }
}

// Weight of an accepted term of level i, w_i(c) = exp(-a D) / (p_i R_i(c))
// with c = sqrt(D) / r_i and R_i the recovery probability
// 1 - (1 - p(c)^K)^L (R_i = 1 with STAG_LSH_LITERAL), from its Chebyshev
// interpolant on the level's range of c (see weight_levels); row layout
// {lo, 2 / (1 - lo), a_0 .. a_32}.  One Clenshaw recurrence replaces the
// collision probability, the two integer powers, the exponential and the
// division of the term.
constexpr int kChebTerms = 33;
constexpr int kChebRow = kChebTerms + 2;

__device__ inline double level_weight(const double* __restrict__ row, double c) {
  const double t = (c - row[0]) * row[1] - 1.0;
  const double t2 = 2.0 * t;
  double b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int k = kChebTerms - 1; k >= 1; --k) {
    const double b0 = __builtin_fma(t2, b1, row[2 + k] - b2);
    b2 = b1;
    b1 = b0;
  }
  return __builtin_fma(t, b1, 0.5 * row[2] - b2);
}

struct LevelConst {
  double p[65], T[65], r[65];
};

// Read-only view of an index for device code.
struct IndexView {
  const float* X;
  const double* xn;  // [n] ||x|| of each point (binary64)
  int dx, d, K1, J, L, K;
  double a;
  int literal;
  const double* cheb;  // [J + 1][kChebRow] term-weight interpolants (level_weight)
  const uint64_t* seg_off;
  const int32_t* members;
  const uint64_t* mkeys;
  const uint64_t* tab_seg_off;
  const uint32_t* seg_cap;
  const uint64_t* tab_key;
  const uint32_t* tab_start;
  const uint32_t* tab_cnt;
  const int32_t* csr;
};

template <int DREG>
__device__ inline void load_point_f32(float* xr, const float* __restrict__ xrow, int d) {
  if constexpr (DREG > 0) {
#pragma unroll
    for (int j = 0; j < DREG; ++j) xr[j] = j < d ? xrow[j] : 0.0f;
  }
}

// Per-wave scratch of a copy walk (LDS).
struct WalkScratch {
  uint64_t qk[64];     // the query's keys of the current level, per table
  int64_t base[64];    // csr index of the query's bucket in each table
  uint32_t pre[64];    // exclusive prefix of the bucket sizes over tables
  int32_t ring[128];   // survivors of the fp32 screen, in candidate order
  double ringD[128];   // their fp64 squared distances
};

// Relative error bound of the fp32 squared distance of d coordinates (one
// rounding per difference, square and accumulation: gamma_{d+2} of unit
// roundoff 2^-24, doubled for margin).
__device__ inline double screen_delta(int d) { return 2.0 * (double)(d + 3) * 0x1.0p-24; }

// Both squared distances of a candidate in one pass over its row (the query
// row is wave-uniform: scalar loads): the fp32 value of the screen (two
// accumulators, alternate coordinates) and the fp64 value of the level test
// (one fused chain over ascending coordinates, the oracle's order).  The row
// is read eight 16-byte pieces at a time, all eight loads issued before
// their products, so that a lane has eight loads in flight instead of one;
// one pass instead of a screen pass and a second pass for the survivors.
__device__ inline float dist2_both(const float* __restrict__ qrow, const float* __restrict__ xrow, int d,
                                   double* D64) {
  const float4* x4 = reinterpret_cast<const float4*>(xrow);
  float D0 = 0.0f, D1 = 0.0f;
  double D = 0.0;
  auto piece = [&](const float4& xv, int h4) {
    const float q0 = qrow[4 * h4], q1 = qrow[4 * h4 + 1], q2 = qrow[4 * h4 + 2], q3 = qrow[4 * h4 + 3];
    float dl = q0 - xv.x;
    D0 = __builtin_fmaf(dl, dl, D0);
    dl = q1 - xv.y;
    D1 = __builtin_fmaf(dl, dl, D1);
    dl = q2 - xv.z;
    D0 = __builtin_fmaf(dl, dl, D0);
    dl = q3 - xv.w;
    D1 = __builtin_fmaf(dl, dl, D1);
    double e = (double)q0 - (double)xv.x;
    D = __builtin_fma(e, e, D);
    e = (double)q1 - (double)xv.y;
    D = __builtin_fma(e, e, D);
    e = (double)q2 - (double)xv.z;
    D = __builtin_fma(e, e, D);
    e = (double)q3 - (double)xv.w;
    D = __builtin_fma(e, e, D);
  };
  const int d4 = d >> 2;
  int h4 = 0;
  for (; h4 + 7 < d4; h4 += 8) {
    const float4 x0 = x4[h4], x1 = x4[h4 + 1], x2 = x4[h4 + 2], x3 = x4[h4 + 3];
    const float4 x5 = x4[h4 + 4], x6 = x4[h4 + 5], x7 = x4[h4 + 6], x8 = x4[h4 + 7];
    piece(x0, h4);
    piece(x1, h4 + 1);
    piece(x2, h4 + 2);
    piece(x3, h4 + 3);
    piece(x5, h4 + 4);
    piece(x6, h4 + 5);
    piece(x7, h4 + 6);
    piece(x8, h4 + 7);
  }
  for (; h4 < d4; ++h4) piece(x4[h4], h4);
  for (int h = 4 * d4; h < d; ++h) {
    const float dl = qrow[h] - xrow[h];
    D0 = __builtin_fmaf(dl, dl, D0);
    const double e = (double)qrow[h] - (double)xrow[h];
    D = __builtin_fma(e, e, D);
  }
  *D64 = D;
  return D0 + D1;
}

// Walks copy t of the estimator for one query (one wave).  Per level, lane l
// resolves the query's bucket in table l; the buckets' members are then
// taken as one flattened list (table, member ascending) in batches of 64, one
// candidate per lane.  A candidate is dropped if it was seen in an earlier
// table of the level or is the query's own point (self_idx >= 0); the rest
// pass an fp32 distance screen that removes only points certainly outside
// the level (bound screen_delta), and the survivors queue up in candidate
// order with their fp64 squared distances (taken in the same pass over the
// row).  Every 64 queued points (and at the end of a level) form a batch in
// which each lane decides the level in fp64 and computes its term:
// on_batch(v, j, valid, i) receives it (0 outside the level), the point j
// and the level i.  Levels whose bit (i - 1) is clear in `levels` are
// skipped (callers pass a mask of the levels with a positive term).
// Returns the number of candidates walked.
template <class F>
__device__ inline int64_t walk_copy(const IndexView& ix, const LevelConst& lc, int t, const uint64_t* __restrict__ qk,
                                    int64_t qs, WalkScratch& ws, const float* __restrict__ qrow, int64_t self_idx,
                                    uint64_t levels, F&& on_batch) {
  const int lane = threadIdx.x & 63;
  const int L = ix.L, d = ix.d;
  const double delta = screen_delta(d);
  // ||q|| (binary64, relative error below 1e-13 for d <= 1024, as ||x||)
  double nq = 0.0;
  for (int c = lane; c < d; c += 64) {
    const double v = qrow[c];
    nq = __builtin_fma(v, v, nq);
  }
  for (int o = 32; o > 0; o >>= 1) nq += __shfl_xor(nq, o);
  const double sq = sqrt(nq);
  int64_t walked = 0;
  for (int i = 1; i <= ix.J; ++i) {  // J <= 64
    if (!((levels >> (i - 1)) & 1)) continue;
    const int seg = t * ix.J + (i - 1);
    const int64_t s0 = (int64_t)ix.seg_off[seg];
    const int64_t cnt = (int64_t)ix.seg_off[seg + 1] - s0;
    if (cnt == 0) continue;
    const uint32_t cap = ix.seg_cap[seg], mask = cap - 1;
    const double Tlo = lc.T[i - 1], Thi = lc.T[i], ri = lc.r[i];
    const double lo_s = Tlo * (1.0 - delta), hi_s = Thi * (1.0 + delta);
    uint32_t c = 0;
    int64_t base = 0;
    if (lane < L) {
      const uint64_t key = qk[((int64_t)seg * L + lane) * qs];
      ws.qk[lane] = key;
      const int64_t tb = (int64_t)ix.tab_seg_off[seg] + (int64_t)lane * cap;
      uint32_t sl = (uint32_t)key & mask;
      while (true) {
        const uint64_t v = ix.tab_key[tb + sl];
        if (v == key) {
          c = ix.tab_cnt[tb + sl];
          base = s0 * L + (int64_t)lane * cnt + ix.tab_start[tb + sl];
          break;
        }
        if (v == kEmpty) break;
        sl = (sl + 1) & mask;
      }
    }
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    const uint32_t total = __shfl(incl, 63);
    walked += total;
    if (lane < L) {
      ws.pre[lane] = incl - c;
      ws.base[lane] = base;
    }
    __builtin_amdgcn_wave_barrier();
    // exact decision and term of the queued points [head, head + count)
    auto drain = [&](uint32_t head, uint32_t count) {
      const bool valid = (uint32_t)lane < count;
      double v = 0.0;
      int32_t j = -1;
      if (valid) {
        j = ws.ring[(head + lane) & 127];
        const double D = ws.ringD[(head + lane) & 127];
        if (D >= Tlo && D < Thi) {
          v = level_weight(ix.cheb + i * kChebRow, sqrt(D) / ri);
        }
      }
      on_batch(v, j, valid, i);
    };
    uint32_t head = 0, tail = 0;
    for (uint32_t k0 = 0; k0 < total; k0 += 64) {
      const uint32_t k = k0 + lane;
      bool keep = false;
      int32_t j = -1;
      double D64 = 0.0;
      if (k < total) {
        int lo = 0, hi = L - 1;  // last table whose prefix is <= k
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (ws.pre[mid] <= k) lo = mid;
          else hi = mid - 1;
        }
        const int l = lo;
        const int32_t u = ix.csr[ws.base[l] + (k - ws.pre[l])];
        j = ix.members[s0 + u];
        const uint64_t* mk = ix.mkeys + (s0 + u) * L;
        bool seen = false;
#pragma unroll 4
        for (int l2 = 0; l2 < l; ++l2) seen |= mk[l2] == ws.qk[l2];
        if (!seen && j != self_idx) {
          // (||q|| - ||x||)^2 <= D <= (||q|| + ||x||)^2, with an absolute slack
          // e above the norms' rounding: a point that these bounds put
          // outside the level by more than the screen's own bound would fail
          // the fp32 screen too, so it is dropped without reading its row
          const double sx = ix.xn[j];
          const double e = 4e-12 * (sq + sx);
          const double up = sq + sx + e, dn = fmax(fabs(sq - sx) - e, 0.0);
          if (up * up * (1.0 + delta) < lo_s || dn * dn * (1.0 - delta) >= hi_s) {
            keep = false;
          } else {
            const double D32 = (double)dist2_both(qrow, ix.X + (int64_t)j * ix.dx, d, &D64);
            keep = D32 >= lo_s && D32 < hi_s;
          }
        }
      }
      const uint64_t km = __ballot(keep);
      const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
      if (keep) {
        ws.ring[(tail + pos) & 127] = j;
        ws.ringD[(tail + pos) & 127] = D64;
      }
      tail += (uint32_t)__popcll(km);
      __builtin_amdgcn_wave_barrier();
      if (tail - head >= 64) {
        drain(head, 64);
        head += 64;
        __builtin_amdgcn_wave_barrier();
      }
    }
    if (tail > head) drain(head, tail - head);
    __builtin_amdgcn_wave_barrier();
  }
  return walked;
}

// One wave per (query, copy): the copy's estimate and candidate counts.
__global__ __launch_bounds__(256) void probe_queries(const float* __restrict__ Q, int ldq, int64_t q0, int64_t mb,
                                                     IndexView ix, LevelConst lc, const uint64_t* __restrict__ qkeys,
                                                     int64_t ntab, int self_excl, double* __restrict__ Scopy,
                                                     int64_t* __restrict__ ncand, int64_t* __restrict__ nacc,
                                                     uint64_t* __restrict__ levels_out) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t pair = (int64_t)blockIdx.x * 4 + wave;
  if (pair >= mb * ix.K1) return;
  const int64_t ql = pair / ix.K1;
  const int t = (int)(pair % ix.K1);
  const float* qrow = Q + (q0 + ql) * ldq;
  __shared__ WalkScratch wsc[4];
  double acc = 0.0;
  int64_t nc = 0, na = 0;
  uint64_t hit = 0;  // levels with a positive term (wave-uniform)
  nc = walk_copy(ix, lc, t, qkeys + ql, mb, wsc[wave], qrow, self_excl ? q0 + ql : -1, ~0ULL,
                 [&](double v, int32_t j, bool valid, int i) {
                   acc += v;
                   na += v > 0.0 ? 1 : 0;
                   if (__ballot(v > 0.0)) hit |= 1ULL << (i - 1);
                 });
  for (int o = 32; o > 0; o >>= 1) {
    acc += __shfl_xor(acc, o);
    na += __shfl_xor(na, o);
  }
  if (lane == 0) {
    Scopy[ql * ix.K1 + t] = acc;
    if (levels_out) levels_out[(q0 + ql) * ix.K1 + t] = hit;
    if (ncand) atomicAdd(reinterpret_cast<unsigned long long*>(ncand + q0 + ql), (unsigned long long)nc);
    if (nacc) atomicAdd(reinterpret_cast<unsigned long long*>(nacc + q0 + ql), (unsigned long long)na);
  }
}

__device__ inline double wave_incl_scan_f64(double v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  return v;
}

// Edge draws from the estimator's terms: one wave per node i (queried against
// the data without its own point).  Lane r < s holds draw r: target
// U(i, r) * sum_t S'_t(i), its copy (cumulative over copies) and remainder;
// each needed copy is walked once, in batches whose inclusive prefix sums
// locate every pending remainder.
__global__ __launch_bounds__(256) void draw_lsh(IndexView ix, LevelConst lc, const uint64_t* __restrict__ qkeys,
                                                int64_t ntab, int64_t q0, int64_t mb, const double* __restrict__ Scopy,
                                                const uint64_t* __restrict__ levels, const double* __restrict__ rest,
                                                int s, uint64_t seed,
                                                int64_t* __restrict__ src, int64_t* __restrict__ dst,
                                                double* __restrict__ w) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ql = (int64_t)blockIdx.x * 4 + wave;
  if (ql >= mb) return;
  const int64_t qi = q0 + ql;
  const float* qrow = ix.X + qi * ix.dx;
  __shared__ WalkScratch wsc[4];
  const double* sc = Scopy + ql * ix.K1;
  double tot = 0.0;
  for (int t = 0; t < ix.K1; ++t) tot += sc[t];
  // this lane's draw
  const bool mine = lane < s;
  int tsel = -1;
  double resid = 0.0;
  int64_t pick = -1;
  if (mine && tot > 0.0) {
    const uint64_t ds = stream_state(seed, kTagDraw, (uint64_t)qi, 0);
    const double u = (double)(mix64_hd(ds + (uint64_t)(lane + 1) * kGamma) >> 11) * 0x1.0p-53;
    const double target = u * tot;
    double c = 0.0;
    for (int t = 0; t < ix.K1; ++t) {
      if (c + sc[t] > target) {
        tsel = t;
        break;
      }
      c += sc[t];
    }
    if (tsel < 0) {
      for (int t = ix.K1 - 1; t >= 0; --t)
        if (sc[t] > 0.0) {
          tsel = t;
          break;
        }
      c = 0.0;
      for (int t = 0; t < tsel; ++t) c += sc[t];
    }
    resid = target - c;
  }
  for (int t = 0; t < ix.K1; ++t) {
    if (__ballot(mine && tsel == t) == 0) continue;
    double running = 0.0;
    int32_t lastj = -1;
    // levels without a positive term change neither the running sum nor the
    // last positive point, so the walk skips them
    const uint64_t lv = levels ? levels[qi * ix.K1 + t] : ~0ULL;
    walk_copy(ix, lc, t, qkeys + ql, mb, wsc[wave], qrow, qi, lv, [&](double v, int32_t j, bool valid, int) {
      const double incl = wave_incl_scan_f64(v);
      const double btot = __shfl(incl, 63);
      const uint64_t pos = __ballot(v > 0.0);
      if (pos) lastj = __shfl(j, 63 - __clzll((long long)pos));
      uint64_t pend = __ballot(mine && tsel == t && pick < 0 && resid < running + btot);
      while (pend) {
        const int r = __ffsll((long long)pend) - 1;
        pend &= pend - 1;
        const double x = __shfl(resid, r);
        // only a positive value can be the crossing (past the last positive
        // value the tree scan may differ from it by a rounding); with none,
        // the draw stays pending for the next block or the fallback below
        const uint64_t over = __ballot(running + incl > x) & pos;
        const int kl = over ? __ffsll((long long)over) - 1 : 0;
        const int32_t jj = __shfl(j, kl);
        if (lane == r && over) pick = jj;
      }
      running += btot;
    });
    if (mine && tsel == t && pick < 0) pick = lastj;  // rounding left the remainder above the total
  }
  if (mine) {
    const int64_t e = qi * s + lane;
    src[e] = qi;
    dst[e] = pick;
    w[e] = pick >= 0 ? 1.0 / ((double)s * (1.0 / rest[qi] + 1.0 / rest[pick])) : 0.0;
  }
}

__global__ void mean_copies(const double* __restrict__ Scopy, int64_t q0, int64_t mb, int K1,
                            double* __restrict__ S_out, double* __restrict__ copies_out) {
  const int64_t ql = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ql >= mb) return;
  double s = 0.0;
  for (int t = 0; t < K1; ++t) {
    const double v = Scopy[ql * K1 + t];
    s += v;
    if (copies_out) copies_out[(q0 + ql) * K1 + t] = v;
  }
  S_out[q0 + ql] = s / (double)K1;
}

__global__ void one_plus(const double* __restrict__ v, int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = 1.0 + v[i];
}

__global__ void zero_i64(int64_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Bucket join (query batches with d <= 128 and L <= 32).  The batch's queries
// are grouped by the bucket they fall in, per table; a wave then takes up to
// 64 queries of one bucket (one per lane, row in registers) against up to
// kJoinMembers members of that bucket, which it stages through LDS
// kJoinChunk rows at a time, so that every member row is read once per 64
// queries instead of once per query.  Per pair: first-table dedupe, self
// exclusion and the fp32 distance screen; the survivors of a staged chunk are
// then settled per lane in member order (fp64 distance, level test, term).
// A lane's partial over its member range goes to tpart; combine_groups adds
// the ranges of a bucket in order and the tables of a copy in order, so a
// query's estimate does not depend on the other queries of its batch.
// ---------------------------------------------------------------------------
constexpr int kJoinMembers = 512;
constexpr int kJoinChunk = 32;

// Bytes of dynamic LDS of one join wave (layout: rows, point ids, member
// norms, member keys, query keys).  With L <= kJoinRegKeys + 1 the query
// keys of the earlier tables are held in registers instead (fewer LDS bytes
// per wave, more waves per CU).
constexpr int kJoinRegKeys = 7;
__host__ __device__ inline int join_lds_rows(int dq) { return kJoinChunk * (dq + 4) * 4; }
__host__ __device__ inline int join_lds_bytes(int dq, int L, bool reg_keys) {
  const int lm1 = L > 1 ? L - 1 : 1;
  return join_lds_rows(dq) + kJoinChunk * 8 + kJoinChunk * lm1 * 8 + (reg_keys ? 0 : lm1 * 64 * 8);
}

// The bucket (global slot) of every (table, query) pair of the batch (pair
// e = table * mb + query), or -1, and the pair's rank among the bucket's
// queries (arrival order; lanes of a wave that share a bucket take one atomic).
__global__ __launch_bounds__(256) void locate_queries(const uint64_t* __restrict__ qkeys, int64_t total, int64_t mb,
                                                      int L, const uint64_t* __restrict__ tab_seg_off,
                                                      const uint32_t* __restrict__ seg_cap,
                                                      const uint64_t* __restrict__ tab_key, int32_t* __restrict__ qslot,
                                                      uint32_t* __restrict__ qrank, uint32_t* __restrict__ qcount) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); e0 < total; e0 += stride) {
    const int64_t e = e0 + lane;
    int32_t slot = -1;
    if (e < total) {
      const int64_t g = e / mb;
      const int64_t seg = g / L;
      const int l = (int)(g % L);
      const uint32_t cap = seg_cap[seg];
      if (cap > 0) {
        const uint64_t key = qkeys[e];
        const int64_t tb = (int64_t)tab_seg_off[seg] + (int64_t)l * cap;
        uint32_t sl = (uint32_t)key & (cap - 1);
        while (true) {
          const uint64_t v = tab_key[tb + sl];
          if (v == key) {
            slot = (int32_t)(tb + sl);
            break;
          }
          if (v == kEmpty) break;
          sl = (sl + 1) & (cap - 1);
        }
      }
      qslot[e] = slot;
    }
    // group the wave's lanes by bucket (ballots only), then let every
    // group's lowest lane take the group's ranks with one atomic, all groups
    // in the same instruction
    int leader_of = lane;
    uint32_t gsize = 0, intra = 0;
    uint64_t pending = __ballot(slot >= 0);
    while (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const int32_t ls = __shfl(slot, leader);
      const uint64_t same = __ballot(slot == ls) & pending;
      if ((same >> lane) & 1ull) {
        leader_of = leader;
        intra = (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
      }
      if (lane == leader) gsize = (uint32_t)__popcll(same);
      pending &= ~same;
    }
    uint32_t base = 0;
    if (gsize > 0) base = atomicAdd(qcount + slot, gsize);
    base = __shfl(base, leader_of);
    if (slot >= 0) qrank[e] = base + intra;
  }
}

__global__ __launch_bounds__(256) void scatter_queries(const int32_t* __restrict__ qslot,
                                                       const uint32_t* __restrict__ qrank, int64_t total, int64_t mb,
                                                       const uint64_t* __restrict__ qstart, int32_t* __restrict__ qlist) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t slot = qslot[e];
    if (slot >= 0) qlist[qstart[slot] + qrank[e]] = (int32_t)(e % mb);
  }
}

// Tasks of a bucket: ceil(queries / 64) x ceil(members / kJoinMembers).
__global__ __launch_bounds__(256) void count_tasks(const uint32_t* __restrict__ qcount,
                                                   const uint32_t* __restrict__ tab_cnt, int64_t nslots,
                                                   uint32_t* __restrict__ ntask) {
  const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= nslots) return;
  const uint32_t nq = qcount[sl], nm = tab_cnt[sl];
  ntask[sl] = (nq > 0 && nm > 0) ? ((nq + 63) / 64) * ((nm + kJoinMembers - 1) / kJoinMembers) : 0u;
}

// Largest index s in [0, n) with v[s] <= x (v ascending, v[0] <= x).
__device__ inline int64_t last_le(const uint64_t* __restrict__ v, int64_t n, uint64_t x) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (v[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int DQ, int QKR>
__global__ __launch_bounds__(64) void join_buckets(IndexView ix, LevelConst lc, const float* __restrict__ Q, int ldq,
                                                   int64_t q0, const uint64_t* __restrict__ qkeys, int64_t mb,
                                                   const uint32_t* __restrict__ qcount,
                                                   const uint64_t* __restrict__ qstart,
                                                   const int32_t* __restrict__ qlist,
                                                   const uint64_t* __restrict__ task_base, int64_t nslots, int nseg,
                                                   int self_excl, double* __restrict__ tpart,
                                                   int64_t* __restrict__ nacc) {
  extern __shared__ __attribute__((aligned(16))) unsigned char jlds[];
  constexpr int RS = DQ + 4;  // LDS row stride (floats)
  const int lane = threadIdx.x;
  const int L = ix.L, d = ix.d, dx = ix.dx;
  const int lm1 = L > 1 ? L - 1 : 1;
  float* rows = reinterpret_cast<float*>(jlds);
  int32_t* jl = reinterpret_cast<int32_t*>(jlds + join_lds_rows(DQ));
  float* nxl = reinterpret_cast<float*>(jl + kJoinChunk);
  uint64_t* mk = reinterpret_cast<uint64_t*>(jlds + join_lds_rows(DQ) + kJoinChunk * 8);
  uint64_t* qk = mk + kJoinChunk * lm1;  // query keys in LDS (QKR == 0)
  uint64_t qkr[QKR > 0 ? QKR : 1];       // or in registers (l <= QKR)

  const int64_t task = blockIdx.x;
  const int64_t slot = last_le(task_base, nslots + 1, (uint64_t)task);
  const int seg = (int)last_le(ix.tab_seg_off, (int64_t)nseg + 1, (uint64_t)slot);
  const uint32_t cap = ix.seg_cap[seg];
  const int l = (int)((slot - (int64_t)ix.tab_seg_off[seg]) / cap);
  const int i = seg % ix.J + 1;
  const int64_t s0 = (int64_t)ix.seg_off[seg];
  const int64_t cnt = (int64_t)ix.seg_off[seg + 1] - s0;
  const uint32_t nq = qcount[slot], nm = ix.tab_cnt[slot];
  const int nmc = (int)((nm + kJoinMembers - 1) / kJoinMembers);
  const int64_t r = task - (int64_t)task_base[slot];
  const int qc = (int)(r / nmc), mc = (int)(r % nmc);
  const int64_t mbase = s0 * L + (int64_t)l * cnt + ix.tab_start[slot];
  const double Tlo = lc.T[i - 1], Thi = lc.T[i], ri = lc.r[i];
  const float Tlo_f = (float)Tlo, Thi_f = (float)Thi;
  // |fl(D) - D| <= ce (|q|^2 + |x|^2) for D = |q|^2 + |x|^2 - 2 q.x with fp32
  // fused dot products and norms (gamma bounds, with margin)
  const float ce = (float)(2 * DQ + 24) * 0x1.0p-24f;

  const uint32_t qp = (uint32_t)qc * 64u + (uint32_t)lane;
  const bool qvalid = qp < nq;
  const int32_t ql = qlist[qstart[slot] + (qvalid ? qp : 0u)];
  const int64_t self_idx = self_excl ? q0 + ql : -1;
  float q[DQ];
  {
    const float* qrow = Q + (q0 + ql) * (int64_t)ldq;
#pragma unroll
    for (int h = 0; h < DQ; ++h) q[h] = h < d ? qrow[h] : 0.0f;
  }
  float qnorm = 0.0f;
#pragma unroll
  for (int h = 0; h < DQ; ++h) qnorm = __builtin_fmaf(q[h], q[h], qnorm);
  if constexpr (QKR > 0) {
#pragma unroll
    for (int l2 = 0; l2 < QKR; ++l2) qkr[l2] = l2 < l ? qkeys[((int64_t)seg * L + l2) * mb + ql] : 0ull;
  } else {
    for (int l2 = 0; l2 < l; ++l2) qk[l2 * 64 + lane] = qkeys[((int64_t)seg * L + l2) * mb + ql];
  }
  if (dx < DQ)
    for (int e = lane; e < kJoinChunk * RS; e += 64) rows[e] = 0.0f;

  double acc = 0.0;
  int64_t na = 0;
  const int dx4 = dx >> 2;
  const int kbeg = mc * kJoinMembers;
  const int kend = (int)min((uint32_t)(kbeg + kJoinMembers), nm);
  for (int k0 = kbeg; k0 < kend; k0 += kJoinChunk) {
    const int nk = min(kJoinChunk, kend - k0);
    __builtin_amdgcn_wave_barrier();
    if (lane < nk) {
      const int32_t u = ix.csr[mbase + k0 + lane];
      jl[lane] = ix.members[s0 + u];
      const uint64_t* mrow = ix.mkeys + (s0 + u) * L;
      for (int l2 = 0; l2 < l; ++l2) mk[lane * lm1 + l2] = mrow[l2];
    }
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < nk * dx4; e += 64) {
      const int rr = e / dx4, c4 = e - rr * dx4;
      const float4 v = reinterpret_cast<const float4*>(ix.X + (int64_t)jl[rr] * dx)[c4];
      *reinterpret_cast<float4*>(&rows[rr * RS + 4 * c4]) = v;
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < nk) {
      float nr = 0.0f;
#pragma unroll
      for (int h4 = 0; h4 < DQ / 4; ++h4) {
        const float4 xv = *reinterpret_cast<const float4*>(&rows[lane * RS + 4 * h4]);
        nr = __builtin_fmaf(xv.x, xv.x, nr);
        nr = __builtin_fmaf(xv.y, xv.y, nr);
        nr = __builtin_fmaf(xv.z, xv.z, nr);
        nr = __builtin_fmaf(xv.w, xv.w, nr);
      }
      nxl[lane] = nr;
    }
    __builtin_amdgcn_wave_barrier();
    uint32_t mask = 0;
    for (int m = 0; m < nk; ++m) {
      const float* xr = &rows[m * RS];
      float p0 = 0.0f, p1 = 0.0f;
#pragma unroll
      for (int h4 = 0; h4 < DQ / 4; ++h4) {
        const float4 xv = *reinterpret_cast<const float4*>(xr + 4 * h4);
        p0 = __builtin_fmaf(q[4 * h4], xv.x, p0);
        p1 = __builtin_fmaf(q[4 * h4 + 1], xv.y, p1);
        p0 = __builtin_fmaf(q[4 * h4 + 2], xv.z, p0);
        p1 = __builtin_fmaf(q[4 * h4 + 3], xv.w, p1);
      }
      const float sn = qnorm + nxl[m];
      const float D32 = __builtin_fmaf(-2.0f, p0 + p1, sn);
      const float E = ce * sn;
      bool keep = qvalid && D32 >= Tlo_f - E && D32 < Thi_f + E;
      if (__ballot(keep)) {
        bool seen = (int64_t)jl[m] == self_idx;
        if constexpr (QKR > 0) {
#pragma unroll
          for (int l2 = 0; l2 < QKR; ++l2)
            if (l2 < l) seen |= mk[m * lm1 + l2] == qkr[l2];
        } else {
          for (int l2 = 0; l2 < l; ++l2) seen |= mk[m * lm1 + l2] == qk[l2 * 64 + lane];
        }
        keep = keep && !seen;
      }
      mask |= keep ? (1u << m) : 0u;
    }
    // survivors, per lane in member order
    while (__ballot(mask != 0u)) {
      if (mask) {
        const int m = __builtin_ctz(mask);
        mask &= mask - 1u;
        const float* xr = &rows[m * RS];
        double D = 0.0;
#pragma unroll
        for (int h4 = 0; h4 < DQ / 4; ++h4) {
          const float4 xv = *reinterpret_cast<const float4*>(xr + 4 * h4);
          const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            float qh = q[4 * h4 + e];
            asm volatile("" : "+v"(qh));  // keeps the widening here (no hoisted fp64 copy of the row)
            const double t0 = (double)qh - (double)xs[e];
            D = __builtin_fma(t0, t0, D);
          }
          if (h4 % 2 == 1) __builtin_amdgcn_sched_barrier(0);
        }
        if (D >= Tlo && D < Thi) {
          acc += level_weight(ix.cheb + i * kChebRow, sqrt(D) / ri);
          ++na;
        }
      }
    }
  }
  tpart[task * 64 + lane] = acc;
  if (qvalid && na > 0 && nacc) atomicAdd(reinterpret_cast<unsigned long long*>(nacc + q0 + ql), (unsigned long long)na);
}

// Per query: the copy sums from the lane partials (bucket ranges in order,
// then the tables and levels of a copy in order) and the candidate count.
__global__ __launch_bounds__(256) void combine_groups(const int32_t* __restrict__ qslot,
                                                      const uint32_t* __restrict__ qrank, int64_t mb, int64_t ntab,
                                                      int K1, const uint32_t* __restrict__ tab_cnt,
                                                      const uint64_t* __restrict__ task_base,
                                                      const double* __restrict__ tpart, int64_t q0,
                                                      double* __restrict__ Scopy, int64_t* __restrict__ ncand) {
  const int64_t ql = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ql >= mb) return;
  const int64_t per_copy = ntab / K1;
  int64_t nc = 0;
  for (int t = 0; t < K1; ++t) {
    double acc = 0.0;
    for (int64_t g = (int64_t)t * per_copy; g < (int64_t)(t + 1) * per_copy; ++g) {
      const int64_t e = g * mb + ql;
      const int32_t slot = qslot[e];
      if (slot < 0) continue;
      const uint32_t rank = qrank[e], nm = tab_cnt[slot];
      const int64_t nmc = (nm + kJoinMembers - 1) / kJoinMembers;
      const int64_t base = (int64_t)task_base[slot] + (int64_t)(rank / 64) * nmc;
      const int lane = (int)(rank % 64);
      double gs = 0.0;
      for (int64_t c = 0; c < nmc; ++c) gs += tpart[(base + c) * 64 + lane];
      acc += gs;
      nc += nm;
    }
    Scopy[ql * K1 + t] = acc;
  }
  if (ncand) ncand[q0 + ql] += nc;
}

__global__ void zero_u32(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------------------
// E2LSH table with near-neighbour listing (the E2LSH class of Sec. "Random
// Projection" / "Boosting the Probability" and its get_near_neighbours): one
// segment holding all n points, L open-addressing tables, CSR members
// ascending within a bucket (built by build_tables_sorted).  A query lists the points
// that collide with it in some table: table by table, ascending within a
// bucket, each point in the first table where it collides.
// ---------------------------------------------------------------------------
// One wave per query.  LIST = false: counts[q]; LIST = true: the list at
// idx_out + offsets[q].
template <bool LIST>
__global__ __launch_bounds__(256) void nn_walk(const uint64_t* __restrict__ qkeys, int64_t m, int L, int64_t n,
                                               uint32_t cap, const uint64_t* __restrict__ tab_key,
                                               const uint32_t* __restrict__ tab_start,
                                               const uint32_t* __restrict__ tab_cnt, const int32_t* __restrict__ csr,
                                               const uint64_t* __restrict__ mkeys, uint32_t* __restrict__ counts,
                                               const uint64_t* __restrict__ offsets, int32_t* __restrict__ idx_out) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t q = (int64_t)blockIdx.x * 4 + wave;
  if (q >= m) return;
  __shared__ uint64_t sqk[4][64];
  __shared__ int64_t sbase[4][64];
  __shared__ uint32_t spre[4][64];
  uint32_t c = 0;
  int64_t base = 0;
  if (lane < L) {
    const uint64_t key = qkeys[q * L + lane];
    sqk[wave][lane] = key;
    const int64_t tb = (int64_t)lane * cap;
    uint32_t sl = (uint32_t)key & (cap - 1);
    while (true) {
      const uint64_t v = tab_key[tb + sl];
      if (v == key) {
        c = tab_cnt[tb + sl];
        base = (int64_t)lane * n + tab_start[tb + sl];
        break;
      }
      if (v == kEmpty) break;
      sl = (sl + 1) & (cap - 1);
    }
  }
  uint32_t incl = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  const uint32_t total = __shfl(incl, 63);
  if (lane < L) {
    spre[wave][lane] = incl - c;
    sbase[wave][lane] = base;
  }
  __builtin_amdgcn_wave_barrier();
  int64_t kept = 0;
  const int64_t out0 = LIST ? (int64_t)offsets[q] : 0;
  for (uint32_t k0 = 0; k0 < total; k0 += 64) {
    const uint32_t k = k0 + lane;
    bool keep = false;
    int32_t j = 0;
    if (k < total) {
      int lo = 0, hi = L - 1;  // last table whose prefix is <= k
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (spre[wave][mid] <= k) lo = mid;
        else hi = mid - 1;
      }
      j = csr[sbase[wave][lo] + (k - spre[wave][lo])];
      const uint64_t* mk = mkeys + (int64_t)j * L;
      bool seen = false;
      for (int l2 = 0; l2 < lo; ++l2) seen |= mk[l2] == sqk[wave][l2];
      keep = !seen;
    }
    const uint64_t km = __ballot(keep);
    if constexpr (LIST) {
      const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
      if (keep) idx_out[out0 + kept + pos] = j;
    }
    kept += __popcll(km);
  }
  if (!LIST && lane == 0) counts[q] = (uint32_t)kept;
}

int ceil_log2_i64(int64_t n) {
  int J = 0;
  while (((int64_t)1 << J) < n) ++J;
  return J;
}

double collision_p_host(double c) {
  if (c <= 0.0) return 1.0;
  const double inv_sqrt_2pi = 0.39894228040143267794;
  return std::erf(2.0 * std::sqrt(2.0) / c) - 0.5 * inv_sqrt_2pi * c * (-std::expm1(-8.0 / (c * c)));
}

double recovery_host(double c, int K, int L) {
  const double x = std::pow(collision_p_host(c), (double)K);
  if (x >= 1.0) return 1.0;
  return -std::expm1((double)L * std::log1p(-x));
}

// Chebyshev interpolants (33 terms) of each level's term weight
// w_i(c) = exp(-a (r_i c)^2) / (p_i R_i(c)) over the level's range of
// c = sqrt(D) / r_i, D in [T_{i-1}, T_i): c in [sqrt(T_{i-1} / T_i), 1].  The
// weight is smooth there (a factor of two in exp(-a D), a recovery
// probability bounded away from 0); the interpolant agrees with the closed
// form to about 2e-14 relative (checked for K in 3..12, L in 4..64 and the
// first 30 levels).
std::vector<double> weight_levels(const LshParams& prm) {
  const int J = prm.shape.J, n = kChebTerms;
  const int K = prm.shape.K, L = prm.shape.L;
  const bool literal = (prm.flags & STAG_LSH_LITERAL) != 0;
  std::vector<double> out((size_t)(J + 1) * kChebRow, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 1; i <= J; ++i) {
    const double lo = std::sqrt(prm.lc_T[i - 1]) / prm.lc_r[i];
    double* row = out.data() + (size_t)i * kChebRow;
    row[0] = lo;
    row[1] = 2.0 / (1.0 - lo);
    std::vector<double> f((size_t)n);
    for (int j = 0; j < n; ++j) {
      const double x = std::cos(pi * (j + 0.5) / n);
      const double c = lo + (1.0 - lo) * (x + 1.0) / 2.0;
      const double rc = prm.lc_r[i] * c;
      const double R = literal ? 1.0 : recovery_host(c, K, L);
      f[(size_t)j] = std::exp(-prm.a * rc * rc) / (prm.lc_p[i] * R);
    }
    for (int k = 0; k < n; ++k) {
      double sum = 0.0;
      for (int j = 0; j < n; ++j) sum += f[(size_t)j] * std::cos(pi * k * (j + 0.5) / n);
      row[2 + k] = 2.0 * sum / n;
    }
  }
  return out;
}

}  // namespace

// Parameter reading for CKNSGaussianKDE(data, a, eps, min_mu, K1, K2_constant,
// p_offset); see the file header.
stag_status lsh_derive_params(int64_t n, double a, double eps, const stag_lsh_params* p, LshParams* out) {
  stag_lsh_params dflt = {};
  if (!p) p = &dflt;
  if (n < 1) return fail(STAG_E_INVAL, "lsh: n must be >= 1");
  if (!(a > 0.0) || !std::isfinite(a)) return fail(STAG_E_INVAL, "lsh: a must be positive and finite");
  if (!(eps > 0.0 && eps < 1.0)) return fail(STAG_E_INVAL, "lsh: eps must be in (0, 1)");
  if (p->p_offset < 0 || p->p_offset > 60) return fail(STAG_E_INVAL, "lsh: p_offset must be in [0, 60]");
  if (p->flags & ~(uint32_t)(STAG_LSH_LITERAL | STAG_LSH_ALL_SAMPLED))
    return fail(STAG_E_INVAL, "lsh: unknown flags 0x%x", p->flags);
  LshParams& s = *out;
  s.flags = p->flags;
  s.seed = p->seed;
  const bool default_mu = !(p->min_mu > 0.0);
  s.shape.mu_min = default_mu ? 1.0 / (double)n : p->min_mu;
  int J = default_mu ? ceil_log2_i64(n) : (int)std::ceil(std::log2(1.0 / s.shape.mu_min));
  if (J < 1) J = 1;
  if (J > 64) return fail(STAG_E_INVAL, "lsh: min_mu too small (more than 64 levels)");
  s.shape.J = J;
  const int L = (p->k2_constant > 0.0) ? (int)std::ceil(std::min(p->k2_constant, 1e6)) : std::max(1, ceil_log2_i64(n));
  if (L > 64) return fail(STAG_E_UNSUPPORTED, "lsh: at most 64 tables per level (K2_constant <= 64)");
  s.shape.L = L;
  int K = 1;
  for (int k = 2; k <= 64; ++k) {
    if (recovery_host(1.0, k, L) >= 1.0 - eps / 4.0) K = k;
    else break;
  }
  s.shape.K = K;
  s.shape.K1 = (p->k1 > 0) ? p->k1 : std::max(1, (int)std::ceil(std::log2((double)n) / (eps * eps)));
  const double ln2 = std::log(2.0);
  s.lc_p[0] = 1.0;
  s.lc_T[0] = 0.0;
  s.lc_r[0] = 0.0;
  s.thr[0] = 0;
  for (int i = 1; i <= J; ++i) {
    double pi;
    if (p->flags & STAG_LSH_ALL_SAMPLED) pi = 1.0;
    else if (default_mu) pi = std::ldexp(1.0, -i - p->p_offset);
    else pi = std::min(1.0, std::ldexp(1.0, -i) / ((double)n * s.shape.mu_min)) * std::ldexp(1.0, -p->p_offset);
    s.lc_p[i] = pi;
    s.thr[i] = (uint64_t)std::ldexp(pi, 53);
    s.lc_T[i] = (double)i * ln2 / a;
    s.lc_r[i] = std::sqrt(s.lc_T[i]);
  }
  s.a = a;
  s.eps = eps;
  s.n = n;
  return STAG_OK;
}

}  // namespace stag

// ---------------------------------------------------------------------------
// index object
// ---------------------------------------------------------------------------
struct stag_lsh_index {
  stag::LshParams prm;
  int d = 0, dx = 0, dg = 0, nch = 0, dreg = 0;
  int64_t nseg = 0, ntab = 0, M = 0, total_slots = 0;
  int device = 0;
  std::vector<uint64_t> h_seg_off;
  std::vector<std::pair<void*, size_t>> owned;  // blocks and their sizes
  char* arena = nullptr;  // current block of small index allocations
  size_t arena_used = 0;
  float* X = nullptr;
  double* xn = nullptr;
  double* G8 = nullptr;
  double* B = nullptr;
  uint64_t* seg_off = nullptr;
  int32_t* members = nullptr;
  uint64_t* mkeys = nullptr;
  uint64_t* tab_seg_off = nullptr;
  uint32_t* seg_cap = nullptr;
  uint64_t* tab_key = nullptr;
  uint32_t* tab_start = nullptr;
  uint32_t* tab_cnt = nullptr;
  int32_t* csr = nullptr;
  double* rlev = nullptr;
  double* cheb = nullptr;
  std::vector<double> h_cheb;
  uint64_t* thr = nullptr;
};

struct stag_e2lsh_table {
  int64_t n = 0;
  int d = 0, K = 0, L = 0, dg = 0;
  uint32_t cap = 0;
  int device = 0;
  std::vector<void*> owned;  // stream-ordered pool blocks
  double* G8 = nullptr;
  double* b = nullptr;
  uint64_t* mkeys = nullptr;
  uint64_t* tab_key = nullptr;
  uint32_t* tab_start = nullptr;
  uint32_t* tab_cnt = nullptr;
  int32_t* csr = nullptr;
  std::vector<uint64_t> h_off;  // host copies of the one-segment layout
  std::vector<uint32_t> h_cap;
};

namespace stag {
namespace {

// Index memory (cached device blocks, reused by later indexes): requests
// below 1 MiB are 256-byte slices of 4 MiB blocks, larger ones blocks of
// their own; all go back to the cache with the index.
template <typename T>
stag_status own_alloc(stag_lsh_index* idx, T** p, size_t count) {
  const size_t bytes = std::max<size_t>((count * sizeof(T) + 255) / 256 * 256, 256);
  const size_t kSmall = (size_t)1 << 20, kBlock = (size_t)4 << 20;
  auto raw = [&](void** v, size_t b) -> stag_status {
    STAG_TRY(cached_alloc(v, b));
    idx->owned.push_back({*v, b});
    return STAG_OK;
  };
  void* v = nullptr;
  if (bytes >= kSmall) {
    STAG_TRY(raw(&v, bytes));
  } else {
    if (idx->arena == nullptr || idx->arena_used + bytes > kBlock) {
      void* blk = nullptr;
      STAG_TRY(raw(&blk, kBlock));
      idx->arena = static_cast<char*>(blk);
      idx->arena_used = 0;
    }
    v = idx->arena + idx->arena_used;
    idx->arena_used += bytes;
  }
  *p = static_cast<T*>(v);
  return STAG_OK;
}

void free_index(stag_lsh_index* idx) {
  if (!idx) return;
  // callers have synchronised the device: nothing uses the memory any more
  for (const auto& b : idx->owned) cached_free(b.first, b.second);
  delete idx;
}

template <typename F>
stag_status dispatch_dreg(int dreg, F&& f) {
  switch (dreg) {
    case 16: return f(std::integral_constant<int, 16>());
    case 32: return f(std::integral_constant<int, 32>());
    case 64: return f(std::integral_constant<int, 64>());
    default: return f(std::integral_constant<int, 0>());
  }
}

__global__ void copy_rows(const float* __restrict__ src, int64_t n, int d, int dx, float* __restrict__ dst) {
  const int64_t total = n * dx;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / dx;
    const int c = (int)(e % dx);
    dst[e] = c < d ? src[r * d + c] : 0.0f;
  }
}

// xn[r] = ||x_r|| in binary64 (one wave per row; any summation order: the
// walk uses it only for bounds with a margin).
__global__ __launch_bounds__(256) void row_norms(const float* __restrict__ X, int64_t n, int dx,
                                                 double* __restrict__ xn) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  double s2 = 0.0;
  for (int c = lane; c < dx; c += 64) {
    const double v = X[r * dx + c];
    s2 = __builtin_fma(v, v, s2);
  }
  for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
  if (lane == 0) xn[r] = sqrt(s2);
}

stag_status create_index(const float* X, int64_t n, int d, double a, double eps, const stag_lsh_params* p,
                         stag_lsh_index* idx, hipStream_t st) {
  STAG_TRY(lsh_derive_params(n, a, eps, p, &idx->prm));
  LshParams& prm = idx->prm;
  const int J = prm.shape.J, L = prm.shape.L, K = prm.shape.K, K1 = prm.shape.K1;
  idx->d = d;
  idx->dx = (int)round_up(d, 4);
  idx->dreg = e2lsh_reg_dim(d);
  idx->dg = idx->dreg > 0 ? idx->dreg : d;
  idx->nch = (int)ceil_div(K, 8);
  idx->nseg = (int64_t)K1 * J;
  idx->ntab = idx->nseg * L;
  const int64_t nproj = idx->ntab * K;
  Workspace ws(st);

  STAG_TRY(own_alloc(idx, &idx->X, (size_t)n * idx->dx));
  hipLaunchKernelGGL(copy_rows, dim3((unsigned)std::min<int64_t>(ceil_div(n * idx->dx, 256), 65536)), dim3(256), 0,
                     st, X, n, d, idx->dx, idx->X);
  STAG_TRY(check_launch("copy_rows"));
  STAG_TRY(own_alloc(idx, &idx->xn, (size_t)n));
  hipLaunchKernelGGL(row_norms, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, idx->X, n, idx->dx, idx->xn);
  STAG_TRY(check_launch("row_norms"));

  // level constants
  STAG_TRY(own_alloc(idx, &idx->rlev, 65));
  STAG_TRY(own_alloc(idx, &idx->thr, 65));
  STAG_HIP(hipMemcpyAsync(idx->rlev, prm.lc_r, sizeof(double) * (J + 1), hipMemcpyHostToDevice, st));
  idx->h_cheb = weight_levels(prm);
  STAG_TRY(own_alloc(idx, &idx->cheb, idx->h_cheb.size()));
  STAG_HIP(hipMemcpyAsync(idx->cheb, idx->h_cheb.data(), sizeof(double) * idx->h_cheb.size(), hipMemcpyHostToDevice,
                          st));
  STAG_HIP(hipMemcpyAsync(idx->thr, prm.thr, sizeof(uint64_t) * (J + 1), hipMemcpyHostToDevice, st));

  // projections and offsets
  const float* G0 = p ? p->G0 : nullptr;
  STAG_TRY(own_alloc(idx, &idx->B, (size_t)nproj));
  if (p && p->b) {
    STAG_HIP(hipMemcpyAsync(idx->B, p->b, sizeof(double) * nproj, hipMemcpyDeviceToDevice, st));
  }
  if (!G0 || !(p && p->b)) {
    float* g = nullptr;
    STAG_TRY(ws.alloc(&g, (size_t)nproj * d));
    double* bb = nullptr;
    STAG_TRY(ws.alloc(&bb, (size_t)nproj));
    {
      ScopedTimer tm("lsh_gen_randomness", st);
      hipLaunchKernelGGL(gen_randomness, dim3((unsigned)std::min<int64_t>(ceil_div(nproj * d, 256), 65536)),
                         dim3(256), 0, st, prm.seed, nproj, d, g, bb);
    }
    STAG_TRY(check_launch("gen_randomness"));
    if (!G0) G0 = g;
    if (!(p && p->b)) STAG_HIP(hipMemcpyAsync(idx->B, bb, sizeof(double) * nproj, hipMemcpyDeviceToDevice, st));
  }
  STAG_TRY(own_alloc(idx, &idx->G8, (size_t)idx->ntab * idx->nch * idx->dg * 8));
  {
    ScopedTimer tm("lsh_scale_projections", st);
    const int64_t tot = idx->ntab * idx->nch * idx->dg * 8;
    hipLaunchKernelGGL(scale_projections, dim3((unsigned)std::min<int64_t>(ceil_div(tot, 256), 65536)), dim3(256), 0,
                       st, G0, idx->ntab, J, L, K, d, idx->dg, idx->nch, idx->rlev, idx->G8);
  }
  STAG_TRY(check_launch("scale_projections"));

  // subsamples
  const int nblk = (int)ceil_div(n, kMaskBlock);
  if (idx->nseg > 65535) return fail(STAG_E_UNSUPPORTED, "lsh: K1*J = %lld segments exceeds 65535", (long long)idx->nseg);
  uint32_t* cnt = nullptr;
  uint64_t* off = nullptr;
  const int64_t ncnt = idx->nseg * nblk;
  STAG_TRY(ws.alloc(&cnt, (size_t)ncnt));
  STAG_TRY(ws.alloc(&off, (size_t)ncnt + 1));
  {
    ScopedTimer tm("lsh_mask", st);
    hipLaunchKernelGGL(mask_count, dim3(nblk, (unsigned)idx->nseg), dim3(256), 0, st, prm.seed, J, n, nblk, idx->thr,
                       cnt);
    STAG_TRY(check_launch("mask_count"));
    STAG_TRY(exclusive_scan_u32(cnt, off, ncnt, ws, st));
  }
  // segment offsets: off[seg * nblk]; bring them to the host (one synchronisation)
  std::vector<uint64_t> all_off((size_t)ncnt + 1);
  STAG_HIP(hipMemcpyAsync(all_off.data(), off, sizeof(uint64_t) * (ncnt + 1), hipMemcpyDeviceToHost, st));
  STAG_HIP(hipStreamSynchronize(st));
  idx->h_seg_off.resize((size_t)idx->nseg + 1);
  for (int64_t s = 0; s < idx->nseg; ++s) idx->h_seg_off[s] = all_off[(size_t)s * nblk];
  idx->h_seg_off[idx->nseg] = all_off[ncnt];
  idx->M = (int64_t)idx->h_seg_off[idx->nseg];
  STAG_TRY(own_alloc(idx, &idx->seg_off, (size_t)idx->nseg + 1));
  STAG_HIP(hipMemcpyAsync(idx->seg_off, idx->h_seg_off.data(), sizeof(uint64_t) * (idx->nseg + 1),
                          hipMemcpyHostToDevice, st));
  STAG_TRY(own_alloc(idx, &idx->members, (size_t)idx->M));
  {
    ScopedTimer tm("lsh_mask", st);
    hipLaunchKernelGGL(mask_scatter, dim3(nblk, (unsigned)idx->nseg), dim3(256), 0, st, prm.seed, J, n, nblk,
                       idx->thr, off, idx->members);
  }
  STAG_TRY(check_launch("mask_scatter"));

  // member keys
  STAG_TRY(own_alloc(idx, &idx->mkeys, (size_t)idx->M * L));
  std::vector<MemberBlock> blocks;
  std::vector<uint32_t> cap((size_t)idx->nseg);
  std::vector<uint64_t> tso((size_t)idx->nseg + 1, 0);
  for (int64_t s = 0; s < idx->nseg; ++s) {
    const int64_t c = (int64_t)(idx->h_seg_off[s + 1] - idx->h_seg_off[s]);
    for (int64_t u0 = 0; u0 < c; u0 += 64) blocks.push_back({(int32_t)s, (int32_t)u0});
    uint32_t cp = 2;
    while ((int64_t)cp < 2 * c) cp <<= 1;
    cap[s] = c > 0 ? cp : 0;
    tso[s + 1] = tso[s] + (uint64_t)cap[s] * L;
  }
  idx->total_slots = (int64_t)tso[idx->nseg];
  if (!blocks.empty()) {
    MemberBlock* dblk = nullptr;
    STAG_TRY(ws.alloc(&dblk, blocks.size()));
    STAG_HIP(hipMemcpyAsync(dblk, blocks.data(), sizeof(MemberBlock) * blocks.size(), hipMemcpyHostToDevice, st));
    ScopedTimer tm("lsh_hash_members", st);
    STAG_TRY(dispatch_dreg(idx->dreg, [&](auto D) {
      hipLaunchKernelGGL(hash_members<decltype(D)::value>, dim3((unsigned)blocks.size()), dim3(256), 0, st, idx->X,
                         idx->dx, d, idx->dg, dblk, idx->seg_off, idx->members, idx->G8, idx->B, K, L, idx->nch,
                         idx->mkeys);
      return check_launch("hash_members");
    }));
  }

  // bucket tables
  STAG_TRY(own_alloc(idx, &idx->seg_cap, (size_t)idx->nseg));
  STAG_TRY(own_alloc(idx, &idx->tab_seg_off, (size_t)idx->nseg + 1));
  STAG_HIP(hipMemcpyAsync(idx->seg_cap, cap.data(), sizeof(uint32_t) * idx->nseg, hipMemcpyHostToDevice, st));
  STAG_HIP(hipMemcpyAsync(idx->tab_seg_off, tso.data(), sizeof(uint64_t) * (idx->nseg + 1), hipMemcpyHostToDevice, st));
  STAG_TRY(own_alloc(idx, &idx->tab_key, (size_t)idx->total_slots));
  STAG_TRY(own_alloc(idx, &idx->tab_start, (size_t)idx->total_slots));
  STAG_TRY(own_alloc(idx, &idx->tab_cnt, (size_t)idx->total_slots));
  STAG_TRY(own_alloc(idx, &idx->csr, (size_t)idx->M * L));
  if (idx->ntab > 0) {
    ScopedTimer tm("lsh_build_tables", st);
    STAG_TRY(build_tables_sorted(L, (int)idx->nseg, idx->M * L, idx->total_slots, idx->seg_off, idx->tab_seg_off,
                                 idx->seg_cap, idx->mkeys, idx->tab_key, idx->tab_start, idx->tab_cnt, idx->csr, ws,
                                 st));
  }
  STAG_HIP(hipGetDevice(&idx->device));
  // the workspace (sort buffers, counts) is released in stream order
  return STAG_OK;
}

IndexView make_view(const stag_lsh_index* idx) {
  const LshParams& prm = idx->prm;
  IndexView v;
  v.X = idx->X;
  v.xn = idx->xn;
  v.dx = idx->dx;
  v.d = idx->d;
  v.K1 = prm.shape.K1;
  v.J = prm.shape.J;
  v.L = prm.shape.L;
  v.K = prm.shape.K;
  v.a = prm.a;
  v.literal = (prm.flags & STAG_LSH_LITERAL) ? 1 : 0;
  v.cheb = idx->cheb;
  v.seg_off = idx->seg_off;
  v.members = idx->members;
  v.mkeys = idx->mkeys;
  v.tab_seg_off = idx->tab_seg_off;
  v.seg_cap = idx->seg_cap;
  v.tab_key = idx->tab_key;
  v.tab_start = idx->tab_start;
  v.tab_cnt = idx->tab_cnt;
  v.csr = idx->csr;
  return v;
}

LevelConst make_levels(const LshParams& prm) {
  LevelConst lc;
  for (int i = 0; i <= 64; ++i) {
    lc.p[i] = i <= prm.shape.J ? prm.lc_p[i] : 0.0;
    lc.T[i] = i <= prm.shape.J ? prm.lc_T[i] : 0.0;
    lc.r[i] = i <= prm.shape.J ? prm.lc_r[i] : 0.0;
  }
  return lc;
}

int64_t query_batch(const stag_lsh_index* idx, int64_t m) {
  int64_t mb = ((int64_t)1 << 30) / (8 * std::max<int64_t>(idx->ntab, 1)) / 64 * 64;
  return std::max<int64_t>(64, std::min(mb, round_up(m, 64)));
}

stag_status hash_query_batch(const stag_lsh_index* idx, const float* Q, int ldq, int64_t q0, int64_t cur,
                             uint64_t* qkeys, hipStream_t st) {
  const LshParams& prm = idx->prm;
  ScopedTimer tm("lsh_hash_queries", st);
  // tables per block: about 2048 blocks (8 waves per SIMD), as few reloads
  // of a query row as that allows
  const int64_t qb = ceil_div(cur, 256);
  const int64_t tpw = std::max<int64_t>(1, std::min<int64_t>(idx->ntab, idx->ntab * qb / 2048));
  const int K = prm.shape.K;
  if ((idx->dreg > 0 || idx->d <= 128) && K <= 64) {
    // one lane per projection: blocks of 4 waves x TW tables, 8 batches of 64 queries each
    // (64 < d <= 128: the lane's coefficients held as fp32)
    const int TW = 64 / K;
    const int qbatches = (int)std::max<int64_t>(8, ceil_div(cur, (int64_t)64 * 65535));  // grid.y <= 65535
    const dim3 grid((unsigned)ceil_div(idx->ntab, 4 * TW), (unsigned)ceil_div(cur, (int64_t)64 * qbatches));
    if (idx->dreg == 0) {
      hipLaunchKernelGGL((hash_lanes<128, true, true>), grid, dim3(256), 0, st, Q, ldq, q0, cur, idx->d, idx->G8,
                         idx->dg, idx->B, K, prm.shape.L, idx->nch, idx->ntab, TW, qbatches, qkeys,
                         (int32_t*)nullptr);
      return check_launch("hash_lanes");
    }
    return dispatch_dreg(idx->dreg, [&](auto D) {
      constexpr int DR = decltype(D)::value;
      if constexpr (DR > 0) {
        hipLaunchKernelGGL((hash_lanes<DR, true>), grid, dim3(256), 0, st, Q, ldq, q0, cur, idx->d, idx->G8,
                           idx->dg, idx->B, K, prm.shape.L, idx->nch, idx->ntab, TW, qbatches, qkeys,
                           (int32_t*)nullptr);
        return check_launch("hash_lanes");
      } else {
        return fail(STAG_E_UNSUPPORTED, "query hashing: no register width");
      }
    });
  }
  return dispatch_dreg(idx->dreg, [&](auto D) {
    hipLaunchKernelGGL(hash_queries<decltype(D)::value>, dim3((unsigned)qb, (unsigned)ceil_div(idx->ntab, tpw)),
                       dim3(256), 0, st, Q, ldq, q0, cur, idx->d, idx->dg, idx->G8, idx->B, prm.shape.K, prm.shape.L,
                       idx->nch, idx->ntab, (int)tpw, qkeys);
    return check_launch("hash_queries");
  });
}

bool join_applies(const stag_lsh_index* idx) {
  return idx->d <= 128 && idx->prm.shape.L <= 32 && idx->total_slots > 0 && idx->total_slots < INT32_MAX;
}

// Copy sums of one hashed query batch through the bucket join.
stag_status join_batch(const stag_lsh_index* idx, const float* Q, int ldq, int64_t q0, int64_t cur, int self_excl,
                       const uint64_t* qkeys, double* scopy, int64_t* ncand, int64_t* nacc, hipStream_t st) {
  const LshParams& prm = idx->prm;
  const int L = prm.shape.L, K1 = prm.shape.K1;
  const int64_t ntab = idx->ntab, nslots = idx->total_slots, pairs = cur * ntab;
  Workspace ws(st);
  int32_t* qslot = nullptr;
  uint32_t* qrank = nullptr;
  uint32_t* qcount = nullptr;
  uint64_t* qstart = nullptr;
  int32_t* qlist = nullptr;
  uint32_t* ntask = nullptr;
  uint64_t* task_base = nullptr;
  STAG_TRY(ws.alloc(&qslot, (size_t)pairs));
  STAG_TRY(ws.alloc(&qrank, (size_t)pairs));
  STAG_TRY(ws.alloc(&qcount, (size_t)nslots));
  STAG_TRY(ws.alloc(&qstart, (size_t)nslots + 1));
  STAG_TRY(ws.alloc(&qlist, (size_t)pairs));
  STAG_TRY(ws.alloc(&ntask, (size_t)nslots));
  STAG_TRY(ws.alloc(&task_base, (size_t)nslots + 1));
  const unsigned gpairs = (unsigned)std::min<int64_t>(ceil_div(pairs, 256), 65536);
  uint64_t ntasks = 0;
  {
    ScopedTimer tm("lsh_join_setup", st);
    hipLaunchKernelGGL(zero_u32, dim3((unsigned)std::min<int64_t>(ceil_div(nslots, 256), 65536)), dim3(256), 0, st,
                       qcount, nslots);
    hipLaunchKernelGGL(locate_queries, dim3(gpairs), dim3(256), 0, st, qkeys, pairs, cur, L, idx->tab_seg_off,
                       idx->seg_cap, idx->tab_key, qslot, qrank, qcount);
    STAG_TRY(check_launch("locate_queries"));
    STAG_TRY(exclusive_scan_u32(qcount, qstart, nslots, ws, st));
    hipLaunchKernelGGL(scatter_queries, dim3(gpairs), dim3(256), 0, st, qslot, qrank, pairs, cur, qstart, qlist);
    STAG_TRY(check_launch("scatter_queries"));
    hipLaunchKernelGGL(count_tasks, dim3((unsigned)ceil_div(nslots, 256)), dim3(256), 0, st, qcount, idx->tab_cnt,
                       nslots, ntask);
    STAG_TRY(check_launch("count_tasks"));
    STAG_TRY(exclusive_scan_u32(ntask, task_base, nslots, ws, st));
    STAG_HIP(hipMemcpyAsync(&ntasks, task_base + nslots, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    STAG_HIP(hipStreamSynchronize(st));
  }
  if (ntasks > (uint64_t)INT32_MAX) return fail(STAG_E_UNSUPPORTED, "lsh: %llu join tasks in one batch",
                                                (unsigned long long)ntasks);
  double* tpart = nullptr;
  STAG_TRY(ws.alloc(&tpart, (size_t)std::max<uint64_t>(ntasks, 1) * 64));
  const IndexView ix = make_view(idx);
  const LevelConst lc = make_levels(prm);
  if (ntasks > 0) {
    ScopedTimer tm("lsh_join", st);
    const int dq = idx->d <= 16 ? 16 : idx->d <= 32 ? 32 : idx->d <= 64 ? 64 : 128;
    const bool reg_keys = L <= kJoinRegKeys + 1;
    const size_t lds = (size_t)join_lds_bytes(dq, L, reg_keys);
    auto launch = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3((unsigned)ntasks), dim3(64), lds, st, ix, lc, Q, ldq, q0, qkeys, cur, qcount,
                         qstart, qlist, task_base, nslots, (int)idx->nseg, self_excl, tpart, nacc);
    };
    if (reg_keys) {
      switch (dq) {
        case 16: launch(join_buckets<16, kJoinRegKeys>); break;
        case 32: launch(join_buckets<32, kJoinRegKeys>); break;
        case 64: launch(join_buckets<64, kJoinRegKeys>); break;
        default: launch(join_buckets<128, kJoinRegKeys>); break;
      }
    } else {
      switch (dq) {
        case 16: launch(join_buckets<16, 0>); break;
        case 32: launch(join_buckets<32, 0>); break;
        case 64: launch(join_buckets<64, 0>); break;
        default: launch(join_buckets<128, 0>); break;
      }
    }
    STAG_TRY(check_launch("join_buckets"));
  }
  {
    ScopedTimer tm("lsh_combine", st);
    hipLaunchKernelGGL(combine_groups, dim3((unsigned)ceil_div(cur, 256)), dim3(256), 0, st, qslot, qrank, cur, ntab,
                       K1, idx->tab_cnt, task_base, tpart, q0, scopy, ncand);
    STAG_TRY(check_launch("combine_groups"));
  }
  return STAG_OK;
}

// Estimates for rows of Q (self_excl: Q is the index's own data and each
// row's own point is left out).  Optional per-copy values and counts.
// keys_buf (optional): the caller's buffer of query_batch(idx, m) x ntab
// keys; when the queries fit one batch it holds their keys on return.
stag_status query_index(const stag_lsh_index* idx, const float* Q, int ldq, int64_t m, int self_excl,
                        double* S_out, double* copies_out, int64_t* ncand, int64_t* nacc, hipStream_t st,
                        uint64_t* levels_out = nullptr, uint64_t* keys_buf = nullptr) {
  const LshParams& prm = idx->prm;
  const int K1 = prm.shape.K1;
  Workspace ws(st);
  const int64_t mb = query_batch(idx, m);
  uint64_t* qkeys = keys_buf;
  double* scopy = nullptr;
  if (!qkeys) STAG_TRY(ws.alloc(&qkeys, (size_t)mb * idx->ntab));
  STAG_TRY(ws.alloc(&scopy, (size_t)mb * K1));
  if (ncand) hipLaunchKernelGGL(zero_i64, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, ncand, m);
  if (nacc) hipLaunchKernelGGL(zero_i64, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, nacc, m);
  const IndexView ix = make_view(idx);
  const LevelConst lc = make_levels(prm);
  for (int64_t q0 = 0; q0 < m; q0 += mb) {
    const int64_t cur = std::min(mb, m - q0);
    STAG_TRY(hash_query_batch(idx, Q, ldq, q0, cur, qkeys, st));
    if (join_applies(idx)) {
      STAG_TRY(join_batch(idx, Q, ldq, q0, cur, self_excl, qkeys, scopy, ncand, nacc, st));
    } else {
      ScopedTimer tm("lsh_probe", st);
      hipLaunchKernelGGL(probe_queries, dim3((unsigned)ceil_div(cur * K1, 4)), dim3(256), 0, st, Q, ldq, q0, cur, ix,
                         lc, qkeys, idx->ntab, self_excl, scopy, ncand, nacc, levels_out);
      STAG_TRY(check_launch("probe_queries"));
    }
    hipLaunchKernelGGL(mean_copies, dim3((unsigned)ceil_div(cur, 256)), dim3(256), 0, st, scopy, q0, cur, K1, S_out,
                       copies_out);
    STAG_TRY(check_launch("mean_copies"));
  }
  return STAG_OK;
}

}  // namespace

// Edge sampling with the CKNS estimator (see draw_lsh): rest_i = mean over
// copies of the estimate of sum_{j != i} k_ij; deg = 1 + rest.
stag_status lsh_sample_edges(const stag_lsh_index* idx, int s, uint64_t seed, int64_t* src, int64_t* dst, double* w,
                             double* deg_out, hipStream_t st) {
  const LshParams& prm = idx->prm;
  const int K1 = prm.shape.K1;
  const int64_t n = prm.n;
  Workspace ws(st);
  double* rest = nullptr;
  double* copies = nullptr;
  STAG_TRY(ws.alloc(&rest, (size_t)n));
  STAG_TRY(ws.alloc(&copies, (size_t)n * K1));
  // with the per-query walk (not the bucket join) the estimate also records,
  // per node and copy, the levels with a positive term for the draws
  uint64_t* levels = nullptr;
  if (!join_applies(idx)) STAG_TRY(ws.alloc(&levels, (size_t)n * K1));
  const int64_t mb = query_batch(idx, n);
  uint64_t* qkeys = nullptr;
  STAG_TRY(ws.alloc(&qkeys, (size_t)mb * idx->ntab));
  STAG_TRY(query_index(idx, idx->X, idx->dx, n, 1, rest, copies, nullptr, nullptr, st, levels, qkeys));
  const IndexView ix = make_view(idx);
  const LevelConst lc = make_levels(prm);
  for (int64_t q0 = 0; q0 < n; q0 += mb) {
    const int64_t cur = std::min(mb, n - q0);
    // with one batch the estimate's keys are still in qkeys
    if (mb < n) STAG_TRY(hash_query_batch(idx, idx->X, idx->dx, q0, cur, qkeys, st));
    ScopedTimer tm("simgraph_draw_lsh", st);
    hipLaunchKernelGGL(draw_lsh, dim3((unsigned)ceil_div(cur, 4)), dim3(256), 0, st, ix, lc, qkeys, idx->ntab, q0,
                       cur, copies + q0 * K1, levels, rest, s, seed, src, dst, w);
    STAG_TRY(check_launch("draw_lsh"));
  }
  if (deg_out) {
    hipLaunchKernelGGL(one_plus, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, rest, n, deg_out);
    STAG_TRY(check_launch("one_plus"));
  }
  return STAG_OK;
}

}  // namespace stag

using namespace stag;

extern "C" {

stag_status stag_lsh_derive(int64_t n, double a, double eps, const stag_lsh_params* p, stag_lsh_shape* out) {
  if (!out) return fail(STAG_E_INVAL, "stag_lsh_derive: out is NULL");
  LshParams prm;
  STAG_TRY(lsh_derive_params(n, a, eps, p, &prm));
  *out = prm.shape;
  return STAG_OK;
}

stag_status stag_lsh_index_create(const float* X, int64_t n, int32_t d, double a, double eps,
                                  const stag_lsh_params* p, stag_lsh_index** out, hipStream_t stream) {
  if (!out) return fail(STAG_E_INVAL, "stag_lsh_index_create: out is NULL");
  *out = nullptr;
  if (!X) return fail(STAG_E_INVAL, "stag_lsh_index_create: X is NULL");
  if (n < 1 || n > 2147483647LL || d < 1 || d > 4096)
    return fail(STAG_E_INVAL, "stag_lsh_index_create: need 1 <= n < 2^31 and 1 <= d <= 4096");
  if ((p && p->G0) != (p && p->b))
    return fail(STAG_E_INVAL, "stag_lsh_index_create: pass both G0 and b, or neither");
  LshParams prm;
  STAG_TRY(lsh_derive_params(n, a, eps, p, &prm));
  clear_error();
  stag_lsh_index* idx = new (std::nothrow) stag_lsh_index();
  if (!idx) return fail(STAG_E_NOMEM, "stag_lsh_index_create: host allocation failed");
  stag_status stt = create_index(X, n, d, a, eps, p, idx, stream);
  if (stt != STAG_OK) {
    (void)hipStreamSynchronize(stream);
    free_index(idx);
    return stt;
  }
  *out = idx;
  return STAG_OK;
}

stag_status stag_lsh_index_shape(const stag_lsh_index* idx, stag_lsh_shape* out) {
  if (!idx || !out) return fail(STAG_E_INVAL, "stag_lsh_index_shape: NULL argument");
  *out = idx->prm.shape;
  return STAG_OK;
}

stag_status stag_lsh_index_query_ex(const stag_lsh_index* idx, const float* Q, int64_t m, double* S_out,
                                    double* S_copies, int64_t* n_cand, int64_t* n_acc, hipStream_t stream) {
  if (!idx || !Q || !S_out) return fail(STAG_E_INVAL, "stag_lsh_index_query: NULL argument");
  if (m < 1) return fail(STAG_E_INVAL, "stag_lsh_index_query: m must be >= 1");
  clear_error();
  return query_index(idx, Q, idx->d, m, 0, S_out, S_copies, n_cand, n_acc, stream);
}

stag_status stag_lsh_index_query(const stag_lsh_index* idx, const float* Q, int64_t m, double* S_out,
                                 hipStream_t stream) {
  return stag_lsh_index_query_ex(idx, Q, m, S_out, nullptr, nullptr, nullptr, stream);
}

stag_status stag_lsh_index_segment(const stag_lsh_index* idx, int32_t t, int32_t i, int64_t* count,
                                   int32_t* members_host, uint64_t* keys_host, hipStream_t stream) {
  if (!idx || !count) return fail(STAG_E_INVAL, "stag_lsh_index_segment: NULL argument");
  const int J = idx->prm.shape.J, L = idx->prm.shape.L;
  if (t < 0 || t >= idx->prm.shape.K1 || i < 1 || i > J)
    return fail(STAG_E_INVAL, "stag_lsh_index_segment: (t, i) out of range");
  const int64_t s = (int64_t)t * J + (i - 1);
  const int64_t s0 = (int64_t)idx->h_seg_off[s], c = (int64_t)idx->h_seg_off[s + 1] - s0;
  *count = c;
  if (c > 0 && members_host)
    STAG_HIP(hipMemcpyAsync(members_host, idx->members + s0, sizeof(int32_t) * c, hipMemcpyDeviceToHost, stream));
  if (c > 0 && keys_host)
    STAG_HIP(hipMemcpyAsync(keys_host, idx->mkeys + s0 * L, sizeof(uint64_t) * c * L, hipMemcpyDeviceToHost, stream));
  STAG_HIP(hipStreamSynchronize(stream));
  return STAG_OK;
}

void stag_lsh_index_destroy(stag_lsh_index* idx) {
  if (!idx) return;
  const int dev = idx->device;
  int cur = dev;
  if (hipGetDevice(&cur) == hipSuccess && cur != dev) (void)hipSetDevice(dev);
  (void)hipDeviceSynchronize();
  free_index(idx);
  if (cur != dev) (void)hipSetDevice(cur);
}

stag_status stag_kde_lsh(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, double a, double eps,
                         const stag_lsh_params* p, double* S_out, hipStream_t stream) {
  if (!Q || !S_out || m < 1) return fail(STAG_E_INVAL, "stag_kde_lsh: invalid query arguments");
  stag_lsh_index* idx = nullptr;
  STAG_TRY(stag_lsh_index_create(X, n, d, a, eps, p, &idx, stream));
  stag_status st = stag_lsh_index_query(idx, Q, m, S_out, stream);
  (void)hipStreamSynchronize(stream);
  stag_lsh_index_destroy(idx);
  return st;
}

namespace {
void e2lsh_table_free(stag_e2lsh_table* t) {
  for (void* p : t->owned) (void)hipFreeAsync(p, nullptr);
  (void)hipStreamSynchronize(nullptr);
  delete t;
}

stag_status e2lsh_query_keys(const stag_e2lsh_table* t, const float* Q, int64_t m, Workspace& ws, uint64_t** qk,
                             hipStream_t st) {
  STAG_TRY(ws.alloc(qk, (size_t)m * t->L));
  return e2lsh_launch(Q, m, t->d, t->G8, t->dg, t->b, t->K, t->L, nullptr, *qk, st);
}
}  // namespace

stag_status stag_e2lsh_table_create(const float* X, int64_t n, int32_t d, const float* G, const double* b, int32_t K,
                                    int32_t L, stag_e2lsh_table** out, hipStream_t stream) {
  if (!out) return fail(STAG_E_INVAL, "stag_e2lsh_table_create: out is NULL");
  *out = nullptr;
  if (!X || !G || !b) return fail(STAG_E_INVAL, "stag_e2lsh_table_create: NULL input pointer");
  if (n < 1 || n > 1073741824LL || d < 1 || d > 4096)
    return fail(STAG_E_INVAL, "stag_e2lsh_table_create: need 1 <= n <= 2^30 and 1 <= d <= 4096");
  if (K < 1 || K > 64 || L < 1 || L > 64) return fail(STAG_E_INVAL, "stag_e2lsh_table_create: need 1 <= K, L <= 64");
  if ((double)n * d >= 2147483648.0 * 4.0) return fail(STAG_E_INVAL, "stag_e2lsh_table_create: n*d too large");
  clear_error();
  stag_e2lsh_table* t = new (std::nothrow) stag_e2lsh_table();
  if (!t) return fail(STAG_E_NOMEM, "stag_e2lsh_table_create: host allocation failed");
  t->n = n;
  t->d = d;
  t->K = K;
  t->L = L;
  (void)hipGetDevice(&t->device);
  uint32_t cap = 2;
  while ((int64_t)cap < 2 * n) cap <<= 1;
  t->cap = cap;
  t->h_off = {0, (uint64_t)n, 0, (uint64_t)cap * L};
  t->h_cap = {cap};
  stag_status st = STAG_OK;
  {
    Workspace ws(stream);
    Workspace tmp(stream);
    auto body = [&]() -> stag_status {
      uint64_t* seg_off = nullptr;
      uint64_t* tso = nullptr;
      uint32_t* segcap = nullptr;
      STAG_TRY(e2lsh_regroup(G, K, L, d, ws, &t->G8, &t->dg, stream));
      STAG_TRY(ws.alloc(&t->b, (size_t)K * L));
      STAG_HIP(hipMemcpyAsync(t->b, b, sizeof(double) * K * L, hipMemcpyDeviceToDevice, stream));
      STAG_TRY(ws.alloc(&t->mkeys, (size_t)n * L));
      STAG_TRY(e2lsh_launch(X, n, d, t->G8, t->dg, t->b, K, L, nullptr, t->mkeys, stream));
      STAG_TRY(ws.alloc(&t->tab_key, (size_t)cap * L));
      STAG_TRY(ws.alloc(&t->tab_start, (size_t)cap * L));
      STAG_TRY(ws.alloc(&t->tab_cnt, (size_t)cap * L));
      STAG_TRY(ws.alloc(&t->csr, (size_t)n * L));
      STAG_TRY(tmp.alloc(&seg_off, 2));
      STAG_TRY(tmp.alloc(&tso, 2));
      STAG_TRY(tmp.alloc(&segcap, 1));
      STAG_HIP(hipMemcpyAsync(seg_off, t->h_off.data(), sizeof(uint64_t) * 2, hipMemcpyHostToDevice, stream));
      STAG_HIP(hipMemcpyAsync(tso, t->h_off.data() + 2, sizeof(uint64_t) * 2, hipMemcpyHostToDevice, stream));
      STAG_HIP(hipMemcpyAsync(segcap, t->h_cap.data(), sizeof(uint32_t), hipMemcpyHostToDevice, stream));
      ScopedTimer tm("e2lsh_table_build", stream);
      return build_tables_sorted(L, 1, n * L, (int64_t)cap * L, seg_off, tso, segcap, t->mkeys, t->tab_key,
                                 t->tab_start, t->tab_cnt, t->csr, tmp, stream);
    };
    st = body();
    t->owned = ws.release();
    (void)hipStreamSynchronize(stream);  // the host copies feed the build
  }
  if (st != STAG_OK) {
    e2lsh_table_free(t);
    return st;
  }
  *out = t;
  return STAG_OK;
}

stag_status stag_e2lsh_table_count(const stag_e2lsh_table* t, const float* Q, int64_t m, int64_t* offsets_out,
                                   hipStream_t stream) {
  if (!t || !Q || !offsets_out) return fail(STAG_E_INVAL, "stag_e2lsh_table_count: NULL argument");
  if (m < 1 || m > 2147483647LL) return fail(STAG_E_INVAL, "stag_e2lsh_table_count: need 1 <= m < 2^31");
  clear_error();
  Workspace ws(stream);
  uint64_t* qk = nullptr;
  uint32_t* cnt = nullptr;
  STAG_TRY(e2lsh_query_keys(t, Q, m, ws, &qk, stream));
  STAG_TRY(ws.alloc(&cnt, (size_t)m));
  {
    ScopedTimer tm("e2lsh_table_query", stream);
    hipLaunchKernelGGL(nn_walk<false>, dim3((unsigned)ceil_div(m, 4)), dim3(256), 0, stream, qk, m, t->L, t->n, t->cap,
                       t->tab_key, t->tab_start, t->tab_cnt, t->csr, t->mkeys, cnt, nullptr, nullptr);
    STAG_TRY(check_launch("nn_walk"));
  }
  return exclusive_scan_u32(cnt, reinterpret_cast<uint64_t*>(offsets_out), m, ws, stream);
}

stag_status stag_e2lsh_table_neighbours(const stag_e2lsh_table* t, const float* Q, int64_t m, const int64_t* offsets,
                                        int32_t* idx_out, hipStream_t stream) {
  if (!t || !Q || !offsets || !idx_out) return fail(STAG_E_INVAL, "stag_e2lsh_table_neighbours: NULL argument");
  if (m < 1 || m > 2147483647LL) return fail(STAG_E_INVAL, "stag_e2lsh_table_neighbours: need 1 <= m < 2^31");
  clear_error();
  Workspace ws(stream);
  uint64_t* qk = nullptr;
  STAG_TRY(e2lsh_query_keys(t, Q, m, ws, &qk, stream));
  ScopedTimer tm("e2lsh_table_query", stream);
  hipLaunchKernelGGL(nn_walk<true>, dim3((unsigned)ceil_div(m, 4)), dim3(256), 0, stream, qk, m, t->L, t->n, t->cap,
                     t->tab_key, t->tab_start, t->tab_cnt, t->csr, t->mkeys, nullptr,
                     reinterpret_cast<const uint64_t*>(offsets), idx_out);
  return check_launch("nn_walk");
}

void stag_e2lsh_table_destroy(stag_e2lsh_table* t) {
  if (!t) return;
  const int dev = t->device;
  int cur = dev;
  if (hipGetDevice(&cur) == hipSuccess && cur != dev) (void)hipSetDevice(dev);
  (void)hipDeviceSynchronize();
  e2lsh_table_free(t);
  if (cur != dev) (void)hipSetDevice(cur);
}

}  // extern "C"
