// Internal interface of the E2LSH hashing kernel (used by the C ABI hash
// entry point and by the CKNS index).
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include "runtime.h"

namespace stag {
constexpr uint64_t kKeySalt = 0x243F6A8885A308D3ULL;
}

namespace stag {

// SplitMix64 finaliser (Steele, Lea & Flood 2014).
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// floor((s + b) / 4) saturated to int32.
__device__ inline int32_t code_of(double s, double b) {
  const double v = floor((s + b) / 4.0);
  if (v >= 2147483647.0) return 2147483647;
  if (v <= -2147483648.0) return (int32_t)(-2147483647 - 1);
  return (int32_t)v;
}

// Sums s[e] = <x, g_e> for KC projections of one table chunk (G8 layout
// [j][8]), as left-to-right binary64 chains over j.  DREG > 0: the point is
// held in registers xr[0..DREG) (zero padded); otherwise read from xrow.
template <int KC, int DREG>
__device__ inline void chunk_sums(const double* xr, const float* __restrict__ xrow, int d, int dg,
                                  const double* __restrict__ g8, double* s) {
#pragma unroll
  for (int e = 0; e < KC; ++e) s[e] = 0.0;
  if constexpr (DREG > 0) {
#pragma unroll
    for (int j = 0; j < DREG; ++j) {
      const double xj = xr[j];
#pragma unroll
      for (int e = 0; e < KC; ++e) s[e] = __builtin_fma(xj, g8[j * 8 + e], s[e]);
    }
  } else {
    // while eight coordinates are in range, their loads are issued before
    // their products (same chains)
    int j = 0;
    for (; j + 8 <= d; j += 8) {
      float xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = xrow[j + u];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int e = 0; e < KC; ++e) s[e] = __builtin_fma((double)xv[u], g8[(j + u) * 8 + e], s[e]);
    }
    for (; j < dg; ++j) {
      const double xj = j < d ? (double)xrow[j] : 0.0;
#pragma unroll
      for (int e = 0; e < KC; ++e) s[e] = __builtin_fma(xj, g8[j * 8 + e], s[e]);
    }
  }
}

template <int KC, int DREG>
__device__ inline uint64_t chunk_fold(uint64_t hkey, const double* xr, const float* __restrict__ xrow, int d,
                                      int dg, const double* __restrict__ g8, const double* __restrict__ bl, int kbase,
                                      int32_t* __restrict__ codes_row) {
  double s[KC];
  chunk_sums<KC, DREG>(xr, xrow, d, dg, g8, s);
#pragma unroll
  for (int e = 0; e < KC; ++e) {
    const int32_t code = code_of(s[e], bl[kbase + e]);
    if (codes_row) codes_row[kbase + e] = code;
    hkey = mix64(hkey ^ (uint64_t)(uint32_t)code);
  }
  return hkey;
}

// Bucket key of one table: K codes in chunks of up to 8 projections (G8 for
// this table is [nch][dg][8], bl its K offsets), folded in code order.
template <int DREG>
__device__ __attribute__((always_inline)) inline uint64_t table_key(int l, const double* xr, const float* __restrict__ xrow, int d, int dg,
                                     const double* __restrict__ g8t, const double* __restrict__ bl, int K, int nch,
                                     int32_t* __restrict__ codes_row) {
  uint64_t hkey = mix64(kKeySalt ^ (uint64_t)(uint32_t)l);
  for (int c = 0; c < nch; ++c) {
    const double* g8 = g8t + (int64_t)c * dg * 8;
    const int kc = K - 8 * c < 8 ? K - 8 * c : 8;
    switch (kc) {
      case 1: hkey = chunk_fold<1, DREG>(hkey, xr, xrow, d, dg, g8, bl, 8 * c, codes_row); break;
      case 2: hkey = chunk_fold<2, DREG>(hkey, xr, xrow, d, dg, g8, bl, 8 * c, codes_row); break;
      case 3: hkey = chunk_fold<3, DREG>(hkey, xr, xrow, d, dg, g8, bl, 8 * c, codes_row); break;
      case 4: hkey = chunk_fold<4, DREG>(hkey, xr, xrow, d, dg, g8, bl, 8 * c, codes_row); break;
      case 5: hkey = chunk_fold<5, DREG>(hkey, xr, xrow, d, dg, g8, bl, 8 * c, codes_row); break;
      case 6: hkey = chunk_fold<6, DREG>(hkey, xr, xrow, d, dg, g8, bl, 8 * c, codes_row); break;
      case 7: hkey = chunk_fold<7, DREG>(hkey, xr, xrow, d, dg, g8, bl, 8 * c, codes_row); break;
      default: hkey = chunk_fold<8, DREG>(hkey, xr, xrow, d, dg, g8, bl, 8 * c, codes_row); break;
    }
  }
  return hkey;
}

// E2LSH hashing with one lane per projection (d <= 64, K <= 64), for the
// CKNS queries (TQ: keys[table * mb + row]) and the E2LSH tables (keys[row *
// ntab + table], codes[(row * ntab + table) * K + e] when codes is not null).
// A wave takes TW = floor(64 / K) whole tables, lane t K + e holding
// projection e of its table t in registers as binary64 (DG values, zero
// padded); the 4 waves of a block share batches of 64 rows, widened to
// binary64 in LDS once per batch and read as broadcasts.  Each lane forms <x, g> for four queries at
// a time as the same left-to-right chain of fused products over the DG
// coordinates as table_key (so codes and keys are bit-identical), takes the
// code, and the 4 TW keys of the four queries are folded by one lane each
// from their table's K codes, gathered in code order with lane shuffles.
// Without scalar coefficient operands the kernel needs no scalar registers
// per coefficient (the per-query kernel spills them through vector lanes).
// code_of without branches (selects), so that the four chains below stay in
// one basic block: floor((s + b) / 4) saturated to int32, the in-range
// conversion being the hardware's (exact for these integral values).
__device__ inline int32_t code_sel(double s, double b) {
  const double v = floor((s + b) / 4.0);
  const int32_t c = __double2int_rz(v);
  return v >= 2147483647.0 ? 2147483647 : (v <= -2147483648.0 ? (int32_t)(-2147483647 - 1) : c);
}

// GF: the lane keeps its coefficients as fp32 (they are fp32 values widened
// exactly) and widens each one where it is used, so that d up to 128 fits
// the registers; dg is the regrouped copy's row width (DG, or d when the
// copy is not padded).
template <int DG, bool TQ, bool GF = false>
__global__ __launch_bounds__(256) void hash_lanes(const float* __restrict__ Q, int ldq, int64_t q0, int64_t mb, int d,
                                                  const double* __restrict__ G8, int dg, const double* __restrict__ B,
                                                  int K, int L, int nch, int64_t ntab, int TW, int qbatches,
                                                  uint64_t* __restrict__ qkeys, int32_t* __restrict__ codes) {
  typedef typename std::conditional<GF, float, double>::type GT;
  __shared__ double xs[64 * DG];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tab0 = ((int64_t)blockIdx.x * 4 + wave) * TW;
  const int ti = lane / K, e = lane - ti * K;
  const int64_t tab = tab0 + ti;
  const bool act = ti < TW && tab < ntab;
  GT g[DG];
  {
    const double* gp = G8 + (act ? tab : 0) * nch * dg * 8 + (e >> 3) * dg * 8 + (e & 7);
#pragma unroll
    for (int j = 0; j < DG; ++j) g[j] = j < dg ? (GT)gp[j * 8] : (GT)0;  // inactive lanes read table 0, never store
  }
  const double bv = act ? B[tab * K + e] : 0.0;
  const int nfold = 4 * TW;
  const int64_t qfirst = (int64_t)blockIdx.y * qbatches * 64;
  for (int qb = 0; qb < qbatches; ++qb) {
    const int64_t qs = qfirst + (int64_t)qb * 64;
    if (qs >= mb) break;  // uniform over the block
    __syncthreads();      // the previous batch's reads are done
    for (int idx = threadIdx.x; idx < 64 * DG; idx += 256) {
      const int r = idx / DG, c = idx - r * DG;
      const int64_t q = qs + r;
      xs[idx] = (q < mb && c < d) ? (double)Q[(q0 + q) * ldq + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 1
    for (int r0 = 0; r0 < 64; r0 += 4) {
      const double* x0 = xs + r0 * DG;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
      for (int j = 0; j < DG; ++j) {
        GT gj = g[j];
        if constexpr (GF) asm volatile("" : "+v"(gj));  // widen here, not once for the whole loop
        const double gd = (double)gj;
        s0 = __builtin_fma(x0[j], gd, s0);
        s1 = __builtin_fma(x0[DG + j], gd, s1);
        s2 = __builtin_fma(x0[2 * DG + j], gd, s2);
        s3 = __builtin_fma(x0[3 * DG + j], gd, s3);
      }

      const int32_t c0 = code_sel(s0, bv), c1 = code_sel(s1, bv), c2 = code_sel(s2, bv), c3 = code_sel(s3, bv);
      if (codes && act) {
        const int32_t cs[4] = {c0, c1, c2, c3};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int64_t q = qs + r0 + k;
          if (q < mb) codes[((q0 + q) * ntab + tab) * K + e] = cs[k];
        }
      }
      for (int f0 = 0; f0 < nfold; f0 += 64) {  // uniform
        const int f = f0 + lane;
        const int fq = f / TW, ft = f - fq * TW;  // query fq of the four, table ft of the wave
        uint64_t h = mix64(kKeySalt ^ (uint64_t)(uint32_t)((tab0 + ft) % L));
#pragma unroll 1
        for (int e2 = 0; e2 < K; ++e2) {
          const int src = (ft * K + e2) & 63;
          const int32_t a0 = __shfl(c0, src), a1 = __shfl(c1, src), a2 = __shfl(c2, src), a3 = __shfl(c3, src);
          const int32_t cc = fq == 0 ? a0 : (fq == 1 ? a1 : (fq == 2 ? a2 : a3));
          h = mix64(h ^ (uint64_t)(uint32_t)cc);
        }
        const int64_t q = qs + r0 + fq, tb = tab0 + ft;
        if (qkeys && f < nfold && tb < ntab && q < mb) {
          if constexpr (TQ) qkeys[tb * mb + q] = h;
          else qkeys[(q0 + q) * ntab + tb] = h;
        }
      }
    }
  }
}

// Loads point row into registers as binary64 (zero padded to DREG).
template <int DREG>
__device__ inline void load_point(double* xr, const float* __restrict__ xrow, int d) {
  if constexpr (DREG > 0) {
#pragma unroll
    for (int j = 0; j < DREG; ++j) xr[j] = j < d ? (double)xrow[j] : 0.0;
  }
}

int e2lsh_reg_dim(int d);
// fp32 [L*K][d] projections -> binary64 regrouped copy in workspace.
stag_status e2lsh_regroup(const float* G, int K, int L, int d, Workspace& ws, double** G8_out, int* dg_out,
                          hipStream_t st);
stag_status e2lsh_launch(const float* X, int64_t n, int d, const double* G8, int dg, const double* b, int K, int L,
                         int32_t* codes, uint64_t* keys, hipStream_t st);

}  // namespace stag
