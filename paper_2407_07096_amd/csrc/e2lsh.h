// Internal interface of the E2LSH hashing kernel (used by the C ABI hash
// entry point and by the CKNS index).
#pragma once

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
    for (int j = 0; j < dg; ++j) {
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
__device__ inline uint64_t table_key(int l, const double* xr, const float* __restrict__ xrow, int d, int dg,
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
