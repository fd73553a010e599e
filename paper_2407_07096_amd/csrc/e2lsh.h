// Internal interface of the E2LSH hashing kernel (used by the C ABI hash
// entry point and by the CKNS index).
#pragma once

#include <hip/hip_runtime.h>

#include "runtime.h"

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

int e2lsh_reg_dim(int d);
// fp32 [L*K][d] projections -> binary64 regrouped copy in workspace.
stag_status e2lsh_regroup(const float* G, int K, int L, int d, Workspace& ws, double** G8_out, int* dg_out,
                          hipStream_t st);
stag_status e2lsh_launch(const float* X, int64_t n, int d, const double* G8, int dg, const double* b, int K, int L,
                         int32_t* codes, uint64_t* keys, hipStream_t st);

}  // namespace stag
