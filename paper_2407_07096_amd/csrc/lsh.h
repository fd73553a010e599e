// Internal interface of the CKNS index (parameter reading shared by the C ABI
// entry points and the edge sampler).
#pragma once

#include "runtime.h"

namespace stag {

struct LshParams {
  stag_lsh_shape shape;
  double lc_p[65], lc_T[65], lc_r[65];
  uint64_t thr[65];
  double a = 0.0, eps = 0.0;
  int64_t n = 0;
  uint64_t seed = 0;
  uint32_t flags = 0;
};

stag_status lsh_derive_params(int64_t n, double a, double eps, const stag_lsh_params* p, LshParams* out);

// Similarity-graph edges from the CKNS estimator of an index built over the
// data itself: s draws per node into src/dst/w [n*s], degrees into deg_out [n]
// (may be NULL).
stag_status lsh_sample_edges(const stag_lsh_index* idx, int s, uint64_t seed, int64_t* src, int64_t* dst, double* w,
                             double* deg_out, hipStream_t st);

}  // namespace stag
