// Random-sampling kernel density: the baseline estimator of the paper's KDE
// comparison (estimate K(q) from a uniformly random sample of the data).
//
// s indices are drawn with replacement from a SplitMix64 counter stream,
// j_r = floor(U_r n) taken with an exact integer product; the sampled rows
// are gathered into a contiguous [s][d] block (one pass, coalesced per row)
// and the exact tiles of kde_tiles.h evaluate all m x s pairs on the matrix
// cores; the reduction scales the sum by the once-rounded n/s.  One sample
// serves every query, so the m x s evaluation is a dense contraction like
// the exact KDE.
#include "runtime.h"
#include "kde_exact.h"

namespace stag {
namespace {

constexpr uint64_t kGammaRs = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kTagSample = 0x52534B44ull;  // "RSKD"

__device__ inline uint64_t rs_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// j_r = floor(U_r n), U_r = (mix(t + (r+1) gamma) >> 11) 2^-53,
// t = mix(mix(mix(seed ^ tag))).
__device__ inline int64_t sample_index(uint64_t seed, int64_t r, int64_t n) {
  const uint64_t t = rs_mix(rs_mix(rs_mix(seed ^ kTagSample)));
  const uint64_t u = rs_mix(t + (uint64_t)(r + 1) * kGammaRs) >> 11;
  const uint64_t hi = __umul64hi(u, (uint64_t)n), lo = u * (uint64_t)n;
  return (int64_t)((hi << 11) | (lo >> 53));
}

// One wave per sampled row: Xs[r] = X[j_r], idx[r] = j_r.
__global__ __launch_bounds__(256) void gather_sample(const float* __restrict__ X, int64_t n, int d, int64_t s,
                                                     uint64_t seed, float* __restrict__ Xs,
                                                     int64_t* __restrict__ idx) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= s) return;
  const int64_t j = sample_index(seed, r, n);
  if (idx && lane == 0) idx[r] = j;
  const float* src = X + j * d;
  float* dst = Xs + r * d;
  for (int c = lane; c < d; c += 64) dst[c] = src[c];
}

}  // namespace
}  // namespace stag

extern "C" stag_status stag_kde_random_sample(const float* X, int64_t n, const float* Q, int64_t m, int32_t d,
                                              double a, int64_t samples, uint64_t seed, int32_t form,
                                              double* S_out, double* bound_out, int64_t* idx_out,
                                              hipStream_t stream) {
  using namespace stag;
  const char* fn = "stag_kde_random_sample";
  if (!X || !Q || !S_out) return fail(STAG_E_INVAL, "%s: NULL pointer argument", fn);
  if (n < 1 || m < 1 || d < 1 || samples < 1) return fail(STAG_E_INVAL, "%s: n, m, d, samples must be >= 1", fn);
  if (!(a > 0.0) || !std::isfinite(a)) return fail(STAG_E_INVAL, "%s: a must be positive and finite", fn);
  if (form < STAG_FORM_FP32 || form > STAG_FORM_BF16_SPLIT3) return fail(STAG_E_INVAL, "%s: unknown form %d", fn, form);
  if (d > 1024) return fail(STAG_E_UNSUPPORTED, "%s: d = %d > 1024 is not supported", fn, d);
  if (d > 256 && form != STAG_FORM_FP32)
    return fail(STAG_E_UNSUPPORTED, "%s: d = %d > 256 is supported by the fp32 form only", fn, d);
  if ((double)n * d >= 2147483648.0 || (double)m * d >= 2147483648.0 || (double)samples * d >= 2147483648.0)
    return fail(STAG_E_INVAL, "%s: n*d, m*d and samples*d must be < 2^31", fn);
  clear_error();
  Workspace ws(stream);
  float* Xs = nullptr;
  STAG_TRY(ws.alloc(&Xs, (size_t)samples * d));
  {
    ScopedTimer tm("rs_gather", stream);
    hipLaunchKernelGGL(gather_sample, dim3((unsigned)ceil_div(samples, 4)), dim3(256), 0, stream, X, n, d, samples,
                       seed, Xs, idx_out);
    STAG_TRY(check_launch("gather_sample"));
  }
  Operands xo, qo;
  STAG_TRY(prepare_operands(form, Xs, samples, d, a, false, ws, &xo, stream));
  STAG_TRY(prepare_operands(form, Q, m, d, a, true, ws, &qo, stream));
  const int P = (int)exact_chunks(xo.rows_pad);
  double* partial = nullptr;
  STAG_TRY(ws.alloc(&partial, (size_t)P * qo.rows_pad));
  STAG_TRY(launch_exact_tiles(xo, qo, partial, TileExtra{}, stream));
  const double scale = (double)n / (double)samples;
  return reduce_with_rescue(partial, P, qo, xo, a, scale, make_bound_model(form, d, a), S_out, bound_out, ws, stream);
}

extern "C" int64_t stag_rs_sample_size(double eps, double mu, int64_t m, double delta) {
  if (!(eps > 0.0 && eps < 1.0) || !(mu > 0.0 && mu <= 1.0) || m < 1 || !(delta > 0.0 && delta < 1.0)) return 0;
  const double s = std::ceil(3.0 * std::log(2.0 * (double)m / delta) / (eps * eps * mu));
  return s < 9.2e18 ? (int64_t)s : 0;
}
