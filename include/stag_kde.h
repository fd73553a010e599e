/*
 * stag_kde.h -- C ABI of the MI355X (gfx950) Gaussian kernel density library.
 *
 * The library computes, on one GPU, the data-parallel core of STAG 2.0's
 * kernel density and similarity-graph methods:
 *
 *   S(q) = sum_{i=1..n} exp(-a ||q - x_i||^2)          (Sec. "Kernel Density
 *          Estimation": the density K(q) = S(q)/n with the Gaussian kernel
 *          k(x) = exp(-a x^2); ExactGaussianKDE computes it in O(dmn)),
 *
 * exactly (tiled all-pairs kernel on the matrix cores) and approximately by the
 * CKNS estimator over E2LSH tables (Sec. "The CKNS Algorithm", Sec. "Random
 * Projection", Sec. "Boosting the Probability"), plus edge sampling of the
 * kernel similarity graph (Sec. "The MS Algorithm", eq. sampling_prob).
 *
 * Conventions for every entry point:
 *   - Matrices are row-major, contiguous, fp32: X is [n][d], Q is [m][d].
 *   - Array arguments are DEVICE pointers (hipMalloc'd or from a tensor)
 *     unless stated otherwise; the caller owns them and the library never
 *     frees caller memory.  Temporary workspace is allocated stream-ordered on
 *     `stream` and released at the end of the call (also stream-ordered).
 *   - Every call is asynchronous on `stream` (NULL = the default stream);
 *     outputs are valid once the stream has been synchronised.
 *   - Every call returns a stag_status.  All argument checks run before any
 *     launch: on STAG_E_INVAL nothing is launched and outputs are untouched.
 *     HIP runtime failures return STAG_E_DEVICE.  stag_last_error() gives a
 *     message for the last non-OK status of the calling thread.
 *   - No C++ exception crosses this interface and nothing aborts the process.
 */
#ifndef STAG_KDE_H
#define STAG_KDE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STAG_OK = 0,
  STAG_E_INVAL = 1,        /* invalid argument (nothing launched) */
  STAG_E_NOMEM = 2,        /* device allocation failed */
  STAG_E_DEVICE = 3,       /* HIP runtime error */
  STAG_E_UNSUPPORTED = 4,  /* valid but unsupported combination */
  STAG_E_BUSY = 5          /* serving loop: request rejected by admission */
} stag_status;

/* Arithmetic form of the exact kernel's cross term q.x (all forms accumulate
 * in fp32 per tile and in fp64 across tiles; norms are fp64). */
typedef enum {
  STAG_FORM_FP32 = 0,        /* fp32 matrix-core products */
  STAG_FORM_BF16_SPLIT = 1,  /* x = hi + lo in bf16, three bf16 products */
  STAG_FORM_FP16_SPLIT = 2,  /* x = hi + lo in fp16, three fp16 products */
  STAG_FORM_BF16_SPLIT3 = 3  /* x = hi + mid + lo in bf16, six bf16 products */
} stag_form;

/* flags of stag_kde_exact */
#define STAG_NORMALIZE 1u  /* return S/n (the paper's K(q)) instead of S */

/* Message describing the last non-OK status returned on this thread (never
 * NULL; empty string if none). */
const char* stag_last_error(void);

/* Library version string, e.g. "0.1.0 gfx950". */
const char* stag_version(void);

/* Per-kernel timing (a tracing aid for benchmarks; off by default).  When
 * enabled, every kernel launch of the library is bracketed by a pair of HIP
 * events on its stream.  stag_timing_report waits for those events, writes
 * one line "name count total_ms" per kernel name into buf (host memory,
 * NUL-terminated, truncated to len), clears the records and returns the size
 * the full report needs. */
void stag_timing_enable(int32_t on);
size_t stag_timing_report(char* buf, size_t len);

/* Collision probability of two points at distance c under K concatenated
 * E2LSH functions repeated over L tables (host function, no device work):
 *   p(c) = erf(2 sqrt 2 / c) - c (1 - exp(-8/c^2)) / (2 sqrt(2 pi)),  p(0) = 1
 *   returns 1 - (1 - p(c)^K)^L
 * (Sec. "Random Projection" closed form; Sec. "Boosting the Probability").
 * K = L = 1 gives p(c).  Returns NaN for c < 0, K < 1 or L < 1. */
double stag_e2lsh_collision_probability(double c, int32_t K, int32_t L);

/* Exact kernel density (Sec. "Kernel Density Estimation"; ExactGaussianKDE
 * query over a matrix of queries).
 *   X [n][d], Q [m][d]  fp32 device, row-major.
 *   a > 0, finite       Gaussian bandwidth parameter of k(x) = exp(-a x^2).
 *   eps                 reserved, pass 0.
 *   form                a stag_form.
 *   flags               STAG_NORMALIZE or 0.
 *   S_out [m]  f64 device: S(q) (or S(q)/n).
 *   bound_out [m] f64 device or NULL: a-priori relative error bound of each
 *                       result (the value is |S_gpu - S| / S <= bound except
 *                       with probability < 1e-9 per result; see the library
 *                       documentation for the model).
 * Limits: 1 <= d <= 256 (STAG_E_UNSUPPORTED above), n, m >= 1,
 * n*d and m*d < 2^31.  FP16_SPLIT additionally needs |x_j| and
 * |2a log2(e) q_j| below 65504; out-of-range inputs give a NaN result.
 * Results are deterministic and do not depend on m or on the other rows of Q
 * (each row's reduction order depends only on n). */
stag_status stag_kde_exact(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, double a,
                           double eps, int32_t form, uint32_t flags, double* S_out, double* bound_out,
                           hipStream_t stream);

/* E2LSH codes and bucket keys (Sec. "Random Projection": h(x) =
 * floor((<x, g> + b) / 4); Sec. "Boosting the Probability": K concatenated
 * functions per table, L tables).
 *   X [n][d] fp32 device.
 *   G [L*K][d] fp32 device: projection vectors, table-major then code index.
 *   b [L*K] f64 device: offsets in [0, 4).
 *   codes_out [n][L][K] int32 device or NULL:
 *       code = floor((s + b) / 4) with s the left-to-right binary64 sum over
 *       j = 0..d-1 of the exact products x_j * g_j; saturated to int32.
 *   keys_out [n][L] uint64 device or NULL: bucket key of table l, the
 *       SplitMix64-finaliser fold h = mix(0x243F6A8885A308D3 ^ l), then
 *       h = mix(h ^ (uint32)code_k) for k = 0..K-1.
 * Limits: 1 <= K <= 64, 1 <= L, L*K <= 2^24, 1 <= d <= 4096.
 * Bit-exact and deterministic. */
stag_status stag_e2lsh_hash(const float* X, int64_t n, int32_t d, const float* G, const double* b, int32_t K,
                            int32_t L, int32_t* codes_out, uint64_t* keys_out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* STAG_KDE_H */
