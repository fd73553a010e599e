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
  STAG_FORM_BF16_SPLIT3 = 3, /* x = hi + mid + lo in bf16, six bf16 products */
  STAG_FORM_AUTO = 4,        /* exact KDE only: the cheapest form whose a-priori bound is <= eps */
  STAG_FORM_FP16_CENTRED = 5, /* exact Gaussian KDE only: data grouped around centres c, one fp16
                                 product (q - c).(x - c) per pair; see stag_kde_exact */
  STAG_FORM_FP16_ADAPTIVE = 6 /* exact Gaussian KDE only: FP16_CENTRED everywhere, FP16_SPLIT where
                                 its bound would matter; see stag_kde_exact */
} stag_form;

/* Kernel functions of Sec. "Kernel Density Estimation" (r = ||q - x||). */
typedef enum {
  STAG_KERNEL_GAUSSIAN = 0,     /* exp(-a r^2) */
  STAG_KERNEL_EXPONENTIAL = 1,  /* exp(-a r) */
  STAG_KERNEL_LOGISTIC = 2      /* 4 / (2 + e^{a r} + e^{-a r}); a = 1 is the paper's */
} stag_kernel;

/* flags of stag_kde_exact */
#define STAG_NORMALIZE 1u     /* return S/n (the paper's K(q)) instead of S */
#define STAG_CHECK_FINITE 2u  /* scan X and Q on the device first; a NaN or Inf is STAG_E_INVAL */

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
 *   eps                 target relative accuracy, used by STAG_FORM_AUTO
 *                       (0 < eps; ignored by the other forms).
 *   form                a stag_form.  STAG_FORM_AUTO scans X and Q once on the
 *                       device (largest norms and elements; one
 *                       synchronisation of `stream`) and takes, in order of
 *                       cost, FP16_SPLIT (if the operands fit fp16's range),
 *                       BF16_SPLIT, BF16_SPLIT3, FP32: the first whose
 *                       a-priori bound at the largest query norm is <= eps;
 *                       FP32 if none is (bound_out then shows it).  The
 *                       result equals that of the chosen form bit for bit.
 *                       The choice rests on the same bound as bound_out,
 *                       whose accumulation term is probabilistic (below), so
 *                       "<= eps" holds except with probability < 1e-9 per
 *                       result, not with certainty.
 *   flags               STAG_NORMALIZE, STAG_CHECK_FINITE (one device scan
 *                       and synchronisation; a NaN or Inf in X or Q is
 *                       STAG_E_INVAL with nothing launched after the scan).
 *   S_out [m]  f64 device: S(q) (or S(q)/n).
 *   bound_out [m] f64 device or NULL: a-priori relative error bound of each
 *                       result (the value is |S_gpu - S| / S <= bound except
 *                       with probability < 1e-9 per result; see the library
 *                       documentation for the model).
 * Small densities: the tiles form each term as 2^E in fp32.  A query whose
 * sum comes out below 2^-60 (its terms may lie below the fp32 range) is
 * recomputed on the device with its exponents shifted by their maximum
 * m_q (a max pass and a second pass over the 128-query tiles that hold
 * such queries; S = sum * 2^m_q, its bound widened by |m_q|); a result below
 * the fp64 range is 0.  Without such queries the two passes end at once.
 * Limits: 1 <= d <= 1024 (d > 256: FP32, FP16_SPLIT or BF16_SPLIT, with
 * STAG_FORM_AUTO taking FP32; STAG_E_UNSUPPORTED otherwise), n, m >= 1,
 * n*d and m*d < 2^31.  FP16_SPLIT additionally needs |x_j| and
 * |2a log2(e) q_j| below 65504; out-of-range inputs give a NaN result.
 * FP16_CENTRED (Gaussian kernel, d <= 256): the rows of X are grouped as for
 * the fp32 form (at most 256 groups from seeded seed rows, each group padded
 * to 32-row tiles) and each group g gets one centre c_g = fl32(mean of its
 * rows).  The data are held once as fl16(x - c_g) with the offsets
 * -a log2(e) ||x - c_g||^2 (fp32 from fp64); per group the tile forms each
 * query's operand fl16(2a log2(e) (q - c_g)) and offset -a log2(e)
 * ||q - c_g||^2, so every pair costs one fp16 matrix-core product instead
 * of the split forms' three.  Each product carries the two fp16 roundings
 * (relative 2^-11 each), so a term's exponent may be off by up to about
 * 2^-10 * 2a log2(e) ||q - c_g|| ||x - c_g||: bound_out states that
 * worst case (with the fp32 terms of the centred fp32 tile), which is far
 * above the typical error because independent roundings cancel in sums of
 * many terms.  STAG_FORM_AUTO never takes this form.  A data row with some
 * |x_j - c_j| >= 65520, or a query with some |2a log2(e) (q_j - c_j)| >=
 * 65520, gives NaN results (all of them, or that query's).
 * FP16_ADAPTIVE (Gaussian kernel, d <= 256): the queries are ordered by
 * their nearest seed of the same grouping, the FP16_CENTRED tiles run over
 * all pairs; per query, the chunks with the smallest FP16_CENTRED bound
 * numerators whose numerators add up to at most 1e-5 of its sum keep their
 * values (the cut taken at a power of 4 of that budget), and every (4096-row
 * chunk, 256-query tile) pair in which some query's chunk is not among them
 * is computed again in the FP16_SPLIT form.  Where the
 * data are clustered and the kernel narrow against the clusters' spacing,
 * few pairs are recomputed and the result has the split form's accuracy at
 * near the single product's cost.  A first estimate runs the selection on
 * every (m_pad / 128 / 8)-th 128-query tile and reads the count back (one
 * synchronisation of `stream`); when more than half of those pairs would be
 * recomputed (wide kernels), the single-product pass is skipped and every
 * pair runs in the split form.  In the single-product pass, a wave of 64
 * queries whose offsets -a log2(e) ||q - c_g||^2 all lie in [-60, 0] for a
 * group sums 2^(E + a log2(e) ||q - c_g||^2) and scales the sums by
 * fl32(2^(-a log2(e) ||q - c_g||^2)) (one rounding more, in its bound).
 * bound_out adds the kept chunks' FP16_CENTRED numerators and the
 * recomputed chunks' FP16_SPLIT bounds.  Sums below 2^-60 are recomputed in
 * the split form (underflow rescue).  Range rules of both forms apply.
 * Results are deterministic.  In every form but FP16_ADAPTIVE they do not
 * depend on m or on the other rows of Q (each row's reduction order depends
 * only on n); in FP16_ADAPTIVE the queries of a 256-query tile decide
 * together which chunks are recomputed, so a row's result (always within
 * its bound) may change with the other rows of Q. */
stag_status stag_kde_exact(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, double a,
                           double eps, int32_t form, uint32_t flags, double* S_out, double* bound_out,
                           hipStream_t stream);

/* stag_kde_exact without device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and results as stag_kde_exact with the
 * Gaussian kernel (bit for bit), except:
 *   - form is FP32, BF16_SPLIT, FP16_SPLIT, BF16_SPLIT3, FP16_CENTRED or FP16_ADAPTIVE (STAG_FORM_AUTO:
 *     STAG_E_UNSUPPORTED) and flags may hold STAG_NORMALIZE only
 *     (STAG_CHECK_FINITE: STAG_E_UNSUPPORTED); eps is not taken;
 *   - every temporary (prepared operands, partial sums, rescue buffers) lives
 *     in a 128 MiB scratch array that the library holds on each device it
 *     runs on until the process ends; a call whose temporaries do not fit is
 *     STAG_E_INVAL before any launch (the split forms take about
 *     (n + m) * d_pad * 4 bytes of split operands (d_pad: d rounded up to 16,
 *     32, 64, 96 ... 256) plus 24 * m_pad * ceil(n / 4096) bytes of partial
 *     sums, m_pad = m rounded up to 128; FP16_ADAPTIVE about (1.5 n + 2 m)
 *     * d_pad * 4 plus 32 * m_pad * ceil(n / 4096) bytes; the error message
 *     states the call's exact need);
 *   - no hipMalloc, hipFree or allocating routine is called; the first call
 *     on a device looks up that device's scratch address once;
 *   - FP16_ADAPTIVE reads its estimate back (one synchronisation of
 *     `stream`), so that form cannot be recorded into a HIP graph.
 * Every call on one device shares that device's scratch: calls that overlap
 * on one device (on different streams, or from several threads) race and
 * give wrong results; serialise them.  The scratch keeps the last call's
 * contents; whatever must start at zero is cleared by each call. */
stag_status stag_kde_exact_noalloc(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, double a,
                                   int32_t form, uint32_t flags, double* S_out, double* bound_out,
                                   hipStream_t stream);

/* Exact kernel density S(q) = sum_i k(||q - x_i||) with any of the three
 * kernel functions of Sec. "Kernel Density Estimation" (stag_kernel); the
 * arguments, limits and determinism are those of stag_kde_exact, which is
 * this call with STAG_KERNEL_GAUSSIAN.
 * The tile computes E = -lambda D, D = ||q||^2 + ||x||^2 - 2 q.x, with
 * lambda = (a log2 e)^2 for the exponential and logistic kernels, and takes
 * y = sqrt(max(-E, 0)) = a r log2(e); FP16_SPLIT then needs
 * |2 (a log2 e)^2 q_j| below 65504.
 * Small densities: as in stag_kde_exact, a sum below 2^-60 is recomputed
 * on the device, here with each term taken as 2^{ys - y}, ys the query's
 * smallest y (from a max pass), and S = sum * 2^{-ys}.
 * Exponential kernel, near pairs: where the computed -E is below 1/4
 * (a r < 1/(2 log2 e), kernel value above 2^-1/2) an error dE in the
 * exponent would move y by up to sqrt(dE); those terms are taken out of the
 * tile sum and evaluated as exp(-a ||q - x||) from fp64 differences of the
 * input rows, in a fixed order (results stay deterministic).  They cost d
 * fp64 operations each and are rare unless many points lie within 1/(2 a
 * log2 e) of a query.  At least 8 of the 32-row data tiles that hold such
 * pairs are taken per query and 4096-row chunk; a query with more keeps the
 * rest in its tile sums and the unrefined bound.
 * bound_out: the a-priori relative error bound per result; for the
 * exponential kernel it uses y^2 >= 1/4 - dE for the terms left to the tile
 * (|dy| <= dE / (2 sqrt(1/4 - dE))), or |dy| <= sqrt(dE) for a query whose
 * near pairs did not all fit; the logistic kernel is flat at r = 0 and keeps
 * a bound of the Gaussian's order.  STAG_FORM_AUTO assumes the near pairs
 * fit.  Unknown kernel: STAG_E_INVAL. */
stag_status stag_kde_exact_kernel(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, int32_t kernel,
                                  double a, double eps, int32_t form, uint32_t flags, double* S_out,
                                  double* bound_out, hipStream_t stream);

/* Random-sampling kernel density (the sampling baseline of Sec. "Kernel
 * Density Estimation" and of the paper's KDE experiments: K(q) estimated from
 * a uniformly random sample of the data).
 *   samples (s >= 1) indices drawn with replacement, j_r = floor(U_r n) taken
 *   exactly, U_r = (mix(t + (r+1) 0x9E3779B97F4A7C15) >> 11) 2^-53,
 *   t = mix(mix(mix(seed ^ 0x52534B44))), mix the SplitMix64 finaliser; one
 *   sample serves every query.
 *   S_out [m] f64 device: (n/s) sum_r exp(-a ||q - x_{j_r}||^2), n/s rounded
 *   once; an unbiased estimate of S(q).
 *   bound_out [m] f64 device or NULL: relative error bound of S_out against
 *   the exact fp64 value of that same estimator (as stag_kde_exact's, small
 *   estimates taking the same underflow rescue).
 *   idx_out [s] int64 device or NULL: the sampled indices.
 * form, d and size limits as stag_kde_exact (samples * d < 2^31). */
stag_status stag_kde_random_sample(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, double a,
                                   int64_t samples, uint64_t seed, int32_t form, double* S_out, double* bound_out,
                                   int64_t* idx_out, hipStream_t stream);

/* Host-only: the sample size ceil(3 ln(2m/delta) / (eps^2 mu)) after which,
 * by the multiplicative Chernoff bound for values in [0, 1] and a union bound
 * over m queries, every query whose density K(q) is at least mu is estimated
 * within a factor 1 +- eps (0 < eps < 1) with probability at least 1 - delta.
 * Returns 0 for invalid arguments. */
int64_t stag_rs_sample_size(double eps, double mu, int64_t m, double delta);

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

/* E2LSH hash table (the E2LSH class: Sec. "Random Projection", "Boosting the
 * Probability"): the keys of the n points of X under L tables of K
 * concatenated hashes, bucketed per table.  Approximate near neighbours of a
 * query (get_near_neighbours) are the points that share its bucket in at
 * least one table.
 *   X [n][d] fp32 device; G [L*K][d] fp32 and b [L*K] f64 device as for
 *   stag_e2lsh_hash (codes and keys are identical to it).  The table copies
 *   what it needs (not X); the caller may free X, G, b after the call.
 * Limits: 1 <= n <= 2^30, 1 <= d <= 4096, 1 <= K, L <= 64, n*d < 2^33.
 * Synchronises `stream` once (the build reads host-side layout data).
 * Errors: STAG_E_INVAL for bad arguments (before any launch), STAG_E_NOMEM. */
typedef struct stag_e2lsh_table stag_e2lsh_table;
stag_status stag_e2lsh_table_create(const float* X, int64_t n, int32_t d, const float* G, const double* b, int32_t K,
                                    int32_t L, stag_e2lsh_table** out, hipStream_t stream);

/* Near-neighbour counts of the m rows of Q [m][d] (fp32 device):
 * offsets_out [m+1] int64 device receives the exclusive prefix sum of the
 * counts (offsets_out[m] = total).  A point is counted once per query. */
stag_status stag_e2lsh_table_count(const stag_e2lsh_table* t, const float* Q, int64_t m, int64_t* offsets_out,
                                   hipStream_t stream);

/* The lists themselves: idx_out [offsets[m]] int32 device (offsets from
 * stag_e2lsh_table_count for the same Q).  Query q's list is at
 * idx_out[offsets[q] .. offsets[q+1]): table by table (table 0 first),
 * ascending point index within a bucket, each point in the first table where
 * it collides with q.  Deterministic. */
stag_status stag_e2lsh_table_neighbours(const stag_e2lsh_table* t, const float* Q, int64_t m, const int64_t* offsets,
                                        int32_t* idx_out, hipStream_t stream);

/* Waits for the device and frees the table (NULL is ignored). */
void stag_e2lsh_table_destroy(stag_e2lsh_table* t);

/* ------------------------------------------------------------------------
 * CKNS approximate kernel density (Sec. "The CKNS Algorithm"; the three
 * CKNSGaussianKDE constructors map onto stag_lsh_params).
 *
 * Reading of the parameters (the paper states them only up to constants):
 *   mu_min  = min_mu > 0 ? min_mu : 1/n
 *   J       = max(1, ceil(log2(1/mu_min))) levels ("log n" subsamples)
 *   p_i     = min(1, 2^-i / (n mu_min)) * 2^-p_offset   (= 2^-i by default)
 *   T_i     = i ln2 / a: level i holds points with T_{i-1} <= D < T_i, i.e.
 *             kernel value in (2^-i, 2^-i+1]; points beyond T_J are not counted
 *   L       = ceil(K2_constant) tables per level (default ceil(log2 n), <= 64)
 *   K       = largest k with 1 - (1 - p(1)^k)^L >= 1 - eps/4
 *   K1      = k1 > 0 ? k1 : ceil(log2(n) / eps^2) independent copies
 *   level i hashes the space scaled by r_i = sqrt(T_i):
 *             g = fp32(g0 / r_i) for the stored N(0,1) vector g0
 * Estimate of copy t: sum over levels i and tables l of every member j of q's
 * bucket not already found in an earlier table of that level, with
 * T_{i-1} <= D < T_i, of exp(-a D) / (p_i R_i), R_i = 1 - (1 - p(sqrt(D)/r_i)^K)^L
 * (R_i = 1 with STAG_LSH_LITERAL, the paper's 2^i weighting).  The result is
 * the mean over copies.  D is the fused-order squared distance: D = fma(e, e,
 * D) over coordinates in order, e = (double)q_h - (double)x_h.
 * Subsample membership: j is in copy t, level i iff
 *   (mix(s + (j+1) 0x9E3779B97F4A7C15) >> 11) < floor(p_i 2^53),
 *   s = mix(mix(mix(seed ^ 0x4D41534B) ^ t) ^ i), mix the SplitMix64 finaliser.
 * ------------------------------------------------------------------------ */
#define STAG_LSH_LITERAL 1u      /* weight 1/p_i only (no recovery reweighting) */
#define STAG_LSH_ALL_SAMPLED 2u  /* test hook: p_i = 1 on every level */

typedef struct {
  double min_mu;       /* <= 0: 1/n */
  int32_t k1;          /* <= 0: ceil(log2(n) / eps^2) */
  double k2_constant;  /* <= 0: ceil(log2 n) */
  int32_t p_offset;    /* >= 0 */
  uint64_t seed;       /* subsampling stream (and default projections) */
  uint32_t flags;      /* STAG_LSH_* */
  const float* G0;     /* device [K1][J][L][K][d] N(0,1) values, or NULL: drawn from seed */
  const double* b;     /* device [K1][J][L][K] offsets in [0,4), or NULL (NULL iff G0 is NULL) */
} stag_lsh_params;

typedef struct {
  int32_t J, L, K, K1;
  double mu_min;
} stag_lsh_shape;

typedef struct stag_lsh_index stag_lsh_index; /* opaque; owns its device arrays */

/* Host-only: the derived shape for (n, a, eps, params); p may be NULL. */
stag_status stag_lsh_derive(int64_t n, double a, double eps, const stag_lsh_params* p, stag_lsh_shape* out);

/* Builds the index over X [n][d] (device fp32, copied; the caller may free X
 * afterwards).  Synchronises `stream` once (segment sizes are read back).
 * Limits: 1 <= n < 2^31, 1 <= d <= 4096, K1*J <= 65535, L <= 64. */
stag_status stag_lsh_index_create(const float* X, int64_t n, int32_t d, double a, double eps,
                                  const stag_lsh_params* p, stag_lsh_index** out, hipStream_t stream);

/* Estimates S(q) for Q [m][d] (device fp32) into S_out [m] (device f64).
 * The index is read-only: concurrent queries on different streams are safe. */
stag_status stag_lsh_index_query(const stag_lsh_index* idx, const float* Q, int64_t m, double* S_out,
                                 hipStream_t stream);

/* As stag_lsh_index_query, plus optional per-copy estimates S_copies [m][K1]
 * (f64), and per query the number of bucket members examined n_cand [m] and
 * of accepted terms n_acc [m] (int64); each may be NULL. */
stag_status stag_lsh_index_query_ex(const stag_lsh_index* idx, const float* Q, int64_t m, double* S_out,
                                    double* S_copies, int64_t* n_cand, int64_t* n_acc, hipStream_t stream);

stag_status stag_lsh_index_shape(const stag_lsh_index* idx, stag_lsh_shape* out);

/* Copies the subsample of copy t (0-based), level i (1-based) to HOST
 * memory: *count points, members_host [count] ascending point indices and
 * keys_host [count][L] their bucket keys (either may be NULL).  Synchronises
 * `stream`. */
stag_status stag_lsh_index_segment(const stag_lsh_index* idx, int32_t t, int32_t i, int64_t* count,
                                   int32_t* members_host, uint64_t* keys_host, hipStream_t stream);

/* Waits for the device and releases the index (NULL is ignored).  Its device
 * memory goes back to a per-device cache of the library, reused by later
 * indexes and returned to the system at process exit. */
void stag_lsh_index_destroy(stag_lsh_index* idx);

/* create + query + destroy. */
stag_status stag_kde_lsh(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, double a, double eps,
                         const stag_lsh_params* p, double* S_out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Similarity-graph edge sampling (Sec. "The MS Algorithm", eq. sampling_prob:
 * edge (i,j) sampled with probability proportional to w/deg(i) + w/deg(j),
 * deg(i) = sum_j k(||x_i - x_j||); approximate_similarity_graph).
 *
 * Every node i draws s neighbours j != i with probability k_ij / rest_i,
 * rest_i = sum_{j != i} k_ij; draw r of node i is output at index i*s + r with
 * weight 1 / (s (1/rest_i + 1/rest_j)), so that the expected sampled weight of
 * each pair equals k_ij (the fully connected graph without self-loops).
 * Duplicates are kept (the caller may merge them); deg(i) = 1 + rest_i.
 * The draw uses U = (mix(s_i + (r+1) 0x9E3779B97F4A7C15) >> 11) 2^-53,
 * s_i = mix(mix(mix(seed ^ 0x44524157) ^ i) ^ 0), inverting the cumulative
 * sum of the row in ascending j.
 *   STAG_SIMGRAPH_EXACT: kernel row sums from one exact tile pass in `form`
 *     (chunk and tile sums), the final 32 values recomputed in fp64; for
 *     d > 256 the form is FP32, FP16_SPLIT or BF16_SPLIT.  Device workspace:
 *     the fp32 sums of every 32-row tile of every row (about n^2 / 8 bytes)
 *     and, for d > 256, where the draws are sorted by tile between the tile
 *     and the row step, about 24 bytes per draw (n * s must then stay below
 *     2^31, else STAG_E_UNSUPPORTED).  Which path runs does not change the
 *     draws.
 *   STAG_SIMGRAPH_LSH: rest_i is the CKNS estimate (eps, lsh params) of
 *     sum_{j != i} k_ij and the draw inverts the estimator's own terms (copy,
 *     level, table, bucket order): E[term of j] = k_ij.
 * Outputs (device): src/dst int64 [n*s], w f64 [n*s], deg f64 [n] or NULL.
 * dst = -1 (w = 0) for a node whose row is empty (all kernel values 0).
 * samples_per_node 0 means ceil(log2 n); at most 64.
 * ------------------------------------------------------------------------ */
/* Host-only: the draws per node s that stag_simgraph_sample and
 * stag_simgraph_sample_tree take for a samples_per_node argument (0 means
 * ceil(log2 n), at least 1), so that a caller can size the outputs; -1 if
 * n < 1 or samples_per_node is outside [0, 64]. */
int32_t stag_simgraph_draws_per_node(int64_t n, int32_t samples_per_node);

#define STAG_SIMGRAPH_EXACT 0
#define STAG_SIMGRAPH_LSH 1

stag_status stag_simgraph_sample(const float* X, int64_t n, int32_t d, double a, int32_t samples_per_node,
                                 int32_t kde_mode, int32_t form, double eps, const stag_lsh_params* lsh,
                                 uint64_t seed, int64_t* src_out, int64_t* dst_out, double* w_out, double* deg_out,
                                 hipStream_t stream);

/* Edge sampling through a KDE tree (Sec. "The MS Algorithm": the sampling
 * probabilities of eq. sampling_prob reached with a KDE algorithm as a black
 * box; here the random-sampling estimator of Sec. "Kernel Density
 * Estimation" per tree node).  Gaussian kernel exp(-a r^2).
 * Tree over the rows in index order: leaves are blocks of 32 rows, h =
 * ceil(log2 ceil(n/32)), node (l, k) holds rows [k 32 2^(h-l),
 * (k+1) 32 2^(h-l)) clipped to [0, n).  A node estimate of sum_{j in node,
 * j != i} k_ij is exact for a node of P <= est_samples rows, else (P/t) times
 * the sum over t = est_samples rows j_c = lo + floor(U_c P) (own row 0).
 * Draw r of node i descends from the root: with estimates eA, eB of the two
 * children and u = U(i, r, l) it goes to A iff u (eA + eB) < eA (if both are
 * 0, to the child with more rows other than i, A on a tie); in the leaf it
 * inverts the cumulative exact values of the leaf's rows (j != i) on
 * u = U(i, r, h), or takes the floor(u m)-th of its m rows other than i when
 * they are all 0.  Degrees: rest_i = the root estimate with degree_samples
 * samples (exact when n <= degree_samples), deg_out[i] = 1 + rest_i; draw
 * (i, j) is output at index i*s + r with weight 1/(s (1/rest_i + 1/rest_j))
 * (0 if one of them is 0).  Every dst is in [0, n) and differs from src.
 * Randomness: SplitMix64 counter streams, output c of stream (seed, tag,
 * a, b) = mix(S + (c+1) 0x9E3779B97F4A7C15), S = mix(mix(mix(seed ^ tag) ^
 * a) ^ b): node samples tag 0x54524545, a = i, b = r << 16 | l << 1 | side
 * (A = 0); descent uniforms tag 0x5452554E, a = i, b = r, c = l; degree
 * samples tag 0x54444547, a = i, b = 0.  U = (output >> 11) 2^-53 and an
 * index floor(U P) is taken exactly in integers.
 * Work: n s draws of h levels x 2 est_samples kernel values + 32 in the leaf,
 * each an fp64 direct-difference distance (no n^2 pass); n degree_samples
 * values for the degrees.  Results are deterministic for a given seed.
 * Arguments: X [n][d] f32 device; 2 <= n < 2^31; 1 <= d <= 1024; a > 0;
 * samples_per_node 0 (= ceil(log2 n)) to 64; est_samples 1 to 32;
 * degree_samples >= 1.  Outputs (device, caller-owned): src/dst int64
 * [n*s], w f64 [n*s], deg_out f64 [n] or NULL.  Invalid arguments:
 * STAG_E_INVAL before any launch. */
stag_status stag_simgraph_sample_tree(const float* X, int64_t n, int32_t d, double a, int32_t samples_per_node,
                                      int32_t est_samples, int64_t degree_samples, uint64_t seed, int64_t* src_out,
                                      int64_t* dst_out, double* w_out, double* deg_out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Spectral clustering (Sec. "Fast Spectral Clustering": a similarity graph,
 * the bottom k eigenvectors of its Laplacian as an embedding in R^k, then
 * k-means on the embedded vertices; spectral_cluster).
 *
 * Graph: an edge list src/dst int64 [n_edges], w f64 [n_edges] (device), as
 * written by stag_simgraph_sample: every edge adds w to A[src][dst] and to
 * A[dst][src] (duplicates add up, a self loop adds 2w to A[i][i]); dst = -1
 * marks an empty draw and is skipped.  Any other index outside [0, n), or a
 * negative or non-finite weight, is STAG_E_INVAL (checked on the device
 * before any further work).  Limits: 1 <= n < 2^31, 0 <= n_edges < 2^30.
 * Laplacian: the normalised N = I - D^{-1/2} A D^{-1/2}, D the row sums of A,
 * with D^{-1/2} = 0 for an isolated vertex.
 * ------------------------------------------------------------------------ */

/* Bottom k eigenpairs of N (1 <= k <= min(56, n)) by Chebyshev-filtered
 * subspace iteration on M = I - N with a block of 8..64 columns, until every
 * residual ||M u_j - theta_j u_j|| <= tol (tol > 0) or after max_iter filter
 * steps (>= 0).  seed selects the random starting block.
 *   eigvals_out [k] f64 device or NULL: eigenvalues of N, ascending.
 *   U_out [n][k] f64 device: row i is vertex i's embedding; column j is the
 *     unit eigenvector of eigvals_out[j], its entry of largest magnitude (the
 *     lowest row among equals) positive.
 *   iters_out (host, may be NULL): filter steps taken.
 * Synchronises `stream` several times per step; deterministic. */
stag_status stag_spectral_embedding(int64_t n, const int64_t* src, const int64_t* dst, const double* w,
                                    int64_t n_edges, int32_t k, double tol, int32_t max_iter, uint64_t seed,
                                    double* eigvals_out, double* U_out, int32_t* iters_out, hipStream_t stream);

/* k-means of the n points P [n][dim] (f64 device) into k clusters (1 <= k <=
 * n, k*dim <= 4096): Lloyd's iteration from init [k][dim] (device) or, with
 * init NULL, from k-means++ seeding.  Every decision is specified:
 *   dist2(p, c) = sum over j ascending of (p_j - c_j)^2, each operation
 *     rounded separately (no fused multiply-add);
 *   U_r = (s >> 11) 2^-53 with s = mix(t + (r+1) 0x9E3779B97F4A7C15),
 *     t = mix(mix(mix(seed ^ 0x4B4D4E53))), mix the SplitMix64 finaliser;
 *   seed 0 = floor(U_0 n) (exact integer product); seed c > 0 = the first
 *     point i with B_b + (sum of D2 over block b up to i) > U_c T, where D2
 *     is the squared distance to the nearest chosen seed, blocks hold 1024
 *     points, B_b is the sum of the block sums before b, T the total (all
 *     sums sequential); if none, the last point with D2 > 0; if T = 0, the
 *     lowest index not chosen yet;
 *   assignment: the nearest centre, ties to the lowest index;
 *   update: per cluster, coordinate sums in the same blocked order divided by
 *     the count; an empty cluster keeps its centre;
 *   stop: after an assignment that changes no label (centres are those the
 *     labels were assigned with), or after max_iter (>= 1) rounds.
 * labels_out [n] int32 device; centroids_out [k][dim] f64 device or NULL;
 * seeds_out [k] int64 device or NULL (-1 with init); iters_out host or NULL
 * (assignment rounds).  Deterministic; synchronises `stream` once per round. */
stag_status stag_kmeans(const double* P, int64_t n, int32_t dim, int32_t k, uint64_t seed, int32_t max_iter,
                        const double* init, int32_t* labels_out, double* centroids_out, int64_t* seeds_out,
                        int32_t* iters_out, hipStream_t stream);

/* stag_spectral_embedding (tol 1e-8, at most 300 steps) followed by
 * stag_kmeans of the embedding (dim = k, k-means++ with the same seed, at
 * most 300 rounds): labels_out [n] int32 device. */
stag_status stag_spectral_cluster(int64_t n, const int64_t* src, const int64_t* dst, const double* w, int64_t n_edges,
                                  int32_t k, uint64_t seed, int32_t* labels_out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Serving loop: continuous batching of kernel-density requests against
 * resident data sets.
 *   - A data set (X, a) is prepared once and stays in device memory in each
 *     of its resident exact forms (a bit mask of 1 << STAG_FORM_* over FP32,
 *     BF16_SPLIT, FP16_SPLIT and BF16_SPLIT3; other bits are STAG_E_INVAL;
 *     the fp32 form with its data tiles centred as in stag_kde_exact) and, on
 *     request, with a CKNS index (stag_lsh_index_create with lsh_eps and the
 *     given parameters) for LSH requests.
 *   - A request is exact (in a resident form, or STAG_FORM_AUTO: the form
 *     the stag_kde_exact rule picks among the resident ones for eps, from
 *     the largest norms of the request's queries and of X; without a split
 *     form whose a-priori bound is <= eps, fp32 if resident) or LSH (the
 *     resident index's estimate, stag_lsh_index_query).
 *   - Requests are queued FIFO and admitted when their workspace footprint
 *     fits the remaining budget (larger than the whole budget: status
 *     STAG_E_BUSY).
 *   - An admitted request is served in chunks of at most chunk_queries
 *     queries.  Every idle stream takes the oldest admitted request with
 *     rows left and packs the next chunk of every admitted request of the
 *     same data set and kind/form (arrival order, one chunk per request) up
 *     to max_batch_queries queries and 1024 chunks into one batch; small
 *     requests arriving behind a large one share its next batches.
 *   - A result is bitwise identical whether its request ran alone, chunked
 *     or batched, and equal to stag_kde_exact in the same form (exact; the
 *     serving loop has no underflow rescue, so sums below 2^-60 keep the
 *     tile's accuracy) or to stag_lsh_index_query on the same index (LSH).
 * Q must be fully written before submission and X before it is added
 * (synchronise their producers: the server works on streams of its own).
 * S_out (and bound_out) are valid once wait/poll reports the request done.
 * A worker thread owned by the server drives the loop and one host thread
 * per stream issues its batches; every function is thread safe.  Latency
 * is measured from submission to completion.
 * ------------------------------------------------------------------------ */
typedef struct stag_server stag_server;

typedef struct {
  uint64_t submitted, completed, failed, rejected, batches, queries;
  double p50_s, p99_s, mean_s, max_s; /* latency of completed requests */
  uint64_t inflight_bytes, peak_inflight_bytes;
} stag_server_stats_t;

#define STAG_REQUEST_EXACT 0
#define STAG_REQUEST_LSH 1

/* budget_bytes 0: 8 GiB; n_streams 0: 4 (at most 16); max_batch_queries 0:
 * 65536; chunk_queries 0: 4096. */
stag_status stag_server_create(size_t budget_bytes, int32_t n_streams, int64_t max_batch_queries,
                               int64_t chunk_queries, stag_server** out);
/* X [n][d] device fp32 (prepared into the server's own buffers).  forms: bit
 * mask of resident exact forms (0 allowed with an index); d > 256: fp32
 * only.  lsh: NULL for no index, else the CKNS parameters (eps = lsh_eps in
 * (0, 1)).  Synchronises.  Errors: STAG_E_INVAL, STAG_E_UNSUPPORTED,
 * STAG_E_NOMEM. */
stag_status stag_server_add_dataset_ex(stag_server* s, const float* X, int64_t n, int32_t d, double a, uint32_t forms,
                                       double lsh_eps, const stag_lsh_params* lsh, int32_t* id_out);
/* One resident exact form, no index. */
stag_status stag_server_add_dataset(stag_server* s, const float* X, int64_t n, int32_t d, double a, int32_t form,
                                    int32_t* id_out);
/* kind STAG_REQUEST_EXACT or STAG_REQUEST_LSH; form a resident form or
 * STAG_FORM_AUTO with eps > 0 (exact only; the AUTO choice scans Q on the
 * device and waits for it); S_out [m] f64 device; bound_out [m] f64 device
 * or NULL (exact only: the per-result bound of the chosen form); form_out
 * (host, or NULL) receives the form (-1 for LSH). */
stag_status stag_server_submit_ex(stag_server* s, int32_t dataset, const float* Q, int64_t m, int32_t kind,
                                  int32_t form, double eps, double* S_out, double* bound_out, int32_t* form_out,
                                  uint64_t* ticket);
/* Exact, in the data set's first resident form (lowest form number). */
stag_status stag_server_submit(stag_server* s, int32_t dataset, const float* Q, int64_t m, double* S_out,
                               uint64_t* ticket);
/* Blocks until the request is done; *result is its status. */
stag_status stag_server_wait(stag_server* s, uint64_t ticket, stag_status* result, double* latency_s);
/* *done = 1 once finished (then *result and *latency_s are set), else 0. */
stag_status stag_server_poll(stag_server* s, uint64_t ticket, int32_t* done, stag_status* result,
                             double* latency_s);
stag_status stag_server_stats(stag_server* s, stag_server_stats_t* out);
/* Stops the loop, waits for the device and frees everything (NULL ignored). */
void stag_server_destroy(stag_server* s);

#ifdef __cplusplus
}
#endif

#endif /* STAG_KDE_H */
