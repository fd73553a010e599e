// FP64 CPU oracle for the Gaussian kernel density hot path of STAG 2.0
// ("Spectral Toolkit of Algorithms for Graphs: Technical Report (2)").
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
// reference that the GPU library is checked against.  Only the test suite,
// the smoke check and the benchmark's CPU-baseline leg load it; the product
// library never links, includes or calls it, and it shares no code with the
// GPU path (no headers, helpers, tables or constants in common).
//
// Precision: everything is IEEE binary64, compiled without -ffast-math and
// with -ffp-contract=off, so every product/sum below is rounded exactly as
// written.  Inputs are fp32 arrays widened exactly to binary64.
//
// Contents (each function cites the passage it follows):
//   orc_kde_exact           - Sec. "Kernel Density Estimation", definition of
//                             K(q) with the Gaussian kernel exp(-a x^2); the
//                             "naive" O(dmn) computation of ExactGaussianKDE.
//   orc_kde_kernel          - the same definition with the exponential and
//                             logistic kernels of that section.
//   orc_collision_probability, orc_boosted_probability
//                           - Sec. "Random Projection" closed form of p(c);
//                             Sec. "Boosting the Probability".
//   orc_e2lsh_hash          - Sec. "Random Projection": h(x) = floor((<x,g>+b)/4),
//                             K concatenated hashes per table, L tables.
//   orc_e2lsh_near_neighbours
//                           - the E2LSH class's get_near_neighbours: points that
//                             share a bucket with the query in some table.
//   orc_lsh_derive, orc_lsh_kde
//                           - Sec. "The CKNS Algorithm": levels L_i, log n
//                             subsamples with probability 2^-i, one LSH table
//                             set per subsample, the importance-weighted sum,
//                             repetition; constructor parameters eps, min_mu,
//                             K1, K2_constant, p_offset of CKNSGaussianKDE.
//   orc_kernel_row, orc_simgraph_exact, orc_simgraph_lsh
//                           - Sec. "The MS Algorithm", eq. (sampling_prob) and
//                             the degree deg_F(i) = sum_j K(||x_i - x_j||),
//                             with exact or CKNS kernel sums.
//   orc_simgraph_tree       - the same section's construction with a KDE
//                             algorithm as a black box: a neighbour is drawn
//                             by descending a binary tree over the data with
//                             random-sampling kernel-sum estimates per node.
//
// Where the paper leaves a detail open, the reading taken is stated at the
// function (level boundaries half-open, log base 2, reweighting by the
// recovery probability, first-table dedupe, SplitMix64 counter randomness).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <vector>

#include <omp.h>

namespace {

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): state advances by the golden-ratio increment and
// each output is the state passed through the 64-bit finaliser below.  The
// c-th output of a generator whose state starts at s is mix(s + (c+1)*gamma),
// which makes it a counter-based generator.
// ---------------------------------------------------------------------------
const uint64_t kGamma = 0x9E3779B97F4A7C15ULL;

uint64_t mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Stream state for (seed, tag, a, b); output c of that stream.
uint64_t counter_bits(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t s = mix(seed ^ tag);
  s = mix(s ^ a);
  s = mix(s ^ b);
  return mix(s + (c + 1) * kGamma);
}

const uint64_t kTagMask = 0x4D41534BULL;   // "MASK": CKNS subsampling
const uint64_t kTagDraw = 0x44524157ULL;   // "DRAW": edge-sampling uniforms
const uint64_t kKeySalt = 0x243F6A8885A308D3ULL;

// Bucket identity of K concatenated E2LSH codes in table l (a 64-bit fold;
// equal code tuples give equal keys, different tables give different keys).
uint64_t bucket_key(int32_t l, const int32_t* codes, int32_t K) {
  uint64_t h = mix(kKeySalt ^ (uint64_t)(uint32_t)l);
  for (int32_t k = 0; k < K; ++k) h = mix(h ^ (uint64_t)(uint32_t)codes[k]);
  return h;
}

// One E2LSH code: floor((<x, g> + b) / 4).  The inner product is the plain
// left-to-right binary64 sum of exact products of fp32 values.
int32_t e2lsh_code(const float* x, const float* g, double b, int32_t d) {
  double s = 0.0;
  for (int32_t j = 0; j < d; ++j) s = s + (double)x[j] * (double)g[j];
  double v = std::floor((s + b) / 4.0);
  if (v >= 2147483647.0) return 2147483647;
  if (v <= -2147483648.0) return (int32_t)(-2147483647 - 1);
  return (int32_t)v;
}

// Squared distance by direct differences (no expansion of the square).
double sqdist_direct(const float* q, const float* x, int32_t d) {
  double D = 0.0;
  for (int32_t j = 0; j < d; ++j) {
    double t = (double)q[j] - (double)x[j];
    D = D + t * t;
  }
  return D;
}

// Squared distance in the fused order used for LSH candidates: the running
// sum is updated with one correctly rounded fused multiply-add per coordinate.
double sqdist_fused(const float* q, const float* x, int32_t d) {
  double D = 0.0;
  for (int32_t j = 0; j < d; ++j) {
    double t = (double)q[j] - (double)x[j];
    D = std::fma(t, t, D);
  }
  return D;
}

// Neumaier compensated summation.
struct KahanSum {
  double s = 0.0, c = 0.0;
  void add(double v) {
    double t = s + v;
    if (std::fabs(s) >= std::fabs(v)) c += (s - t) + v;
    else c += (v - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

// p(c) of Sec. "Random Projection", rearranged so that exp(8/c^2) is never
// formed: c * e^{-8/c^2} (e^{8/c^2} - 1) = c (1 - e^{-8/c^2}).
double collision_p(double c) {
  if (c <= 0.0) return 1.0;
  const double pi = 3.14159265358979323846;
  return std::erf(2.0 * std::sqrt(2.0) / c) - c * (1.0 - std::exp(-8.0 / (c * c))) / (2.0 * std::sqrt(2.0 * pi));
}

// 1 - (1 - p^K)^L in a form that keeps relative accuracy for small p^K.
double boosted_p(double c, int32_t K, int32_t L) {
  double x = std::pow(collision_p(c), (double)K);
  if (x >= 1.0) return 1.0;
  return -std::expm1((double)L * std::log1p(-x));
}

struct LshShape {
  int32_t J, L, K, K1;
  double mu_min;
  double p[65];       // p[i], i = 1..J: sampling probability of level i
  uint64_t thr[65];   // keep j iff (bits >> 11) < thr[i]
  double T[65];       // T[0] = 0, T[i] = i ln2 / a: level i holds T[i-1] <= D < T[i]
  double r[65];       // r[i] = sqrt(T[i]): distance scale of level i's hashes
};

const uint32_t kFlagLiteral = 1u;     // weight 2^i only (no recovery reweighting)
const uint32_t kFlagAllSampled = 2u;  // test hook: p_i = 1 for every level

int ceil_log2_int(int64_t n) {  // smallest J with 2^J >= n
  int J = 0;
  while (((int64_t)1 << J) < n) ++J;
  return J;
}

// Parameter reading for CKNSGaussianKDE(data, a, eps, min_mu, K1, K2_constant,
// p_offset).  Returns 0 on success, nonzero on invalid arguments.
int derive(int64_t n, double a, double eps, double min_mu, int32_t k1, double k2c, int32_t p_offset,
           uint32_t flags, LshShape* s) {
  if (n < 1 || !(a > 0.0) || !std::isfinite(a) || !(eps > 0.0 && eps < 1.0) || p_offset < 0) return 1;
  const bool default_mu = !(min_mu > 0.0);
  s->mu_min = default_mu ? 1.0 / (double)n : min_mu;
  // "log n" levels: J = ceil(log2(1/mu_min)), at least 1.
  int J = default_mu ? ceil_log2_int(n) : (int)std::ceil(std::log2(1.0 / s->mu_min));
  if (J < 1) J = 1;
  if (J > 64) return 2;
  s->J = J;
  // L tables per level: ceil(K2_constant), default ceil(log2 n).
  int L = (k2c > 0.0) ? (int)std::ceil(k2c) : std::max(1, ceil_log2_int(n));
  s->L = L;
  // K: largest k with recovery 1-(1-p(1)^k)^L >= 1 - eps/4 at unit scaled distance.
  int K = 1;
  for (int k = 2; k <= 64; ++k) {
    if (boosted_p(1.0, k, L) >= 1.0 - eps / 4.0) K = k; else break;
  }
  s->K = K;
  // K1 copies: ceil(eps^-2 log2 n).
  s->K1 = (k1 > 0) ? k1 : std::max(1, (int)std::ceil(std::log2((double)n) / (eps * eps)));
  const double ln2 = std::log(2.0);
  s->p[0] = 1.0; s->thr[0] = 0; s->T[0] = 0.0; s->r[0] = 0.0;
  for (int i = 1; i <= J; ++i) {
    double p;
    if (flags & kFlagAllSampled) p = 1.0;
    else if (default_mu) p = std::ldexp(1.0, -i - p_offset);
    else p = std::min(1.0, std::ldexp(1.0, -i) / ((double)n * s->mu_min)) * std::ldexp(1.0, -p_offset);
    s->p[i] = p;
    s->thr[i] = (uint64_t)std::ldexp(p, 53);
    s->T[i] = (double)i * ln2 / a;
    s->r[i] = std::sqrt(s->T[i]);
  }
  return 0;
}

}  // namespace

extern "C" {

uint64_t orc_mix64(uint64_t z) { return mix(z); }

uint64_t orc_counter_bits(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, uint64_t c) {
  return counter_bits(seed, tag, a, b, c);
}

uint64_t orc_bucket_key(int32_t l, const int32_t* codes, int32_t K) { return bucket_key(l, codes, K); }

double orc_collision_probability(double c) { return collision_p(c); }

double orc_boosted_probability(double c, int32_t K, int32_t L) { return boosted_p(c, K, L); }

// Gaussian kernel value exp(-a ||p1 - p2||^2) (Sec. "Kernel Density
// Estimation" user's guide, gaussian_kernel(a, p1, p2)).
double orc_gaussian_kernel(double a, const float* p1, const float* p2, int32_t d) {
  return std::exp(-a * sqdist_direct(p1, p2, d));
}

// Exact kernel density sum S(q) = sum_i exp(-a ||q - x_i||^2) for every row q
// of Q (Sec. "Kernel Density Estimation": K(q) = S(q)/n; ExactGaussianKDE
// query, O(dmn)).  The sum is formed with a max shift: with
// M = max_i(-a D_i), log S = M + log(sum_i exp(-a D_i - M)), the inner sum
// compensated and taken over i ascending.  S_out receives S (0 if it
// underflows), logS_out (if not NULL) receives log S.
void orc_kde_exact(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, double a,
                   double* S_out, double* logS_out, int32_t nthreads) {
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<double> E((size_t)n);
#pragma omp for schedule(static)
    for (int64_t qi = 0; qi < m; ++qi) {
      const float* q = Q + (size_t)qi * d;
      double M = -INFINITY;
      for (int64_t i = 0; i < n; ++i) {
        E[i] = -a * sqdist_direct(q, X + (size_t)i * d, d);
        if (E[i] > M) M = E[i];
      }
      KahanSum acc;
      for (int64_t i = 0; i < n; ++i) acc.add(std::exp(E[i] - M));
      const double sum = acc.value();
      const double lg = M + std::log(sum);
      // exp(M) * sum keeps S = n exact when every point equals q; below
      // exp(-700) the scaled form would lose bits to subnormals.
      S_out[qi] = (M > -700.0) ? std::exp(M) * sum : std::exp(lg);
      if (logS_out) logS_out[qi] = lg;
    }
  }
}

// Kernel functions of Sec. "Kernel Density Estimation" as functions of the
// distance r = ||q - x|| (kernel ids: 0 Gaussian, 1 exponential, 2 logistic):
//   Gaussian     exp(-a r^2)
//   exponential  exp(-a r)
//   logistic     4 / (2 + e^{a r} + e^{-a r}); the paper writes it without a
//                bandwidth, which is the case a = 1 here.
double kernel_of_distance(int32_t kernel, double a, double r) {
  switch (kernel) {
    case 0: return std::exp(-a * r * r);
    case 1: return std::exp(-a * r);
    default: {
      const double u = a * r;
      return 4.0 / (2.0 + std::exp(u) + std::exp(-u));
    }
  }
}

// S(q) = sum_i k(||q - x_i||) for every row q of Q, with the kernel chosen by
// id as above: the definition of K(q) = S(q)/n written out, r_i = sqrt(D_i)
// from the direct-difference squared distance, the terms summed over i
// ascending with compensation.  Returns -1 for an unknown kernel id.
int32_t orc_kde_kernel(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, int32_t kernel, double a,
                       double* S_out, int32_t nthreads) {
  if (kernel < 0 || kernel > 2) return -1;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t qi = 0; qi < m; ++qi) {
    const float* q = Q + (size_t)qi * d;
    KahanSum acc;
    for (int64_t i = 0; i < n; ++i)
      acc.add(kernel_of_distance(kernel, a, std::sqrt(sqdist_direct(q, X + (size_t)i * d, d))));
    S_out[qi] = acc.value();
  }
  return 0;
}

// One kernel value k(r) (the same functions, for pins of their shape).
double orc_kernel_value(int32_t kernel, double a, double r) { return kernel_of_distance(kernel, a, r); }

// Kernel values of one data point against all others: out[j] = exp(-a D_ij).
void orc_kernel_row(const float* X, int64_t n, int32_t d, double a, int64_t i, double* out) {
  const float* xi = X + (size_t)i * d;
  for (int64_t j = 0; j < n; ++j) out[j] = std::exp(-a * sqdist_direct(xi, X + (size_t)j * d, d));
}

// E2LSH codes and bucket keys (Sec. "Random Projection" and "Boosting the
// Probability").  G is [L*K][d] (table-major, then code), b is [L*K] in
// [0,4).  codes_out [n][L][K] and keys_out [n][L] may each be NULL.
void orc_e2lsh_hash(const float* X, int64_t n, int32_t d, const float* G, const double* b, int32_t K,
                    int32_t L, int32_t* codes_out, uint64_t* keys_out, int32_t nthreads) {
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t i = 0; i < n; ++i) {
    std::vector<int32_t> codes((size_t)K);
    const float* x = X + (size_t)i * d;
    for (int32_t l = 0; l < L; ++l) {
      for (int32_t k = 0; k < K; ++k) {
        int32_t p = l * K + k;
        codes[k] = e2lsh_code(x, G + (size_t)p * d, b[p], d);
        if (codes_out) codes_out[((size_t)i * L + l) * K + k] = codes[k];
      }
      if (keys_out) keys_out[(size_t)i * L + l] = bucket_key(l, codes.data(), K);
    }
  }
}

// Near neighbours under an E2LSH table of L tables with K codes each (Sec.
// "Random Projection", "Boosting the Probability"; the get_near_neighbours
// method of the E2LSH class): the points whose key equals the query's in at
// least one table.  The paper returns them as a set; the listing order taken
// here is table by table (0 first), ascending point index within a table,
// each point only in the first table where it collides.  counts_out [m];
// idx_out, if not NULL, receives the lists back to back (sum of counts).
void orc_e2lsh_near_neighbours(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, const float* G,
                               const double* b, int32_t K, int32_t L, int64_t* counts_out, int32_t* idx_out,
                               int32_t nthreads) {
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  std::vector<uint64_t> kx((size_t)n * L), kq((size_t)m * L);
  orc_e2lsh_hash(X, n, d, G, b, K, L, nullptr, kx.data(), nthreads);
  orc_e2lsh_hash(Q, m, d, G, b, K, L, nullptr, kq.data(), nthreads);
  auto first_table = [&](int64_t q, int64_t j) {  // first colliding table, or L
    for (int32_t l = 0; l < L; ++l)
      if (kx[(size_t)j * L + l] == kq[(size_t)q * L + l]) return l;
    return L;
  };
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t q = 0; q < m; ++q) {
    int64_t c = 0;
    for (int64_t j = 0; j < n; ++j) c += first_table(q, j) < L ? 1 : 0;
    counts_out[q] = c;
  }
  if (!idx_out) return;
  std::vector<int64_t> off((size_t)m + 1, 0);
  for (int64_t q = 0; q < m; ++q) off[(size_t)q + 1] = off[(size_t)q] + counts_out[q];
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t q = 0; q < m; ++q) {
    int64_t w = off[(size_t)q];
    for (int32_t l = 0; l < L; ++l)
      for (int64_t j = 0; j < n; ++j)
        if (first_table(q, j) == l) idx_out[w++] = (int32_t)j;
  }
}

// Parameters of the CKNS structure.  shape_i32 <- {J, L, K, K1};
// p, T, r are [J+1] (index 0 unused / zero), thr likewise.
int32_t orc_lsh_derive(int64_t n, double a, double eps, double min_mu, int32_t k1, double k2c,
                       int32_t p_offset, uint32_t flags, int32_t* shape_i32, double* mu_min_out,
                       double* p, uint64_t* thr, double* T, double* r) {
  LshShape s;
  int rc = derive(n, a, eps, min_mu, k1, k2c, p_offset, flags, &s);
  if (rc) return rc;
  shape_i32[0] = s.J; shape_i32[1] = s.L; shape_i32[2] = s.K; shape_i32[3] = s.K1;
  if (mu_min_out) *mu_min_out = s.mu_min;
  for (int i = 0; i <= s.J; ++i) {
    if (p) p[i] = s.p[i];
    if (thr) thr[i] = s.thr[i];
    if (T) T[i] = s.T[i];
    if (r) r[i] = s.r[i];
  }
  return 0;
}

// Subsample membership of copy t, level i: j is kept iff the 53 high bits of
// the counter draw (seed, MASK, t, i, j) fall below thr (i.e. U < p_i).
void orc_lsh_mask(uint64_t seed, int32_t t, int32_t i, int64_t n, uint64_t thr, uint8_t* keep) {
  for (int64_t j = 0; j < n; ++j)
    keep[j] = (counter_bits(seed, kTagMask, (uint64_t)t, (uint64_t)i, (uint64_t)j) >> 11) < thr ? 1 : 0;
}

// CKNS kernel density estimate (Sec. "The CKNS Algorithm").
//
// For each copy t < K1 and level i = 1..J:
//   * subsample S_{t,i} = { j : U(t,i,j) < p_i };
//   * L tables of K concatenated E2LSH functions on the space scaled by
//     1/r_i: projection g = fp32(g0 / r_i) from the stored N(0,1) vectors
//     G0[t][i-1][l][k][:], offsets b[t][i-1][l][k];
//   * a bucket map per table over S_{t,i}, members in ascending j.
// Query q, copy t: for i = 1..J, l = 0..L-1, every member j of q's bucket in
// table l (ascending j) that has not collided with q in an earlier table
// l' < l of the same level; keep it if T_{i-1} <= D < T_i (level L_i) and add
//     exp(-a D) / (p_i * R_i),   R_i = 1 - (1 - p(sqrt(D)/r_i)^K)^L
// (R_i = 1 under the literal 2^i weighting).  The estimate is the mean of the
// K1 copies.  D is the fused-order squared distance.
//
// Returns 0 on success.  n_cand[q] counts bucket members examined (with
// repeats across tables), n_acc[q] the accepted terms; S_copies is [m][K1].
int32_t orc_lsh_kde(const float* X, int64_t n, int32_t d, const float* Q, int64_t m, double a,
                    double eps, double min_mu, int32_t k1, double k2c, int32_t p_offset, uint64_t seed,
                    uint32_t flags, const float* G0, const double* B, double* S_out, int64_t* n_cand,
                    int64_t* n_acc, double* S_copies, int32_t nthreads) {
  LshShape s;
  int rc = derive(n, a, eps, min_mu, k1, k2c, p_offset, flags, &s);
  if (rc) return rc;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  const int J = s.J, L = s.L, K = s.K, K1 = s.K1;
  std::vector<double> St((size_t)m * K1, 0.0);
  std::vector<int64_t> cand((size_t)m, 0), acc((size_t)m, 0);
  std::vector<float> g((size_t)L * K * d);
  std::vector<int32_t> members;
  std::vector<uint64_t> mkeys;
  for (int t = 0; t < K1; ++t) {
    for (int i = 1; i <= J; ++i) {
      // scaled projections of this level
      const size_t base = ((size_t)t * J + (i - 1)) * (size_t)L * K;
      for (size_t e = 0; e < (size_t)L * K * d; ++e)
        g[e] = (float)((double)G0[base * d + e] / s.r[i]);
      const double* bb = B + base;
      // subsample
      members.clear();
      for (int64_t j = 0; j < n; ++j)
        if ((counter_bits(seed, kTagMask, (uint64_t)t, (uint64_t)i, (uint64_t)j) >> 11) < s.thr[i])
          members.push_back((int32_t)j);
      const int64_t ns = (int64_t)members.size();
      mkeys.assign((size_t)ns * L, 0);
#pragma omp parallel for schedule(static) num_threads(nthreads)
      for (int64_t u = 0; u < ns; ++u) {
        std::vector<int32_t> codes((size_t)K);
        const float* x = X + (size_t)members[u] * d;
        for (int l = 0; l < L; ++l) {
          for (int k = 0; k < K; ++k)
            codes[k] = e2lsh_code(x, &g[((size_t)l * K + k) * d], bb[l * K + k], d);
          mkeys[(size_t)u * L + l] = bucket_key(l, codes.data(), K);
        }
      }
      // bucket maps: key -> positions u (ascending, hence ascending j)
      std::vector<std::unordered_map<uint64_t, std::vector<int64_t>>> tab((size_t)L);
      for (int64_t u = 0; u < ns; ++u)
        for (int l = 0; l < L; ++l) tab[l][mkeys[(size_t)u * L + l]].push_back(u);
      const double Tlo = s.T[i - 1], Thi = s.T[i], pi = s.p[i], ri = s.r[i];
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
      for (int64_t qi = 0; qi < m; ++qi) {
        const float* q = Q + (size_t)qi * d;
        std::vector<uint64_t> qk((size_t)L);
        std::vector<int32_t> codes((size_t)K);
        for (int l = 0; l < L; ++l) {
          for (int k = 0; k < K; ++k) codes[k] = e2lsh_code(q, &g[((size_t)l * K + k) * d], bb[l * K + k], d);
          qk[l] = bucket_key(l, codes.data(), K);
        }
        double sum = St[(size_t)qi * K1 + t];
        for (int l = 0; l < L; ++l) {
          auto it = tab[l].find(qk[l]);
          if (it == tab[l].end()) continue;
          for (int64_t u : it->second) {
            cand[qi] += 1;
            bool seen = false;
            for (int l2 = 0; l2 < l; ++l2)
              if (mkeys[(size_t)u * L + l2] == qk[l2]) { seen = true; break; }
            if (seen) continue;
            const double D = sqdist_fused(q, X + (size_t)members[u] * d, d);
            if (!(D >= Tlo && D < Thi)) continue;
            double R = 1.0;
            if (!(flags & kFlagLiteral)) R = boosted_p(std::sqrt(D) / ri, K, L);
            sum += std::exp(-a * D) / (pi * R);
            acc[qi] += 1;
          }
        }
        St[(size_t)qi * K1 + t] = sum;
      }
    }
  }
  for (int64_t qi = 0; qi < m; ++qi) {
    double tot = 0.0;
    for (int t = 0; t < K1; ++t) tot += St[(size_t)qi * K1 + t];
    S_out[qi] = tot / (double)K1;
    if (n_cand) n_cand[qi] = cand[qi];
    if (n_acc) n_acc[qi] = acc[qi];
    if (S_copies)
      for (int t = 0; t < K1; ++t) S_copies[(size_t)qi * K1 + t] = St[(size_t)qi * K1 + t];
  }
  return 0;
}

// Uniform in [0,1) of draw r at node i (53 high bits of the counter draw).
double orc_draw_uniform(uint64_t seed, int64_t i, int32_t r) {
  return (double)(counter_bits(seed, kTagDraw, (uint64_t)i, 0, (uint64_t)r) >> 11) * 0x1.0p-53;
}

// Similarity-graph edge sampling from exact kernel values (Sec. "The MS
// Algorithm").  deg(i) = sum_j k(x_i, x_j) (self term included).  Each node i
// draws s neighbours j != i with probability k_ij / (deg(i) - 1) by inverse
// CDF over j ascending on the uniform U(i, r); every draw (i, j) is emitted
// with weight k_ij / (s (P_i(j) + P_j(i))), which makes the expected sampled
// weight of every pair equal to k_ij (eq. sampling_prob).  Output is
// node-major, draw-minor: entry i*s + r.  deg_out [n] may be NULL.
void orc_simgraph_exact(const float* X, int64_t n, int32_t d, double a, int32_t s, uint64_t seed,
                        int64_t* src, int64_t* dst, double* w, double* deg_out, double* margin_out,
                        int32_t nthreads) {
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  std::vector<double> rest((size_t)n);  // deg(i) - 1 = sum over j != i
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<double> row((size_t)n);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      orc_kernel_row(X, n, d, a, i, row.data());
      KahanSum ks;
      for (int64_t j = 0; j < n; ++j)
        if (j != i) ks.add(row[j]);
      rest[i] = ks.value();
    }
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      orc_kernel_row(X, n, d, a, i, row.data());
      for (int32_t r = 0; r < s; ++r) {
        const double target = orc_draw_uniform(seed, i, r) * rest[i];
        double c = 0.0;
        int64_t pick = -1, last = -1;
        double before = 0.0;
        for (int64_t j = 0; j < n; ++j) {
          if (j == i) continue;
          if (row[j] > 0.0) last = j;
          before = c;
          c = c + row[j];
          if (c > target) { pick = j; break; }
        }
        const size_t e = (size_t)i * s + r;
        // relative distance of the target to the nearest cumulative boundary
        if (margin_out) margin_out[e] = pick >= 0 ? std::min(target - before, c - target) / rest[i] : 0.0;
        if (pick < 0) pick = last;  // rounding left the target above the total
        src[e] = i;
        dst[e] = pick;
        if (pick < 0) { w[e] = 0.0; continue; }
        w[e] = 1.0 / ((double)s * (1.0 / rest[i] + 1.0 / rest[pick]));
      }
    }
  }
  if (deg_out)
    for (int64_t i = 0; i < n; ++i) deg_out[i] = rest[i] + 1.0;
}


// Edge sampling with the CKNS estimator in place of exact degrees (the
// similarity-graph construction on top of the LSH kernel density estimate).
// Every node i is queried against the data with its own point excluded:
// S'_t(i) is copy t's estimate of sum_{j != i} k_ij, accumulated in the
// canonical order (level, table, bucket member ascending);
// rest_i = mean_t S'_t(i), deg(i) = 1 + rest_i.  A draw takes the target
// U(i, r) * sum_t S'_t(i), picks the copy whose cumulative estimate passes
// it, then the term of that copy whose cumulative sum passes the remainder;
// its point j is the neighbour, with weight 1/(s (1/rest_i + 1/rest_j)).
// margin_out: relative distance of the target to the nearest boundary.
int32_t orc_simgraph_lsh(const float* X, int64_t n, int32_t d, double a, double eps, double min_mu, int32_t k1,
                         double k2c, int32_t p_offset, uint64_t lsh_seed, uint32_t flags, const float* G0,
                         const double* B, int32_t s, uint64_t draw_seed, int64_t* src, int64_t* dst, double* w,
                         double* deg_out, double* margin_out, int32_t nthreads) {
  LshShape sh;
  int rc = derive(n, a, eps, min_mu, k1, k2c, p_offset, flags, &sh);
  if (rc) return rc;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  const int J = sh.J, L = sh.L, K = sh.K, K1 = sh.K1;
  // terms[(node * K1 + t)] = ordered (j, value)
  std::vector<std::vector<std::pair<int32_t, double>>> terms((size_t)n * K1);
  std::vector<float> g((size_t)L * K * d);
  std::vector<int32_t> members;
  std::vector<uint64_t> mkeys;
  for (int t = 0; t < K1; ++t) {
    for (int i = 1; i <= J; ++i) {
      const size_t base = ((size_t)t * J + (i - 1)) * (size_t)L * K;
      for (size_t e = 0; e < (size_t)L * K * d; ++e) g[e] = (float)((double)G0[base * d + e] / sh.r[i]);
      const double* bb = B + base;
      members.clear();
      for (int64_t j = 0; j < n; ++j)
        if ((counter_bits(lsh_seed, kTagMask, (uint64_t)t, (uint64_t)i, (uint64_t)j) >> 11) < sh.thr[i])
          members.push_back((int32_t)j);
      const int64_t ns = (int64_t)members.size();
      mkeys.assign((size_t)ns * L, 0);
#pragma omp parallel for schedule(static) num_threads(nthreads)
      for (int64_t u = 0; u < ns; ++u) {
        std::vector<int32_t> codes((size_t)K);
        const float* x = X + (size_t)members[u] * d;
        for (int l = 0; l < L; ++l) {
          for (int k = 0; k < K; ++k) codes[k] = e2lsh_code(x, &g[((size_t)l * K + k) * d], bb[l * K + k], d);
          mkeys[(size_t)u * L + l] = bucket_key(l, codes.data(), K);
        }
      }
      std::vector<std::unordered_map<uint64_t, std::vector<int64_t>>> tab((size_t)L);
      for (int64_t u = 0; u < ns; ++u)
        for (int l = 0; l < L; ++l) tab[l][mkeys[(size_t)u * L + l]].push_back(u);
      const double Tlo = sh.T[i - 1], Thi = sh.T[i], pi = sh.p[i], ri = sh.r[i];
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
      for (int64_t qi = 0; qi < n; ++qi) {
        const float* q = X + (size_t)qi * d;
        std::vector<uint64_t> qk((size_t)L);
        std::vector<int32_t> codes((size_t)K);
        for (int l = 0; l < L; ++l) {
          for (int k = 0; k < K; ++k) codes[k] = e2lsh_code(q, &g[((size_t)l * K + k) * d], bb[l * K + k], d);
          qk[l] = bucket_key(l, codes.data(), K);
        }
        auto& out = terms[(size_t)qi * K1 + t];
        for (int l = 0; l < L; ++l) {
          auto it = tab[l].find(qk[l]);
          if (it == tab[l].end()) continue;
          for (int64_t u : it->second) {
            bool seen = false;
            for (int l2 = 0; l2 < l; ++l2)
              if (mkeys[(size_t)u * L + l2] == qk[l2]) { seen = true; break; }
            if (seen) continue;
            const int32_t j = members[u];
            if (j == qi) continue;
            const double D = sqdist_fused(q, X + (size_t)j * d, d);
            if (!(D >= Tlo && D < Thi)) continue;
            double R = 1.0;
            if (!(flags & kFlagLiteral)) R = boosted_p(std::sqrt(D) / ri, K, L);
            out.push_back({j, std::exp(-a * D) / (pi * R)});
          }
        }
      }
    }
  }
  std::vector<double> St((size_t)n * K1), rest((size_t)n);
  for (int64_t qi = 0; qi < n; ++qi) {
    double tot = 0.0;
    for (int t = 0; t < K1; ++t) {
      double sum = 0.0;
      for (auto& pr : terms[(size_t)qi * K1 + t]) sum += pr.second;
      St[(size_t)qi * K1 + t] = sum;
      tot += sum;
    }
    rest[qi] = tot / (double)K1;
  }
  for (int64_t qi = 0; qi < n; ++qi) {
    double tot = 0.0;
    for (int t = 0; t < K1; ++t) tot += St[(size_t)qi * K1 + t];
    for (int32_t r = 0; r < s; ++r) {
      const size_t e = (size_t)qi * s + r;
      src[e] = qi;
      dst[e] = -1;
      w[e] = 0.0;
      if (margin_out) margin_out[e] = 0.0;
      if (!(tot > 0.0)) continue;
      const double target = orc_draw_uniform(draw_seed, qi, r) * tot;
      double c = 0.0;
      int tsel = -1;
      for (int t = 0; t < K1; ++t) {
        if (c + St[(size_t)qi * K1 + t] > target) { tsel = t; break; }
        c += St[(size_t)qi * K1 + t];
      }
      if (tsel < 0) {  // rounding: last copy with mass
        for (int t = K1 - 1; t >= 0; --t)
          if (St[(size_t)qi * K1 + t] > 0.0) { tsel = t; break; }
        c = 0.0;
        for (int t = 0; t < tsel; ++t) c += St[(size_t)qi * K1 + t];
      }
      const double resid = target - c;
      const auto& tl = terms[(size_t)qi * K1 + tsel];
      double cc = 0.0, before = 0.0;
      int64_t pick = -1;
      for (auto& pr : tl) {
        before = cc;
        cc = cc + pr.second;
        if (cc > resid) { pick = pr.first; break; }
      }
      if (pick < 0) {
        pick = tl.back().first;
      } else if (margin_out) {
        margin_out[e] = std::min(resid - before, cc - resid) / tot;
      }
      dst[e] = pick;
      w[e] = 1.0 / ((double)s * (1.0 / rest[qi] + 1.0 / rest[pick]));
    }
  }
  if (deg_out)
    for (int64_t i = 0; i < n; ++i) deg_out[i] = 1.0 + rest[i];
  return 0;
}


// ---------------------------------------------------------------------------
// k-means for the third step of spectral clustering (Sec. "Fast Spectral
// Clustering": k-means on the embedded points).  Lloyd's iteration with
// k-means++ seeding (Arthur & Vassilvitskii 2007: first centre uniform, each
// further centre drawn with probability proportional to the squared distance
// to the nearest chosen centre).  The paper names k-means only; the seeding,
// the tie rules and the summation orders below are this library's reading,
// written out so that every decision is reproducible:
//   dist2(p, c)  = sum over j ascending of (p_j - c_j)^2, each subtraction,
//                  product and addition rounded (no fused operations);
//   U_r          = (counter_bits(seed, "KMNS", 0, 0, r) >> 11) 2^-53;
//   first centre = floor(U_0 n), taken exactly with integer arithmetic;
//   centre c > 0 = the first point i with Cum(i) > U_c T, where D2(i) is the
//                  squared distance to the nearest chosen centre, points are
//                  grouped in blocks of 1024, S_b is the sequential sum of D2
//                  over block b, B_b the sequential sum of S_0..S_{b-1},
//                  Cum(i) = B_b + (sequential sum of D2 over block b up to and
//                  including i) and T = B_{nb}; if no point qualifies (U_c T
//                  rounded up to T) the last point with D2 > 0; if T = 0 the
//                  lowest index not chosen yet;
//   assignment   = argmin over centres of dist2, ties to the lowest centre;
//   update       = per cluster, coordinate sums in the same blocked order
//                  (sequential over the points of a block, then over blocks),
//                  divided by the count; an empty cluster keeps its centre;
//   stop         = after an assignment that changes no label (the centres are
//                  then those the labels were assigned with) or after max_iter
//                  assignment + update rounds.
// ---------------------------------------------------------------------------
const uint64_t kTagKmeans = 0x4B4D4E53ULL;  // "KMNS"
const int64_t kKmBlock = 1024;

double dist2_seq(const double* p, const double* c, int32_t dim) {
  double s = 0.0;
  for (int32_t j = 0; j < dim; ++j) {
    const double t = p[j] - c[j];
    s = s + t * t;
  }
  return s;
}

double kmeans_uniform(uint64_t seed, int64_t r) {
  return (double)(counter_bits(seed, kTagKmeans, 0, 0, (uint64_t)r) >> 11) * 0x1.0p-53;
}

// Returns 0, or -1 for invalid sizes.  init (k x dim) replaces the seeding
// when not NULL; seeds_out (k) receives the seeded point indices (-1 with init).
int32_t orc_kmeans(const double* P, int64_t n, int32_t dim, int32_t k, uint64_t seed, int32_t max_iter,
                   const double* init, int32_t* labels, double* C, int32_t* iters_out, int64_t* seeds_out) {
  if (n < 1 || dim < 1 || k < 1 || k > n || max_iter < 1) return -1;
  const int64_t nb = (n + kKmBlock - 1) / kKmBlock;
  if (init) {
    std::memcpy(C, init, sizeof(double) * (size_t)k * dim);
    if (seeds_out)
      for (int32_t c = 0; c < k; ++c) seeds_out[c] = -1;
  } else {
    std::vector<double> D2((size_t)n, INFINITY);
    std::vector<char> chosen((size_t)n, 0);
    const uint64_t u0 = counter_bits(seed, kTagKmeans, 0, 0, 0) >> 11;
    int64_t pick = (int64_t)(((unsigned __int128)u0 * (uint64_t)n) >> 53);
    for (int32_t c = 0; c < k; ++c) {
      if (c > 0) {
        const double* last = C + (size_t)(c - 1) * dim;
        for (int64_t i = 0; i < n; ++i) D2[i] = std::min(D2[i], dist2_seq(P + (size_t)i * dim, last, dim));
        std::vector<double> B((size_t)nb + 1, 0.0);
        for (int64_t b = 0; b < nb; ++b) {
          double sb = 0.0;
          for (int64_t i = b * kKmBlock; i < std::min(n, (b + 1) * kKmBlock); ++i) sb = sb + D2[i];
          B[b + 1] = B[b] + sb;
        }
        const double T = B[nb];
        pick = -1;
        if (T > 0.0) {
          const double t = kmeans_uniform(seed, c) * T;
          for (int64_t b = 0; b < nb && pick < 0; ++b) {
            if (!(B[b + 1] > t)) continue;
            double cum = 0.0;
            for (int64_t i = b * kKmBlock; i < std::min(n, (b + 1) * kKmBlock); ++i) {
              cum = cum + D2[i];
              if (B[b] + cum > t) {
                pick = i;
                break;
              }
            }
          }
          if (pick < 0)
            for (int64_t i = n - 1; i >= 0 && pick < 0; --i)
              if (D2[i] > 0.0) pick = i;
        } else {
          for (int64_t i = 0; i < n && pick < 0; ++i)
            if (!chosen[i]) pick = i;
        }
      }
      chosen[pick] = 1;
      if (seeds_out) seeds_out[c] = pick;
      std::memcpy(C + (size_t)c * dim, P + (size_t)pick * dim, sizeof(double) * dim);
    }
  }
  for (int64_t i = 0; i < n; ++i) labels[i] = -1;
  std::vector<double> tot((size_t)k * dim), acc((size_t)k * dim);
  std::vector<int64_t> cnt((size_t)k);
  int32_t it = 0;
  while (it < max_iter) {
    ++it;
    bool changed = false;
    for (int64_t i = 0; i < n; ++i) {
      const double* p = P + (size_t)i * dim;
      int32_t best = 0;
      double bd = dist2_seq(p, C, dim);
      for (int32_t c = 1; c < k; ++c) {
        const double dc = dist2_seq(p, C + (size_t)c * dim, dim);
        if (dc < bd) {
          bd = dc;
          best = c;
        }
      }
      if (labels[i] != best) changed = true;
      labels[i] = best;
    }
    if (!changed) break;
    std::fill(tot.begin(), tot.end(), 0.0);
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t b = 0; b < nb; ++b) {
      std::fill(acc.begin(), acc.end(), 0.0);
      for (int64_t i = b * kKmBlock; i < std::min(n, (b + 1) * kKmBlock); ++i) {
        const int32_t l = labels[i];
        cnt[l] += 1;
        for (int32_t j = 0; j < dim; ++j) acc[(size_t)l * dim + j] = acc[(size_t)l * dim + j] + P[(size_t)i * dim + j];
      }
      for (size_t e = 0; e < tot.size(); ++e) tot[e] = tot[e] + acc[e];
    }
    for (int32_t c = 0; c < k; ++c)
      if (cnt[c] > 0)
        for (int32_t j = 0; j < dim; ++j) C[(size_t)c * dim + j] = tot[(size_t)c * dim + j] / (double)cnt[c];
  }
  *iters_out = it;
  return 0;
}


// ---------------------------------------------------------------------------
// Random-sampling KDE (the baseline of Sec. "Kernel Density Estimation" and of
// the experiments: estimate K(q) from a uniformly random sample of the data).
// Reading: s indices drawn independently and uniformly with replacement,
//   j_r = floor(U_r n), U_r = (counter_bits(seed, "RSKD", 0, 0, r) >> 11) 2^-53,
// taken exactly with integer arithmetic; one sample serves all queries; the
// estimate of S(q) = n K(q) is (n/s) sum_r exp(-a ||q - x_{j_r}||^2), the sum
// compensated over r ascending and scaled by the once-rounded n/s.
// Sample size for a (1 +- eps) estimate of every one of m queries whose
// density is at least mu, with failure probability at most delta: the
// multiplicative Chernoff bound for s independent values in [0, 1] with mean
// K >= mu, P(|mean - K| > eps K) <= 2 exp(-eps^2 K s / 3), and a union bound
// over the m queries give s = ceil(3 ln(2m/delta) / (eps^2 mu)).
// ---------------------------------------------------------------------------
const uint64_t kTagSample = 0x52534B44ULL;  // "RSKD"

int64_t sample_index(uint64_t seed, int64_t r, int64_t n) {
  const uint64_t u = counter_bits(seed, kTagSample, 0, 0, (uint64_t)r) >> 11;
  return (int64_t)(((unsigned __int128)u * (uint64_t)n) >> 53);
}

void orc_kde_random_sample(const float* X, int64_t n, const float* Q, int64_t m, int32_t d, double a, int64_t s,
                           uint64_t seed, double* S_out, int64_t* idx_out, int32_t nthreads) {
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  std::vector<int64_t> idx((size_t)s);
  for (int64_t r = 0; r < s; ++r) idx[r] = sample_index(seed, r, n);
  if (idx_out) std::memcpy(idx_out, idx.data(), sizeof(int64_t) * (size_t)s);
  const double scale = (double)n / (double)s;
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t qi = 0; qi < m; ++qi) {
    const float* q = Q + (size_t)qi * d;
    KahanSum acc;
    for (int64_t r = 0; r < s; ++r) acc.add(std::exp(-a * sqdist_direct(q, X + (size_t)idx[r] * d, d)));
    S_out[qi] = acc.value() * scale;
  }
}

int64_t orc_rs_sample_size(double eps, double mu, int64_t m, double delta) {
  return (int64_t)std::ceil(3.0 * std::log(2.0 * (double)m / delta) / (eps * eps * mu));
}

// ---------------------------------------------------------------------------
// Edge sampling through a KDE tree (Sec. "The MS Algorithm": each edge (i, j)
// is sampled with probability close to eq. (sampling_prob), the kernel sums
// coming from a KDE algorithm used as a black box).  The black box here is
// the random-sampling estimator of Sec. "Kernel Density Estimation".
//
// Tree: leaves are blocks of 32 consecutive rows, nb = ceil(n/32) of them;
// h = ceil(log2 nb); node (l, k), l = 0..h, holds rows
// [k 32 2^(h-l), (k+1) 32 2^(h-l)) clipped to [0, n).
// est(i, node, stream): with P rows in the node, if P <= t the exact sum of
// k_ij over its rows j != i (ascending j); otherwise (P/t) sum_c k_{i,j_c}
// [j_c != i] over c = 0..t-1 ascending, j_c = lo + floor(U_c P), U_c the c-th
// 53-bit uniform of the stream.  Both are unbiased for sum_{j in node, j != i}.
// Draw (i, r): from the root, at level l with children A, B (B possibly
// empty): eA = est(i, A, (i, r, l, 0)), eB = est(i, B, (i, r, l, 1)),
// u = U(i, r, l); go to A iff u (eA + eB) < eA; if eA + eB = 0, to the child
// with more rows other than i (A on a tie).  At the leaf (level h): values
// k_ij of its rows (0 for j = i) and their running sum c_j in row order,
// total T, target u T with u = U(i, r, h): j = the first row with c_j >
// target (the last positive one if rounding leaves none); if T = 0 the
// floor(u m)-th of the leaf's m rows other than i.
// Degrees: rest_i = est(i, root, degree stream of i) with t_deg samples
// (exact when n <= t_deg); deg_out[i] = 1 + rest_i; a draw (i, j) gets the
// weight 1/(s (1/rest_i + 1/rest_j)) (0 when an estimate is 0).
// margin_out: the smallest relative distance of a decision's target to its
// boundary along the draw's path (|u (eA+eB) - eA| / (eA+eB) per level, the
// leaf's as in orc_simgraph_exact); 1 where no decision was random.
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {
const uint64_t kTagTree = 0x54524545ULL;     // "TREE": node-estimate samples
const uint64_t kTagTreeU = 0x5452554EULL;    // "TRUN": descent uniforms
const uint64_t kTagTreeDeg = 0x54444547ULL;  // "TDEG": degree samples

double tree_u53(uint64_t bits) { return (double)(bits >> 11) * 0x1.0p-53; }

int64_t tree_pick(uint64_t bits, int64_t P) {
  return (int64_t)(((unsigned __int128)(bits >> 11) * (uint64_t)P) >> 53);
}

double gauss_k(const float* X, int32_t d, double a, int64_t i, int64_t j) {
  return std::exp(-a * sqdist_direct(X + (size_t)i * d, X + (size_t)j * d, d));
}

// est(i, [lo, hi)) with t samples from stream (tag, i, b).
double tree_estimate(const float* X, int32_t d, double a, int64_t i, int64_t lo, int64_t hi, int64_t t,
                     uint64_t seed, uint64_t tag, uint64_t b) {
  const int64_t P = hi - lo;
  if (P <= 0) return 0.0;
  double s = 0.0;
  if (P <= t) {
    for (int64_t j = lo; j < hi; ++j)
      if (j != i) s = s + gauss_k(X, d, a, i, j);
    return s;
  }
  for (int64_t c = 0; c < t; ++c) {
    const int64_t j = lo + tree_pick(counter_bits(seed, tag, (uint64_t)i, b, (uint64_t)c), P);
    if (j != i) s = s + gauss_k(X, d, a, i, j);
  }
  return s * ((double)P / (double)t);
}
}  // namespace

extern "C" {

// Draws are made for the rows i in [i_lo, i_hi) only (all rows: 0, n), output
// at (i - i_lo) s + r; the degrees always cover every row.
void orc_simgraph_tree(const float* X, int64_t n, int32_t d, double a, int32_t s, int32_t t, int64_t t_deg,
                       uint64_t seed, int64_t i_lo, int64_t i_hi, int64_t* src, int64_t* dst, double* w,
                       double* deg_out, double* margin_out, int32_t nthreads) {
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  const int64_t nb = (n + 31) / 32;
  int h = 0;
  while (((int64_t)1 << h) < nb) ++h;
  std::vector<double> rest((size_t)n);
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t i = 0; i < n; ++i) rest[i] = tree_estimate(X, d, a, i, 0, n, t_deg, seed, kTagTreeDeg, 0);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
  for (int64_t i = i_lo; i < i_hi; ++i) {
    for (int32_t r = 0; r < s; ++r) {
      int64_t k = 0;
      double margin = 1.0;
      for (int l = 0; l < h; ++l) {
        const int64_t span = (int64_t)32 << (h - l - 1);  // rows per child
        const int64_t aLo = std::min(n, 2 * k * span), aHi = std::min(n, (2 * k + 1) * span);
        const int64_t bLo = aHi, bHi = std::min(n, (2 * k + 2) * span);
        const uint64_t b0 = ((uint64_t)r << 16) | ((uint64_t)l << 1);
        const double eA = tree_estimate(X, d, a, i, aLo, aHi, t, seed, kTagTree, b0);
        const double eB = tree_estimate(X, d, a, i, bLo, bHi, t, seed, kTagTree, b0 | 1);
        const double u = tree_u53(counter_bits(seed, kTagTreeU, (uint64_t)i, (uint64_t)r, (uint64_t)l));
        const double tot = eA + eB;
        bool left;
        if (tot > 0.0) {
          const double x = u * tot;
          left = x < eA;
          margin = std::min(margin, std::fabs(x - eA) / tot);
        } else {
          const int64_t mA = (aHi - aLo) - (i >= aLo && i < aHi ? 1 : 0);
          const int64_t mB = (bHi - bLo) - (i >= bLo && i < bHi ? 1 : 0);
          left = mA >= mB;
        }
        k = left ? 2 * k : 2 * k + 1;
      }
      const int64_t lo = std::min(n, k * 32), hi = std::min(n, (k + 1) * 32);
      const double u = tree_u53(counter_bits(seed, kTagTreeU, (uint64_t)i, (uint64_t)r, (uint64_t)h));
      double T = 0.0;
      for (int64_t j = lo; j < hi; ++j)
        if (j != i) T = T + gauss_k(X, d, a, i, j);
      int64_t pick = -1;
      if (T > 0.0) {
        const double target = u * T;
        double c = 0.0, before = 0.0;
        int64_t last = -1;
        for (int64_t j = lo; j < hi; ++j) {
          const double v = j != i ? gauss_k(X, d, a, i, j) : 0.0;
          if (v > 0.0) last = j;
          before = c;
          c = c + v;
          if (c > target) {
            pick = j;
            margin = std::min(margin, std::min(target - before, c - target) / T);
            break;
          }
        }
        if (pick < 0) { pick = last; margin = 0.0; }
      } else {
        const int64_t m = (hi - lo) - (i >= lo && i < hi ? 1 : 0);
        int64_t idx = (int64_t)(u * (double)m);
        for (int64_t j = lo; j < hi; ++j) {
          if (j == i) continue;
          if (idx-- == 0) { pick = j; break; }
        }
      }
      const size_t e = (size_t)(i - i_lo) * s + r;
      src[e] = i;
      dst[e] = pick;
      w[e] = (rest[i] > 0.0 && rest[pick] > 0.0) ? 1.0 / ((double)s * (1.0 / rest[i] + 1.0 / rest[pick])) : 0.0;
      if (margin_out) margin_out[e] = margin;
    }
  }
  if (deg_out)
    for (int64_t i = 0; i < n; ++i) deg_out[i] = 1.0 + rest[i];
}

}  // extern "C"
