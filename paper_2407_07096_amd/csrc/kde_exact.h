// Internal interface of the exact kernel-density tiles, shared by the C ABI
// entry point, the similarity-graph sampler and the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "runtime.h"

namespace stag {

// Operand set of one side (data or queries) in a given form.
struct Operands {
  int form = 0;
  int64_t rows = 0, rows_pad = 0;
  int d = 0, dp = 0;
  void* part[3] = {nullptr, nullptr, nullptr};  // fp32 copy or split parts, [rows_pad][dp]
  float* off = nullptr;                         // -a log2(e) ||row||^2 (padding rows: -1e30 for data)
  void* aug = nullptr;                          // 8 x bf16 augmentation operand per row (split forms)
  double* nrm = nullptr;                        // ||row||^2, fp64, [rows]
  unsigned long long* max_nrm_bits = nullptr;   // max ||row||^2 (fp64 bits)
  // Centred data (fp32 form, d <= 256): rows grouped into compact 32-row
  // tiles, part[0] holds fl32(x - c_T) and off holds -a log2(e) ||x - c_T||^2
  // (padding rows -1e30); centre [rows_pad/32][dp] fp32 c_T, radius
  // [rows_pad/32] max ||x - c_T|| (rounded up).  rows_pad is an upper bound
  // of the padded row count; the count itself is *n_pad_dev (device).
  // Centred fp16 data (STAG_FORM_FP16_CENTRED, d <= 256): the same grouping
  // with one centre c_g per group: part[0] holds fl16(x - c_g) [rows_pad][dp],
  // off -a log2(e) ||x - c_g||^2 (NaN for a row outside fp16's range),
  // tgroup [rows_pad/32] the group of each tile, centre [K_pad][dp] fp32 c_g,
  // radius [K_pad] max ||x - c_g|| over the group (rounded up).
  bool centred = false;
  float* centre = nullptr;
  float* radius = nullptr;
  int64_t* n_pad_dev = nullptr;
  int* tgroup = nullptr;
};

// Temporaries of the centring's grouping (kde_centre.hip).
struct CentreTemp {
  int K = 0, K_pad = 0;
  int64_t nblk = 0;
  float *seeds = nullptr, *hn = nullptr, *ref = nullptr;
  uint8_t* label = nullptr;
  uint32_t *hist = nullptr, *count = nullptr, *goff = nullptr;
  int* map = nullptr;
  // fp16 form: per-tile fp64 coordinate sums [rows_pad/32][dp] (group means)
  double* tsum = nullptr;
};
// Upper bound of the padded row count of centred data of n rows.
int64_t centred_rows_max(int64_t n);
// Centred data operands of n rows (buffers from ws, no launch), the
// temporaries of their grouping (from a workspace that may be released once
// the preparation has run), and the preparation from X [n][d] (a_tile: the
// kernel's bandwidth, a for the Gaussian).
stag_status alloc_centred_operands(int64_t n, int d, Workspace& ws, Operands* out);
stag_status alloc_centre_temp(const Operands& o, Workspace& ws, CentreTemp* t);
stag_status prep_centred_operands(const float* X, double a_tile, const Operands& o, const CentreTemp& t,
                                  hipStream_t st);
// Queries ordered by their nearest seed of the data's grouping (the data's
// seeds), so that a 256-query tile holds queries of few groups: perm
// [m_pad] maps a sorted position to its query row (-1: padding).
struct QuerySort {
  int64_t nblk = 0;
  uint8_t* label = nullptr;
  uint32_t *hist = nullptr, *count = nullptr, *goff = nullptr;
  int64_t* total = nullptr;
  int* perm = nullptr;
};
stag_status alloc_query_sort(int64_t m, int64_t m_pad, int K, Workspace& ws, QuerySort* qs);
stag_status sort_queries(const float* Q, int64_t m, int64_t m_pad, int d, int dp, const CentreTemp& t,
                         const QuerySort& qs, hipStream_t st);
// The same for the centred fp16 form (group centres; o.form ==
// STAG_FORM_FP16_CENTRED, temporaries from alloc_centre_temp).
stag_status alloc_centred_h_operands(int64_t n, int d, Workspace& ws, Operands* out);
stag_status prep_centred_h_operands(const float* X, double a_tile, const Operands& o, const CentreTemp& t,
                                    hipStream_t st);

// Rounding-error model of one result.  The tiles produce the exponent
// E = -lambda D (base 2; lambda = la) with an absolute error of at most
//   dE = c_acc (cross + offs) + c_split cross + c_off offs,
// cross = 2 la ||q|| max||x||, offs = la (||q||^2 + max||x||^2).  The
// relative error of every kernel value, and so of the sum, is then at most
//   Gaussian     2^dE - 1
//   exponential  2^(sqrt(dE) + dy) - 1     (|sqrt(u) - sqrt(v)| <= sqrt|u - v|)
//   logistic     e^(dE / (4 log2(e)^2) + ln2 dy) - 1 + 5 ulp
// plus c_tail (exp2, the 16-term fp32 tile sums).  For the logistic kernel
// |d ln k / d(r^2)| <= 1/4 bounds the effect of the exponent error, and
// dy = 2^-23 min(150, sqrt(la) (||q|| + max||x||)) is the rounding of
// y = sqrt(-E) (terms with y > 150 are below 2^-150 and flush to zero).
// Exponential kernel: terms with computed y^2 = -E below this are evaluated
// exactly from the input rows (the tile's near pairs).
constexpr double kNearY2 = 0.25;

struct BoundModel {
  double la, c_acc, c_split, c_off, c_tail;
  // centred fp32 tile: each term's exponent error is at most c_cent M_T,
  // M_T = la (||q - c_T|| + R_T)^2 + |shift| (accumulated per tile in the
  // kernel, weighted by the tile's sum)
  double c_cent = 0.0;
  int kern = 0;          // a stag_kernel
  double near_y2 = 0.0;  // exponential kernel: terms with computed y^2 below this are exact
};

// extra (underflow rescue): Gaussian, a further offset magnitude carried by
// the accumulators (the shift |m_q|, in exponent units); exponential and
// logistic, the shift ys of y = sqrt(-E) (terms up to y = 150 + ys count).
// Sum of col[p * stride] over p = 0 .. P-1, added in increasing p (the loads
// issued eight at a time, so that a thread does not wait on each in turn).
__device__ inline double chunk_sum(const double* __restrict__ col, int P, int64_t stride) {
  double s = 0.0;
  int p = 0;
  for (; p + 8 <= P; p += 8) {
    double v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = col[(int64_t)(p + i) * stride];
#pragma unroll
    for (int i = 0; i < 8; ++i) s += v[i];
  }
  for (; p < P; ++p) s += col[(int64_t)p * stride];
  return s;
}

__host__ __device__ inline double relative_bound(const BoundModel& bm, double qn, double xm, double extra = 0.0) {
  const double ln2 = 0.69314718055994530942;
  const double cross = 2.0 * bm.la * sqrt(qn) * sqrt(xm);
  const double offs = bm.la * (qn + xm) + (bm.kern == 0 ? extra : 0.0);
  const double dE = bm.c_acc * (cross + offs) + bm.c_split * cross + bm.c_off * offs;
  if (bm.kern == 0) return expm1(ln2 * dE) + bm.c_tail;
  const double dy = 0x1.0p-23 * fmin(150.0 + extra, sqrt(bm.la) * (sqrt(qn) + sqrt(xm)));
  if (bm.kern == 1) {
    // A term left to the tile has computed y^2 >= near_y2, so its true y^2 is
    // >= near_y2 - dE and |dy| <= dE / (2 sqrt(near_y2 - dE)); without that
    // floor, y -> 0 gives |dy| <= sqrt(dE).
    const double dyE = bm.near_y2 > 2.0 * dE ? dE / (2.0 * sqrt(bm.near_y2 - dE)) : sqrt(dE);
    return expm1(ln2 * (dyE + dy)) + bm.c_tail;
  }
  const double log2e = 1.4426950408889634074;
  return expm1(dE / (4.0 * log2e * log2e) + ln2 * dy) + bm.c_tail + 5.0 * 0x1.0p-23;
}

// Epilogue options of the tiles: the kernel function, and for edge sampling
// (Gaussian only) two optional outputs: drop the diagonal
// when a data set is queried against itself, and write per-32-row-tile
// partial sums tp[query * ntile + tile] (fp32; ntile, the row stride, is at
// least padded data rows / 32 and a multiple of 16).
struct TileExtra {
  int kernel = 0;  // a stag_kernel; self and tp need the Gaussian
  // Exponential kernel, near pairs: a value whose computed -E is below near_e
  // (of a query < m_rows) is taken out of the tile sum and replaced by
  // exp(-a ||q - x||) from fp64 direct differences of the input rows
  // near_x[row * d], near_q[query * d].  Off when near_x is null.  A query
  // with more near pairs than the tile can hold gets near_over[query] = 1
  // (the array starts at zero) and keeps the excess in its tile sums.
  const float* near_x = nullptr;
  int* near_over = nullptr;
  const float* near_q = nullptr;
  int d = 0;
  float near_e = 0.0f;
  double a = 0.0;
  int64_t m_rows = 0;
  int self = 0;
  float* tp = nullptr;
  int64_t ntile = 0;
  // Gaussian underflow rescue: max_pass makes each partial the largest
  // exponent E of its (chunk, query) instead of a sum; with qtile_active, a
  // workgroup whose 128-query tile has flag 0 returns at once (its partials
  // are not written).
  int max_pass = 0;
  const int* qtile_active = nullptr;
  // exponential / logistic in the rescue's second pass: per query the shift
  // ys (smallest y = sqrt(-E)); the terms are 2^{ys - y}
  const float* yshift = nullptr;
  // centred data: bpart[chunk][query] = sum over the chunk's tiles of the
  // tile's kernel sum times (2^{c_cent M_T} - 1), the bound's numerator
  double* bpart = nullptr;
  float c_cent = 0.0f;
  // split tiles: with cflag, only the (chunk, 256-query tile) pairs with
  // cflag[chunk * ceil(m_pad / 256) + tile] != 0 run (the others return at
  // once, their partials not written)
  const uint8_t* cflag = nullptr;
  // the adaptive form's estimate on sampled query tiles (a timer of its own);
  // with qsel_n > 0 the centred fp16 tile launches only the workgroups that
  // hold the 128-query tiles qsel[0 .. qsel_n) (at most kMaxSel of them)
  int sample = 0;
  static constexpr int kMaxSel = 16;
  int qsel_n = 0;
  int qsel[kMaxSel] = {};
  int h1c_chunks = 0;  // chunks of the centred fp16 tile's grid (set by its launcher)
  // centred fp16 tile, Gaussian sums: a wave whose queries all have their
  // offset alpha in [-60, 0] for a group starts its accumulators from beta
  // alone and scales its tile sums by 2^alpha (a query's bits then depend on
  // the other queries of its wave)
  int fold_alpha = 0;
};

int exact_padded_dim(int d);  // 0 if unsupported
int form_parts(int form);
size_t form_element_bytes(int form);
int64_t exact_chunks(int64_t n_pad);
// lambda of the tiles for a kernel: a log2(e) (Gaussian), (a log2(e))^2
// (exponential, logistic); operands are prepared with a / log2(e) * lambda.
double kernel_tile_a(int kernel, double a);
BoundModel make_bound_model(int form, int d, double a_tile, int kernel = 0);

stag_status prepare_operands(int form, const float* src, int64_t rows, int d, double a, bool is_query,
                             Workspace& ws, Operands* out, hipStream_t st);
// The two halves of prepare_operands: the operand set's buffers from ws (no
// launch), then the preparation kernel into them.
stag_status alloc_operands(int form, int64_t rows, int d, bool is_query, Workspace& ws, Operands* out);
stag_status prep_operands(const float* src, double a, bool is_query, const Operands& o, hipStream_t st);
// Prepares `rows` query rows into a batch operand set (allocated by the
// caller for batch.rows_pad rows) starting at row0 (a multiple of the query
// tile, query_tile_rows()).
stag_status prep_query_into(int form, const float* src, int64_t rows, int d, double a, const Operands& batch,
                            int64_t row0, hipStream_t st, bool centred = false);
// Largest squared row norm (fp64 bits), largest |element| (fp32 bits) and a
// non-finite flag of A [rows][d], into caller device words (cleared first;
// asynchronous on st).
stag_status row_stats_async(const float* A, int64_t rows, int d, unsigned long long* nrm_bits, unsigned int* abs_bits,
                            int* bad, hipStream_t st);
// The form the STAG_FORM_AUTO rule takes among the resident ones (bit mask of
// 1 << form) for the Gaussian kernel: the first of fp16 split (if the
// operands fit fp16), bf16 split, bf16 three-way whose a-priori bound at the
// largest norms is <= eps, else fp32 if resident, else the resident split
// form of smallest bound; -1 if none is resident.
int choose_resident_form(uint32_t resident, int d, double a, double eps, double max_nrm_q, double max_nrm_x,
                         float max_abs_q, float max_abs_x);
int64_t query_tile_rows();
stag_status launch_exact_tiles(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                               hipStream_t st);
// A Gaussian sum below this is recomputed with its exponents shifted by
// their maximum (its terms may lie below the fp32 range of the tile).
constexpr double kRescueBelow = 0x1.0p-60;

// Shift of the underflow rescue: for the flagged queries (flag[q] != 0, their
// 128-query tiles in qtile_flag) m_q = the largest exponent E over the data
// (a max pass of the tiles; self: leave out the diagonal of a data set
// queried against itself), shift[q] = m_q and off2[q] = fl32(-a_tile log2(e)
// ||q||^2 - m_q); other queries keep their offset and shift 0.  off2 and
// shift have qo.rows_pad entries.
stag_status rescue_offsets(const Operands& xo, const Operands& qo, int P, double a_tile, int self, const int* flag,
                           const int* qtile_flag, float* off2, double* shift, Workspace& ws, hipStream_t st);
// As rescue_offsets, with the max pass's partials pmax [P][qo.rows_pad] from
// the caller.
stag_status rescue_offsets_into(const Operands& xo, const Operands& qo, int P, double a_tile, int self,
                                const int* flag, const int* qtile_flag, double* pmax, float* off2, double* shift,
                                hipStream_t st);
// Buffers of the underflow rescue of one call (flag [m], qflag [m_pad/128],
// pmax and p2 [P][m_pad]; Gaussian: shift, off2 [m_pad]; other kernels:
// yshift [m_pad]).
struct RescueBuffers {
  int *flag = nullptr, *qflag = nullptr;
  double *pmax = nullptr, *p2 = nullptr, *shift = nullptr;
  float *off2 = nullptr, *yshift = nullptr;
};
stag_status alloc_rescue(int kernel, int P, const Operands& qo, Workspace& ws, RescueBuffers* rb);
stag_status reduce_with_rescue_into(const double* partial, int P, const Operands& qo, const Operands& xo,
                                    double a_tile, double scale, const BoundModel& bm, const RescueBuffers& rb,
                                    double* S_out, double* bound_out, hipStream_t st);
// launch_reduce for the Gaussian kernel with the underflow rescue: sums
// below 2^-60 are recomputed with their exponents shifted by their maximum
// (two more tile passes over the 128-query tiles that hold such queries).
stag_status reduce_with_rescue(const double* partial, int P, const Operands& qo, const Operands& xo, double a_tile,
                               double scale, const BoundModel& bm, double* S_out, double* bound_out, Workspace& ws,
                               hipStream_t st);
stag_status launch_reduce(const double* partial, int P, const Operands& qo, const Operands& xo, double scale,
                          const BoundModel& bm, double* S_out, double* bound_out, hipStream_t st,
                          const int* near_over = nullptr, int* flag = nullptr, int* qtile_flag = nullptr);

}  // namespace stag
