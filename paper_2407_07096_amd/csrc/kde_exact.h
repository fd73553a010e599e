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
};

// Rounding-error model of one result, in base-2 exponent units:
//   dE <= c_acc (cross + offs) + c_split cross + c_off offs
// with cross = 2 a log2(e) ||q|| max||x|| and offs = a log2(e)(||q||^2 + max||x||^2);
// relative bound = 2^dE - 1 + c_tail.
struct BoundModel {
  double la, c_acc, c_split, c_off, c_tail;
};

__host__ __device__ inline double relative_bound(const BoundModel& bm, double qn, double xm) {
  const double cross = 2.0 * bm.la * sqrt(qn) * sqrt(xm);
  const double offs = bm.la * (qn + xm);
  const double dE = bm.c_acc * (cross + offs) + bm.c_split * cross + bm.c_off * offs;
  return expm1(0.69314718055994530942 * dE) + bm.c_tail;
}

// Optional epilogue outputs of the tiles (edge sampling): drop the diagonal
// when a data set is queried against itself, and write per-32-row-tile
// partial sums tp[query * ntile + tile] (fp32; ntile, the row stride, is at
// least padded data rows / 32 and a multiple of 8).
struct TileExtra {
  int self = 0;
  float* tp = nullptr;
  int64_t ntile = 0;
};

int exact_padded_dim(int d);  // 0 if unsupported
int form_parts(int form);
size_t form_element_bytes(int form);
int64_t exact_chunks(int64_t n_pad);
BoundModel make_bound_model(int form, int d, double a);

stag_status prepare_operands(int form, const float* src, int64_t rows, int d, double a, bool is_query,
                             Workspace& ws, Operands* out, hipStream_t st);
// Prepares `rows` query rows into a batch operand set (allocated by the
// caller for batch.rows_pad rows) starting at row0 (a multiple of the query
// tile, query_tile_rows()).
stag_status prep_query_into(int form, const float* src, int64_t rows, int d, double a, const Operands& batch,
                            int64_t row0, hipStream_t st);
int64_t query_tile_rows();
stag_status launch_exact_tiles(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                               hipStream_t st);
stag_status launch_reduce(const double* partial, int P, const Operands& qo, const Operands& xo, double scale,
                          const BoundModel& bm, double* S_out, double* bound_out, hipStream_t st);

}  // namespace stag
