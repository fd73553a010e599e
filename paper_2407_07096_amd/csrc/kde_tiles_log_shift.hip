// Exact kernel density tiles, epilogue mode kModeLogShift (the logistic kernel in
// the underflow rescue's second pass).
#include "kde_tiles.h"

namespace stag {

stag_status launch_tiles_log_shift(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                                   hipStream_t st) {
  return tiles::launch_tiles<tiles::kModeLogShift>(xo, qo, partial, ex, st);
}

}  // namespace stag
