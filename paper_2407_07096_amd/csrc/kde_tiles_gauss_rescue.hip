// Exact kernel density tiles, epilogue mode kModeGaussRescue (the Gaussian sum of the underflow rescue).
#include "kde_tiles.h"

namespace stag {

stag_status launch_tiles_gauss_rescue(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                                      hipStream_t st) {
  return tiles::launch_tiles<tiles::kModeGaussRescue>(xo, qo, partial, ex, st);
}

}  // namespace stag
