// Exact kernel density tiles, epilogue mode kModeGauss.
#include "kde_tiles.h"

namespace stag {

stag_status launch_tiles_gauss(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                               hipStream_t st) {
  return tiles::launch_tiles<tiles::kModeGauss>(xo, qo, partial, ex, st);
}

}  // namespace stag
