// Exact kernel density tiles, epilogue mode kModeGaussExtra.
#include "kde_tiles.h"

namespace stag {

stag_status launch_tiles_gauss_extra(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                                     hipStream_t st) {
  return tiles::launch_tiles<tiles::kModeGaussExtra>(xo, qo, partial, ex, st);
}

}  // namespace stag
