// Exact kernel density tiles, epilogue mode kModeExponential.
#include "kde_tiles.h"

namespace stag {

stag_status launch_tiles_exponential(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                                     hipStream_t st) {
  return tiles::launch_tiles<tiles::kModeExponential>(xo, qo, partial, ex, st);
}

}  // namespace stag
