// Exact kernel density tiles, epilogue mode kModeMax (largest exponent per chunk and query).
#include "kde_tiles.h"

namespace stag {

stag_status launch_tiles_max(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                             hipStream_t st) {
  return tiles::launch_tiles<tiles::kModeMax>(xo, qo, partial, ex, st);
}

}  // namespace stag
