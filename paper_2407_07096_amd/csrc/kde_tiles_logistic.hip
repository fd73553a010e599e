// Exact kernel density tiles, epilogue mode kModeLogistic.
#include "kde_tiles.h"

namespace stag {

stag_status launch_tiles_logistic(const Operands& xo, const Operands& qo, double* partial, const TileExtra& ex,
                                  hipStream_t st) {
  return tiles::launch_tiles<tiles::kModeLogistic>(xo, qo, partial, ex, st);
}

}  // namespace stag
