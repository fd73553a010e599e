// Exact kernel density tiles, epilogue mode kModeGaussExtraRescue (the edge
// sampler's self pass in the underflow rescue).
#include "kde_tiles.h"

namespace stag {

stag_status launch_tiles_gauss_extra_rescue(const Operands& xo, const Operands& qo, double* partial,
                                            const TileExtra& ex, hipStream_t st) {
  return tiles::launch_tiles<tiles::kModeGaussExtraRescue>(xo, qo, partial, ex, st);
}

}  // namespace stag
