// Stable device radix sort of (uint32 key, uint32 value) pairs (internal).
#pragma once

#include "runtime.h"

namespace stag {

// Sorts the n pairs (keys, vals) by the low key_bits bits of the key,
// keeping the input order among equal keys (LSD, 8 bits per pass).  The
// inputs are left unchanged; the sorted pairs go to keys_out / vals_out.
// key_bits in [1, 32]; n < 2^31.
stag_status radix_sort_pairs_u32(const uint32_t* keys, const uint32_t* vals, uint32_t* keys_out, uint32_t* vals_out,
                                 int64_t n, int key_bits, Workspace& ws, hipStream_t st);

}  // namespace stag
