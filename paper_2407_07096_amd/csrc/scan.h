// Device-wide exclusive prefix sum of uint32 counts into uint64 offsets.
#pragma once

#include "runtime.h"

namespace stag {

// out[i] = sum_{k<i} in[k] for i in [0, n], so out[n] is the total.
stag_status exclusive_scan_u32(const uint32_t* in, uint64_t* out, int64_t n, Workspace& ws, hipStream_t st);

}  // namespace stag
