// Stream-ordered zero fill done by a kernel, for buffers that are cleared in
// code a caller may record into a HIP graph (memset nodes are avoided there).
#include "runtime.h"

namespace stag {
namespace {

__global__ void __launch_bounds__(256) zero_words(uint32_t* __restrict__ p, size_t words,
                                                  unsigned char* __restrict__ tail, int ntail) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < words; i += stride) p[i] = 0u;
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(256) zero_bytes(unsigned char* __restrict__ p, size_t bytes) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < bytes; i += stride) p[i] = 0;
}

}  // namespace

stag_status zero_async(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return STAG_OK;
  const size_t per = 256;
  if (((uintptr_t)p & 3u) == 0) {
    size_t words = bytes / 4;
    int ntail = (int)(bytes % 4);
    size_t blocks = (words + per - 1) / per;
    if (blocks < 1) blocks = 1;
    if (blocks > 2048) blocks = 2048;
    zero_words<<<(unsigned)blocks, (unsigned)per, 0, st>>>(static_cast<uint32_t*>(p), words,
                                                         static_cast<unsigned char*>(p) + words * 4,
                                                         ntail);
  } else {
    size_t blocks = (bytes + per - 1) / per;
    if (blocks > 2048) blocks = 2048;
    zero_bytes<<<(unsigned)blocks, (unsigned)per, 0, st>>>(static_cast<unsigned char*>(p), bytes);
  }
  return check_launch("zero_async");
}

}  // namespace stag
