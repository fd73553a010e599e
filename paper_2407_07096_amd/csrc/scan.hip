// Exclusive prefix sum, three phases: per-block scan with block totals,
// recursive scan of the totals, add of the block offsets.
#include "scan.h"

namespace stag {
namespace {

constexpr int kScanBlock = 1024;  // elements per block (4 per thread)

__device__ inline uint64_t wave_incl_scan(uint64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  return v;
}

// Block-level exclusive scan of 1024 values (4 per thread); returns the
// block total through *total.
template <typename T>
__device__ inline void block_scan4(const T* vin, uint64_t* vout, uint64_t* total) {
  __shared__ uint64_t wsum[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t loc[4], run = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    loc[k] = run;
    run += (uint64_t)vin[k];
  }
  const uint64_t incl = wave_incl_scan(run);
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint64_t wbase = 0;
  for (int w = 0; w < wave; ++w) wbase += wsum[w];
  const uint64_t base = wbase + incl - run;
#pragma unroll
  for (int k = 0; k < 4; ++k) vout[k] = base + loc[k];
  *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

template <typename T>
__global__ __launch_bounds__(256) void scan_blocks(const T* __restrict__ in, int64_t n, uint64_t* __restrict__ out,
                                                   uint64_t* __restrict__ block_tot) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
  T v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = base + k < n ? in[base + k] : (T)0;
  uint64_t o[4], tot;
  block_scan4<T>(v, o, &tot);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (base + k < n) out[base + k] = o[k];
  if (threadIdx.x == 0) block_tot[blockIdx.x] = tot;
}

__global__ void add_offsets(uint64_t* __restrict__ out, int64_t n, const uint64_t* __restrict__ block_off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += block_off[i / kScanBlock];
}

// out[n] = the grand total (the last entry of the scanned block offsets, or
// the one block's total)
__global__ void write_total(uint64_t* __restrict__ out, int64_t n, const uint64_t* __restrict__ total) {
  out[n] = total[0];
}

template <typename T>
stag_status scan_impl(const T* in, uint64_t* out, int64_t n, Workspace& ws, hipStream_t st) {
  const int64_t nb = ceil_div(n, kScanBlock);
  uint64_t* tot = nullptr;
  STAG_TRY(ws.alloc(&tot, (size_t)nb));
  hipLaunchKernelGGL(scan_blocks<T>, dim3((unsigned)nb), dim3(256), 0, st, in, n, out, tot);
  STAG_TRY(check_launch("scan_blocks"));
  const uint64_t* total = tot;  // one block: its total is the grand total
  if (nb > 1) {
    uint64_t* off = nullptr;
    STAG_TRY(ws.alloc(&off, (size_t)nb + 1));
    STAG_TRY(scan_impl<uint64_t>(tot, off, nb, ws, st));
    hipLaunchKernelGGL(add_offsets, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, out, n, off);
    STAG_TRY(check_launch("add_offsets"));
    total = off + nb;
  }
  hipLaunchKernelGGL(write_total, dim3(1), dim3(1), 0, st, out, n, total);
  return check_launch("write_total");
}

}  // namespace

stag_status exclusive_scan_u32(const uint32_t* in, uint64_t* out, int64_t n, Workspace& ws, hipStream_t st) {
  return scan_impl<uint32_t>(in, out, n, ws, st);
}

}  // namespace stag
