// Stable LSD radix sort of (uint32 key, uint32 value) pairs, 8 bits per pass.
//
// One pass over digit shift s:
//   radix_hist     every workgroup counts the digits of its 4096 items into
//                  hist[digit * nblocks + block] (digit-major)
//   exclusive scan of hist: the destination of the first item with digit d in
//                  block b is offs[d * nblocks + b] (all smaller digits, then
//                  the same digit in earlier blocks)
//   radix_scatter  every workgroup walks its items in order, 256 at a time;
//                  within a wave the lanes holding the same digit are found
//                  with 8 ballots (one per digit bit) and ranked by lane; the
//                  per-wave counts of the round and the running per-digit
//                  counts of earlier rounds give each item its place.
// Items therefore keep their input order among equal digits, which makes
// every pass, and the whole sort, stable.
#include "sort.h"

#include "scan.h"

namespace stag {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                         // rounds per workgroup
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 items

__global__ __launch_bounds__(kSortThreads) void radix_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                           int64_t nblocks, uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter(const uint32_t* __restrict__ keys,
                                                              const uint32_t* __restrict__ vals, int64_t n, int shift,
                                                              int64_t nblocks, const uint64_t* __restrict__ offs,
                                                              uint32_t* __restrict__ keys_out,
                                                              uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t running[256];
  __shared__ uint32_t wcount[4][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  running[tid] = 0;
  for (int w = 0; w < 4; ++w) wcount[w][tid] = 0;
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + tid;
    const bool valid = i < n;
    const uint32_t key = valid ? keys[i] : 0u;
    const uint32_t val = valid ? vals[i] : 0u;
    const uint32_t digit = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (digit >> b) & 1u;
      const uint64_t ones = __ballot(bit);
      peers &= bit ? ones : ~ones;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    if (valid && rank == 0) wcount[wave][digit] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t before = running[digit];
      for (int w = 0; w < wave; ++w) before += wcount[w][digit];
      const uint64_t dst = offs[(int64_t)digit * nblocks + blockIdx.x] + before + rank;
      keys_out[dst] = key;
      vals_out[dst] = val;
    }
    __syncthreads();
    running[tid] += wcount[0][tid] + wcount[1][tid] + wcount[2][tid] + wcount[3][tid];
    for (int w = 0; w < 4; ++w) wcount[w][tid] = 0;
    __syncthreads();
  }
}

}  // namespace

stag_status radix_sort_pairs_u32(const uint32_t* keys, const uint32_t* vals, uint32_t* keys_out, uint32_t* vals_out,
                                 int64_t n, int key_bits, Workspace& ws, hipStream_t st) {
  if (n < 0 || n >= ((int64_t)1 << 31) || key_bits < 1 || key_bits > 32)
    return fail(STAG_E_INVAL, "radix_sort_pairs_u32: bad size");
  if (n == 0) return STAG_OK;
  const int passes = (key_bits + 7) / 8;
  const int64_t nblocks = ceil_div(n, kSortTile);
  uint32_t *hist = nullptr, *tk = nullptr, *tv = nullptr;
  uint64_t* offs = nullptr;
  STAG_TRY(ws.alloc(&hist, (size_t)256 * nblocks));
  STAG_TRY(ws.alloc(&offs, (size_t)256 * nblocks + 1));
  if (passes > 1) {
    STAG_TRY(ws.alloc(&tk, (size_t)n));
    STAG_TRY(ws.alloc(&tv, (size_t)n));
  }
  // ping-pong so that the last pass writes keys_out / vals_out
  const uint32_t* src_k = keys;
  const uint32_t* src_v = vals;
  ScopedTimer tm("radix_sort", st);
  for (int p = 0; p < passes; ++p) {
    const bool last = p == passes - 1;
    uint32_t* dk = ((passes - 1 - p) & 1) ? tk : keys_out;
    uint32_t* dv = ((passes - 1 - p) & 1) ? tv : vals_out;
    if (last) {
      dk = keys_out;
      dv = vals_out;
    }
    hipLaunchKernelGGL(radix_hist, dim3((unsigned)nblocks), dim3(kSortThreads), 0, st, src_k, n, 8 * p, nblocks, hist);
    STAG_TRY(check_launch("radix_hist"));
    STAG_TRY(exclusive_scan_u32(hist, offs, 256 * nblocks, ws, st));
    hipLaunchKernelGGL(radix_scatter, dim3((unsigned)nblocks), dim3(kSortThreads), 0, st, src_k, src_v, n, 8 * p,
                       nblocks, offs, dk, dv);
    STAG_TRY(check_launch("radix_scatter"));
    src_k = dk;
    src_v = dv;
  }
  return STAG_OK;
}

}  // namespace stag
