// E2LSH codes and bucket keys (Sec. "Random Projection": h(x) =
// floor((<x, g> + b) / 4) with g ~ N(0, I_d), b ~ U[0,4); Sec. "Boosting the
// Probability": K functions concatenated per table, L tables).
//
// Bit-exact definition: <x, g> is the left-to-right binary64 sum over
// j = 0..d-1 of x_j * g_j.  With fp32 x and g each product is exact in
// binary64, so a fused multiply-add per coordinate rounds exactly like the
// separate add.  The bucket key of table l folds the K codes with the
// SplitMix64 finaliser.
//
// Kernel layout: one lane per point, so every lane runs its own sequential
// fp64 chain; the projections are wave-uniform and come from scalar loads of
// a regrouped binary64 copy G8[l][chunk][j][8] (8 projections of one table
// per 64-byte line), so one scalar load feeds 8 FMAs of every lane.  Points of
// dimension <= 64 sit in registers as binary64; larger ones are read from
// the (cached) row per coordinate.
#include "e2lsh.h"
#include "runtime.h"

namespace stag {

namespace {

// Regroup fp32 projections [L*K][d] (table-major) into binary64
// G8[l][c][j][e] = g[l*K + 8c + e][j] (zero for 8c+e >= K or j >= d).
__global__ void regroup_projections(const float* __restrict__ G, int K, int L, int d, int dg, int nch,
                                    double* __restrict__ G8) {
  const int64_t total = (int64_t)L * nch * dg * 8;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(idx & 7);
    const int64_t r = idx >> 3;
    const int j = (int)(r % dg);
    const int64_t lc = r / dg;
    const int c = (int)(lc % nch);
    const int l = (int)(lc / nch);
    const int k = 8 * c + e;
    double v = 0.0;
    if (k < K && j < d) v = (double)G[((int64_t)l * K + k) * d + j];
    G8[idx] = v;
  }
}

// One lane per point; wave w of block (bx, by) hashes tables
// [(by*4 + w)*tpw, +tpw) of points [bx*64, +64).
template <int DREG>
__global__ __launch_bounds__(256) void e2lsh_kernel(const float* __restrict__ X, int64_t n, int d, int dg,
                                                    const double* __restrict__ G8, const double* __restrict__ b,
                                                    int K, int L, int nch, int tpw, int32_t* __restrict__ codes,
                                                    uint64_t* __restrict__ keys) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool live = i < n;
  const int64_t irow = live ? i : 0;
  const float* xrow = X + irow * d;
  double xr[DREG > 0 ? DREG : 1];
  load_point<DREG>(xr, xrow, d);
  const int l0 = (blockIdx.y * 4 + wave) * tpw;
  for (int l = l0; l < l0 + tpw && l < L; ++l) {
    int32_t* crow = (codes && live) ? codes + (irow * L + l) * K : nullptr;
    const uint64_t hkey = table_key<DREG>(l, xr, xrow, d, dg, G8 + (int64_t)l * nch * dg * 8, b + (int64_t)l * K, K,
                                          nch, crow);
    if (keys && live) keys[irow * L + l] = hkey;
  }
}

}  // namespace

int e2lsh_reg_dim(int d) {
  if (d <= 16) return 16;
  if (d <= 32) return 32;
  if (d <= 64) return 64;
  return 0;
}

stag_status e2lsh_regroup(const float* G, int K, int L, int d, Workspace& ws, double** G8_out, int* dg_out,
                          hipStream_t st) {
  const int dreg = e2lsh_reg_dim(d);
  const int dg = dreg > 0 ? dreg : d;
  const int nch = (int)ceil_div(K, 8);
  double* G8 = nullptr;
  STAG_TRY(ws.alloc(&G8, (size_t)L * nch * dg * 8));
  const int64_t total = (int64_t)L * nch * dg * 8;
  const int blocks = (int)std::min<int64_t>(ceil_div(total, 256), 65536);
  ScopedTimer tm("e2lsh_regroup", st);
  hipLaunchKernelGGL(regroup_projections, dim3(blocks), dim3(256), 0, st, G, K, L, d, dg, nch, G8);
  STAG_TRY(check_launch("regroup_projections"));
  *G8_out = G8;
  *dg_out = dg;
  return STAG_OK;
}

stag_status e2lsh_launch(const float* X, int64_t n, int d, const double* G8, int dg, const double* b, int K, int L,
                         int32_t* codes, uint64_t* keys, hipStream_t st) {
  const int nch = (int)ceil_div(K, 8);
  const int64_t pblocks = ceil_div(n, 64);
  // spread tables over waves so that the grid has enough work
  int tpw = 1;
  while (tpw < L && (pblocks * ceil_div(L, 4 * tpw) > 65536 || ceil_div(L, 4 * tpw) > 65535)) tpw *= 2;
  const dim3 grid((unsigned)pblocks, (unsigned)ceil_div(L, 4 * tpw));
  const int dreg = e2lsh_reg_dim(d);
  ScopedTimer tm("e2lsh_hash", st);
  if ((dreg > 0 || d <= 128) && K <= 64) {
    // one lane per projection: blocks of 4 waves x TW tables, 8 batches of 64 points each
    // (64 < d <= 128: the lane's coefficients held as fp32)
    const int TW = 64 / K;
    const int qbatches = (int)std::max<int64_t>(8, ceil_div(n, (int64_t)64 * 65535));  // grid.y <= 65535
    const dim3 lgrid((unsigned)ceil_div(L, 4 * TW), (unsigned)ceil_div(n, (int64_t)64 * qbatches));
    switch (dreg) {
      case 16:
        hipLaunchKernelGGL((hash_lanes<16, false>), lgrid, dim3(256), 0, st, X, d, (int64_t)0, n, d, G8, dg, b, K, L,
                           nch, (int64_t)L, TW, qbatches, keys, codes);
        break;
      case 32:
        hipLaunchKernelGGL((hash_lanes<32, false>), lgrid, dim3(256), 0, st, X, d, (int64_t)0, n, d, G8, dg, b, K, L,
                           nch, (int64_t)L, TW, qbatches, keys, codes);
        break;
      case 64:
        hipLaunchKernelGGL((hash_lanes<64, false>), lgrid, dim3(256), 0, st, X, d, (int64_t)0, n, d, G8, dg, b, K, L,
                           nch, (int64_t)L, TW, qbatches, keys, codes);
        break;
      default:
        hipLaunchKernelGGL((hash_lanes<128, false, true>), lgrid, dim3(256), 0, st, X, d, (int64_t)0, n, d, G8, dg, b,
                           K, L, nch, (int64_t)L, TW, qbatches, keys, codes);
        break;
    }
    return check_launch("hash_lanes");
  }
  switch (dreg) {
    case 16:
      hipLaunchKernelGGL(e2lsh_kernel<16>, grid, dim3(256), 0, st, X, n, d, dg, G8, b, K, L, nch, tpw, codes, keys);
      break;
    case 32:
      hipLaunchKernelGGL(e2lsh_kernel<32>, grid, dim3(256), 0, st, X, n, d, dg, G8, b, K, L, nch, tpw, codes, keys);
      break;
    case 64:
      hipLaunchKernelGGL(e2lsh_kernel<64>, grid, dim3(256), 0, st, X, n, d, dg, G8, b, K, L, nch, tpw, codes, keys);
      break;
    default:
      hipLaunchKernelGGL(e2lsh_kernel<0>, grid, dim3(256), 0, st, X, n, d, dg, G8, b, K, L, nch, tpw, codes, keys);
      break;
  }
  return check_launch("e2lsh_kernel");
}

}  // namespace stag

extern "C" stag_status stag_e2lsh_hash(const float* X, int64_t n, int32_t d, const float* G, const double* b,
                                       int32_t K, int32_t L, int32_t* codes_out, uint64_t* keys_out,
                                       hipStream_t stream) {
  using namespace stag;
  if (!X || !G || !b) return fail(STAG_E_INVAL, "stag_e2lsh_hash: NULL input pointer");
  if (!codes_out && !keys_out) return fail(STAG_E_INVAL, "stag_e2lsh_hash: both outputs are NULL");
  if (n < 1 || d < 1 || d > 4096) return fail(STAG_E_INVAL, "stag_e2lsh_hash: need n >= 1 and 1 <= d <= 4096");
  if (K < 1 || K > 64 || L < 1 || (int64_t)K * L > (1 << 24))
    return fail(STAG_E_INVAL, "stag_e2lsh_hash: need 1 <= K <= 64, L >= 1, K*L <= 2^24");
  if ((double)n * d >= 2147483648.0 * 4.0) return fail(STAG_E_INVAL, "stag_e2lsh_hash: n*d too large");
  clear_error();
  Workspace ws(stream);
  double* G8 = nullptr;
  int dg = 0;
  STAG_TRY(e2lsh_regroup(G, K, L, d, ws, &G8, &dg, stream));
  return e2lsh_launch(X, n, d, G8, dg, b, K, L, codes_out, keys_out, stream);
}
