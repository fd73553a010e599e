// Spectral clustering of a weighted graph (Sec. "Fast Spectral Clustering":
// similarity graph -> bottom k eigenvectors of the Laplacian -> k-means on
// the embedded vertices).
//
// Graph.  The edge list (src, dst, w) is read as the symmetric adjacency A
// (every edge adds w at (src, dst) and at (dst, src); dst = -1 marks an empty
// draw).  Its 2E entries are keyed by row and put in row order by a stable
// radix sort, so each CSR row lists its entries in edge order and every row
// sum below is taken in a fixed order.  The Laplacian is the normalised
// N = I - D^{-1/2} A D^{-1/2}; the CSR values become the entries of
// M = D^{-1/2} A D^{-1/2} (spectrum in [-1, 1]), whose top eigenvectors are
// N's bottom ones (eigenvalue lambda = 1 - theta).
//
// Eigenvectors: Chebyshev-filtered subspace iteration (Zhou & Saad 2007) on
// a block of b = 8..64 columns (n x b, fp64, row-major, padded to a power of
// two bp):
//   filter     Y <- T_p((M - sigma) / e) V, the Chebyshev polynomial of
//              degree p that is bounded by 1 on the unwanted interval
//              [-1, c] (c = the block's smallest Ritz value) and grows fast
//              above it; three-term recurrence, one fused SpMM per degree
//   orthonormalise twice by Cholesky QR (Gram matrix V^T V = R^T R on the
//              host, V <- V R^{-1}; by its eigen-decomposition, V <- V Q L^{-1/2},
//              if a pivot fails)
//   Rayleigh-Ritz  W = M V, H = V^T W, H = Z diag(theta) Z^T on the host,
//              V <- V Z, W <- W Z (theta descending)
//   stop       when the k leading residuals ||W_j - theta_j V_j|| <= tol.
// Only b x b matrices cross to the host (cyclic Jacobi there); every n-sized
// operation is a kernel below, every reduction in a fixed order, so results
// are bitwise reproducible.
//
// k-means: Lloyd's iteration with k-means++ seeding, the decisions taken in
// the stated order (squared distances summed over coordinates in order
// without fused operations, seeding sums in blocks of 1024 points, ties to
// the lowest index; see include/stag_kde.h).
#include <algorithm>
#include <cmath>
#include <vector>

#include "runtime.h"
#include "scan.h"
#include "sort.h"

namespace stag {
namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kTagSpectral = 0x53504543ull;  // "SPEC": initial block
constexpr uint64_t kTagKmeans = 0x4B4D4E53ull;    // "KMNS": k-means++ uniforms
constexpr int kKmBlock = 1024;                    // points per seeding/update block
constexpr int kMaxBlockCols = 64;
constexpr int kGramRows = 256;                    // rows per Gram workgroup

__host__ __device__ inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Output c of the counter stream (seed, tag): mix(state + (c+1) gamma),
// state = mix(mix(mix(seed ^ tag) ^ 0) ^ 0).
__host__ __device__ inline uint64_t stream_bits(uint64_t seed, uint64_t tag, uint64_t c) {
  const uint64_t s = sm_mix(sm_mix(sm_mix(seed ^ tag)));
  return sm_mix(s + (c + 1) * kGamma);
}

// ---------------------------------------------------------------------------
// Graph build
// ---------------------------------------------------------------------------
// Entry 2e is (row src, column dst), entry 2e+1 (row dst, column src); an
// empty draw gets the key n on both (sorted past every row).  Invalid edges
// raise *bad.
__global__ void edge_entries(const int64_t* __restrict__ src, const int64_t* __restrict__ dst,
                             const double* __restrict__ w, int64_t E, int64_t n, uint32_t* __restrict__ keys,
                             uint32_t* __restrict__ vals, uint32_t* __restrict__ rowcnt, int* __restrict__ bad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int64_t s = src[e], t = dst[e];
  uint32_t k0 = (uint32_t)n, k1 = (uint32_t)n;
  const bool s_ok = s >= 0 && s < n;
  if (t == -1) {
    if (!s_ok) atomicOr(bad, 1);
  } else {
    const double we = w[e];
    if (!s_ok || t < 0 || t >= n || !(we >= 0.0) || !(we < INFINITY)) {
      atomicOr(bad, 1);
    } else {
      k0 = (uint32_t)s;
      k1 = (uint32_t)t;
      atomicAdd(&rowcnt[s], 1u);
      atomicAdd(&rowcnt[t], 1u);
    }
  }
  keys[2 * e] = k0;
  vals[2 * e] = (uint32_t)(2 * e);
  keys[2 * e + 1] = k1;
  vals[2 * e + 1] = (uint32_t)(2 * e + 1);
}

__global__ void csr_fill(const uint32_t* __restrict__ sorted_vals, const uint64_t* __restrict__ rowptr, int64_t n,
                         int64_t cap, const int64_t* __restrict__ src, const int64_t* __restrict__ dst,
                         const double* __restrict__ w, int32_t* __restrict__ col, double* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap || i >= (int64_t)rowptr[n]) return;
  const uint32_t v = sorted_vals[i];
  const int64_t e = v >> 1;
  col[i] = (int32_t)((v & 1u) ? src[e] : dst[e]);
  val[i] = w[e];
}

// deg(r) = row sum in CSR order; dinv = deg^{-1/2} (0 for an isolated vertex).
__global__ void row_dinv(const uint64_t* __restrict__ rowptr, const double* __restrict__ val, int64_t n,
                         double* __restrict__ deg, double* __restrict__ dinv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double s = 0.0;
  for (uint64_t i = rowptr[r]; i < rowptr[r + 1]; ++i) s += val[i];
  deg[r] = s;
  dinv[r] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
}

__global__ void normalise_vals(const uint64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                               const double* __restrict__ dinv, int64_t n, double* __restrict__ val) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double dr = dinv[r];
  for (uint64_t i = rowptr[r]; i < rowptr[r + 1]; ++i) val[i] = dr * val[i] * dinv[col[i]];
}

// ---------------------------------------------------------------------------
// Block operations (X [n][bp] fp64 row-major, the first b columns in use)
// ---------------------------------------------------------------------------
// Y = alpha (M X) + beta X + gamma Z; LPR lanes per row, two columns per lane.
template <int LPR>
__global__ __launch_bounds__(256) void spmm_comb(const uint64_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col, const double* __restrict__ val,
                                                 int64_t n, const double2* __restrict__ X,
                                                 const double2* __restrict__ Z, double2* __restrict__ Y, double alpha,
                                                 double beta, double gamma) {
  constexpr int RPB = 256 / LPR;
  const int64_t r = (int64_t)blockIdx.x * RPB + threadIdx.x / LPR;
  const int c = threadIdx.x % LPR;
  if (r >= n) return;
  double ax = 0.0, ay = 0.0;
  const uint64_t e1 = rowptr[r + 1];
  for (uint64_t i = rowptr[r]; i < e1; ++i) {
    const double v = val[i];
    const double2 x = X[(int64_t)col[i] * LPR + c];
    ax = fma(v, x.x, ax);
    ay = fma(v, x.y, ay);
  }
  const double2 xr = X[r * LPR + c];
  double yx = alpha * ax + beta * xr.x;
  double yy = alpha * ay + beta * xr.y;
  if (Z) {
    const double2 z = Z[r * LPR + c];
    yx += gamma * z.x;
    yy += gamma * z.y;
  }
  Y[r * LPR + c] = make_double2(yx, yy);
}

// Partial Gram matrices A^T B over kGramRows rows per workgroup, rows in
// order; part [nblk][b][b].
__global__ __launch_bounds__(256) void gram_partial(const double* __restrict__ A, const double* __restrict__ B,
                                                    int64_t n, int bp, int b, double* __restrict__ part) {
  __shared__ double sa[32 * kMaxBlockCols];
  __shared__ double sb[32 * kMaxBlockCols];
  const int tid = threadIdx.x;
  const int bb = b * b;
  const int64_t r0 = (int64_t)blockIdx.x * kGramRows;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int rr = 0; rr < kGramRows; rr += 32) {
    for (int v = tid; v < 32 * bp; v += 256) {
      const int64_t row = r0 + rr + v / bp;
      const int cc = v % bp;
      sa[(v / bp) * kMaxBlockCols + cc] = row < n ? A[row * bp + cc] : 0.0;
      sb[(v / bp) * kMaxBlockCols + cc] = row < n ? B[row * bp + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q;
      if (e < bb) {
        const int i = e / b, j = e % b;
        double s = acc[q];
        for (int t = 0; t < 32; ++t) s = fma(sa[t * kMaxBlockCols + i], sb[t * kMaxBlockCols + j], s);
        acc[q] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q;
    if (e < bb) part[(int64_t)blockIdx.x * bb + e] = acc[q];
  }
}

// Sum of v[k * stride] over k < count in order; the loads are issued eight at
// a time so that they overlap, the additions stay sequential.
__device__ inline double ordered_sum(const double* __restrict__ v, int64_t count, int64_t stride) {
  double s = 0.0;
  int64_t k = 0;
  for (; k + 8 <= count; k += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = v[(k + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += t[u];
  }
  for (; k < count; ++k) s += v[k * stride];
  return s;
}

__global__ void gram_final(const double* __restrict__ part, int64_t nblk, int bb, double* __restrict__ G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= bb) return;
  G[e] = ordered_sum(part + e, nblk, bb);
}

// Y[:, :b] = X[:, :b] R (R b x b row-major), Y[:, b:bp] = 0.
__global__ __launch_bounds__(256) void apply_small(const double* __restrict__ X, int64_t n, int bp, int b,
                                                   const double* __restrict__ R, double* __restrict__ Y) {
  __shared__ double sR[kMaxBlockCols * kMaxBlockCols];
  __shared__ double sx[256];
  const int tid = threadIdx.x;
  for (int v = tid; v < b * b; v += 256) sR[v] = R[v];
  const int rpb = 256 / bp;
  const int64_t row = (int64_t)blockIdx.x * rpb + tid / bp;
  const int j = tid % bp;
  sx[tid] = row < n ? X[row * bp + j] : 0.0;
  __syncthreads();
  if (row >= n) return;
  double y = 0.0;
  if (j < b) {
    const double* xr = &sx[(tid / bp) * bp];
    for (int i = 0; i < b; ++i) y = fma(xr[i], sR[i * b + j], y);
  }
  Y[row * bp + j] = y;
}

// R = W - V diag(theta) on the first b columns.
__global__ void residual_block(const double* __restrict__ W, const double* __restrict__ V,
                               const double* __restrict__ theta, int64_t n, int bp, int b, double* __restrict__ R) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * bp) return;
  const int j = (int)(i % bp);
  R[i] = j < b ? W[i] - theta[j] * V[i] : 0.0;
}

__global__ void init_block(double* __restrict__ V, int64_t n, int bp, int b, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * bp) return;
  const int j = (int)(i % bp);
  const int64_t r = i / bp;
  double v = 0.0;
  if (j < b) v = (double)(stream_bits(seed, kTagSpectral, (uint64_t)(r * b + j)) >> 11) * 0x1.0p-52 - 1.0;
  V[i] = v;
}

// Column j < k: the entry of largest magnitude (lowest row on ties) per
// workgroup of 256 rows, then over workgroups in order.
__global__ __launch_bounds__(256) void col_absmax_partial(const double* __restrict__ V, int64_t n, int bp, int k,
                                                          double* __restrict__ pv, int64_t* __restrict__ pi) {
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    double best = -1.0;
    int64_t bi = -1;
    for (int64_t r = r0; r < min(n, r0 + 256); ++r) {
      const double a = fabs(V[r * bp + j]);
      if (a > best) {
        best = a;
        bi = r;
      }
    }
    pv[(int64_t)blockIdx.x * k + j] = best;
    pi[(int64_t)blockIdx.x * k + j] = bi;
  }
}

__global__ void col_sign(const double* __restrict__ pv, const int64_t* __restrict__ pi, int64_t nblk,
                         const double* __restrict__ V, int bp, int k, double* __restrict__ sign) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double best = -1.0;
  int64_t bi = 0;
  for (int64_t g = 0; g < nblk; ++g) {
    if (pv[g * k + j] > best) {
      best = pv[g * k + j];
      bi = pi[g * k + j];
    }
  }
  sign[j] = V[bi * bp + j] < 0.0 ? -1.0 : 1.0;
}

__global__ void extract_embedding(const double* __restrict__ V, int64_t n, int bp, int k,
                                  const double* __restrict__ sign, double* __restrict__ U) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * k) return;
  const int64_t r = i / k;
  const int j = (int)(i % k);
  U[i] = sign[j] * V[r * bp + j];
}

__global__ void eig_out(const double* __restrict__ theta, int k, double* __restrict__ lam) {
  const int j = threadIdx.x;
  if (j < k) lam[j] = 1.0 - theta[j];
}

// ---------------------------------------------------------------------------
// Host dense helpers (b <= 64)
// ---------------------------------------------------------------------------
// Cyclic Jacobi eigen-decomposition of the symmetric b x b matrix A
// (row-major); eigenvalues descending in w, eigenvectors as the columns of Z.
void jacobi_eigen(std::vector<double> A, int b, std::vector<double>& w, std::vector<double>& Z) {
  Z.assign((size_t)b * b, 0.0);
  for (int i = 0; i < b; ++i) Z[(size_t)i * b + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < b; ++i)
      for (int j = 0; j < b; ++j) {
        const double v = A[(size_t)i * b + j] * A[(size_t)i * b + j];
        tot += v;
        if (i != j) off += v;
      }
    // relative off-diagonal size 1e-14: below it further sweeps only trade
    // rounding noise
    if (off <= 1e-28 * tot || off == 0.0) break;
    for (int p = 0; p < b - 1; ++p)
      for (int q = p + 1; q < b; ++q) {
        const double apq = A[(size_t)p * b + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * b + p], aqq = A[(size_t)q * b + q];
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int r = 0; r < b; ++r) {  // A <- A J (columns p, q)
          const double arp = A[(size_t)r * b + p], arq = A[(size_t)r * b + q];
          A[(size_t)r * b + p] = c * arp - s * arq;
          A[(size_t)r * b + q] = s * arp + c * arq;
        }
        for (int r = 0; r < b; ++r) {  // A <- J^T A (rows p, q)
          const double apr = A[(size_t)p * b + r], aqr = A[(size_t)q * b + r];
          A[(size_t)p * b + r] = c * apr - s * aqr;
          A[(size_t)q * b + r] = s * apr + c * aqr;
        }
        A[(size_t)p * b + q] = A[(size_t)q * b + p] = 0.0;  // zero by construction of the rotation
        for (int r = 0; r < b; ++r) {
          const double zrp = Z[(size_t)r * b + p], zrq = Z[(size_t)r * b + q];
          Z[(size_t)r * b + p] = c * zrp - s * zrq;
          Z[(size_t)r * b + q] = s * zrp + c * zrq;
        }
      }
  }
  std::vector<int> ord((size_t)b);
  for (int i = 0; i < b; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int x, int y) { return A[(size_t)x * b + x] > A[(size_t)y * b + y]; });
  w.resize((size_t)b);
  std::vector<double> Zs((size_t)b * b);
  for (int c = 0; c < b; ++c) {
    w[c] = A[(size_t)ord[c] * b + ord[c]];
    for (int r = 0; r < b; ++r) Zs[(size_t)r * b + c] = Z[(size_t)r * b + ord[c]];
  }
  Z.swap(Zs);
}

// Upper-triangular R with G = R^T R (b x b, row-major), returned as R^{-1};
// false if a pivot is not positive (then the caller orthonormalises by the
// eigen-decomposition instead).
bool cholesky_inverse(const std::vector<double>& G, int b, std::vector<double>& Rinv) {
  std::vector<double> R((size_t)b * b, 0.0);
  for (int j = 0; j < b; ++j) {
    double dj = G[(size_t)j * b + j];
    for (int k = 0; k < j; ++k) dj -= R[(size_t)k * b + j] * R[(size_t)k * b + j];
    if (!(dj > 0.0) || !std::isfinite(dj)) return false;
    const double rjj = std::sqrt(dj);
    R[(size_t)j * b + j] = rjj;
    for (int i = j + 1; i < b; ++i) {
      double v = G[(size_t)j * b + i];
      for (int k = 0; k < j; ++k) v -= R[(size_t)k * b + j] * R[(size_t)k * b + i];
      R[(size_t)j * b + i] = v / rjj;
    }
  }
  // back substitution, column by column: R X = I
  Rinv.assign((size_t)b * b, 0.0);
  for (int c = 0; c < b; ++c)
    for (int i = c; i >= 0; --i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = i + 1; k <= c; ++k) v -= R[(size_t)i * b + k] * Rinv[(size_t)k * b + c];
      Rinv[(size_t)i * b + c] = v / R[(size_t)i * b + i];
    }
  return true;
}

// ---------------------------------------------------------------------------
// Subspace iteration driver
// ---------------------------------------------------------------------------
struct Csr {
  int64_t n = 0;
  uint64_t* rowptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
};

stag_status build_normalised(int64_t n, const int64_t* src, const int64_t* dst, const double* w, int64_t E,
                             Workspace& ws, Csr* g, hipStream_t st) {
  const int64_t ne = 2 * E;
  uint32_t *keys = nullptr, *vals = nullptr, *sk = nullptr, *sv = nullptr, *rowcnt = nullptr;
  int* bad = nullptr;
  STAG_TRY(ws.alloc(&keys, (size_t)std::max<int64_t>(ne, 1)));
  STAG_TRY(ws.alloc(&vals, (size_t)std::max<int64_t>(ne, 1)));
  STAG_TRY(ws.alloc(&sk, (size_t)std::max<int64_t>(ne, 1)));
  STAG_TRY(ws.alloc(&sv, (size_t)std::max<int64_t>(ne, 1)));
  STAG_TRY(ws.alloc(&rowcnt, (size_t)n));
  STAG_TRY(ws.alloc(&bad, 1));
  STAG_TRY(ws.alloc(&g->rowptr, (size_t)n + 1));
  STAG_TRY(ws.alloc(&g->col, (size_t)std::max<int64_t>(ne, 1)));
  STAG_TRY(ws.alloc(&g->val, (size_t)std::max<int64_t>(ne, 1)));
  double *deg = nullptr, *dinv = nullptr;
  STAG_TRY(ws.alloc(&deg, (size_t)n));
  STAG_TRY(ws.alloc(&dinv, (size_t)n));
  g->n = n;
  STAG_HIP(hipMemsetAsync(rowcnt, 0, sizeof(uint32_t) * (size_t)n, st));
  STAG_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
  ScopedTimer tm("graph_build", st);
  if (E > 0) {
    hipLaunchKernelGGL(edge_entries, dim3((unsigned)ceil_div(E, 256)), dim3(256), 0, st, src, dst, w, E, n, keys,
                       vals, rowcnt, bad);
    STAG_TRY(check_launch("edge_entries"));
  }
  int hbad = 0;
  STAG_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  STAG_HIP(hipStreamSynchronize(st));
  if (hbad)
    return fail(STAG_E_INVAL, "graph: an edge has src or dst outside [0, n) (dst = -1 aside) or a negative or "
                              "non-finite weight");
  int key_bits = 1;
  while (key_bits < 32 && ((uint64_t)n >> key_bits) != 0) ++key_bits;
  if (ne > 0) STAG_TRY(radix_sort_pairs_u32(keys, vals, sk, sv, ne, key_bits, ws, st));
  STAG_TRY(exclusive_scan_u32(rowcnt, g->rowptr, n, ws, st));
  if (ne > 0) {
    hipLaunchKernelGGL(csr_fill, dim3((unsigned)ceil_div(ne, 256)), dim3(256), 0, st, sv, g->rowptr, n, ne, src, dst,
                       w, g->col, g->val);
    STAG_TRY(check_launch("csr_fill"));
  }
  hipLaunchKernelGGL(row_dinv, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, g->rowptr, g->val, n, deg, dinv);
  STAG_TRY(check_launch("row_dinv"));
  hipLaunchKernelGGL(normalise_vals, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, g->rowptr, g->col, dinv, n,
                     g->val);
  return check_launch("normalise_vals");
}

class Subspace {
 public:
  Subspace(const Csr& g, int bp, int b, Workspace& ws, hipStream_t st) : g_(g), bp_(bp), b_(b), ws_(ws), st_(st) {}
  ~Subspace() {
    if (pinned_) {
      (void)hipStreamSynchronize(st_);
      (void)hipHostFree(pinned_);
    }
  }
  Subspace(const Subspace&) = delete;
  Subspace& operator=(const Subspace&) = delete;

  stag_status init() {
    // staging of the b x b uploads (matrix, Ritz values); the host rewrites
    // it only after a Gram read-back has synchronised the stream
    STAG_HIP(hipHostMalloc(reinterpret_cast<void**>(&pinned_), sizeof(double) * (kMaxBlockCols * kMaxBlockCols + kMaxBlockCols)));
    const size_t nb = (size_t)g_.n * bp_;
    for (double** p : {&V_, &W_, &Y0_, &Y1_, &T_}) STAG_TRY(ws_.alloc(p, nb));
    nblk_ = ceil_div(g_.n, kGramRows);
    STAG_TRY(ws_.alloc(&part_, (size_t)nblk_ * b_ * b_));
    STAG_TRY(ws_.alloc(&G_, (size_t)b_ * b_));
    STAG_TRY(ws_.alloc(&R_, (size_t)b_ * b_));
    STAG_TRY(ws_.alloc(&theta_, (size_t)kMaxBlockCols));
    return STAG_OK;
  }

  // Y = alpha M X + beta X + gamma Z
  stag_status spmm(const double* X, const double* Z, double* Y, double alpha, double beta, double gamma) {
    ScopedTimer tm("spectral_spmm", st_);
    const int lpr = bp_ / 2;
    const int64_t grid = ceil_div(g_.n, 256 / lpr);
    auto X2 = reinterpret_cast<const double2*>(X);
    auto Z2 = reinterpret_cast<const double2*>(Z);
    auto Y2 = reinterpret_cast<double2*>(Y);
    switch (lpr) {
      case 4:
        hipLaunchKernelGGL(spmm_comb<4>, dim3((unsigned)grid), dim3(256), 0, st_, g_.rowptr, g_.col, g_.val, g_.n, X2,
                           Z2, Y2, alpha, beta, gamma);
        break;
      case 8:
        hipLaunchKernelGGL(spmm_comb<8>, dim3((unsigned)grid), dim3(256), 0, st_, g_.rowptr, g_.col, g_.val, g_.n, X2,
                           Z2, Y2, alpha, beta, gamma);
        break;
      case 16:
        hipLaunchKernelGGL(spmm_comb<16>, dim3((unsigned)grid), dim3(256), 0, st_, g_.rowptr, g_.col, g_.val, g_.n, X2,
                           Z2, Y2, alpha, beta, gamma);
        break;
      default:
        hipLaunchKernelGGL(spmm_comb<32>, dim3((unsigned)grid), dim3(256), 0, st_, g_.rowptr, g_.col, g_.val, g_.n, X2,
                           Z2, Y2, alpha, beta, gamma);
    }
    return check_launch("spmm_comb");
  }

  // host <- A^T B (b x b)
  stag_status gram(const double* A, const double* B, std::vector<double>& out) {
    {
      ScopedTimer tm("spectral_gram", st_);
      hipLaunchKernelGGL(gram_partial, dim3((unsigned)nblk_), dim3(256), 0, st_, A, B, g_.n, bp_, b_, part_);
      STAG_TRY(check_launch("gram_partial"));
      hipLaunchKernelGGL(gram_final, dim3((unsigned)ceil_div(b_ * b_, 256)), dim3(256), 0, st_, part_, nblk_, b_ * b_,
                         G_);
      STAG_TRY(check_launch("gram_final"));
    }
    out.resize((size_t)b_ * b_);
    STAG_HIP(hipMemcpyAsync(out.data(), G_, sizeof(double) * out.size(), hipMemcpyDeviceToHost, st_));
    STAG_HIP(hipStreamSynchronize(st_));
    return STAG_OK;
  }

  // device R <- host R (b x b), through the pinned staging buffer
  stag_status upload(const std::vector<double>& R) {
    std::copy(R.begin(), R.end(), pinned_);
    STAG_HIP(hipMemcpyAsync(R_, pinned_, sizeof(double) * R.size(), hipMemcpyHostToDevice, st_));
    return STAG_OK;
  }

  // Y = X R with the uploaded R
  stag_status apply(const double* X, double* Y) {
    ScopedTimer tm("spectral_apply", st_);
    hipLaunchKernelGGL(apply_small, dim3((unsigned)ceil_div(g_.n, 256 / bp_)), dim3(256), 0, st_, X, g_.n, bp_, b_,
                       R_, Y);
    return check_launch("apply_small");
  }

  // Twice: V <- V R^{-1} from the Cholesky factor of V^T V (Cholesky QR), or,
  // if that breaks down, V <- V Q L^{-1/2} from its eigen-decomposition.
  stag_status orthonormalise() {
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<double> G, R;
      STAG_TRY(gram(V_, V_, G));
      if (!cholesky_inverse(G, b_, R)) {
        std::vector<double> lam, Q;
        jacobi_eigen(G, b_, lam, Q);
        const double floor_ = std::max(lam[0], 1e-300) * 1e-30;
        R.assign((size_t)b_ * b_, 0.0);
        for (int c = 0; c < b_; ++c) {
          const double sc = 1.0 / std::sqrt(std::max(lam[c], floor_));
          for (int r = 0; r < b_; ++r) R[(size_t)r * b_ + c] = Q[(size_t)r * b_ + c] * sc;
        }
      }
      STAG_TRY(upload(R));
      STAG_TRY(apply(V_, T_));
      std::swap(V_, T_);
    }
    return STAG_OK;
  }

  // W = M V, H = V^T W = Z theta Z^T, V <- V Z, W <- W Z.
  stag_status rayleigh_ritz() {
    STAG_TRY(spmm(V_, nullptr, W_, 1.0, 0.0, 0.0));
    std::vector<double> H, Z;
    STAG_TRY(gram(V_, W_, H));
    for (int i = 0; i < b_; ++i)  // symmetrise the rounding
      for (int j = i + 1; j < b_; ++j) {
        const double m = 0.5 * (H[(size_t)i * b_ + j] + H[(size_t)j * b_ + i]);
        H[(size_t)i * b_ + j] = H[(size_t)j * b_ + i] = m;
      }
    jacobi_eigen(H, b_, theta_h_, Z);
    STAG_TRY(upload(Z));
    STAG_TRY(apply(V_, T_));
    std::swap(V_, T_);
    STAG_TRY(apply(W_, T_));
    std::swap(W_, T_);
    double* th = pinned_ + kMaxBlockCols * kMaxBlockCols;
    std::copy(theta_h_.begin(), theta_h_.end(), th);
    STAG_HIP(hipMemcpyAsync(theta_, th, sizeof(double) * b_, hipMemcpyHostToDevice, st_));
    return STAG_OK;
  }

  // Largest residual norm over the first k Ritz pairs.
  stag_status max_residual(int k, double* out) {
    hipLaunchKernelGGL(residual_block, dim3((unsigned)ceil_div(g_.n * bp_, 256)), dim3(256), 0, st_, W_, V_, theta_,
                       g_.n, bp_, b_, T_);
    STAG_TRY(check_launch("residual_block"));
    std::vector<double> G;
    STAG_TRY(gram(T_, T_, G));
    double m = 0.0;
    for (int j = 0; j < k; ++j) m = std::max(m, std::sqrt(std::max(G[(size_t)j * b_ + j], 0.0)));
    *out = m;
    return STAG_OK;
  }

  // V <- T_p((M - c)/e) V by the three-term recurrence
  //   Y_0 = V, Y_1 = (M - c) V / e, Y_{j+1} = 2 (M - c) Y_j / e - Y_{j-1},
  // rotating three buffers (V_, Y1_, Y0_); the result becomes V_.
  stag_status filter(int p, double lo, double hi) {
    const double e = 0.5 * (hi - lo), c = 0.5 * (hi + lo);
    double* buf[3] = {V_, Y1_, Y0_};  // Y_{j-1}, Y_j, spare
    STAG_TRY(spmm(buf[0], nullptr, buf[1], 1.0 / e, -c / e, 0.0));
    for (int j = 2; j <= p; ++j) {
      STAG_TRY(spmm(buf[1], buf[0], buf[2], 2.0 / e, -2.0 * c / e, -1.0));
      double* t = buf[0];
      buf[0] = buf[1];
      buf[1] = buf[2];
      buf[2] = t;
    }
    V_ = buf[1];
    Y1_ = buf[0];
    Y0_ = buf[2];
    return STAG_OK;
  }

  stag_status run(int k, double tol, int max_iter, uint64_t seed, int* iters) {
    hipLaunchKernelGGL(init_block, dim3((unsigned)ceil_div(g_.n * bp_, 256)), dim3(256), 0, st_, V_, g_.n, bp_, b_,
                       seed);
    STAG_TRY(check_launch("init_block"));
    STAG_TRY(orthonormalise());
    STAG_TRY(rayleigh_ritz());
    int it = 0;
    for (;;) {
      double res = 0.0;
      STAG_TRY(max_residual(k, &res));
      if (res <= tol || it >= max_iter) break;
      ++it;
      const double cut = std::min(theta_h_[b_ - 1], 1.0 - 1e-12);
      const double lo = -1.0;
      const double e = 0.5 * (cut - lo), c = 0.5 * (cut + lo);
      const double xt = (1.0 - c) / e;  // image of the spectrum's top
      int p = 30;
      if (xt > 1.0) p = (int)std::floor(std::acosh(1e6) / std::acosh(xt));
      p = std::max(2, std::min(30, p));
      STAG_TRY(filter(p, lo, cut));
      STAG_TRY(orthonormalise());
      STAG_TRY(rayleigh_ritz());
    }
    *iters = it;
    return STAG_OK;
  }

  const double* V() const { return V_; }
  const double* theta() const { return theta_; }

 private:
  const Csr& g_;
  int bp_, b_;
  Workspace& ws_;
  hipStream_t st_;
  int64_t nblk_ = 0;
  double *V_ = nullptr, *W_ = nullptr, *Y0_ = nullptr, *Y1_ = nullptr, *T_ = nullptr;
  double *part_ = nullptr, *G_ = nullptr, *R_ = nullptr, *theta_ = nullptr;
  double* pinned_ = nullptr;
  std::vector<double> theta_h_;
};

// ---------------------------------------------------------------------------
// k-means kernels (fp64; distances and sums without fused operations)
// ---------------------------------------------------------------------------
__device__ inline double dist2_rn(const double* p, const double* c, int dim) {
  double s = 0.0;
  for (int j = 0; j < dim; ++j) {
    const double t = __dsub_rn(p[j], c[j]);
    s = __dadd_rn(s, __dmul_rn(t, t));
  }
  return s;
}

// D2[i] = min(D2[i], dist2(P_i, centre)); first = 1 initialises D2.
__global__ void km_d2_update(const double* __restrict__ P, int64_t n, int dim, const double* __restrict__ centre,
                             int first, double* __restrict__ D2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = dist2_rn(P + i * dim, centre, dim);
  D2[i] = first ? d : fmin(D2[i], d);
}

// S[b] = sequential sum of D2 over block b (one workgroup per block: the
// values are staged in LDS with coalesced loads, then added in order).
__global__ __launch_bounds__(256) void km_block_sums(const double* __restrict__ D2, int64_t n,
                                                     double* __restrict__ S) {
  __shared__ double v[kKmBlock];
  const int64_t b = blockIdx.x;
  const int64_t base = b * kKmBlock;
  const int cnt = (int)min((int64_t)kKmBlock, n - base);
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) v[i] = D2[base + i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < cnt; ++i) s = __dadd_rn(s, v[i]);
  S[b] = s;
}

// One thread: picks centre c (c == 0: uniform; else D^2 sampling in the
// blocked order, with the documented fallbacks) and copies its row to C.
__global__ void km_pick(const double* __restrict__ P, int64_t n, int dim, const double* __restrict__ D2,
                        const double* __restrict__ S, int64_t nb, uint64_t seed, int c, unsigned char* chosen,
                        double* __restrict__ C, int64_t* __restrict__ seeds) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint64_t u = stream_bits(seed, kTagKmeans, (uint64_t)c) >> 11;
  int64_t pick = -1;
  if (c == 0) {
    const uint64_t hi = __umul64hi(u, (uint64_t)n), lo = u * (uint64_t)n;
    pick = (int64_t)((hi << 11) | (lo >> 53));
  } else {
    double T = 0.0;
    for (int64_t b = 0; b < nb; ++b) T = __dadd_rn(T, S[b]);
    if (T > 0.0) {
      const double t = __dmul_rn((double)u * 0x1.0p-53, T);
      double B = 0.0;
      for (int64_t b = 0; b < nb && pick < 0; ++b) {
        const double B1 = __dadd_rn(B, S[b]);
        if (B1 > t) {
          double cum = 0.0;
          const int64_t e = min(n, (b + 1) * (int64_t)kKmBlock);
          for (int64_t i = b * kKmBlock; i < e; ++i) {
            cum = __dadd_rn(cum, D2[i]);
            if (__dadd_rn(B, cum) > t) {
              pick = i;
              break;
            }
          }
        }
        B = B1;
      }
      for (int64_t i = n - 1; i >= 0 && pick < 0; --i)
        if (D2[i] > 0.0) pick = i;
    } else {
      for (int64_t i = 0; i < n && pick < 0; ++i)
        if (!chosen[i]) pick = i;
    }
  }
  if (pick < 0) pick = 0;  // unreachable for finite inputs
  chosen[pick] = 1;
  if (seeds) seeds[c] = pick;
  for (int j = 0; j < dim; ++j) C[(int64_t)c * dim + j] = P[pick * dim + j];
}

// label = argmin over centres (ties to the lowest); *changed |= any change.
__global__ __launch_bounds__(256) void km_assign(const double* __restrict__ P, int64_t n, int dim,
                                                 const double* __restrict__ C, int k, int32_t* __restrict__ labels,
                                                 int* __restrict__ changed) {
  extern __shared__ double sC[];
  for (int v = threadIdx.x; v < k * dim; v += blockDim.x) sC[v] = C[v];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* p = P + i * dim;
  int best = 0;
  double bd = dist2_rn(p, sC, dim);
  for (int c = 1; c < k; ++c) {
    const double dc = dist2_rn(p, sC + c * dim, dim);
    if (dc < bd) {
      bd = dc;
      best = c;
    }
  }
  if (labels[i] != best) {
    labels[i] = best;
    atomicOr(changed, 1);
  }
}

// Per block of 1024 points: coordinate sums per cluster, points in order
// (lane j owns coordinate j of every cluster), and counts.
__global__ __launch_bounds__(64) void km_block_accum(const double* __restrict__ P, const int32_t* __restrict__ labels,
                                                     int64_t n, int dim, int k, double* __restrict__ part,
                                                     int64_t* __restrict__ cnt) {
  extern __shared__ double acc[];  // [k][dim]
  const int lane = threadIdx.x;
  for (int v = lane; v < k * dim; v += 64) acc[v] = 0.0;
  __syncthreads();
  const int64_t b = blockIdx.x;
  const int64_t e = min(n, (b + 1) * (int64_t)kKmBlock);
  for (int64_t i = b * kKmBlock; i < e; ++i) {
    const int l = labels[i];
    for (int j = lane; j < dim; j += 64) acc[l * dim + j] = __dadd_rn(acc[l * dim + j], P[i * dim + j]);
  }
  __syncthreads();
  for (int v = lane; v < k * dim; v += 64) part[b * k * dim + v] = acc[v];
  if (lane == 0) {
    for (int c = 0; c < k; ++c) cnt[b * k + c] = 0;
    for (int64_t i = b * kKmBlock; i < e; ++i) cnt[b * k + labels[i]] += 1;
  }
}

__global__ void km_update(const double* __restrict__ part, const int64_t* __restrict__ cnt, int64_t nb, int dim, int k,
                          double* __restrict__ C) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= k * dim) return;
  const int c = v / dim;
  double s = 0.0;
  int64_t m = 0;
  int64_t b = 0;
  for (; b + 8 <= nb; b += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      t[u] = part[(b + u) * k * dim + v];
      m += cnt[(b + u) * k + c];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s = __dadd_rn(s, t[u]);
  }
  for (; b < nb; ++b) {
    s = __dadd_rn(s, part[b * k * dim + v]);
    m += cnt[b * k + c];
  }
  if (m > 0) C[v] = __ddiv_rn(s, (double)m);
}

__global__ void fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

stag_status kmeans_impl(const double* P, int64_t n, int dim, int k, uint64_t seed, int max_iter, const double* init,
                        int32_t* labels, double* C_out, int64_t* seeds, int* iters, Workspace& ws, hipStream_t st) {
  const int64_t nb = ceil_div(n, kKmBlock);
  double *C = nullptr, *D2 = nullptr, *S = nullptr, *part = nullptr;
  int64_t* cnt = nullptr;
  int* changed = nullptr;
  unsigned char* chosen = nullptr;
  STAG_TRY(ws.alloc(&C, (size_t)k * dim));
  STAG_TRY(ws.alloc(&part, (size_t)nb * k * dim));
  STAG_TRY(ws.alloc(&cnt, (size_t)nb * k));
  STAG_TRY(ws.alloc(&changed, 1));
  ScopedTimer tm("kmeans", st);
  if (init) {
    STAG_HIP(hipMemcpyAsync(C, init, sizeof(double) * (size_t)k * dim, hipMemcpyDeviceToDevice, st));
    if (seeds) {
      std::vector<int64_t> neg((size_t)k, -1);
      STAG_HIP(hipMemcpyAsync(seeds, neg.data(), sizeof(int64_t) * (size_t)k, hipMemcpyHostToDevice, st));
      STAG_HIP(hipStreamSynchronize(st));
    }
  } else {
    STAG_TRY(ws.alloc(&D2, (size_t)n));
    STAG_TRY(ws.alloc(&S, (size_t)nb));
    STAG_TRY(ws.alloc(&chosen, (size_t)n));
    STAG_HIP(hipMemsetAsync(chosen, 0, (size_t)n, st));
    for (int c = 0; c < k; ++c) {
      if (c > 0) {
        hipLaunchKernelGGL(km_d2_update, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, P, n, dim,
                           C + (int64_t)(c - 1) * dim, c == 1 ? 1 : 0, D2);
        STAG_TRY(check_launch("km_d2_update"));
        hipLaunchKernelGGL(km_block_sums, dim3((unsigned)nb), dim3(256), 0, st, D2, n, S);
        STAG_TRY(check_launch("km_block_sums"));
      }
      hipLaunchKernelGGL(km_pick, dim3(1), dim3(64), 0, st, P, n, dim, D2, S, nb, seed, c, chosen, C, seeds);
      STAG_TRY(check_launch("km_pick"));
    }
  }
  hipLaunchKernelGGL(fill_i32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, labels, n, -1);
  STAG_TRY(check_launch("fill_i32"));
  const size_t lds_c = sizeof(double) * (size_t)k * dim;
  int it = 0;
  while (it < max_iter) {
    ++it;
    STAG_HIP(hipMemsetAsync(changed, 0, sizeof(int), st));
    hipLaunchKernelGGL(km_assign, dim3((unsigned)ceil_div(n, 256)), dim3(256), lds_c, st, P, n, dim, C, k, labels,
                       changed);
    STAG_TRY(check_launch("km_assign"));
    int h = 0;
    STAG_HIP(hipMemcpyAsync(&h, changed, sizeof(int), hipMemcpyDeviceToHost, st));
    STAG_HIP(hipStreamSynchronize(st));
    if (!h) break;
    hipLaunchKernelGGL(km_block_accum, dim3((unsigned)nb), dim3(64), lds_c, st, P, labels, n, dim, k, part, cnt);
    STAG_TRY(check_launch("km_block_accum"));
    hipLaunchKernelGGL(km_update, dim3((unsigned)ceil_div(k * dim, 256)), dim3(256), 0, st, part, cnt, nb, dim, k, C);
    STAG_TRY(check_launch("km_update"));
  }
  if (C_out) STAG_HIP(hipMemcpyAsync(C_out, C, sizeof(double) * (size_t)k * dim, hipMemcpyDeviceToDevice, st));
  STAG_HIP(hipStreamSynchronize(st));
  if (iters) *iters = it;
  return STAG_OK;
}

int block_cols(int k) {
  int bp = 8;
  while (bp < k + 8) bp *= 2;
  return bp;
}

stag_status check_graph_args(const char* fn, int64_t n, const int64_t* src, const int64_t* dst, const double* w,
                             int64_t E, int32_t k) {
  if (n < 1 || n >= ((int64_t)1 << 31)) return fail(STAG_E_INVAL, "%s: n must be in [1, 2^31)", fn);
  if (E < 0 || E >= ((int64_t)1 << 30)) return fail(STAG_E_INVAL, "%s: n_edges must be in [0, 2^30)", fn);
  if (E > 0 && (!src || !dst || !w)) return fail(STAG_E_INVAL, "%s: NULL edge array", fn);
  if (k < 1 || k > 56 || k > n) return fail(STAG_E_INVAL, "%s: k must be in [1, min(56, n)]", fn);
  return STAG_OK;
}

stag_status embedding_impl(int64_t n, const int64_t* src, const int64_t* dst, const double* w, int64_t E, int32_t k,
                           double tol, int32_t max_iter, uint64_t seed, double* lam_out, double* U_out,
                           int32_t* iters_out, Workspace& ws, hipStream_t st) {
  Csr g;
  STAG_TRY(build_normalised(n, src, dst, w, E, ws, &g, st));
  const int bp = block_cols(k);
  const int b = (int)std::min<int64_t>(n, bp);
  Subspace sub(g, bp, b, ws, st);
  STAG_TRY(sub.init());
  int it = 0;
  STAG_TRY(sub.run(k, tol, max_iter, seed, &it));
  // signs, embedding, eigenvalues
  const int64_t nblk = ceil_div(n, 256);
  double *pv = nullptr, *sign = nullptr;
  int64_t* pi = nullptr;
  STAG_TRY(ws.alloc(&pv, (size_t)nblk * k));
  STAG_TRY(ws.alloc(&pi, (size_t)nblk * k));
  STAG_TRY(ws.alloc(&sign, (size_t)k));
  hipLaunchKernelGGL(col_absmax_partial, dim3((unsigned)nblk), dim3(64), 0, st, sub.V(), n, bp, k, pv, pi);
  STAG_TRY(check_launch("col_absmax_partial"));
  hipLaunchKernelGGL(col_sign, dim3(1), dim3(64), 0, st, pv, pi, nblk, sub.V(), bp, k, sign);
  STAG_TRY(check_launch("col_sign"));
  hipLaunchKernelGGL(extract_embedding, dim3((unsigned)ceil_div(n * k, 256)), dim3(256), 0, st, sub.V(), n, bp, k,
                     sign, U_out);
  STAG_TRY(check_launch("extract_embedding"));
  if (lam_out) {
    hipLaunchKernelGGL(eig_out, dim3(1), dim3(64), 0, st, sub.theta(), k, lam_out);
    STAG_TRY(check_launch("eig_out"));
  }
  STAG_HIP(hipStreamSynchronize(st));
  if (iters_out) *iters_out = it;
  return STAG_OK;
}

}  // namespace
}  // namespace stag

extern "C" stag_status stag_spectral_embedding(int64_t n, const int64_t* src, const int64_t* dst, const double* w,
                                               int64_t n_edges, int32_t k, double tol, int32_t max_iter,
                                               uint64_t seed, double* eigvals_out, double* U_out, int32_t* iters_out,
                                               hipStream_t stream) {
  using namespace stag;
  STAG_TRY(check_graph_args("stag_spectral_embedding", n, src, dst, w, n_edges, k));
  if (!U_out) return fail(STAG_E_INVAL, "stag_spectral_embedding: NULL U_out");
  if (!(tol > 0.0) || max_iter < 0) return fail(STAG_E_INVAL, "stag_spectral_embedding: tol > 0, max_iter >= 0");
  clear_error();
  Workspace ws(stream);
  return embedding_impl(n, src, dst, w, n_edges, k, tol, max_iter, seed, eigvals_out, U_out, iters_out, ws, stream);
}

extern "C" stag_status stag_kmeans(const double* P, int64_t n, int32_t dim, int32_t k, uint64_t seed,
                                   int32_t max_iter, const double* init, int32_t* labels_out, double* centroids_out,
                                   int64_t* seeds_out, int32_t* iters_out, hipStream_t stream) {
  using namespace stag;
  if (!P || !labels_out) return fail(STAG_E_INVAL, "stag_kmeans: NULL pointer argument");
  if (n < 1 || n >= ((int64_t)1 << 31) || dim < 1 || k < 1 || k > n || max_iter < 1)
    return fail(STAG_E_INVAL, "stag_kmeans: need 1 <= k <= n < 2^31, dim >= 1, max_iter >= 1");
  if ((int64_t)k * dim > 4096) return fail(STAG_E_UNSUPPORTED, "stag_kmeans: k * dim must be <= 4096");
  clear_error();
  Workspace ws(stream);
  int it = 0;
  STAG_TRY(kmeans_impl(P, n, dim, k, seed, max_iter, init, labels_out, centroids_out, seeds_out, &it, ws, stream));
  if (iters_out) *iters_out = it;
  return STAG_OK;
}

extern "C" stag_status stag_spectral_cluster(int64_t n, const int64_t* src, const int64_t* dst, const double* w,
                                             int64_t n_edges, int32_t k, uint64_t seed, int32_t* labels_out,
                                             hipStream_t stream) {
  using namespace stag;
  STAG_TRY(check_graph_args("stag_spectral_cluster", n, src, dst, w, n_edges, k));
  if (!labels_out) return fail(STAG_E_INVAL, "stag_spectral_cluster: NULL labels_out");
  clear_error();
  Workspace ws(stream);
  double* U = nullptr;
  STAG_TRY(ws.alloc(&U, (size_t)n * k));
  STAG_TRY(embedding_impl(n, src, dst, w, n_edges, k, 1e-8, 300, seed, nullptr, U, nullptr, ws, stream));
  int it = 0;
  return kmeans_impl(U, n, k, k, seed, 300, nullptr, labels_out, nullptr, nullptr, &it, ws, stream);
}
