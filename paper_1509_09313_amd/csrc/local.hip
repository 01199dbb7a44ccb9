// The other local NLS solvers of Algorithm 1: multiplicative updates (MU,
// Eq. muupdate) and HALS (Eq. halsupdate).  Given the FP64 Gram matrix G of
// the fixed factor and the FP32 right-hand sides R, every row x of X (a row
// of W, or a row of H^T) is updated in place and independently:
//   MU   x_j <- x_j r_j / (x^T G)_j          (all j from the old x)
//   HALS x_i <- [r_i - sum_{l != i} G_li x_l]_+ / G_ii   (i in order, each
//        step using the values already updated in this sweep)
// An index with G_ii <= 1e-14 max_l G_ll is pinned at 0 (as in BPP), and MU
// sets x_j = 0 where (x^T G)_j <= 0.  Arithmetic is FP64, one rounding to FP32
// per entry when the row is stored.
//
// One lane per row, 64 rows per wavefront-sized block.  The rows of R and X
// are staged through LDS (coalesced loads and stores); G, padded to K x K with
// zeros, sits in LDS and is read at the same address by every lane.  HALS
// keeps the row in registers rotated so that the current index is always in
// slot 0 (no register indexing by a loop variable).  The cost is 2 k^2 FP64
// flops per row, as the paper counts it (2 (m + n) k^2 per iteration).
#include "nmf_common.h"

namespace {

constexpr int kRows = 64;

template <int K, int SOLVER>
__global__ __launch_bounds__(64) void k_local(int k, int64_t rows, const double* __restrict__ G,
                                              const float* __restrict__ R, int64_t ldr, float* __restrict__ X,
                                              int64_t ldx) {
  __shared__ double Gs[K * K];
  __shared__ float rt[kRows][K + 1];
  __shared__ float xt[kRows][K + 1];
  const int l = threadIdx.x;
  for (int e = l; e < K * K; e += 64) {
    const int q = e / K, p = e % K;
    Gs[e] = (q < k && p < k) ? G[q * k + p] : 0.0;
  }
  __syncthreads();
  double dmax = 0.0;
  for (int q = 0; q < k; ++q) dmax = fmax(dmax, Gs[q * K + q]);
  const double thr = 1e-14 * dmax;

  for (int64_t r0 = (int64_t)blockIdx.x * kRows; r0 < rows; r0 += (int64_t)gridDim.x * kRows) {
    const int64_t nr = rows - r0 < kRows ? rows - r0 : kRows;
    __syncthreads();
    for (int e = l; e < kRows * K; e += 64) {
      const int row = e / K, c = e % K;
      const bool in = row < nr && c < k;
      rt[row][c] = in ? R[(r0 + row) * ldr + c] : 0.0f;
      xt[row][c] = in ? X[(r0 + row) * ldx + c] : 0.0f;
    }
    __syncthreads();
    double x[K];
#pragma unroll
    for (int c = 0; c < K; ++c) x[c] = (double)xt[l][c];
    if (SOLVER == NMF_SOLVER_HALS) {
      // x[q] holds x_{(i + q) mod K}; the new x_i goes to the end
#pragma unroll 1
      for (int i = 0; i < K; ++i) {
        double s = (double)rt[l][i];
#pragma unroll
        for (int q = 1; q < K; ++q) s -= Gs[((i + q) & (K - 1)) * K + i] * x[q];
        const double gii = Gs[i * K + i];
        const double xi = (i < k && gii > thr) ? fmax(s, 0.0) / gii : 0.0;
#pragma unroll
        for (int q = 0; q < K - 1; ++q) x[q] = x[q + 1];
        x[K - 1] = xi;
      }
#pragma unroll
      for (int c = 0; c < K; ++c) xt[l][c] = (float)x[c];
    } else {
#pragma unroll 1
      for (int j = 0; j < K; ++j) {
        double d = 0.0;
#pragma unroll
        for (int q = 0; q < K; ++q) d += x[q] * Gs[q * K + j];
        const double xj = (double)xt[l][j], rj = (double)rt[l][j];
        const bool ok = j < k && Gs[j * K + j] > thr && d > 0.0;
        xt[l][j] = ok ? (float)(xj * rj / d) : 0.0f;
      }
    }
    __syncthreads();
    for (int e = l; e < kRows * K; e += 64) {
      const int row = e / K, c = e % K;
      if (row < nr && c < k) X[(r0 + row) * ldx + c] = xt[row][c];
    }
  }
}

template <int K>
void launch_k(int solver, int k, int64_t rows, const double* G, const float* R, int64_t ldr, float* X, int64_t ldx,
              hipStream_t s) {
  int64_t blocks = nmf::cdiv(rows, kRows);
  if (blocks > 8192) blocks = 8192;
  if (solver == NMF_SOLVER_HALS)
    hipLaunchKernelGGL((k_local<K, NMF_SOLVER_HALS>), dim3((unsigned)blocks), dim3(64), 0, s, k, rows, G, R, ldr,
                       X, ldx);
  else
    hipLaunchKernelGGL((k_local<K, NMF_SOLVER_MU>), dim3((unsigned)blocks), dim3(64), 0, s, k, rows, G, R, ldr, X,
                       ldx);
}

}  // namespace

namespace nmf {

int local_update_launch(int solver, int k, int64_t rows, const double* G, const float* R, int64_t ldr, float* X,
                        int64_t ldx, hipStream_t s) {
  if (rows == 0) return NMF_OK;
  if (k <= 8)
    launch_k<8>(solver, k, rows, G, R, ldr, X, ldx, s);
  else if (k <= 16)
    launch_k<16>(solver, k, rows, G, R, ldr, X, ldx, s);
  else if (k <= 32)
    launch_k<32>(solver, k, rows, G, R, ldr, X, ldx, s);
  else
    launch_k<64>(solver, k, rows, G, R, ldr, X, ldx, s);
  return launch_status("local update");
}

}  // namespace nmf

extern "C" int nmf_local_update(int solver, int k, int64_t rows, const double* G, const float* R, int64_t ldr,
                                float* X, int64_t ldx, void* stream) {
  if (solver != NMF_SOLVER_HALS && solver != NMF_SOLVER_MU)
    return nmf::fail(NMF_EINVAL, "nmf_local_update: solver must be NMF_SOLVER_HALS or NMF_SOLVER_MU");
  if (!nmf::valid_k(k)) return nmf::fail(NMF_EINVAL, "nmf_local_update: k=%d outside [1,64]", k);
  if (rows < 0 || ldr < k || ldx < k) return nmf::fail(NMF_EINVAL, "nmf_local_update: bad sizes");
  if (rows > 0 && (!G || !R || !X)) return nmf::fail(NMF_EINVAL, "nmf_local_update: null pointer");
  return nmf::local_update_launch(solver, k, rows, G, R, ldr, X, ldx, nmf::as_stream(stream));
}
