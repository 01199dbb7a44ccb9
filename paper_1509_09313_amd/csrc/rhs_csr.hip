// Sparse right-hand sides: R (rows x k) = A_csr * Y (cols x k).
//
// The sparse case of the local products ("2 nnz(A) k flops", Section
// "Computation Cost"): CSR(A) with Ht gives A H^T, CSR(A^T) with W gives
// (W^T A)^T.  One wavefront per CSR row (or one half-wavefront when k <= 32):
// the row's (column, value) pairs are read once and broadcast, lane l gathers
// Y[col][l] (a k-float row of Y, coalesced), and products are accumulated in
// FP64 in storage order.  Eight nonzeros are in flight per step.
#include "nmf_common.h"

namespace {

constexpr int kUnroll = 8;

template <int LPR>
__global__ __launch_bounds__(256) void k_spmm(int64_t rows, int k, const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ colidx, const float* __restrict__ vals,
                                              const float* __restrict__ Y, int64_t ldy, float* __restrict__ R,
                                              int64_t ldr) {
  constexpr int RPW = 64 / LPR;
  const int lane = threadIdx.x & 63;
  const int sub = lane / LPR, l = lane % LPR;
  const bool lane_ok = l < k;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * RPW; base < rows; base += nwaves * RPW) {
    const int64_t i = base + sub;
    if (i >= rows) continue;
    const int64_t p0 = rowptr[i], p1 = rowptr[i + 1];
    double acc = 0.0;
    int64_t p = p0;
    for (; p + kUnroll <= p1; p += kUnroll) {
      int c[kUnroll];
      float v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        c[u] = colidx[p + u];
        v[u] = vals[p + u];
      }
      float y[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) y[u] = lane_ok ? Y[(int64_t)c[u] * ldy + l] : 0.0f;
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) acc += (double)v[u] * (double)y[u];
    }
    for (; p < p1; ++p) {
      const int c = colidx[p];
      const float y = lane_ok ? Y[(int64_t)c * ldy + l] : 0.0f;
      acc += (double)vals[p] * (double)y;
    }
    if (lane_ok) R[i * ldr + l] = (float)acc;
  }
}

}  // namespace

namespace nmf {

int rhs_csr_launch(int64_t rows, int64_t cols, int k, const int64_t* rowptr, const int32_t* colidx,
                   const float* vals, const float* Y, int64_t ldy, float* R, int64_t ldr, hipStream_t s) {
  (void)cols;
  if (rows == 0) return NMF_OK;
  const int rpw = k <= 32 ? 2 : 1;
  const int64_t waves = cdiv(rows, rpw);
  int64_t blocks = cdiv(waves, 4);
  if (blocks > 16384) blocks = 16384;
  mark_begin(s);
  if (k <= 32)
    hipLaunchKernelGGL(k_spmm<32>, dim3((unsigned)blocks), dim3(256), 0, s, rows, k, rowptr, colidx, vals, Y, ldy,
                       R, ldr);
  else
    hipLaunchKernelGGL(k_spmm<64>, dim3((unsigned)blocks), dim3(256), 0, s, rows, k, rowptr, colidx, vals, Y, ldy,
                       R, ldr);
  mark_end(s);
  return launch_status("rhs csr");
}

}  // namespace nmf

extern "C" int nmf_rhs_csr(int64_t rows, int64_t cols, int k, const int64_t* rowptr, const int32_t* colidx,
                           const float* vals, const float* Y, int64_t ldy, float* R, int64_t ldr, void* stream) {
  if (!nmf::valid_k(k)) return nmf::fail(NMF_EINVAL, "nmf_rhs_csr: k=%d outside [1,64]", k);
  if (rows < 0 || cols < 0 || ldy < k || ldr < k) return nmf::fail(NMF_EINVAL, "nmf_rhs_csr: bad sizes");
  if (rows > 0 && (!rowptr || !R)) return nmf::fail(NMF_EINVAL, "nmf_rhs_csr: null pointer");
  if (rows > 0 && cols > 0 && (!colidx || !vals || !Y)) return nmf::fail(NMF_EINVAL, "nmf_rhs_csr: null pointer");
  return nmf::rhs_csr_launch(rows, cols, k, rowptr, colidx, vals, Y, ldy, R, ldr, nmf::as_stream(stream));
}
