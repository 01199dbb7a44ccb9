// Split-precision (BF16x3) right-hand sides.
//
// x = hi + lo with hi = bf16_rne(x) and lo = bf16_rne(x - hi) (x - hi is
// exact in FP32), and R = A_hi Y_hi + A_hi Y_lo + A_lo Y_hi with FP32
// accumulation: the lo*lo term (relative size 2^-16 per operand pair) is
// dropped.  Bytes per entry of A stay 4 (two BF16 planes), so the product is
// HBM-bound where the FP32 MFMA form is compute-bound.
#include "nmf_common.h"

namespace {

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t bias = 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)((u + bias) >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__global__ void k_split(int64_t rows, int64_t cols, const float* __restrict__ X, int64_t ldx, uint16_t* __restrict__ hi,
                        uint16_t* __restrict__ lo, int64_t ldo) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e - r * cols;
    const float x = X[r * ldx + c];
    const uint16_t h = bf16_rne(x);
    hi[r * ldo + c] = h;
    lo[r * ldo + c] = bf16_rne(x - bf16_to_f32(h));
  }
}

// Transposed split through a 64 x 64 LDS tile: planes of X^T (cols x rows).
__global__ __launch_bounds__(256) void k_split_t(int64_t rows, int64_t cols, const float* __restrict__ X, int64_t ldx,
                                                 uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int64_t ldo) {
  __shared__ float tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t r = r0 + rr, c = c0 + tx;
    tile[rr][tx] = (r < rows && c < cols) ? X[r * ldx + c] : 0.0f;
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t c = c0 + cc, r = r0 + tx;
    if (c < cols && r < rows) {
      const float x = tile[tx][cc];
      const uint16_t h = bf16_rne(x);
      hi[c * ldo + r] = h;
      lo[c * ldo + r] = bf16_rne(x - bf16_to_f32(h));
    }
  }
}

}  // namespace

namespace nmf {

int bf16x3_plan(int side, int64_t m, int64_t n, int k, Carver& c, void** scratch) {
  (void)side; (void)m; (void)n; (void)k; (void)c;
  *scratch = nullptr;
  return NMF_OK;
}

int bf16x3_launch(int side, int64_t m, int64_t n, int k, const uint16_t* B_hi, const uint16_t* B_lo, int64_t ldb,
                  const float* Y, int64_t ldy, float* R, int64_t ldr, void* scratch, hipStream_t s) {
  (void)side; (void)m; (void)n; (void)k; (void)B_hi; (void)B_lo; (void)ldb; (void)Y; (void)ldy; (void)R; (void)ldr;
  (void)scratch; (void)s;
  return fail(NMF_EUNSUPPORTED, "nmf_rhs_dense: BF16X3 is not built yet");
}

}  // namespace nmf

extern "C" int nmf_split_bf16(int64_t rows, int64_t cols, const float* X, int64_t ldx, uint16_t* hi, uint16_t* lo,
                              int64_t ldo, int transpose, void* stream) {
  if (rows < 0 || cols < 0 || ldx < cols) return nmf::fail(NMF_EINVAL, "nmf_split_bf16: bad sizes");
  if (ldo < (transpose ? rows : cols)) return nmf::fail(NMF_EINVAL, "nmf_split_bf16: ldo too small");
  if (rows * cols > 0 && (!X || !hi || !lo)) return nmf::fail(NMF_EINVAL, "nmf_split_bf16: null pointer");
  if (rows * cols == 0) return NMF_OK;
  hipStream_t s = nmf::as_stream(stream);
  if (!transpose) {
    int64_t blocks = nmf::cdiv(rows * cols, 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_split, dim3((unsigned)blocks), dim3(256), 0, s, rows, cols, X, ldx, hi, lo, ldo);
  } else {
    const int64_t gx = nmf::cdiv(cols, 64), gy = nmf::cdiv(rows, 64);
    if (gy > 65535) return nmf::fail(NMF_EINVAL, "nmf_split_bf16: too many rows");
    hipLaunchKernelGGL(k_split_t, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, rows, cols, X, ldx, hi, lo, ldo);
  }
  return nmf::launch_status("nmf_split_bf16");
}
