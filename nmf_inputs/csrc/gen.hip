// Device-side synthetic input generation (Philox-4x32-10, SC'11 definition).
//
// This library only builds input matrices; it contains none of the
// factorisation's arithmetic.  Every value is addressed by (key, counter) with
// key = (seed, matrix id) and counter = (row, col, 0, 0); U[0,1) takes the top
// 24 bits of output word 0 times 2^-24, so float32 holds it exactly.  Sums of
// products are accumulated in float64 in index order with products that are
// exact (24-bit x 24-bit), and this file is compiled without floating-point
// contraction, so the host recipes in nmf_inputs.configs reproduce every
// element bit for bit.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint32_t philox_w0(uint32_t c0, uint32_t c1, uint32_t k0, uint32_t k1) {
  uint32_t c2 = 0, c3 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return c0;
}

__device__ __forceinline__ float u01(uint32_t seed, uint32_t mid, uint64_t row, uint64_t col) {
  return (float)(philox_w0((uint32_t)row, (uint32_t)col, seed, mid) >> 8) * (1.0f / 16777216.0f);
}

// out[r * ld_r + c * ld_c] = U(seed, mid, row0 + r, col0 + c)
__global__ void k_uniform(uint32_t seed, uint32_t mid, int64_t row0, int64_t rows, int64_t col0,
                          int64_t cols, float* out, int64_t ld_r, int64_t ld_c) {
  const int64_t total = rows * cols;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / cols, c = t - r * cols;
    out[r * ld_r + c * ld_c] = u01(seed, mid, row0 + r, col0 + c);
  }
}

constexpr int kTileRows = 16;
constexpr int kMaxRank = 64;

// Planted: A[i,j] = fl32( sum_l W0[i,l] * H0[l,j] + noise * u[i,j] ).
// W0 is m x r (row-major), H0t is n x r (H0 transposed), both exact U[0,1).
__global__ void k_planted(uint32_t seed, uint32_t mid_noise, int64_t m, int64_t n, int r, double noise,
                          const float* __restrict__ W0, const float* __restrict__ H0t, float* A,
                          int64_t lda) {
  __shared__ float ws[kTileRows][kMaxRank];
  const int64_t col_tiles = (n + blockDim.x - 1) / blockDim.x;
  const int64_t row_tiles = (m + kTileRows - 1) / kTileRows;
  for (int64_t tile = blockIdx.x; tile < row_tiles * col_tiles; tile += gridDim.x) {
    const int64_t rt = tile / col_tiles, ct = tile - rt * col_tiles;
    const int64_t i0 = rt * kTileRows;
    __syncthreads();
    for (int t = threadIdx.x; t < kTileRows * r; t += blockDim.x) {
      const int ii = t / r, l = t - ii * r;
      ws[ii][l] = (i0 + ii < m) ? W0[(i0 + ii) * r + l] : 0.0f;
    }
    __syncthreads();
    const int64_t j = ct * blockDim.x + threadIdx.x;
    if (j >= n) continue;
    float h[kMaxRank];
#pragma unroll
    for (int l = 0; l < kMaxRank; ++l) h[l] = (l < r) ? H0t[j * r + l] : 0.0f;
    for (int ii = 0; ii < kTileRows && i0 + ii < m; ++ii) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < kMaxRank; ++l)
        if (l < r) s = s + (double)ws[ii][l] * (double)h[l];
      const double e = noise * (double)u01(seed, mid_noise, i0 + ii, j);
      A[(i0 + ii) * lda + j] = (float)(s + e);
    }
  }
}

constexpr int kVideoRank = 10;

// Video-like: B = fl64(sum_{l<10} Wb[i,l] Hb[l,j]) * 0.1; foreground where u < 0.02
// takes an independent U[0,1) value.  Wb is m x 10, Hbt is n x 10.
__global__ void k_video(uint32_t seed, uint32_t mid_fgmask, uint32_t mid_fgval, int64_t m, int64_t n,
                        const float* __restrict__ Wb, const float* __restrict__ Hbt, float* A,
                        int64_t lda) {
  __shared__ float ws[kTileRows][kVideoRank];
  const int64_t col_tiles = (n + blockDim.x - 1) / blockDim.x;
  const int64_t row_tiles = (m + kTileRows - 1) / kTileRows;
  for (int64_t tile = blockIdx.x; tile < row_tiles * col_tiles; tile += gridDim.x) {
    const int64_t rt = tile / col_tiles, ct = tile - rt * col_tiles;
    const int64_t i0 = rt * kTileRows;
    __syncthreads();
    for (int t = threadIdx.x; t < kTileRows * kVideoRank; t += blockDim.x) {
      const int ii = t / kVideoRank, l = t - ii * kVideoRank;
      ws[ii][l] = (i0 + ii < m) ? Wb[(i0 + ii) * kVideoRank + l] : 0.0f;
    }
    __syncthreads();
    const int64_t j = ct * blockDim.x + threadIdx.x;
    if (j >= n) continue;
    float h[kVideoRank];
#pragma unroll
    for (int l = 0; l < kVideoRank; ++l) h[l] = Hbt[j * kVideoRank + l];
    for (int ii = 0; ii < kTileRows && i0 + ii < m; ++ii) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < kVideoRank; ++l) s = s + (double)ws[ii][l] * (double)h[l];
      s = s * 0.1;
      const int64_t i = i0 + ii;
      if (u01(seed, mid_fgmask, i, j) < 0.02f) s = (double)u01(seed, mid_fgval, i, j);
      A[i * lda + j] = (float)s;
    }
  }
}

int grid_for(int64_t work, int block) {
  int64_t g = (work + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

extern "C" {

int nmfin_uniform(uint32_t seed, uint32_t mid, int64_t row0, int64_t rows, int64_t col0, int64_t cols,
                  float* out, int64_t ld_r, int64_t ld_c, void* stream) {
  if (rows < 0 || cols < 0 || (rows * cols > 0 && out == nullptr)) return 1;
  if (rows * cols == 0) return 0;
  hipLaunchKernelGGL(k_uniform, dim3(grid_for(rows * cols, 256)), dim3(256), 0, (hipStream_t)stream,
                     seed, mid, row0, rows, col0, cols, out, ld_r, ld_c);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

int nmfin_planted(uint32_t seed, uint32_t mid_noise, int64_t m, int64_t n, int r, double noise,
                  const float* W0, const float* H0t, float* A, int64_t lda, void* stream) {
  if (m < 0 || n < 0 || r < 1 || r > kMaxRank || lda < n) return 1;
  if (m * n == 0) return 0;
  const int64_t tiles = ((m + kTileRows - 1) / kTileRows) * ((n + 255) / 256);
  hipLaunchKernelGGL(k_planted, dim3(grid_for(tiles, 1)), dim3(256), 0, (hipStream_t)stream, seed,
                     mid_noise, m, n, r, noise, W0, H0t, A, lda);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

int nmfin_video(uint32_t seed, uint32_t mid_fgmask, uint32_t mid_fgval, int64_t m, int64_t n,
                const float* Wb, const float* Hbt, float* A, int64_t lda, void* stream) {
  if (m < 0 || n < 0 || lda < n) return 1;
  if (m * n == 0) return 0;
  const int64_t tiles = ((m + kTileRows - 1) / kTileRows) * ((n + 255) / 256);
  hipLaunchKernelGGL(k_video, dim3(grid_for(tiles, 1)), dim3(256), 0, (hipStream_t)stream, seed,
                     mid_fgmask, mid_fgval, m, n, Wb, Hbt, A, lda);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

}  // extern "C"
