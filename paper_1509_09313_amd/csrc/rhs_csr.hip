// Sparse right-hand sides: R (rows x k) = A_csr * Y (cols x k).
//
// The sparse case of the local products ("2 nnz(A) k flops", Section
// "Computation Cost"): CSR(A) with Ht gives A H^T, CSR(A^T) with W gives
// (W^T A)^T.  One wavefront per CSR row; lane l < k owns column l of the
// row's result.  The row's (column, value) pairs are brought in 128 at a time
// by one load per lane, then broadcast lane by lane (a register read, no
// memory), and the rows of Y they name are gathered 32 at a time, back to
// back.  Products are accumulated in FP64 in storage order and rounded once.
//
// The cost is the gather: every nonzero pulls a 4k-byte row of Y from
// wherever it is cached (Y of the sparse workload is tens of MB, above an
// XCD's 4 MB L2).  A row of Y that straddles cache lines costs an extra
// line, so the ANLS driver copies Y to a line-aligned leading dimension
// (csr_pad_ld) before the product.
#include "nmf_common.h"

namespace {

// A row's entries are taken kBlock at a time: two loads per lane bring in
// their (column, value) pairs; the Y rows are gathered kChunk at a time.
constexpr int kChunk = 32;
constexpr int kBlock = 128;
// buffer-resource word 3 for plain 32-bit loads (range-checked: an offset
// past the byte count reads 0)
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Y[c][lc]: with BUF a buffer load (one lane offset shared by every gather,
// the row offset in a scalar register; Y below 4 GiB), else a global load.
template <bool BUF>
__device__ __forceinline__ float gather(const float* __restrict__ Y, __amdgpu_buffer_rsrc_t rs, int c, int64_t ldy,
                                        unsigned lc) {
  if (BUF)
    return __uint_as_float(
        __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(lc * 4u), (int)((uint32_t)c * (uint32_t)ldy * 4u), 0));
  return Y[(int64_t)c * ldy + lc];
}

// One wavefront per row.  Index loads are clamped to the row and lanes >= k
// read column 0 of Y, so every load is in bounds and unconditional (the
// gathers of a chunk issue back to back); entries past the row's end are
// zeroed by selects.  y_bytes: Y's extent (the buffer range with BUF).
template <bool BUF>
__global__ __launch_bounds__(256) void k_spmm(int64_t rows, int k, const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ colidx, const float* __restrict__ vals,
                                              const float* __restrict__ Y, int64_t ldy, uint32_t y_bytes,
                                              float* __restrict__ R, int64_t ldr) {
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)Y, (short)0, (int)y_bytes, kRsrcWord3);
  const unsigned l = threadIdx.x & 63;
  const bool lane_ok = l < (unsigned)k;
  const unsigned lc = lane_ok ? l : 0;
  const int64_t wave = uniform_i64(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < rows; i += nwaves) {
    const int64_t p1 = rowptr[i + 1];
    double acc = 0.0;
    for (int64_t p = rowptr[i]; p < p1; p += kBlock) {
      const int64_t e0 = p + l < p1 ? p + l : p1 - 1;
      const int64_t e1 = p + 64 + l < p1 ? p + 64 + l : p1 - 1;
      // the index stream is read once: non-temporal loads leave the L2 to
      // the gathered rows of Y
      const int ca = __builtin_nontemporal_load(colidx + e0), cb = __builtin_nontemporal_load(colidx + e1);
      const float va = __builtin_nontemporal_load(vals + e0), vb = __builtin_nontemporal_load(vals + e1);
#pragma unroll
      for (int h = 0; h < kBlock / kChunk; ++h) {
        const int64_t q = p + h * kChunk;
        if (q >= p1) break;
        const int cr = h < 2 ? ca : cb;
        const float vr = h < 2 ? va : vb;
        float y[kChunk], v[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          const int src = (h & 1) * kChunk + u;
          const int c = __builtin_amdgcn_readlane(cr, src);
          const float vu = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vr), src));
          const bool in = q + u < p1;
          v[u] = in ? vu : 0.0f;
          const float yu = gather<BUF>(Y, rs, c, ldy, lc);
          y[u] = in ? yu : 0.0f;
        }
        // storage order; an entry past the row's end adds an exact +0.0,
        // which leaves the sum's bits alone (a sum started from +0.0 is
        // never -0.0)
#pragma unroll
        for (int u = 0; u < kChunk; ++u) acc += (double)v[u] * (double)y[u];
      }
    }
    if (lane_ok) R[i * ldr + l] = (float)acc;
  }
}

// dst (rows x k, ldd) = src (rows x k, lds); one wave per row.
__global__ __launch_bounds__(256) void k_copy_rows(int64_t rows, int k, const float* __restrict__ src, int64_t lds,
                                                   float* __restrict__ dst, int64_t ldd) {
  const int l = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < rows; i += nwaves)
    if (l < k) dst[i * ldd + l] = src[i * lds + l];
}

}  // namespace

namespace nmf {

int64_t csr_pad_ld(int k) {
  if (k > 32) return cdiv(k, 32) * 32;  // whole 128-byte lines
  int64_t ld = 1;
  while (ld < k) ld <<= 1;  // a power of two: rows never straddle a line
  return ld;
}

int rhs_csr_launch(int64_t rows, int64_t cols, int k, const int64_t* rowptr, const int32_t* colidx,
                   const float* vals, const float* Y, int64_t ldy, float* R, int64_t ldr, float* ypad,
                   hipStream_t s) {
  if (rows == 0) return NMF_OK;
  if (ypad && cols > 0 && ldy != csr_pad_ld(k)) {
    int64_t cb = cdiv(cols, 4);
    if (cb > 16384) cb = 16384;
    hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)cb), dim3(256), 0, s, cols, k, Y, ldy, ypad, csr_pad_ld(k));
    Y = ypad;
    ldy = csr_pad_ld(k);
  }
  int64_t blocks = cdiv(rows, 4);
  if (blocks > 16384) blocks = 16384;
  // Y's extent; buffer loads take 32-bit offsets
  const int64_t y_bytes = cols > 0 ? ((cols - 1) * ldy + k) * (int64_t)sizeof(float) : 0;
  const bool buf = y_bytes <= (int64_t)UINT32_MAX;
  const uint32_t yb = buf ? (uint32_t)y_bytes : 0;
  mark_begin(s);
  if (buf)
    hipLaunchKernelGGL(k_spmm<true>, dim3((unsigned)blocks), dim3(256), 0, s, rows, k, rowptr, colidx, vals, Y, ldy,
                       yb, R, ldr);
  else
    hipLaunchKernelGGL(k_spmm<false>, dim3((unsigned)blocks), dim3(256), 0, s, rows, k, rowptr, colidx, vals, Y,
                       ldy, yb, R, ldr);
  mark_end(s);
  return launch_status("rhs csr");
}

}  // namespace nmf

extern "C" int nmf_rhs_csr(int64_t rows, int64_t cols, int k, const int64_t* rowptr, const int32_t* colidx,
                           const float* vals, const float* Y, int64_t ldy, float* R, int64_t ldr, void* stream) {
  if (!nmf::valid_k(k)) return nmf::fail(NMF_EINVAL, "nmf_rhs_csr: k=%d outside [1,64]", k);
  if (rows < 0 || cols < 0 || cols > INT32_MAX || ldy < k || ldr < k)
    return nmf::fail(NMF_EINVAL, "nmf_rhs_csr: bad sizes");
  if (rows > 0 && (!rowptr || !R)) return nmf::fail(NMF_EINVAL, "nmf_rhs_csr: null pointer");
  if (rows > 0 && cols > 0 && (!colidx || !vals || !Y)) return nmf::fail(NMF_EINVAL, "nmf_rhs_csr: null pointer");
  return nmf::rhs_csr_launch(rows, cols, k, rowptr, colidx, vals, Y, ldy, R, ldr, nullptr, nmf::as_stream(stream));
}
