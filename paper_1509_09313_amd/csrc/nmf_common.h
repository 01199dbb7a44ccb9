// Internal helpers shared by the libnmf translation units: error reporting,
// workspace carving, launch checks and small device utilities.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stddef.h>
#include <stdint.h>

#include "libnmf.h"

namespace nmf {

// Thread-local error message behind nmf_last_error().
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);

inline int launch_status(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NMF_EHIP, "%s: %s", what, hipGetErrorString(e));
  return NMF_OK;
}

#define NMF_TRY(expr)          \
  do {                         \
    const int _rc = (expr);    \
    if (_rc != NMF_OK) return _rc; \
  } while (0)

// Carves 256-byte-aligned sub-buffers out of a caller workspace.  With a null
// base it only measures, so one routine both sizes and lays out a workspace.
struct Carver {
  char* base;
  size_t cap;
  size_t off = 0;
  Carver(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  bool fits() const { return off <= cap; }
};

inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

inline bool valid_k(int k) { return k >= 1 && k <= 64; }

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---- internal launchers shared between translation units -------------------
int gram_plan(int64_t rows, int k, Carver& c, double** partial, int* nblocks);
// With yth (optional) the kernel also writes the transposed BF16 split of X
// (hi to yth, lo to ytl: KP x ldt, X row r at column r, zero for columns
// k <= i < KP and rows rows <= r < ldt; ldt a multiple of 64): the Y planes
// of a BF16x3 product whose contraction runs over the rows of X.
int gram_launch(int64_t rows, int k, const float* X, int64_t ldx, double* G, double* partial,
                int nblocks, hipStream_t s, uint16_t* yth = nullptr, uint16_t* ytl = nullptr, int64_t ldt = 0,
                int KP = 0);

int rhs_dense_plan(int side, int64_t m, int64_t n, int k, int prec, Carver& c, void** scratch);
// y_ready: (BF16x3) the transposed Y planes in scratch are already written
int rhs_dense_launch(int side, int64_t m, int64_t n, int k, const float* A, int64_t lda, const void* Bt,
                     const float* Y, int64_t ldy, float* R, int64_t ldr, int prec, void* scratch, hipStream_t s,
                     bool y_ready = false);
// The transposed Y planes of a BF16x3 product inside its scratch block
void bf16x3_y_planes(int side, int64_t m, int64_t n, int k, void* scratch, uint16_t** yth, uint16_t** ytl,
                     int64_t* ldt, int* KP);

// CSR products.  csr_pad_ld: a leading dimension for Y whose rows never
// straddle a 128-byte line; with ypad (cols x csr_pad_ld(k) floats) Y is
// first copied there.
int64_t csr_pad_ld(int k);
int rhs_csr_launch(int64_t rows, int64_t cols, int k, const int64_t* rowptr, const int32_t* colidx,
                   const float* vals, const float* Y, int64_t ldy, float* R, int64_t ldr, float* ypad,
                   hipStream_t s);

int local_update_launch(int solver, int k, int64_t rows, const double* G, const float* R, int64_t ldr, float* X,
                        int64_t ldx, hipStream_t s);

// dot_partial (optional, bpp_blocks(k, batch) entries): per-block sums of
// R[b][i] X[b][i] over the stored solutions; status_counts (optional, two
// entries): the capped and fell-back problems are added to [0] and [1].
int bpp_launch(int k, int64_t batch, const double* G, const float* R, int64_t ldr, float* X,
               int64_t ldx, const uint64_t* mask_in, uint64_t* mask_out, uint8_t* rounds,
               uint8_t* status, int max_rounds, int warm_cap, uint64_t* counters, hipStream_t s,
               double* dot_partial = nullptr, uint64_t* status_counts = nullptr);
// workgroups (and dot_partial entries) of a bpp_launch of this size
int64_t bpp_blocks(int k, int64_t batch);

// Zero-fills a rows x cols FP32 block with leading dimension ld (a kernel, so
// it is safe inside captured graphs).
int zero_f32(float* p, int64_t rows, int64_t cols, int64_t ld, hipStream_t s);

// Deterministic FP64 dot product  out[0] = sum_i a[i] * b[i]  over `len`
// elements of two FP32 arrays.
int dot_plan(int64_t len, Carver& c, double** partial, int* nblocks);
int dot_f32_launch(int64_t len, const float* a, const float* b, double* out, double* partial,
                   int nblocks, hipStream_t s);

// Kernel-level timing hook: when set (by the ANLS driver), the product
// launchers record these events right around their main kernel.
struct KernelMark {
  hipEvent_t begin = nullptr;
  hipEvent_t end = nullptr;
};
KernelMark& kernel_mark();
inline void mark_begin(hipStream_t s) {
  if (kernel_mark().begin) hipEventRecord(kernel_mark().begin, s);
}
inline void mark_end(hipStream_t s) {
  if (kernel_mark().end) hipEventRecord(kernel_mark().end, s);
}

}  // namespace nmf

// ---- device helpers -----------------------------------------------------------

// Orders a wavefront's own LDS writes before its subsequent LDS reads by other
// lanes of the same wavefront (no workgroup barrier needed).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The BF16 split of the BF16x3 products: hi = bf16_rne(x), lo =
// bf16_rne(x - hi) (round to nearest even; x - hi is exact in FP32).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t bias = 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)((u + bias) >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
