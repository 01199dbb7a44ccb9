// Objective of Eq. NMF: r = ||A - W H||_F / ||A||_F, and ||A||_F^2.
//
// DIRECT, dense: each wavefront owns a 32-row strip of W and walks 32-column
// tiles of A; the W H tile comes from v_mfma_f32_32x32x2_f32 (FP32 products
// of FP32 factors, FP32 accumulation over k), the residual entries and A's
// entries are squared and summed in FP64.  A is read once.
// DIRECT, CSR: ||A||^2 - 2 sum_nnz a_ij (W H)_ij + <W^T W, H H^T>, all FP64
// (the sum over nonzeros is sum_i W_i . (A H^T)_i with (A H^T)_i in FP64).
// TRACE: ||A||^2 - 2 <A^T W, H^T> + <W^T W, H H^T> in FP64 from quantities
// the iteration already has (cheap, but it cancels when r is small).
// All sums are block partials combined in a fixed order (deterministic).
#include <math.h>

#include "nmf_common.h"

typedef float v16f __attribute__((ext_vector_type(16)));

namespace {

constexpr int kRedThreads = 256;

// out = sum of partial[0..n) in a fixed order (strided per thread, then tree).
__global__ void k_reduce_sum(int64_t n, int width, const double* __restrict__ partial, double* __restrict__ out) {
  __shared__ double s[kRedThreads];
  for (int c = 0; c < width; ++c) {
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kRedThreads) acc += partial[i * width + c];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kRedThreads / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = s[0];
    __syncthreads();
  }
}

template <typename T>
__global__ void k_dot(int64_t len, const T* __restrict__ a, const T* __restrict__ b, double* __restrict__ partial) {
  __shared__ double s[kRedThreads];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < len; i += (int64_t)gridDim.x * kRedThreads)
    acc += (double)a[i] * (double)b[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kRedThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

// sum of squares of a rows x cols FP32 block with leading dimension ld
__global__ void k_sumsq(int64_t rows, int64_t cols, int64_t ld, const float* __restrict__ a,
                        double* __restrict__ partial) {
  __shared__ double s[kRedThreads];
  double acc = 0.0;
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; e < total; e += (int64_t)gridDim.x * kRedThreads) {
    const int64_t r = e / cols, c = e - r * cols;
    const double v = a[r * ld + c];
    acc += v * v;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kRedThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

constexpr int kObjColTiles = 64;  // 32-column tiles per wavefront

// One wavefront per (32-row strip, range of 32-column tiles).  partial[w] =
// {sum (a - wh)^2, sum a^2}.
template <int NS>
__global__ __launch_bounds__(64) void k_obj_dense(int64_t m, int64_t n, int k, const float* __restrict__ A,
                                                  int64_t lda, const float* __restrict__ W,
                                                  const float* __restrict__ Ht, double* __restrict__ partial) {
  const int lane = threadIdx.x, i = lane & 31, h = lane >> 5;
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  const int64_t tile0 = (int64_t)blockIdx.y * kObjColTiles;
  float wa[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = 2 * s + h;
    wa[s] = (r0 + i < m && c < k) ? W[(r0 + i) * k + c] : 0.0f;
  }
  double sr = 0.0, sa = 0.0;
  const int64_t ntiles = (n + 31) / 32;
  const int64_t tend = (tile0 + kObjColTiles < ntiles) ? tile0 + kObjColTiles : ntiles;
  // the next tile's H^T operands and A entries are loaded while the current
  // tile is reduced (A, read once, with non-temporal loads) (acc[v] = (W Ht^T)[r0 + ii][c0 + i], ii = (v&3) + 8(v>>2) + 4h)
  float hn[NS], an[16];
#define NMF_OBJ_LOAD(TL)                                                              \
  do {                                                                                \
    const int64_t jn_ = (TL) * 32 + i;                                                \
    _Pragma("unroll") for (int s_ = 0; s_ < NS; ++s_) {                               \
      const int c_ = 2 * s_ + h;                                                      \
      hn[s_] = (jn_ < n && c_ < k) ? Ht[jn_ * k + c_] : 0.0f;                         \
    }                                                                                 \
    _Pragma("unroll") for (int v_ = 0; v_ < 16; ++v_) {                               \
      const int64_t row_ = r0 + (v_ & 3) + 8 * (v_ >> 2) + 4 * h;                     \
      an[v_] = (jn_ < n && row_ < m) ? __builtin_nontemporal_load(A + row_ * lda + jn_) : 0.0f; \
    }                                                                                 \
  } while (0)
  if (tile0 < tend) NMF_OBJ_LOAD(tile0);
  for (int64_t tl = tile0; tl < tend; ++tl) {
    float hb[NS], av[16];
#pragma unroll
    for (int s = 0; s < NS; ++s) hb[s] = hn[s];
#pragma unroll
    for (int v = 0; v < 16; ++v) av[v] = an[v];
    if (tl + 1 < tend) NMF_OBJ_LOAD(tl + 1);
    const int64_t jc = tl * 32 + i;
    v16f acc = v16f{};
#pragma unroll
    for (int s = 0; s < NS; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wa[s], hb[s], acc, 0, 0, 0);
    if (jc < n) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = r0 + (v & 3) + 8 * (v >> 2) + 4 * h;
        if (row < m) {
          const double a = av[v];
          const double e = a - (double)acc[v];
          sr += e * e;
          sa += a * a;
        }
      }
    }
  }
#undef NMF_OBJ_LOAD
  sr = wave_sum_f64(sr);
  sa = wave_sum_f64(sa);
  if (lane == 0) {
    const int64_t w = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    partial[2 * w] = sr;
    partial[2 * w + 1] = sa;
  }
}

// Sparse: partial[w] = {sum_i W_i . (A Ht)_i, sum a^2} over the wave's rows.
__global__ __launch_bounds__(256) void k_obj_csr(int64_t m, int k, const int64_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ colidx, const float* __restrict__ vals,
                                                 const float* __restrict__ W, const float* __restrict__ Ht,
                                                 double* __restrict__ partial) {
  __shared__ double s[4][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t gw = (int64_t)blockIdx.x * 4 + wave;
  const int64_t nw = (int64_t)gridDim.x * 4;
  double cross = 0.0, sa = 0.0;
  for (int64_t i = gw; i < m; i += nw) {
    double u = 0.0;
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      const double a = vals[p];
      if (lane < k) u += a * (double)Ht[(int64_t)colidx[p] * k + lane];
      if (lane == 0) sa += a * a;
    }
    if (lane < k) cross += (double)W[i * k + lane] * u;
  }
  cross = wave_sum_f64(cross);
  sa = wave_sum_f64(sa);
  if (lane == 0) {
    s[wave][0] = cross;
    s[wave][1] = sa;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double c = 0.0, q = 0.0;
    for (int w = 0; w < 4; ++w) {
      c += s[w][0];
      q += s[w][1];
    }
    partial[2 * blockIdx.x] = c;
    partial[2 * blockIdx.x + 1] = q;
  }
}

// out = {r, res2, fro2}; mode 0: res2 given; mode 1: res2 = fro2 - 2 cross + gdot
__global__ void k_obj_finish(int mode, const double* __restrict__ sums, const double* __restrict__ fro2_in,
                             const double* __restrict__ cross, const double* __restrict__ gdot,
                             double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double res2, fro2;
  if (mode == 0) {
    res2 = sums[0];
    fro2 = sums[1];
  } else {
    fro2 = fro2_in[0];
    res2 = fro2 - 2.0 * cross[0] + gdot[0];
  }
  out[0] = fro2 > 0.0 ? sqrt(fmax(res2, 0.0) / fro2) : 0.0;
  out[1] = res2;
  out[2] = fro2;
}

// The trace expansion in one block: cross = the sum of the dot kernel's
// per-block partials (fixed order), gdot = <G_W, G_H>_F over kk entries, then
// out = {r, res2, fro2} with res2 = fro2 - 2 cross + gdot; r is also stored
// to *r_copy when that is given.
__global__ void k_trace_finish(int64_t nparts, const double* __restrict__ partial, int64_t kk,
                               const double* __restrict__ GW, const double* __restrict__ GH,
                               const double* __restrict__ fro2_in, double* __restrict__ out,
                               double* __restrict__ r_copy) {
  __shared__ double s[2][kRedThreads];
  double c = 0.0, g = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += kRedThreads) c += partial[i];
  for (int64_t i = threadIdx.x; i < kk; i += kRedThreads) g += GW[i] * GH[i];
  s[0][threadIdx.x] = c;
  s[1][threadIdx.x] = g;
  __syncthreads();
  for (int off = kRedThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s[0][threadIdx.x] += s[0][threadIdx.x + off];
      s[1][threadIdx.x] += s[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double fro2 = fro2_in[0];
    const double res2 = fro2 - 2.0 * s[0][0] + s[1][0];
    const double r = fro2 > 0.0 ? sqrt(fmax(res2, 0.0) / fro2) : 0.0;
    out[0] = r;
    out[1] = res2;
    out[2] = fro2;
    if (r_copy) r_copy[0] = r;
  }
}

__global__ void k_zero_f32(float* __restrict__ p, int64_t rows, int64_t cols, int64_t ld) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e - r * cols;
    p[r * ld + c] = 0.0f;
  }
}

int red_blocks(int64_t len) {
  int64_t b = nmf::cdiv(len, 4 * kRedThreads);
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

struct ObjPlan {
  double* sums = nullptr;     // final {res2, fro2} or {cross, sumsq}
  double* partial = nullptr;  // block partials
  int64_t nparts = 0;
  double* GW = nullptr;
  double* GH = nullptr;
  double* gpart = nullptr;    // gram partials
  int gblocks = 0;
  double* gdot = nullptr;
  double* dpart = nullptr;
  int dblocks = 0;
};

void dense_grid(int64_t m, int64_t n, int64_t* gx, int64_t* gy) {
  *gx = nmf::cdiv(m, 32);
  *gy = nmf::cdiv(nmf::cdiv(n, 32), kObjColTiles);
}

void plan_objective(const nmf_matrix* A, int k, int mode, nmf::Carver& c, ObjPlan* P) {
  P->sums = c.take<double>(4);
  P->gdot = c.take<double>(1);
  if (mode == NMF_OBJ_DIRECT && A->kind == NMF_DENSE) {
    int64_t gx, gy;
    dense_grid(A->m, A->n, &gx, &gy);
    P->nparts = gx * gy;
    P->partial = c.take<double>((size_t)P->nparts * 2);
    return;
  }
  P->GW = c.take<double>((size_t)k * k);
  P->GH = c.take<double>((size_t)k * k);
  const int64_t rows = A->m > A->n ? A->m : A->n;
  nmf::gram_plan(rows, k, c, &P->gpart, &P->gblocks);
  if (mode == NMF_OBJ_DIRECT) {  // CSR
    P->nparts = red_blocks(A->m);
    P->partial = c.take<double>((size_t)P->nparts * 2);
  } else {
    const int64_t len = A->n * k;
    P->dblocks = red_blocks(len);
    P->dpart = c.take<double>((size_t)P->dblocks);
  }
}

int check_matrix(const nmf_matrix* A, const char* who) {
  if (!A) return nmf::fail(NMF_EINVAL, "%s: matrix is null", who);
  if (A->m < 0 || A->n < 0) return nmf::fail(NMF_EINVAL, "%s: negative size", who);
  if (A->kind == NMF_DENSE) {
    if (A->lda < A->n) return nmf::fail(NMF_EINVAL, "%s: lda < n", who);
    if (A->m > 0 && A->n > 0 && !A->A) return nmf::fail(NMF_EINVAL, "%s: A is null", who);
  } else if (A->kind == NMF_CSR) {
    if ((A->m > 0 && !A->rowptr) || (A->n > 0 && !A->rowptr_t))
      return nmf::fail(NMF_EINVAL, "%s: CSR pointers are null", who);
  } else {
    return nmf::fail(NMF_EINVAL, "%s: bad matrix kind %d", who, A->kind);
  }
  return NMF_OK;
}

}  // namespace

namespace nmf {

int zero_f32(float* p, int64_t rows, int64_t cols, int64_t ld, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return NMF_OK;
  int64_t blocks = cdiv(rows * cols, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)blocks), dim3(256), 0, s, p, rows, cols, ld);
  return launch_status("zero fill");
}

int dot_plan(int64_t len, Carver& c, double** partial, int* nblocks) {
  *nblocks = red_blocks(len);
  *partial = c.take<double>((size_t)*nblocks);
  return NMF_OK;
}

int dot_f32_launch(int64_t len, const float* a, const float* b, double* out, double* partial, int nblocks,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_dot<float>, dim3(nblocks), dim3(kRedThreads), 0, s, len, a, b, partial);
  NMF_TRY(launch_status("dot f32"));
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(kRedThreads), 0, s, (int64_t)nblocks, 1, partial, out);
  return launch_status("dot reduce");
}

int trace_finish_launch(int nblocks, const double* partial, int k, const double* GW, const double* GH,
                        const double* fro2, double* out, double* r_copy, hipStream_t s);

// {r, res2, fro2} of the trace expansion, with cross = <a, b> over len FP32
// elements (a = R, b = the factor just solved for) and the Gram inner product
// <G_W, G_H>_F; used by the ANLS driver too.  Two launches.
int trace_objective_launch(int64_t len, const float* a, const float* b, int k, const double* GW, const double* GH,
                           const double* fro2, double* partial, int nblocks, double* out, double* r_copy,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_dot<float>, dim3(nblocks), dim3(kRedThreads), 0, s, len, a, b, partial);
  NMF_TRY(launch_status("objective cross term"));
  return trace_finish_launch(nblocks, partial, k, GW, GH, fro2, out, r_copy, s);
}

// The same with the cross term already summed per block into partial[0 .. nblocks)
// (the BPP kernel does so for the rows it solves).
int trace_finish_launch(int nblocks, const double* partial, int k, const double* GW, const double* GH,
                        const double* fro2, double* out, double* r_copy, hipStream_t s) {
  hipLaunchKernelGGL(k_trace_finish, dim3(1), dim3(kRedThreads), 0, s, (int64_t)nblocks, partial, (int64_t)k * k, GW,
                     GH, fro2, out, r_copy);
  return launch_status("objective finish");
}

}  // namespace nmf

extern "C" int nmf_fro2_workspace_bytes(const nmf_matrix* A, size_t* bytes) {
  if (!bytes) return nmf::fail(NMF_EINVAL, "nmf_fro2_workspace_bytes: bytes is null");
  NMF_TRY(check_matrix(A, "nmf_fro2_workspace_bytes"));
  nmf::Carver c(nullptr, 0);
  c.take<double>(1024);
  *bytes = c.off;
  return NMF_OK;
}

extern "C" int nmf_fro2(const nmf_matrix* A, double* out, void* ws, size_t ws_bytes, void* stream) {
  NMF_TRY(check_matrix(A, "nmf_fro2"));
  if (!out) return nmf::fail(NMF_EINVAL, "nmf_fro2: out is null");
  if (A->kind == NMF_CSR && (A->nnz < 0 || (A->nnz > 0 && !A->vals)))
    return nmf::fail(NMF_EINVAL, "nmf_fro2: bad nnz / vals");
  nmf::Carver c(ws, ws_bytes);
  double* partial = c.take<double>(1024);
  if (!ws || !c.fits()) return nmf::fail(NMF_EWORKSPACE, "nmf_fro2: workspace too small");
  hipStream_t s = nmf::as_stream(stream);
  if (A->kind == NMF_CSR) {
    const int nb = red_blocks(A->nnz);
    return nmf::dot_f32_launch(A->nnz, A->vals, A->vals, out, partial, nb, s);
  }
  const int nb = red_blocks(A->m * A->n);
  hipLaunchKernelGGL(k_sumsq, dim3(nb), dim3(kRedThreads), 0, s, A->m, A->n, A->lda, A->A, partial);
  NMF_TRY(nmf::launch_status("fro2"));
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(kRedThreads), 0, s, (int64_t)nb, 1, partial, out);
  return nmf::launch_status("fro2 reduce");
}

extern "C" int nmf_objective_workspace_bytes(const nmf_matrix* A, int k, int mode, size_t* bytes) {
  if (!bytes) return nmf::fail(NMF_EINVAL, "nmf_objective_workspace_bytes: bytes is null");
  NMF_TRY(check_matrix(A, "nmf_objective_workspace_bytes"));
  if (!nmf::valid_k(k) || (mode != NMF_OBJ_DIRECT && mode != NMF_OBJ_TRACE))
    return nmf::fail(NMF_EINVAL, "nmf_objective_workspace_bytes: bad k or mode");
  nmf::Carver c(nullptr, 0);
  ObjPlan P;
  plan_objective(A, k, mode, c, &P);
  *bytes = c.off;
  return NMF_OK;
}

extern "C" int nmf_objective(const nmf_matrix* A, int k, const float* W, const float* Ht, int mode,
                             const double* G_W, const double* G_H, const float* R_H, double* out, void* ws,
                             size_t ws_bytes, void* stream) {
  NMF_TRY(check_matrix(A, "nmf_objective"));
  if (!nmf::valid_k(k)) return nmf::fail(NMF_EINVAL, "nmf_objective: k=%d outside [1,64]", k);
  if (mode != NMF_OBJ_DIRECT && mode != NMF_OBJ_TRACE) return nmf::fail(NMF_EINVAL, "nmf_objective: bad mode");
  if (!out || (A->m > 0 && !W) || (A->n > 0 && !Ht)) return nmf::fail(NMF_EINVAL, "nmf_objective: null pointer");
  if (mode == NMF_OBJ_TRACE && (!G_W || !G_H || !R_H || !A->fro2))
    return nmf::fail(NMF_EINVAL, "nmf_objective: TRACE needs G_W, G_H, R_H and A->fro2");
  nmf::Carver c(ws, ws_bytes);
  ObjPlan P;
  plan_objective(A, k, mode, c, &P);
  if (!ws || !c.fits()) return nmf::fail(NMF_EWORKSPACE, "nmf_objective: workspace %zu < %zu bytes", ws_bytes, c.off);
  hipStream_t s = nmf::as_stream(stream);
  const int64_t m = A->m, n = A->n;

  if (mode == NMF_OBJ_TRACE) {
    return nmf::trace_objective_launch(n * k, R_H, Ht, k, G_W, G_H, A->fro2, P.dpart, P.dblocks, out, nullptr, s);
  }
  if (A->kind == NMF_DENSE) {
    int64_t gx, gy;
    dense_grid(m, n, &gx, &gy);
    if (gx * gy > 0) {
      const dim3 grid((unsigned)gx, (unsigned)gy);
      if (k <= 32)
        hipLaunchKernelGGL(k_obj_dense<16>, grid, dim3(64), 0, s, m, n, k, A->A, A->lda, W, Ht, P.partial);
      else
        hipLaunchKernelGGL(k_obj_dense<32>, grid, dim3(64), 0, s, m, n, k, A->A, A->lda, W, Ht, P.partial);
      NMF_TRY(nmf::launch_status("objective dense"));
      hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(kRedThreads), 0, s, gx * gy, 2, P.partial, P.sums);
      NMF_TRY(nmf::launch_status("objective reduce"));
    } else {
      return nmf::fail(NMF_EINVAL, "nmf_objective: empty matrix");
    }
    hipLaunchKernelGGL(k_obj_finish, dim3(1), dim3(64), 0, s, 0, P.sums, nullptr, nullptr, nullptr, out);
    return nmf::launch_status("objective finish");
  }
  // CSR direct
  hipLaunchKernelGGL(k_obj_csr, dim3((unsigned)P.nparts), dim3(256), 0, s, m, k, A->rowptr, A->colidx, A->vals, W,
                     Ht, P.partial);
  NMF_TRY(nmf::launch_status("objective csr"));
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(kRedThreads), 0, s, P.nparts, 2, P.partial, P.sums);
  NMF_TRY(nmf::launch_status("objective reduce"));
  NMF_TRY(nmf::gram_launch(m, k, W, k, P.GW, P.gpart, P.gblocks, s));
  NMF_TRY(nmf::gram_launch(n, k, Ht, k, P.GH, P.gpart, P.gblocks, s));
  // gdot into sums[2]; fro2 = sums[1]
  hipLaunchKernelGGL(k_dot<double>, dim3(1), dim3(kRedThreads), 0, s, (int64_t)k * k, P.GW, P.GH, P.gdot);
  NMF_TRY(nmf::launch_status("objective gram dot"));
  hipLaunchKernelGGL(k_obj_finish, dim3(1), dim3(64), 0, s, 1, nullptr, P.sums + 1, P.sums, P.gdot, out);
  return nmf::launch_status("objective finish");
}
