// Gram matrix G = X^T X for a tall FP32 matrix X (rows x k), FP64 result.
//
// The local Gram products of Algorithm 1 / Algorithm 3 (H H^T from Ht, W^T W
// from W).  Work is HBM-streaming over X (rows * k * 4 bytes) with k^2/2 FP64
// multiply-adds per row: each block stages a tile of rows in LDS and every
// thread accumulates a 4 x 4 block of the upper triangle of G for one slice of
// the tile's rows; slices and then blocks are combined in a fixed order, so
// the FP64 result does not depend on scheduling.  Optionally the same pass
// writes X's transposed BF16 split (the Y planes of a BF16x3 product that
// contracts over the rows of X) from the staged tiles, sparing that product
// its own pass over X.
#include <mutex>

#include "batched.h"
#include "nmf_common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kTileRows = 64;
constexpr int kMaxBlocks = 1024;

// Sums X[t*64 .. t*64+64)^T X[...] over the 64-row tiles t = t_begin,
// t_begin + t_step, ... < t_end into out[e * out_stride] (both triangles,
// e = i * k + j).  KW (32 or 64) lanes load one row of a tile: thread t loads
// column t % KW of rows t / KW + step * (256 / KW), so every load of a tile
// has its address from one base and a stride; the next tile is loaded into
// registers while the current one is used.  Starts and ends with a barrier-
// safe use of its LDS, so a persistent loop may call it repeatedly.
template <int KW>
__device__ __forceinline__ void gram_tiles(int64_t rows, int k, const float* __restrict__ X, int64_t ldx,
                                           int64_t t_begin, int64_t t_end, int64_t t_step, double* __restrict__ out,
                                           int64_t out_stride, uint16_t* __restrict__ yth = nullptr,
                                           uint16_t* __restrict__ ytl = nullptr, int64_t ldt = 0, int KP = 0) {
  constexpr int kRowsPerPass = kThreads / KW;
  constexpr int kLoads = kTileRows / kRowsPerPass;
  __shared__ float tile[kTileRows][64 + 4];
  __shared__ double red[kThreads * 4];  // slice reduction scratch (re-used)
  const int kp = (k + 3) & ~3;
  const int kt = kp >> 2;                 // 4-wide column blocks
  const int npairs = kt * (kt + 1) / 2;   // upper-triangular block pairs
  const int slices = kThreads / npairs;   // >= 1 because npairs <= 136
  const int t = threadIdx.x;
  const int slice = t / npairs;
  const int pair = t - slice * npairs;
  const bool active = slice < slices;
  // pair -> (bi, bj) with bi <= bj
  int bi = 0, rem = pair;
  while (rem >= kt - bi) { rem -= kt - bi; ++bi; }
  const int bj = bi + rem;
  const int lc = t % KW, lr = t / KW;
  const bool col_ok = lc < k;

  double acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.0;

  float stage[kLoads];
  int64_t tl = t_begin;
  if (tl < t_end) {
    const int64_t rb = tl * kTileRows + lr;
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int64_t r = rb + u * kRowsPerPass;
      stage[u] = (col_ok && r < rows) ? X[r * ldx + lc] : 0.0f;
    }
  }
  for (; tl < t_end; tl += t_step) {
    const int64_t r0 = tl * kTileRows;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kLoads; ++u) tile[lr + u * kRowsPerPass][lc] = stage[u];
    __syncthreads();
    if (yth) {
      // the tile's transposed BF16 split: plane row i, columns r0 .. r0 + 63
      // (columns past k and rows past the end are staged as zero)
      for (int e = t; e < KP * kTileRows; e += kThreads) {
        const int i = e / kTileRows, rr = e - i * kTileRows;
        const float x = tile[rr][i];
        const uint16_t h = bf16_rne(x);
        yth[i * ldt + r0 + rr] = h;
        ytl[i * ldt + r0 + rr] = bf16_rne(x - bf16_to_f32(h));
      }
    }
    const int64_t tn = tl + t_step;
    if (tn < t_end) {
      const int64_t rb = tn * kTileRows + lr;
#pragma unroll
      for (int u = 0; u < kLoads; ++u) {
        const int64_t r = rb + u * kRowsPerPass;
        stage[u] = (col_ok && r < rows) ? X[r * ldx + lc] : 0.0f;
      }
    }
    if (active) {
      const int nr = (int)((rows - r0) < kTileRows ? (rows - r0) : kTileRows);
      for (int rr = slice; rr < nr; rr += slices) {
        const float4 a = *reinterpret_cast<const float4*>(&tile[rr][4 * bi]);
        const float4 b = *reinterpret_cast<const float4*>(&tile[rr][4 * bj]);
        const double av[4] = {a.x, a.y, a.z, a.w};
        const double bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
        for (int ii = 0; ii < 4; ++ii)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) acc[ii * 4 + jj] += av[ii] * bv[jj];
      }
    }
  }
  // combine slices in order, four entries of the 4 x 4 block at a time
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    __syncthreads();
    if (active) {
#pragma unroll
      for (int e = 0; e < 4; ++e) red[t * 4 + e] = acc[q * 4 + e];
    }
    __syncthreads();
    if (active && slice == 0) {
      double s[4] = {0.0, 0.0, 0.0, 0.0};
      for (int sl = 0; sl < slices; ++sl)
#pragma unroll
        for (int e = 0; e < 4; ++e) s[e] += red[(sl * npairs + pair) * 4 + e];
      const int ii = q;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = 4 * bi + ii, gj = 4 * bj + e;
        if (gi < k && gj < k) {
          out[(int64_t)(gi * k + gj) * out_stride] = s[e];
          out[(int64_t)(gj * k + gi) * out_stride] = s[e];
        }
      }
    }
  }
  __syncthreads();
}

// Partials are stored entry-major, partial[e * nblocks + block], so that the
// reduction reads each entry's partials contiguously.
template <int KW>
__global__ __launch_bounds__(kThreads) void k_gram_partial(int64_t rows, int k, const float* __restrict__ X,
                                                           int64_t ldx, double* __restrict__ partial,
                                                           uint16_t* __restrict__ yth, uint16_t* __restrict__ ytl,
                                                           int64_t ldt, int KP) {
  const int64_t ntiles = (rows + kTileRows - 1) / kTileRows;
  gram_tiles<KW>(rows, k, X, ldx, blockIdx.x, ntiles, gridDim.x, partial + blockIdx.x, gridDim.x, yth, ytl, ldt, KP);
}

// Grouped form: item i sums its own tile range into its own k x k partial.
__global__ __launch_bounds__(kThreads) void k_gram_grouped(const nmf::GramItem* __restrict__ items, int64_t n) {
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const nmf::GramItem it = items[i];
    gram_tiles<64>(it.rows, it.k, it.X, it.ldx, it.tile0, it.tile0 + it.ntiles, 1, it.partial, 1);
  }
}

// Grouped reduction: G[e] = sum over the instance's item partials in order.
__global__ __launch_bounds__(256) void k_gram_reduce_grouped(const nmf::GramReduceItem* __restrict__ items,
                                                             int64_t n) {
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const nmf::GramReduceItem it = items[i];
    const int64_t e = it.e0 + threadIdx.x;
    const int64_t kk = (int64_t)it.k * it.k;
    if (e < kk) {
      double s = 0.0;
      for (int sl = 0; sl < it.nslots; ++sl) s += it.partial[sl * kk + e];
      it.G[e] = s;
    }
  }
}

// One wavefront per entry of G: lane l sums partials l, l + 64, ... in order,
// then the 64 lane sums are combined by a fixed butterfly.
__global__ __launch_bounds__(256) void k_gram_reduce(int k, int nblocks, const double* __restrict__ partial,
                                                     double* __restrict__ G) {
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= k * k) return;
  const double* p = partial + (int64_t)e * nblocks;
  double s = 0.0;
  for (int b = lane; b < nblocks; b += 64) s += p[b];
  s = wave_sum_f64(s);
  if (lane == 0) G[e] = s;
}

int gram_blocks(int64_t rows) {
  const int64_t tiles = (rows + kTileRows - 1) / kTileRows;
  return (int)(tiles < 1 ? 1 : (tiles > kMaxBlocks ? kMaxBlocks : tiles));
}

}  // namespace

namespace nmf {

int gram_plan(int64_t rows, int k, Carver& c, double** partial, int* nblocks) {
  *nblocks = gram_blocks(rows);
  *partial = c.take<double>((size_t)(*nblocks) * k * k);
  return NMF_OK;
}

int gram_launch(int64_t rows, int k, const float* X, int64_t ldx, double* G, double* partial, int nblocks,
                hipStream_t s, uint16_t* yth, uint16_t* ytl, int64_t ldt, int KP) {
  // the split needs every 64-row tile of the planes (ldt of them) and
  // KP <= the staged width (32 or 64)
  if (yth && (!ytl || ldt < cdiv(rows, kTileRows) * kTileRows || ldt % kTileRows || KP < k ||
              KP > (k <= 32 ? 32 : 64)))
    return fail(NMF_EINVAL, "gram: bad split planes");
  if (k <= 32)
    hipLaunchKernelGGL(k_gram_partial<32>, dim3(nblocks), dim3(kThreads), 0, s, rows, k, X, ldx, partial, yth, ytl,
                       ldt, KP);
  else
    hipLaunchKernelGGL(k_gram_partial<64>, dim3(nblocks), dim3(kThreads), 0, s, rows, k, X, ldx, partial, yth, ytl,
                       ldt, KP);
  NMF_TRY(launch_status("gram partial"));
  hipLaunchKernelGGL(k_gram_reduce, dim3((k * k + 3) / 4), dim3(256), 0, s, k, nblocks, partial, G);
  return launch_status("gram reduce");
}

int gram_grouped_launch(const GramItem* items, int64_t n, int grid, hipStream_t s) {
  if (n == 0) return NMF_OK;
  hipLaunchKernelGGL(k_gram_grouped, dim3((unsigned)grid), dim3(kThreads), 0, s, items, n);
  return launch_status("gram (grouped)");
}

int gram_reduce_grouped_launch(const GramReduceItem* items, int64_t n, int grid, hipStream_t s) {
  if (n == 0) return NMF_OK;
  hipLaunchKernelGGL(k_gram_reduce_grouped, dim3((unsigned)grid), dim3(256), 0, s, items, n);
  return launch_status("gram reduce (grouped)");
}

int gram_grouped_occupancy(int which, int* per_cu) {
  hipError_t e = hipErrorInvalidValue;
  if (which == kCapGram) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_gram_grouped, kThreads, 0);
  return e == hipSuccess ? NMF_OK : NMF_EHIP;
}

}  // namespace nmf

extern "C" int nmf_gram_workspace_bytes(int64_t rows, int k, size_t* bytes) {
  if (!bytes || rows < 0 || !nmf::valid_k(k)) return nmf::fail(NMF_EINVAL, "nmf_gram_workspace_bytes: bad arguments");
  nmf::Carver c(nullptr, 0);
  double* p;
  int nb;
  nmf::gram_plan(rows, k, c, &p, &nb);
  *bytes = c.off;
  return NMF_OK;
}

extern "C" int nmf_gram(int64_t rows, int k, const float* X, int64_t ldx, double* G, void* ws, size_t ws_bytes,
                        void* stream) {
  if (!nmf::valid_k(k)) return nmf::fail(NMF_EINVAL, "nmf_gram: k=%d outside [1,64]", k);
  if (rows < 0 || (rows > 0 && ldx < k)) return nmf::fail(NMF_EINVAL, "nmf_gram: rows=%lld ldx=%lld", (long long)rows, (long long)ldx);
  if (!G || (rows > 0 && !X)) return nmf::fail(NMF_EINVAL, "nmf_gram: null pointer");
  nmf::Carver c(ws, ws_bytes);
  double* partial;
  int nb;
  nmf::gram_plan(rows, k, c, &partial, &nb);
  if (!c.fits() || !ws) return nmf::fail(NMF_EWORKSPACE, "nmf_gram: workspace %zu < %zu bytes", ws_bytes, c.off);
  return nmf::gram_launch(rows, k, X, ldx, G, partial, nb, nmf::as_stream(stream));
}

// ---- the variant without a workspace ------------------------------------------
// The block partials of nmf_gram_noalloc live in this file-scope device array
// instead of a caller workspace: kMaxBlocks partials of a 64 x 64 matrix
// (32 MiB), enough for every valid (rows, k).  Each device holds its own copy
// for the life of the process.  In host code `scratch` only names the array:
// its device address comes from hipGetSymbolAddress, taken once per device.
static __device__ __align__(256) double scratch[NMF_GRAM_NOALLOC_SCRATCH_BYTES / sizeof(double)];
static_assert(NMF_GRAM_NOALLOC_SCRATCH_BYTES == (size_t)kMaxBlocks * 64 * 64 * sizeof(double),
              "the scratch holds kMaxBlocks partials at k = 64");

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on its first use).
int scratch_address(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return nmf::fail(NMF_EHIP, "nmf_gram_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return nmf::fail(NMF_EUNSUPPORTED, "nmf_gram_noalloc: device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return nmf::fail(NMF_EHIP, "nmf_gram_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return NMF_OK;
}

}  // namespace

extern "C" int nmf_gram_noalloc(int64_t rows, int k, const float* X, int64_t ldx, double* G, void* stream) {
  if (!nmf::valid_k(k)) return nmf::fail(NMF_EINVAL, "nmf_gram_noalloc: k=%d outside [1,64]", k);
  if (rows < 0 || (rows > 0 && ldx < k))
    return nmf::fail(NMF_EINVAL, "nmf_gram_noalloc: rows=%lld ldx=%lld", (long long)rows, (long long)ldx);
  if (!G || (rows > 0 && !X)) return nmf::fail(NMF_EINVAL, "nmf_gram_noalloc: null pointer");
  const int nb = gram_blocks(rows);
  const size_t need = (size_t)nb * k * k * sizeof(double);
  if (need > NMF_GRAM_NOALLOC_SCRATCH_BYTES)
    return nmf::fail(NMF_EINVAL, "nmf_gram_noalloc: %zu bytes of partials exceed the %zu-byte scratch", need,
                     (size_t)NMF_GRAM_NOALLOC_SCRATCH_BYTES);
  double* partial = nullptr;
  NMF_TRY(scratch_address(&partial));
  // every partial slot the reduction reads is written by the partial kernel
  // first, so nothing left by an earlier call is read
  return nmf::gram_launch(rows, k, X, ldx, G, partial, nb, nmf::as_stream(stream));
}
