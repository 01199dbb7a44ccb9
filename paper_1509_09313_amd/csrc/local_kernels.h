// Kernels of the other local NLS solvers of Algorithm 1: multiplicative updates (MU,
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
// One lane per row, one wavefront per 64-row tile.  G is the same for every
// lane, so it is read through the scalar cache into SGPRs (a v_fma_f64 takes
// one SGPR-pair operand): staging it in LDS would return 64 copies of every
// element to the VGPRs and make the LDS return path the bound.  The kernel is
// instantiated per k so that every offset into G is an immediate, rows of G
// load as 8-double scalar bursts, and the row x lives in k FP64 registers with
// static indices.  G is symmetric (a Gram matrix), so column l of G is read
// as row l.  The rows of X and R pass through a per-wave LDS tile (odd pitch,
// conflict-free) so that global loads and stores are coalesced.  The cost is
// 2 k^2 FP64 flops per row, as the paper counts it (2 (m + n) k^2 per
// iteration), and 12 k bytes of HBM traffic per row (R read, X read and
// written).
#pragma once

#include <atomic>
#include <cstdint>
#include <utility>

#include "nmf_common.h"

namespace nmf {
namespace local {

typedef const __attribute__((address_space(4))) double* GPtr;

constexpr int kLocalBlocks = 4096;

// f(integral_constant<int, 0>) ... f(integral_constant<int, N - 1>): the
// outer sweeps are written out at compile time, so every index into the row
// registers is a constant however large k is (a loop over the k^2 body would
// exceed the unroller's size limit from k = 48, and a loop variable indexing
// x puts x in scratch memory).  The inner loops stay small enough to unroll.
template <typename F, int... I>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}

template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// A 64-row tile of a row-major FP32 matrix (k = K columns, leading dimension
// ld) to and from LDS (pitch K | 1).  Lanes cover PW = the power of two >= K
// columns of 64 / PW rows per instruction, so each instruction reads or
// writes whole rows (coalesced) from one scalar row base.  For a full tile
// all loads are issued before the first is used (one memory round trip); the
// lanes past column K-1 load column K-1 again and drop it, so no load leaves
// the row.  The last, partial tile takes a guarded loop.
template <int K>
struct TileMap {
  static constexpr int PW = K <= 1 ? 1 : K <= 2 ? 2 : K <= 4 ? 4 : K <= 8 ? 8 : K <= 16 ? 16 : K <= 32 ? 32 : 64;
  static constexpr int RPI = 64 / PW;  // rows per instruction
  static constexpr int NI = 64 / RPI;  // instructions per tile
  static constexpr int P = K | 1;
};

template <int K>
__device__ __forceinline__ void stage_in(float* __restrict__ T, const float* __restrict__ src, int64_t ld, int64_t r0,
                                         int nr, int lane) {
  using M = TileMap<K>;
  const int sub = lane / M::PW, c = lane % M::PW, cc = c < K ? c : K - 1;
  const float* p = src + (r0 + sub) * ld + cc;
  float* t = T + sub * M::P + c;
  if (nr == 64) {
    float v[M::NI];
#pragma unroll
    for (int i = 0; i < M::NI; ++i) v[i] = p[(int64_t)(i * M::RPI) * ld];
    if (c < K) {
#pragma unroll
      for (int i = 0; i < M::NI; ++i) t[i * M::RPI * M::P] = v[i];
    }
  } else {
#pragma unroll 4
    for (int i = 0; i < M::NI; ++i) {
      const int row = i * M::RPI + sub;
      if (c < K) t[i * M::RPI * M::P] = row < nr ? p[(int64_t)(i * M::RPI) * ld] : 0.0f;
    }
  }
}

template <int K>
__device__ __forceinline__ void stage_out(const float* __restrict__ T, float* __restrict__ dst, int64_t ld,
                                          int64_t r0, int nr, int lane) {
  using M = TileMap<K>;
  const int sub = lane / M::PW, c = lane % M::PW;
  if (c >= K) return;
  float* p = dst + (r0 + sub) * ld + c;
  const float* t = T + sub * M::P + c;
  if (nr == 64) {
#pragma unroll
    for (int i = 0; i < M::NI; ++i) p[(int64_t)(i * M::RPI) * ld] = t[i * M::RPI * M::P];
  } else {
#pragma unroll 4
    for (int i = 0; i < M::NI; ++i)
      if (i * M::RPI + sub < nr) p[(int64_t)(i * M::RPI) * ld] = t[i * M::RPI * M::P];
  }
}

template <int K, int SOLVER>
__global__ __launch_bounds__(64) void k_local(int64_t rows, const double* __restrict__ Gin,
                                              const float* __restrict__ R, int64_t ldr, float* __restrict__ X,
                                              int64_t ldx) {
  constexpr int P = K | 1;  // tile pitch in floats
  __shared__ float T[64 * P];
  const GPtr G0 = (GPtr)Gin;
  const int lane = threadIdx.x;

  double dmax = 0.0;
#pragma unroll
  for (int q = 0; q < K; ++q) dmax = fmax(dmax, G0[q * K + q]);
  const double thr = 1e-14 * dmax;
  // lane j < K holds 1 / G_jj (0 marks a pinned index); the sweeps fetch it
  // with readlane, keeping LDS (and its wait counter, shared with the scalar
  // loads) out of them
  double inv_mine = 0.0;
  if (lane < K) {
    const double g = Gin[lane * K + lane];
    inv_mine = g > thr ? 1.0 / g : 0.0;
  }
  const int inv_lo = __double2loint(inv_mine), inv_hi = __double2hiint(inv_mine);

  const int64_t ntiles = (rows + 63) / 64;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * 64;
    const int nr = rows - r0 < 64 ? (int)(rows - r0) : 64;
    const float* Tl = T + lane * P;
    double x[K];
    __syncthreads();
    stage_in<K>(T, X, ldx, r0, nr, lane);
    __syncthreads();
    static_for<K>([&](auto C) __attribute__((always_inline)) { x[C] = (double)Tl[C]; });
    __syncthreads();
    stage_in<K>(T, R, ldr, r0, nr, lane);
    __syncthreads();
    float* Tw = T + lane * P;
    // opaque per tile: keeps the scalar loads of G inside the loop (hoisted,
    // k^2 values would not fit in SGPRs)
    GPtr G = G0;
    asm volatile("" : "+s"(G));
    if constexpr (SOLVER == NMF_SOLVER_HALS) {
      static_for<K>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = I;
        double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < K; ++q) {
          if (q != i) a[q & 3] = fma(G[i * K + q], x[q], a[q & 3]);
          // at most one 8-double burst of G ahead of its use: scheduling the
          // loads of later rows early runs out of SGPRs
          if ((q & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        const double s = (double)Tl[i] - ((a[0] + a[1]) + (a[2] + a[3]));
        const double inv = __hiloint2double(__builtin_amdgcn_readlane(inv_hi, i),
                                            __builtin_amdgcn_readlane(inv_lo, i));
        x[i] = fmax(s, 0.0) * inv;
      });
      static_for<K>([&](auto C) __attribute__((always_inline)) { Tw[C] = (float)x[C]; });
    } else {
      static_for<K>([&](auto J) __attribute__((always_inline)) {
        constexpr int j = J;
        double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < K; ++q) a[q & 3] = fma(G[j * K + q], x[q], a[q & 3]);
        const double d = (a[0] + a[1]) + (a[2] + a[3]);
        const double rj = (double)Tl[j];
        const double inv = __hiloint2double(__builtin_amdgcn_readlane(inv_hi, j),
                                            __builtin_amdgcn_readlane(inv_lo, j));
        // 1 / d from the hardware estimate and two Newton steps y <- y (2 - d y)
        // (each doubles the correct bits), in place of the division sequence
        double y = __builtin_amdgcn_rcp(d);
        y = fma(y, fma(-d, y, 1.0), y);
        y = fma(y, fma(-d, y, 1.0), y);
        Tw[j] = (inv > 0.0 && d > 0.0) ? (float)(x[j] * rj * y) : 0.0f;
      });
    }
    __syncthreads();
    stage_out<K>(T, X, ldx, r0, nr, lane);
  }
}

// Workgroups of k_local<K, SOLVER> resident on the whole device at once
// (occupancy calculator; kLocalBlocks if it cannot be queried), per device.
template <int K, int SOLVER>
int64_t resident_blocks() {
  constexpr int kDevices = 64;
  static std::atomic<int> cache[kDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevices) return kLocalBlocks;
  int cap = cache[dev].load(std::memory_order_relaxed);
  if (cap > 0) return cap;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_local<K, SOLVER>, 64, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu <= 0 ||
      cus <= 0) {
    (void)hipGetLastError();
    return kLocalBlocks;
  }
  cap = per_cu * cus;
  cache[dev].store(cap, std::memory_order_relaxed);
  return cap;
}

// One workgroup (a wavefront) per 64-row tile, at most as many as are
// resident at once (a persistent walk: the per-workgroup set-up of the
// pinned-index reciprocals is amortised over several tiles).
template <int K, int SOLVER>
void launch_solver(int64_t rows, const double* G, const float* R, int64_t ldr, float* X, int64_t ldx,
                   hipStream_t s) {
  int64_t blocks = nmf::cdiv(rows, 64);
  const int64_t cap = resident_blocks<K, SOLVER>();
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL((k_local<K, SOLVER>), dim3((unsigned)blocks), dim3(64), 0, s, rows, G, R, ldr, X, ldx);
}

template <int K>
void launch_k(int solver, int64_t rows, const double* G, const float* R, int64_t ldr, float* X, int64_t ldx,
              hipStream_t s) {
  if (solver == NMF_SOLVER_HALS)
    launch_solver<K, NMF_SOLVER_HALS>(rows, G, R, ldr, X, ldx, s);
  else
    launch_solver<K, NMF_SOLVER_MU>(rows, G, R, ldr, X, ldx, s);
}

typedef void (*LaunchFn)(int, int64_t, const double*, const float*, int64_t, float*, int64_t, hipStream_t);

// t[K - 1] = launch_k<K> for K in [LO, LO + sizeof...(I))
template <int LO, int... I>
void fill(LaunchFn* t, std::integer_sequence<int, I...>) {
  ((t[LO + I - 1] = &launch_k<LO + I>), ...);
}

// The instantiations are spread over three sources (k <= 44, 45..56,
// 57..64: about equal sums of k^2, the compile cost) built in parallel.
void fill_k1_44(LaunchFn* t);
void fill_k45_56(LaunchFn* t);
void fill_k57_64(LaunchFn* t);

}  // namespace local
}  // namespace nmf
