// Split-precision (BF16x3) right-hand sides.
//
// x = hi + lo with hi = bf16_rne(x) and lo = bf16_rne(x - hi) (x - hi is
// exact in FP32), and R = A_hi Y_hi + A_hi Y_lo + A_lo Y_hi with FP32
// accumulation: the lo*lo term (relative size 2^-16 per operand pair) is
// dropped.  Bytes per entry of A stay 4 (two BF16 planes), so the product is
// HBM-bound where the FP32 MFMA form is compute-bound.
#include <atomic>

#include "batched.h"
#include "nmf_common.h"

namespace {

// Padded BF16 operand: B (rows x cols) as two row-major planes of Rp x Cp
// BF16 values, Rp = rows rounded up to kTR, Cp = cols rounded up to kTC, zero
// in the padding: the hi plane, then the lo plane.  Row-major rows keep the 8
// rows a wavefront loads per instruction spread over memory channels.
constexpr int kTR = 128;
constexpr int kTC = 64;

// B = X (transpose 0) or X^T (transpose 1); one block per 64 x 64 block of B.
__global__ __launch_bounds__(256) void k_split_planes(int64_t rows, int64_t cols, const float* __restrict__ X,
                                                      int64_t ldx, int transpose, int64_t Rp, int64_t Cp,
                                                      uint16_t* __restrict__ out) {
  __shared__ float tile[64][65];
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;  // block origin in B
  const int64_t brows = transpose ? cols : rows, bcols = transpose ? rows : cols;
  uint16_t* hi = out;
  uint16_t* lo = out + Rp * Cp;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  if (!transpose) {
    for (int ii = ty; ii < 64; ii += 4) {
      const int64_t i = i0 + ii, j = j0 + tx;
      const float x = (i < brows && j < bcols) ? X[i * ldx + j] : 0.0f;
      const uint16_t h = bf16_rne(x);
      hi[i * Cp + j] = h;
      lo[i * Cp + j] = bf16_rne(x - bf16_to_f32(h));
    }
  } else {
    for (int jj = ty; jj < 64; jj += 4) {  // X row j0 + jj, columns i0 + tx
      const int64_t j = j0 + jj, i = i0 + tx;
      tile[jj][tx] = (i < brows && j < bcols) ? X[j * ldx + i] : 0.0f;
    }
    __syncthreads();
    for (int ii = ty; ii < 64; ii += 4) {
      const int64_t i = i0 + ii, j = j0 + tx;
      const float x = tile[tx][ii];
      const uint16_t h = bf16_rne(x);
      hi[i * Cp + j] = h;
      lo[i * Cp + j] = bf16_rne(x - bf16_to_f32(h));
    }
  }
}

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

__device__ __forceinline__ v16f mfma_bf16(v8bf a, v8bf b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Y (K x k FP32, ld ldy) -> transposed BF16 planes Yth, Ytl (KP x ldt), rows
// i >= k and columns >= K zero.  One block per 64 rows of Y (from row K0).
__device__ __forceinline__ void split_y_chunk(int64_t K, int k, int KP, const float* __restrict__ Y, int64_t ldy,
                                              uint16_t* __restrict__ Yth, uint16_t* __restrict__ Ytl, int64_t ldt,
                                              int64_t K0) {
  __shared__ float tile[64][65];
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int kk = e / 64, c = e - kk * 64;
    tile[kk][c] = (K0 + kk < K && c < k) ? Y[(K0 + kk) * ldy + c] : 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < KP * 64; e += 256) {
    const int i = e / 64, kk = e - i * 64;
    const int64_t col = K0 + kk;
    if (col < ldt) {
      const float x = tile[kk][i];
      const uint16_t h = bf16_rne(x);
      Yth[i * ldt + col] = h;
      Ytl[i * ldt + col] = bf16_rne(x - bf16_to_f32(h));
    }
  }
}

__global__ __launch_bounds__(256) void k_split_y(int64_t K, int k, int KP, const float* __restrict__ Y, int64_t ldy,
                                                 uint16_t* __restrict__ Yth, uint16_t* __restrict__ Ytl, int64_t ldt) {
  split_y_chunk(K, k, KP, Y, ldy, Yth, Ytl, ldt, (int64_t)blockIdx.x * 64);
}

__global__ __launch_bounds__(256) void k_split_y_grouped(const nmf::SplitYItem* __restrict__ items, int64_t n) {
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const nmf::SplitYItem it = items[i];
    split_y_chunk(it.K, it.k, it.KP, it.Y, it.ldy, it.Yth, it.Ytl, it.ldt, it.K0);
  }
}

constexpr int kBTM = kTR;          // rows of B per block (4 waves x 32)
constexpr int kBTK = kTC;          // contraction chunk (BF16 elements)
constexpr int kBPitch = kBTK + 8;  // LDS pitch in uint16 (144 bytes: conflict-free 16-byte reads)

// One tile of 32 NW rows (NW wavefronts of 64 threads: 128 rows for the
// single-product kernels, 64 or 128 for the grouped ones) of R = B * Y over
// the 64-column chunks [kc0, kc1) of the contraction, written to out (ld
// ldp); B in the padded BF16 form (planes Rp x Cp), Y as transposed BF16
// planes (KP x ldt, ldt = Cp, zero past K).  Wave w holds D_t[i][j] =
// R[row0 + 32w + j][32t + i] and accumulates three MFMAs per 16-wide K step
// (Yhi Bhi + Ylo Bhi + Yhi Blo).  Barrier-safe for repeated calls from a
// persistent loop.
typedef unsigned int v4u_t __attribute__((ext_vector_type(4)));

// The planes of A are read once per launch: non-temporal loads stream them
// without displacing the reused operand from the caches, and reach a higher
// read bandwidth than plain loads on this part.
__device__ __forceinline__ uint4 load_stream(const uint16_t* p) {
  const v4u_t v = __builtin_nontemporal_load(reinterpret_cast<const v4u_t*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

template <int NT, int NW = 4>
__device__ __forceinline__ void bf16x3_tile(int64_t rows, int k, const uint16_t* __restrict__ B, int64_t Rp,
                                            int64_t nkc, const uint16_t* __restrict__ Yth,
                                            const uint16_t* __restrict__ Ytl, int64_t ldt, float* __restrict__ out,
                                            int64_t ldp, int64_t row0, int64_t kc0, int64_t kc1) {
  constexpr int KP = 32 * NT;
  constexpr int TM = 32 * NW;     // rows of the tile
  constexpr int NTH = 64 * NW;    // threads
  constexpr int RPP = NTH / 8;    // rows one load pass covers (8 threads per 128-byte row)
  constexpr int YL = KP / RPP;    // load passes over each Y plane
  static_assert(TM == 4 * RPP && YL >= 1 && YL <= 4, "tile staging layout");
  __shared__ __align__(16) uint16_t Bs[2][TM * kBPitch];
  __shared__ __align__(16) uint16_t Ys[2][KP * kBPitch];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int j = lane & 31, h = lane >> 5;
  const int64_t Cp = nkc * kTC;
  const uint16_t* Bh = B + row0 * Cp;

  v16f acc[NT];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) acc[tt] = v16f{};

  // A chunk in flight: the staging registers of one 64-column chunk (explicit
  // members: no arrays, which keeps them out of scratch).
  struct Stage {
    uint4 bh0, bh1, bh2, bh3, bl0, bl1, bl2, bl3, yh0, yl0, yh1, yl1, yh2, yl2, yh3, yl3;
  };
  auto load = [&](Stage& S, int64_t kc) __attribute__((always_inline)) {
    const int64_t c0 = kc * kTC;
    const uint16_t* ph = Bh + (int64_t)(t >> 3) * Cp + c0 + 8 * (t & 7);
    const uint16_t* pl = ph + Rp * Cp;
    const int64_t rs = RPP * Cp;
    S.bh0 = load_stream(ph);
    S.bh1 = load_stream(ph + rs);
    S.bh2 = load_stream(ph + 2 * rs);
    S.bh3 = load_stream(ph + 3 * rs);
    S.bl0 = load_stream(pl);
    S.bl1 = load_stream(pl + rs);
    S.bl2 = load_stream(pl + 2 * rs);
    S.bl3 = load_stream(pl + 3 * rs);
    const int64_t yo = (int64_t)(t >> 3) * ldt + c0 + 8 * (t & 7);
    S.yh0 = *reinterpret_cast<const uint4*>(Yth + yo);
    S.yl0 = *reinterpret_cast<const uint4*>(Ytl + yo);
    if (YL > 1) {
      S.yh1 = *reinterpret_cast<const uint4*>(Yth + yo + RPP * ldt);
      S.yl1 = *reinterpret_cast<const uint4*>(Ytl + yo + RPP * ldt);
    }
    if (YL > 2) {
      S.yh2 = *reinterpret_cast<const uint4*>(Yth + yo + 2 * RPP * ldt);
      S.yl2 = *reinterpret_cast<const uint4*>(Ytl + yo + 2 * RPP * ldt);
      S.yh3 = *reinterpret_cast<const uint4*>(Yth + yo + 3 * RPP * ldt);
      S.yl3 = *reinterpret_cast<const uint4*>(Ytl + yo + 3 * RPP * ldt);
    }
  };
  const int so = (t >> 3) * kBPitch + 8 * (t & 7);
  auto store = [&](const Stage& S) __attribute__((always_inline)) {
    *reinterpret_cast<uint4*>(&Bs[0][so]) = S.bh0;
    *reinterpret_cast<uint4*>(&Bs[0][so + RPP * kBPitch]) = S.bh1;
    *reinterpret_cast<uint4*>(&Bs[0][so + 2 * RPP * kBPitch]) = S.bh2;
    *reinterpret_cast<uint4*>(&Bs[0][so + 3 * RPP * kBPitch]) = S.bh3;
    *reinterpret_cast<uint4*>(&Bs[1][so]) = S.bl0;
    *reinterpret_cast<uint4*>(&Bs[1][so + RPP * kBPitch]) = S.bl1;
    *reinterpret_cast<uint4*>(&Bs[1][so + 2 * RPP * kBPitch]) = S.bl2;
    *reinterpret_cast<uint4*>(&Bs[1][so + 3 * RPP * kBPitch]) = S.bl3;
    *reinterpret_cast<uint4*>(&Ys[0][so]) = S.yh0;
    *reinterpret_cast<uint4*>(&Ys[1][so]) = S.yl0;
    if (YL > 1) {
      *reinterpret_cast<uint4*>(&Ys[0][so + RPP * kBPitch]) = S.yh1;
      *reinterpret_cast<uint4*>(&Ys[1][so + RPP * kBPitch]) = S.yl1;
    }
    if (YL > 2) {
      *reinterpret_cast<uint4*>(&Ys[0][so + 2 * RPP * kBPitch]) = S.yh2;
      *reinterpret_cast<uint4*>(&Ys[1][so + 2 * RPP * kBPitch]) = S.yl2;
      *reinterpret_cast<uint4*>(&Ys[0][so + 3 * RPP * kBPitch]) = S.yh3;
      *reinterpret_cast<uint4*>(&Ys[1][so + 3 * RPP * kBPitch]) = S.yl3;
    }
  };
  auto compute = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < kBTK / 16; ++s) {
      const int off = 16 * s + 8 * h;
      const v8bf bh = *reinterpret_cast<const v8bf*>(&Bs[0][(32 * w + j) * kBPitch + off]);
      const v8bf bl = *reinterpret_cast<const v8bf*>(&Bs[1][(32 * w + j) * kBPitch + off]);
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
        const v8bf yh = *reinterpret_cast<const v8bf*>(&Ys[0][(32 * tt + j) * kBPitch + off]);
        const v8bf yl = *reinterpret_cast<const v8bf*>(&Ys[1][(32 * tt + j) * kBPitch + off]);
        acc[tt] = mfma_bf16(yh, bh, acc[tt]);
        acc[tt] = mfma_bf16(yl, bh, acc[tt]);
        acc[tt] = mfma_bf16(yh, bl, acc[tt]);
      }
    }
  };
  // the 64-row form keeps one chunk in flight (two staging sets take it past
  // 256 VGPRs)
  if (NW == 4 && kc1 - kc0 >= 4) {
    // Two chunks in flight: the loads of chunk c + 2 are issued while chunk
    // c + 1 is still arriving.  The main loop's loads are unconditional, so
    // each wait is for the older set only; the last two or three chunks
    // follow in straight-line code.
    Stage A, B;
    load(A, kc0);
    __builtin_amdgcn_sched_barrier(0);  // same issue order as in the loop
    load(B, kc0 + 1);
    int64_t kc = kc0;
    for (; kc + 3 < kc1; kc += 2) {
      __syncthreads();
      store(A);
      __syncthreads();
      load(A, kc + 2);
      compute();
      __syncthreads();
      store(B);
      __syncthreads();
      load(B, kc + 3);
      compute();
    }
    const bool three = kc + 2 < kc1;
    __syncthreads();
    store(A);
    __syncthreads();
    if (three) load(A, kc + 2);
    compute();
    __syncthreads();
    store(B);
    __syncthreads();
    compute();
    if (three) {
      __syncthreads();
      store(A);
      __syncthreads();
      compute();
    }
  } else {
    Stage A;
    if (kc0 < kc1) load(A, kc0);
    for (int64_t kc = kc0; kc < kc1; ++kc) {
      __syncthreads();
      store(A);
      __syncthreads();
      if (kc + 1 < kc1) load(A, kc + 1);
      compute();
    }
  }
  // The finished tile goes out through LDS (the B staging buffer, idle now)
  // so that the stores cover whole rows (straight from the MFMA layout each
  // store instruction touches 32 rows with 8 bytes each), and the stores are
  // non-temporal: written while A streams in, ordinary stores slow the read
  // stream more (10^6 x 2400, k = 30: 1.715 ms scattered, 1.688 through LDS,
  // 1.620 through LDS non-temporal; 1.417 with no output at all).
  constexpr int OP = KP + 1;  // odd pitch: conflict-free column writes
  static_assert(TM * OP * sizeof(float) <= sizeof(Bs), "output tile exceeds the staging buffer");
  float* O = reinterpret_cast<float*>(&Bs[0][0]);
  __syncthreads();
#pragma unroll
  for (int tt = 0; tt < NT; ++tt)
#pragma unroll
    for (int v = 0; v < 16; ++v) O[(32 * w + j) * OP + 32 * tt + (v & 3) + 8 * (v >> 2) + 4 * h] = acc[tt][v];
  __syncthreads();
  const int nr = rows - row0 < TM ? (int)(rows - row0) : TM;
  for (int e = t; e < nr * k; e += NTH) {
    const int row = e / k, c = e - row * k;
    __builtin_nontemporal_store(O[row * OP + c], &out[(row0 + row) * ldp + c]);
  }
  __syncthreads();
}

// R (rows x k) = B (rows x K) * Y (K x k) with B in the padded BF16 form
// (planes Rp x Cp) and Y as transposed BF16 planes (KP x ldt, ldt = Cp, zero
// past K).  The grid is one-dimensional and XCD-aware: workgroups are
// dispatched to the 8 XCDs round-robin, so launch index L runs on XCD L % 8;
// L is remapped to the logical tile (L % 8) * (grid / 8) + L / 8, which gives
// every XCD a contiguous range of logical tiles, row tile fastest.  All row
// tiles of one K-range then run on the same XCD and share that range of Y in
// its L2.  The K index of a logical tile selects a range of 64-column chunks
// (split-K); its partial goes to P + split * split_stride.  SIDE
// (NMF_SIDE_W / NMF_SIDE_H) does not change the code; it only gives the two
// products distinct kernel names in traces.
template <int NT, int SIDE>
__global__ __launch_bounds__(256) void k_rhs_bf16x3(int64_t rows, int k, const uint16_t* __restrict__ B, int64_t Rp,
                                                    int64_t nkc,
                                                    const uint16_t* __restrict__ Yth, const uint16_t* __restrict__ Ytl,
                                                    int64_t ldt, float* __restrict__ P, int64_t ldp, int64_t kc_per_split,
                                                    int64_t split_stride, int64_t ntiles, int64_t nsplit) {
  const int64_t per_xcd = gridDim.x / 8;
  const int64_t lid = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (lid >= ntiles * nsplit) return;
  const int64_t bx = lid % ntiles, by = lid / ntiles;
  const int64_t kc0 = by * kc_per_split;
  const int64_t kc1 = (kc0 + kc_per_split < nkc) ? kc0 + kc_per_split : nkc;
  bf16x3_tile<NT>(rows, k, B, Rp, nkc, Yth, Ytl, ldt, P + by * split_stride, ldp, bx * kBTM, kc0, kc1);
}

// Grouped form: a persistent walk over tiles of many products, 128 rows per
// tile (four wavefronts) ...
template <int NT>
__global__ __launch_bounds__(256) void k_rhs_bf16x3_grouped(const nmf::Bf16Item* __restrict__ items, int64_t n) {
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const nmf::Bf16Item it = items[i];
    bf16x3_tile<NT, 4>(it.rows, it.k, it.B, it.Rp, it.nkc, it.Yth, it.Ytl, it.ldt, it.out, it.ldp, it.row0, it.kc0,
                       it.kc1);
  }
}

// ... or 64 rows (two wavefronts, one chunk in flight).
template <int NT>
__global__ __launch_bounds__(128) void k_rhs_bf16x3_grouped64(
    const nmf::Bf16Item* __restrict__ items, int64_t n) {
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const nmf::Bf16Item it = items[i];
    bf16x3_tile<NT, 2>(it.rows, it.k, it.B, it.Rp, it.nkc, it.Yth, it.Ytl, it.ldt, it.out, it.ldp, it.row0, it.kc0,
                       it.kc1);
  }
}

__global__ void k_reduce_splits(int64_t rows, int k, int S, const float* __restrict__ P, int64_t split_stride,
                                float* __restrict__ R, int64_t ldr) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= rows * k) return;
  const int64_t row = e / k;
  const int c = (int)(e - row * k);
  double s = 0.0;
  for (int sp = 0; sp < S; ++sp) s += (double)P[sp * split_stride + e];
  R[row * ldr + c] = (float)s;
}

__global__ __launch_bounds__(256) void k_reduce_splits_grouped(const nmf::SplitReduceItem* __restrict__ items,
                                                               int64_t n) {
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const nmf::SplitReduceItem it = items[i];
    const int64_t e = it.e0 + threadIdx.x;
    if (e < it.rows * it.k) {
      const int64_t row = e / it.k;
      const int c = (int)(e - row * it.k);
      double s = 0.0;
      for (int sp = 0; sp < it.S; ++sp) s += (double)it.P[sp * it.stride + e];
      it.R[row * it.ldr + c] = (float)s;
    }
  }
}

struct Bf16Plan {
  int64_t rows, K, nkc, ldt;
  int KP, S;
  int64_t kcps;
};

// Workgroups of the product kernel that fit on the device at once (all CUs),
// from the occupancy calculator; 0 if it cannot be queried.  Cached per
// device and per K width.
constexpr int kMaxDevices = 64;
std::atomic<int> g_capacity[kMaxDevices][2];

int bf16_capacity(int KP) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
  const int which = KP == 32 ? 0 : 1;
  int cap = g_capacity[dev][which].load(std::memory_order_relaxed);
  if (cap > 0) return cap;
  int per_cu = 0, cus = 0;
  const hipError_t e1 = which == 0
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rhs_bf16x3<1, NMF_SIDE_H>, 256, 0)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rhs_bf16x3<2, NMF_SIDE_H>, 256, 0);
  const hipError_t e2 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e1 != hipSuccess || e2 != hipSuccess || per_cu <= 0 || cus <= 0) {
    (void)hipGetLastError();
    return 0;
  }
  cap = per_cu * cus;
  g_capacity[dev][which].store(cap, std::memory_order_relaxed);
  return cap;
}

// Workspace is sized for at most kMaxBlocksSized concurrent workgroups, so
// the split count used at launch (from the device's capacity) never exceeds
// the one the workspace was sized for.
constexpr int64_t kMaxBlocksSized = 4096;

// capacity <= 0: sizing for the workspace (upper bound of the split count).
// Otherwise the split count makes rows-tiles x splits fit the device at once
// (no partial second wave of workgroups) when there are fewer row tiles than
// resident workgroups.
Bf16Plan bf16_plan(int side, int64_t m, int64_t n, int k, int capacity) {
  Bf16Plan p;
  p.rows = side == NMF_SIDE_W ? m : n;
  p.K = side == NMF_SIDE_W ? n : m;
  p.KP = k <= 32 ? 32 : 64;
  p.nkc = (p.K + kTC - 1) / kTC;
  p.ldt = p.nkc * kTC;
  const int64_t tiles = nmf::cdiv(p.rows, kBTM);
  const int64_t cap = capacity > 0 && capacity < kMaxBlocksSized ? capacity : kMaxBlocksSized;
  int64_t S = cap / (tiles > 0 ? tiles : 1);
  // Long contractions with at least as many row tiles as resident
  // workgroups: the split count (up to kTailSplits) that fills whole rounds
  // of resident workgroups best.  A partial last round of such long-lived
  // workgroups streams below the full rate (172,800 rows: 4.7% slower per
  // tile than two whole rounds).  Sizing (capacity 0) takes the largest
  // split this can choose.
  constexpr int64_t kTailSplits = 8, kTailMinChunks = 1024;
  if (p.nkc >= kTailMinChunks) {
    if (capacity <= 0) {
      if (S < kTailSplits) S = kTailSplits;
    } else if (tiles >= cap) {
      int64_t best = 1;
      double best_waste = 1e30;
      for (int64_t sp = 1; sp <= kTailSplits; ++sp) {
        const int64_t items = tiles * sp, rounds = (items + cap - 1) / cap;
        const double waste = (double)(rounds * cap) / (double)items - 1.0;
        if (waste < best_waste - 0.01) {  // a larger split must gain over 1% of a round
          best_waste = waste;
          best = sp;
        }
      }
      S = best;
    }
  }
  const int64_t maxS = p.nkc / 32 > 1 ? p.nkc / 32 : 1;
  if (S > maxS) S = maxS;
  if (S > 65535) S = 65535;
  if (S < 1) S = 1;
  p.kcps = nmf::cdiv(p.nkc, S);
  p.S = (int)nmf::cdiv(p.nkc, p.kcps);
  if (p.S < 1) p.S = 1;
  return p;
}

}  // namespace

namespace nmf {

size_t bf16_padded_bytes(int64_t rows, int64_t cols) {
  return (size_t)2 * (size_t)(cdiv(rows, kTR) * kTR) * (size_t)(cdiv(cols, kTC) * kTC) * sizeof(uint16_t);
}

int bf16x3_plan(int side, int64_t m, int64_t n, int k, Carver& c, void** scratch) {
  const Bf16Plan p = bf16_plan(side, m, n, k, 0);
  // the scratch block starts with the two Y planes, then the split partials
  uint16_t* y = c.take<uint16_t>((size_t)2 * p.KP * p.ldt);
  if (p.S > 1) c.take<float>((size_t)p.S * p.rows * k);
  *scratch = y;
  return NMF_OK;
}

// Longest FP32 accumulation (products per accumulator) of a launch on the
// current device: three products per contraction index over one split.
int64_t bf16x3_chain(int side, int64_t m, int64_t n, int k) {
  const int KP = k <= 32 ? 32 : 64;
  const Bf16Plan p = bf16_plan(side, m, n, k, bf16_capacity(KP));
  return 3 * p.kcps * kTC;
}

void bf16x3_y_planes(int side, int64_t m, int64_t n, int k, void* scratch, uint16_t** yth, uint16_t** ytl,
                     int64_t* ldt, int* KP) {
  const Bf16Plan p = bf16_plan(side, m, n, k, 0);
  *yth = static_cast<uint16_t*>(scratch);
  *ytl = *yth + (size_t)p.KP * p.ldt;
  *ldt = p.ldt;
  *KP = p.KP;
}

int bf16x3_launch(int side, int64_t m, int64_t n, int k, const void* Bt, const float* Y, int64_t ldy, float* R,
                  int64_t ldr, void* scratch, hipStream_t s, bool y_ready) {
  const int KP = k <= 32 ? 32 : 64;
  const Bf16Plan p = bf16_plan(side, m, n, k, bf16_capacity(KP));
  if (p.rows == 0) return NMF_OK;
  if (p.K == 0) return zero_f32(R, p.rows, k, ldr, s);
  uint16_t* yth = static_cast<uint16_t*>(scratch);
  uint16_t* ytl = yth + (size_t)p.KP * p.ldt;
  // the partials follow the planes at the next 256-byte boundary (as carved)
  const size_t plane_bytes = (size_t)2 * p.KP * p.ldt * sizeof(uint16_t);
  float* partial = reinterpret_cast<float*>(static_cast<char*>(scratch) + ((plane_bytes + 255) & ~size_t(255)));
  if (!y_ready) {
    hipLaunchKernelGGL(k_split_y, dim3((unsigned)cdiv(p.ldt, 64)), dim3(256), 0, s, p.K, k, p.KP, Y, ldy, yth, ytl,
                       p.ldt);
    NMF_TRY(launch_status("rhs bf16x3: split Y"));
  }
  float* P = p.S > 1 ? partial : R;
  const int64_t ldp = p.S > 1 ? k : ldr;
  const int64_t stride = p.S > 1 ? p.rows * k : 0;
  const int64_t ntiles = cdiv(p.rows, kBTM);
  const dim3 grid((unsigned)(cdiv(ntiles * p.S, 8) * 8));
  const uint16_t* B = static_cast<const uint16_t*>(Bt);
  mark_begin(s);
  const int64_t Rp = cdiv(p.rows, kBTM) * kBTM;
  auto kern = side == NMF_SIDE_W ? (p.KP == 32 ? k_rhs_bf16x3<1, NMF_SIDE_W> : k_rhs_bf16x3<2, NMF_SIDE_W>)
                                  : (p.KP == 32 ? k_rhs_bf16x3<1, NMF_SIDE_H> : k_rhs_bf16x3<2, NMF_SIDE_H>);
  hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, p.rows, k, B, Rp, p.nkc, yth, ytl, p.ldt, P, ldp, p.kcps, stride,
                     ntiles, (int64_t)p.S);
  mark_end(s);
  NMF_TRY(launch_status("rhs bf16x3"));
  if (p.S > 1) {
    hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)cdiv(p.rows * k, 256)), dim3(256), 0, s, p.rows, k, p.S,
                       partial, stride, R, ldr);
    NMF_TRY(launch_status("rhs bf16x3: reduce"));
  }
  return NMF_OK;
}

int split_y_grouped_launch(const SplitYItem* items, int64_t n, int grid, hipStream_t s) {
  if (n == 0) return NMF_OK;
  hipLaunchKernelGGL(k_split_y_grouped, dim3((unsigned)grid), dim3(256), 0, s, items, n);
  return launch_status("split Y (grouped)");
}

int bf16x3_grouped_launch(int NT, int tile_rows, const Bf16Item* items, int64_t n, int grid, hipStream_t s) {
  if (n == 0) return NMF_OK;
  if (tile_rows == 64) {
    if (NT == 1)
      hipLaunchKernelGGL(k_rhs_bf16x3_grouped64<1>, dim3((unsigned)grid), dim3(128), 0, s, items, n);
    else
      hipLaunchKernelGGL(k_rhs_bf16x3_grouped64<2>, dim3((unsigned)grid), dim3(128), 0, s, items, n);
  } else {
    if (NT == 1)
      hipLaunchKernelGGL(k_rhs_bf16x3_grouped<1>, dim3((unsigned)grid), dim3(256), 0, s, items, n);
    else
      hipLaunchKernelGGL(k_rhs_bf16x3_grouped<2>, dim3((unsigned)grid), dim3(256), 0, s, items, n);
  }
  return launch_status("rhs bf16x3 (grouped)");
}

int split_reduce_grouped_launch(const SplitReduceItem* items, int64_t n, int grid, hipStream_t s) {
  if (n == 0) return NMF_OK;
  hipLaunchKernelGGL(k_reduce_splits_grouped, dim3((unsigned)grid), dim3(256), 0, s, items, n);
  return launch_status("split reduce (grouped)");
}

int bf16_grouped_occupancy(int which, int* per_cu) {
  hipError_t e = hipErrorInvalidValue;
  if (which == kCapSplitY) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_split_y_grouped, 256, 0);
  if (which == kCapBf16NT1)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_rhs_bf16x3_grouped<1>, 256, 0);
  if (which == kCapBf16NT2)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_rhs_bf16x3_grouped<2>, 256, 0);
  if (which == kCapBf16NT1T64)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_rhs_bf16x3_grouped64<1>, 128, 0);
  if (which == kCapBf16NT2T64)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_rhs_bf16x3_grouped64<2>, 128, 0);
  if (which == kCapReduce)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_reduce_splits_grouped, 256, 0);
  return e == hipSuccess ? NMF_OK : NMF_EHIP;
}

}  // namespace nmf

extern "C" size_t nmf_split_bf16_bytes(int64_t rows, int64_t cols, int transpose) {
  if (rows < 0 || cols < 0) return 0;
  return transpose ? nmf::bf16_padded_bytes(cols, rows) : nmf::bf16_padded_bytes(rows, cols);
}

extern "C" int nmf_split_bf16(int64_t rows, int64_t cols, const float* X, int64_t ldx, int transpose, void* out,
                              void* stream) {
  if (rows < 0 || cols < 0 || ldx < cols) return nmf::fail(NMF_EINVAL, "nmf_split_bf16: bad sizes");
  if (rows * cols > 0 && (!X || !out)) return nmf::fail(NMF_EINVAL, "nmf_split_bf16: null pointer");
  if (rows * cols == 0) return NMF_OK;
  const int64_t brows = transpose ? cols : rows, bcols = transpose ? rows : cols;
  const int64_t Rp = nmf::cdiv(brows, kTR) * kTR, Cp = nmf::cdiv(bcols, kTC) * kTC;
  if (Rp / 64 > 65535) return nmf::fail(NMF_EINVAL, "nmf_split_bf16: too many rows");
  hipLaunchKernelGGL(k_split_planes, dim3((unsigned)(Cp / 64), (unsigned)(Rp / 64)), dim3(256), 0,
                     nmf::as_stream(stream), rows, cols, X, ldx, transpose, Rp, Cp, static_cast<uint16_t*>(out));
  return nmf::launch_status("nmf_split_bf16");
}
