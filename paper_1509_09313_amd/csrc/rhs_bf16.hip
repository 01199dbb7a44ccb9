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


typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

__device__ __forceinline__ v16f mfma_bf16(v8bf a, v8bf b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Y (K x k FP32, ld ldy) -> transposed BF16 planes Yth, Ytl (KP x ldt), rows
// i >= k and columns >= K zero.  One block per 64 rows of Y.
__global__ __launch_bounds__(256) void k_split_y(int64_t K, int k, int KP, const float* __restrict__ Y, int64_t ldy,
                                                 uint16_t* __restrict__ Yth, uint16_t* __restrict__ Ytl, int64_t ldt) {
  __shared__ float tile[64][65];
  const int64_t K0 = (int64_t)blockIdx.x * 64;
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

constexpr int kBTM = 128;          // rows of B per block (4 waves x 32)
constexpr int kBTK = 64;           // contraction chunk (BF16 elements)
constexpr int kBPitch = kBTK + 8;  // LDS pitch in uint16 (144 bytes: conflict-free 16-byte reads)

// R (rows x k) = B (rows x K) * Y (K x k) with B and Y given as BF16 planes:
// D_t[i][j] = R[row0 + 32w + j][32t + i] from three MFMAs per 16-wide K step
// (Yhi Bhi + Ylo Bhi + Yhi Blo).  blockIdx.y selects a K range (split-K);
// its partial goes to P + y * split_stride.
template <int NT, bool VEC>
__global__ __launch_bounds__(256) void k_rhs_bf16x3(int64_t rows, int64_t K, int k, const uint16_t* __restrict__ Bh,
                                                    const uint16_t* __restrict__ Bl, int64_t ldb,
                                                    const uint16_t* __restrict__ Yth, const uint16_t* __restrict__ Ytl,
                                                    int64_t ldt, float* __restrict__ P, int64_t ldp,
                                                    int64_t k_per_split, int64_t split_stride) {
  constexpr int KP = 32 * NT;
  __shared__ __align__(16) uint16_t Bs[2][kBTM * kBPitch];
  __shared__ __align__(16) uint16_t Ys[2][KP * kBPitch];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int j = lane & 31, h = lane >> 5;
  const int64_t row0 = (int64_t)blockIdx.x * kBTM;
  const int64_t kb = (int64_t)blockIdx.y * k_per_split;
  const int64_t ke = (kb + k_per_split < K) ? kb + k_per_split : K;

  v16f acc[NT];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) acc[tt] = v16f{};

  uint4 rb[2][4];
  uint4 ry[2][NT];
  auto load = [&](int64_t c0) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int q = t + 256 * s;
      const int rr = q >> 3, c8 = q & 7;
      const int64_t r = row0 + rr, c = c0 + 8 * c8;
#pragma unroll
      for (int pl = 0; pl < 2; ++pl) {
        const uint16_t* src = (pl ? Bl : Bh) + r * ldb + c;
        if (VEC && r < rows && c + 7 < ke) {
          rb[pl][s] = *reinterpret_cast<const uint4*>(src);
        } else {
          uint16_t v[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = (r < rows && c + e < ke) ? src[e] : (uint16_t)0;
          rb[pl][s] = make_uint4(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16),
                                 v[4] | ((uint32_t)v[5] << 16), v[6] | ((uint32_t)v[7] << 16));
        }
      }
    }
#pragma unroll
    for (int s = 0; s < NT; ++s) {
      const int q = t + 256 * s;
      const int ii = q >> 3, c8 = q & 7;
      const int64_t c = c0 + 8 * c8;
#pragma unroll
      for (int pl = 0; pl < 2; ++pl) {
        const uint16_t* src = (pl ? Ytl : Yth) + (int64_t)ii * ldt + c;
        if (c + 7 < ke) {
          ry[pl][s] = *reinterpret_cast<const uint4*>(src);
        } else {
          uint16_t v[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = (c + e < ke) ? src[e] : (uint16_t)0;
          ry[pl][s] = make_uint4(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16),
                                 v[4] | ((uint32_t)v[5] << 16), v[6] | ((uint32_t)v[7] << 16));
        }
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int q = t + 256 * s;
      const int rr = q >> 3, c8 = q & 7;
#pragma unroll
      for (int pl = 0; pl < 2; ++pl) *reinterpret_cast<uint4*>(&Bs[pl][rr * kBPitch + 8 * c8]) = rb[pl][s];
    }
#pragma unroll
    for (int s = 0; s < NT; ++s) {
      const int q = t + 256 * s;
      const int ii = q >> 3, c8 = q & 7;
#pragma unroll
      for (int pl = 0; pl < 2; ++pl) *reinterpret_cast<uint4*>(&Ys[pl][ii * kBPitch + 8 * c8]) = ry[pl][s];
    }
  };

  if (kb < ke) load(kb);
  for (int64_t c0 = kb; c0 < ke; c0 += kBTK) {
    __syncthreads();
    store();
    __syncthreads();
    if (c0 + kBTK < ke) load(c0 + kBTK);
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
  }
  float* out = P + (int64_t)blockIdx.y * split_stride;
  const int64_t r = row0 + 32 * w + j;
  if (r < rows) {
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int c = 32 * tt + (v & 3) + 8 * (v >> 2) + 4 * h;
        if (c < k) out[r * ldp + c] = acc[tt][v];
      }
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

struct Bf16Plan {
  int64_t rows, K, ldt;
  int KP, S;
  int64_t kps;
};

Bf16Plan bf16_plan(int side, int64_t m, int64_t n, int k) {
  Bf16Plan p;
  p.rows = side == NMF_SIDE_W ? m : n;
  p.K = side == NMF_SIDE_W ? n : m;
  p.KP = k <= 32 ? 32 : 64;
  p.ldt = (p.K + 7) / 8 * 8;
  const int64_t tiles = nmf::cdiv(p.rows, kBTM);
  int64_t S = nmf::cdiv(1024, tiles);
  const int64_t maxS = p.K / 2048 > 1 ? p.K / 2048 : 1;
  if (S > maxS) S = maxS;
  if (S > 65535) S = 65535;
  if (S < 1) S = 1;
  int64_t kps = nmf::cdiv(p.K, S);
  kps = (kps + kBTK - 1) / kBTK * kBTK;
  if (kps < kBTK) kps = kBTK;
  p.kps = kps;
  p.S = (int)nmf::cdiv(p.K, kps);
  if (p.S < 1) p.S = 1;
  return p;
}

struct Bf16Scratch {
  uint16_t* yth;
  uint16_t* ytl;
  float* partial;
};

}  // namespace

namespace nmf {

int bf16x3_plan(int side, int64_t m, int64_t n, int k, Carver& c, void** scratch) {
  const Bf16Plan p = bf16_plan(side, m, n, k);
  // the scratch block starts with the two Y planes, then the split partials
  uint16_t* y = c.take<uint16_t>((size_t)2 * p.KP * p.ldt);
  if (p.S > 1) c.take<float>((size_t)p.S * p.rows * k);
  *scratch = y;
  return NMF_OK;
}

int bf16x3_launch(int side, int64_t m, int64_t n, int k, const uint16_t* B_hi, const uint16_t* B_lo, int64_t ldb,
                  const float* Y, int64_t ldy, float* R, int64_t ldr, void* scratch, hipStream_t s) {
  const Bf16Plan p = bf16_plan(side, m, n, k);
  if (p.rows == 0) return NMF_OK;
  if (p.K == 0) return zero_f32(R, p.rows, k, ldr, s);
  uint16_t* yth = static_cast<uint16_t*>(scratch);
  uint16_t* ytl = yth + (size_t)p.KP * p.ldt;
  // the partials follow the planes at the next 256-byte boundary (as carved)
  const size_t plane_bytes = (size_t)2 * p.KP * p.ldt * sizeof(uint16_t);
  float* partial = reinterpret_cast<float*>(static_cast<char*>(scratch) + ((plane_bytes + 255) & ~size_t(255)));
  hipLaunchKernelGGL(k_split_y, dim3((unsigned)cdiv(p.ldt, 64)), dim3(256), 0, s, p.K, k, p.KP, Y, ldy, yth, ytl,
                     p.ldt);
  NMF_TRY(launch_status("rhs bf16x3: split Y"));
  const bool vec = (ldb % 8 == 0) && ((uintptr_t)B_hi % 16 == 0) && ((uintptr_t)B_lo % 16 == 0);
  float* P = p.S > 1 ? partial : R;
  const int64_t ldp = p.S > 1 ? k : ldr;
  const int64_t stride = p.S > 1 ? p.rows * k : 0;
  const dim3 grid((unsigned)cdiv(p.rows, kBTM), (unsigned)p.S);
#define NMF_BF16_LAUNCH(NT_, V_)                                                                            \
  hipLaunchKernelGGL((k_rhs_bf16x3<NT_, V_>), grid, dim3(256), 0, s, p.rows, p.K, k, B_hi, B_lo, ldb, yth, ytl, \
                     p.ldt, P, ldp, p.kps, stride)
  if (p.KP == 32) {
    if (vec) NMF_BF16_LAUNCH(1, true); else NMF_BF16_LAUNCH(1, false);
  } else {
    if (vec) NMF_BF16_LAUNCH(2, true); else NMF_BF16_LAUNCH(2, false);
  }
#undef NMF_BF16_LAUNCH
  NMF_TRY(launch_status("rhs bf16x3"));
  if (p.S > 1) {
    hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)cdiv(p.rows * k, 256)), dim3(256), 0, s, p.rows, k, p.S,
                       partial, stride, R, ldr);
    NMF_TRY(launch_status("rhs bf16x3: reduce"));
  }
  return NMF_OK;
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
