// Dense right-hand sides of the two ANLS updates (Algorithm 1):
//   side W:  R (m x k) = A (m x n) * Ht (n x k)        = A H^T
//   side H:  R (n x k) = A^T (n x m) * W (m x k)       = (W^T A)^T
// These are the "MM" local products of the paper (Algorithm 3's V_ij and
// Y_ij at p = 1).  k <= 64 is the short dimension; A is streamed once.
//
// FP32 path: v_mfma_f32_32x32x2_f32.  Output tiles are 32 (k) x 32 (rows of
// A or columns of A).  The contraction index inside one K-chunk is permuted
// freely (A and B operands use the same permutation) so that every lane's
// operand comes from one 16-byte load.
//   side W stages 128 x 32 tiles of A and of the transposed Y in LDS (rows of
//     A are contracted along their contiguous dimension, so lanes need
//     different rows), two chunks in flight; when A has too few row tiles to
//     fill the device (A^T of a tall matrix: Ht = A^T W over a resident FP32
//     A^T), the contraction is split into S column ranges whose FP32
//     partials are summed in FP64 in a fixed order;
//   side H needs no LDS: lane (j, h) loads A[r + h][c0 + 4j .. +3] with one
//     16-byte load (a 512-byte contiguous segment per half-wave) and feeds
//     four MFMAs, one per component, with the next rows' loads issued before
//     the current rows' MFMAs; the rows of A are split into S ranges whose
//     FP32 partials are summed in FP64 in a fixed order.
// BF16X3 path (tiled BF16 operand): see rhs_bf16.hip.
#include "nmf_common.h"

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ v16f mfma32(float a, float b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// A is read once per launch: non-temporal loads stream it without
// displacing the reused operand from the caches, and reach a higher read
// bandwidth than plain loads on this part.
__device__ __forceinline__ float4 load_stream(const float* p) {
  const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

// ---------------------------------------------------------------- side W --
constexpr int kWTM = 128;  // rows of A per block (4 waves x 32)
constexpr int kWTK = 32;   // contraction chunk (columns of A)
constexpr int kWPitch = kWTK + 4;

template <int NT, bool VEC>
__global__ __launch_bounds__(256) void k_rhs_w_f32(int64_t m, int64_t n, int k, const float* __restrict__ A,
                                                   int64_t lda, const float* __restrict__ Y, int64_t ldy,
                                                   float* __restrict__ R, int64_t ldr) {
  constexpr int KP = 32 * NT;
  constexpr int YP = KP + 4;
  constexpr int YPER = KP * kWTK / 256;  // Y values staged per thread
  __shared__ __align__(16) float As[kWTM * kWPitch];
  __shared__ __align__(16) float Ys[kWTK * YP];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int j = lane & 31, h = lane >> 5;
  const int64_t row0 = (int64_t)blockIdx.x * kWTM;

  v16f acc[NT];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) acc[tt] = v16f{};

  float4 ra[4];
  float ry[YPER];
  auto load = [&](int64_t n0) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int q = t + 256 * s;
      const int rr = q >> 3, c4 = q & 7;
      const int64_t r = row0 + rr, c = n0 + 4 * c4;
      const float* src = A + r * lda + c;
      if (VEC && r < m && c + 3 < n) {
        ra[s] = load_stream(src);
      } else {
        ra[s].x = (r < m && c + 0 < n) ? src[0] : 0.0f;
        ra[s].y = (r < m && c + 1 < n) ? src[1] : 0.0f;
        ra[s].z = (r < m && c + 2 < n) ? src[2] : 0.0f;
        ra[s].w = (r < m && c + 3 < n) ? src[3] : 0.0f;
      }
    }
#pragma unroll
    for (int s = 0; s < YPER; ++s) {
      const int e = t + 256 * s;
      const int kk = e / KP, cc = e - kk * KP;
      ry[s] = (n0 + kk < n && cc < k) ? Y[(n0 + kk) * ldy + cc] : 0.0f;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int q = t + 256 * s;
      const int rr = q >> 3, c4 = q & 7;
      *reinterpret_cast<float4*>(&As[rr * kWPitch + 4 * c4]) = ra[s];
    }
#pragma unroll
    for (int s = 0; s < YPER; ++s) {
      const int e = t + 256 * s;
      const int kk = e / KP, cc = e - kk * KP;
      Ys[kk * YP + cc] = ry[s];
    }
  };

  load(0);
  for (int64_t n0 = 0; n0 < n; n0 += kWTK) {
    __syncthreads();
    store();
    __syncthreads();
    if (n0 + kWTK < n) load(n0 + kWTK);
#pragma unroll
    for (int sg = 0; sg < kWTK / 8; ++sg) {
      const float4 a4 = *reinterpret_cast<const float4*>(&As[(32 * w + j) * kWPitch + 8 * sg + 4 * h]);
      const float av[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = 8 * sg + 4 * h + q;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) acc[tt] = mfma32(Ys[kk * YP + 32 * tt + j], av[q], acc[tt]);
      }
    }
  }
  // D_tt[i][j] = R[row0 + 32w + j][32 tt + i]; lane holds i = (v&3) + 8(v>>2) + 4h.
  // Each 32-column part of the tile goes out through LDS (the A staging
  // buffer) so that the stores cover whole row segments: straight from the
  // MFMA layout every store instruction touches 32 rows with 8 bytes each
  // (1.97 -> 1.84 ms at 10^6 x 2400, k = 30).  The stores stay ordinary:
  // non-temporal ones save 0.01 ms here and cost the BPP that reads R 0.06.
  constexpr int OP = 33;
  static_assert(kWTM * OP <= kWTM * kWPitch, "output part exceeds the staging buffer");
  const int nr = m - row0 < kWTM ? (int)(m - row0) : kWTM;
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    const int cw = k - 32 * tt < 32 ? k - 32 * tt : 32;  // columns of this part
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 16; ++v) As[(32 * w + j) * OP + (v & 3) + 8 * (v >> 2) + 4 * h] = acc[tt][v];
    __syncthreads();
    for (int e = t; e < nr * cw; e += 256) {
      const int row = e / cw, c = e - row * cw;
      R[(row0 + row) * ldr + 32 * tt + c] = As[row * OP + c];
    }
  }
}

// Side W, streaming form (A 16-byte aligned with lda % 4 == 0): the
// structure of the BF16x3 product kernel with FP32 operands.  Each block owns
// 128 rows of A and walks the contraction in 32-column chunks (16 KB of A per
// chunk: small staging sets give three blocks per CU; 64-column chunks, two
// blocks per CU, measured 8% slower); Y comes transposed and zero-padded (Yt,
// KP x ldt with ldt a multiple of 64), so a lane reads
// four consecutive contraction indices of its Y column as one 16-byte LDS
// read, as it does for its row of A.  Two chunks are in flight in two register
// staging sets, with unconditional loads (rows past m are clamped to m - 1:
// a row only feeds its own output row, which is not stored) so each wait is
// for the older set only.  A ragged last chunk (n not a multiple of 64) is
// loaded element by element with zeros past n.  The finished tile leaves
// through LDS as whole rows.
constexpr int kSC = 32;            // contraction chunk (columns of A)
constexpr int kSPitch = kSC + 4;   // LDS pitch in floats (== 4 mod 32: conflict-free 16-byte reads)
constexpr int kSRowsPass = 256 / (kSC / 4);  // rows one staging pass covers
constexpr int kSPassA = kWTM / kSRowsPass;   // passes over the 128-row A tile

// blockIdx.y = s takes contraction columns [s cps, (s + 1) cps) and writes
// its product to R + s pstride (a single range: cps >= n, pstride 0).
template <int NT>
__global__ __launch_bounds__(256) void k_rhs_w_f32s(int64_t m, int64_t n, int k, const float* __restrict__ A,
                                                    int64_t lda, const float* __restrict__ Yt, int64_t ldt,
                                                    float* __restrict__ R, int64_t ldr, int64_t cps,
                                                    int64_t pstride) {
  {
    const int64_t cs0 = (int64_t)blockIdx.y * cps;
    A += cs0;
    Yt += cs0;
    n = n - cs0 < cps ? n - cs0 : cps;
    R += (int64_t)blockIdx.y * pstride;
  }
  constexpr int KP = 32 * NT;
  constexpr int kPassY = KP / kSRowsPass;
  __shared__ __align__(16) float As[kWTM * kSPitch];
  __shared__ __align__(16) float Ys[KP * kSPitch];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int j = lane & 31, h = lane >> 5;
  const int64_t row0 = (int64_t)blockIdx.x * kWTM;
  const int64_t nfull = n / kSC;  // whole chunks

  v16f acc[NT];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) acc[tt] = v16f{};

  // thread t stages rows lr + kSRowsPass s of the tile, columns lc .. lc + 3
  const int lr = t / (kSC / 4), lc = 4 * (t % (kSC / 4));
  const int64_t rlast = m - 1 - row0;
  const float* a_base = A + (row0 + lr) * lda + lc;
  struct Stage {
    float4 a[kSPassA];
    float4 y[kPassY];
  };
  // row lr + kSRowsPass s of the tile, clamped to the last row of A
  auto arow = [&](int s) __attribute__((always_inline)) -> const float* {
    const int r = lr + kSRowsPass * s;
    return r <= rlast ? a_base + (int64_t)kSRowsPass * s * lda : a_base + (rlast - lr) * lda;
  };
  auto load = [&](Stage& S, int64_t c0) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < kSPassA; ++s) S.a[s] = load_stream(arow(s) + c0);
    const float* yp = Yt + (int64_t)lr * ldt + c0 + lc;
#pragma unroll
    for (int s = 0; s < kPassY; ++s) S.y[s] = *reinterpret_cast<const float4*>(yp + (int64_t)kSRowsPass * s * ldt);
  };
  // the ragged last chunk: element loads, zero past column n
  auto load_tail = [&](Stage& S, int64_t c0) __attribute__((always_inline)) {
    const int64_t c = c0 + lc;
#pragma unroll
    for (int s = 0; s < kSPassA; ++s) {
      const float* p = arow(s) + c0;
      S.a[s].x = c + 0 < n ? p[0] : 0.0f;
      S.a[s].y = c + 1 < n ? p[1] : 0.0f;
      S.a[s].z = c + 2 < n ? p[2] : 0.0f;
      S.a[s].w = c + 3 < n ? p[3] : 0.0f;
    }
    const float* yp = Yt + (int64_t)lr * ldt + c0 + lc;
#pragma unroll
    for (int s = 0; s < kPassY; ++s) S.y[s] = *reinterpret_cast<const float4*>(yp + (int64_t)kSRowsPass * s * ldt);
  };
  const int so = lr * kSPitch + lc;
  auto store = [&](const Stage& S) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < kSPassA; ++s) *reinterpret_cast<float4*>(&As[so + kSRowsPass * s * kSPitch]) = S.a[s];
#pragma unroll
    for (int s = 0; s < kPassY; ++s) *reinterpret_cast<float4*>(&Ys[so + kSRowsPass * s * kSPitch]) = S.y[s];
  };
  // lane (j, h) takes contraction indices 8 g + 4 h + q for the q-th MFMA of
  // group g, for A and Y alike
  auto compute = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int g = 0; g < kSC / 8; ++g) {
      const int off = 8 * g + 4 * h;
      const float4 a4 = *reinterpret_cast<const float4*>(&As[(32 * w + j) * kSPitch + off]);
      const float av[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
        const float4 y4 = *reinterpret_cast<const float4*>(&Ys[(32 * tt + j) * kSPitch + off]);
        const float yv[4] = {y4.x, y4.y, y4.z, y4.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[tt] = mfma32(yv[q], av[q], acc[tt]);
      }
    }
  };
  if (nfull >= 4) {
    Stage S0, S1;
    load(S0, 0);
    __builtin_amdgcn_sched_barrier(0);  // same issue order as in the loop
    load(S1, kSC);
    int64_t c = 0;
    for (; c + 3 < nfull; c += 2) {
      __syncthreads();
      store(S0);
      __syncthreads();
      load(S0, (c + 2) * kSC);
      compute();
      __syncthreads();
      store(S1);
      __syncthreads();
      load(S1, (c + 3) * kSC);
      compute();
    }
    const bool three = c + 2 < nfull;
    __syncthreads();
    store(S0);
    __syncthreads();
    if (three) load(S0, (c + 2) * kSC);
    compute();
    __syncthreads();
    store(S1);
    __syncthreads();
    compute();
    if (three) {
      __syncthreads();
      store(S0);
      __syncthreads();
      compute();
    }
  } else {
    Stage S0;
    if (nfull > 0) load(S0, 0);
    for (int64_t c = 0; c < nfull; ++c) {
      __syncthreads();
      store(S0);
      __syncthreads();
      if (c + 1 < nfull) load(S0, (c + 1) * kSC);
      compute();
    }
  }
  if (nfull * kSC < n) {
    Stage S0;
    load_tail(S0, nfull * kSC);
    __syncthreads();
    store(S0);
    __syncthreads();
    compute();
  }
  // D_tt[i][j] = R[row0 + 32w + j][32 tt + i]; lane holds i = (v&3) + 8(v>>2) + 4h.
  // Each 32-column part leaves through LDS as whole row segments.
  constexpr int OP = 33;  // odd pitch: conflict-free column writes
  static_assert(kWTM * OP <= kWTM * kSPitch, "output part exceeds the staging buffer");
  const int nr = m - row0 < kWTM ? (int)(m - row0) : kWTM;
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    const int cw = k - 32 * tt < 32 ? k - 32 * tt : 32;  // columns of this part
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 16; ++v) As[(32 * w + j) * OP + (v & 3) + 8 * (v >> 2) + 4 * h] = acc[tt][v];
    __syncthreads();
    for (int e = t; e < nr * cw; e += 256) {
      const int row = e / cw, c = e - row * cw;
      R[(row0 + row) * ldr + 32 * tt + c] = As[row * OP + c];
    }
  }
}

// Yt (KP x ldt) = Y^T (Y: K x k, ld ldy), zero in rows >= k and columns >= K.
__global__ __launch_bounds__(256) void k_transpose_y(int64_t K, int k, int KP, const float* __restrict__ Y,
                                                     int64_t ldy, float* __restrict__ Yt, int64_t ldt) {
  __shared__ float tile[64][65];
  const int64_t K0 = (int64_t)blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int kk = e / 64, c = e - kk * 64;
    tile[kk][c] = (K0 + kk < K && c < k) ? Y[(K0 + kk) * ldy + c] : 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < KP * 64; e += 256) {
    const int i = e / 64, kk = e - i * 64;
    Yt[i * ldt + K0 + kk] = tile[kk][i];
  }
}

// ---------------------------------------------------------------- side H --
constexpr int kHCols = 128;  // columns of A per wave
constexpr int kHUnroll = 8;  // row pairs in flight per lane

// The grid is one-dimensional and XCD-aware (launch index L runs on XCD
// L % 8; L -> logical (L % 8) * (grid / 8) + L / 8, column group fastest), so
// all column groups of one row range run on one XCD and share that range of
// Y in its L2.
template <int NT, bool VEC>
__global__ __launch_bounds__(64) void k_rhs_h_f32(int64_t m, int64_t n, int k, const float* __restrict__ A,
                                                  int64_t lda, const float* __restrict__ Y, int64_t ldy,
                                                  float* __restrict__ P, int64_t ldp, int64_t rows_per_split,
                                                  int64_t split_stride, int64_t ngroups, int64_t nsplit) {
  const int64_t per_xcd = gridDim.x / 8;
  const int64_t lid = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (lid >= ngroups * nsplit) return;
  const int64_t gx = lid % ngroups, gy = lid / ngroups;
  const int lane = threadIdx.x;
  const int j = lane & 31, h = lane >> 5;
  const int64_t c0 = gx * kHCols;
  const int64_t col = c0 + 4 * j;
  const int64_t r_begin = gy * rows_per_split;
  const int64_t r_end = (r_begin + rows_per_split < m) ? r_begin + rows_per_split : m;

  v16f acc[4][NT];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) acc[q][tt] = v16f{};

  for (int64_t r = r_begin; r < r_end; r += 2 * kHUnroll) {
    float4 a[kHUnroll];
    float wv[kHUnroll][NT];
#pragma unroll
    for (int u = 0; u < kHUnroll; ++u) {
      const int64_t rr = r + 2 * u + h;
      const bool rok = rr < r_end;
      const float* src = A + rr * lda + col;
      if (VEC && rok && col + 3 < n) {
        a[u] = load_stream(src);
      } else {
        a[u].x = (rok && col + 0 < n) ? src[0] : 0.0f;
        a[u].y = (rok && col + 1 < n) ? src[1] : 0.0f;
        a[u].z = (rok && col + 2 < n) ? src[2] : 0.0f;
        a[u].w = (rok && col + 3 < n) ? src[3] : 0.0f;
      }
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
        const int c = 32 * tt + j;
        wv[u][tt] = (rok && c < k) ? Y[rr * ldy + c] : 0.0f;
      }
    }
#pragma unroll
    for (int u = 0; u < kHUnroll; ++u) {
      const float av[4] = {a[u].x, a[u].y, a[u].z, a[u].w};
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) acc[q][tt] = mfma32(wv[u][tt], av[q], acc[q][tt]);
    }
  }
  // D_{q,tt}[i][j] = R[c0 + 4j + q][32 tt + i]
  float* out = P + gy * split_stride;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t row = col + q;
    if (row >= n) continue;
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int c = 32 * tt + (v & 3) + 8 * (v >> 2) + 4 * h;
        if (c < k) out[row * ldp + c] = acc[q][tt][v];
      }
  }
}

// Side H, streaming form (A 16-byte aligned with lda % 4 == 0): the same
// per-lane scheme as k_rhs_h_f32 with the loads of the next 16 rows issued
// before the MFMAs of the current ones (two register sets).  Every load is
// unconditional: rows are clamped to m - 1, columns past n to the row's last
// 16-byte segment and Y columns past k to k - 1, all valid addresses.  A row
// outside [r_begin, r_end) or a Y column past k then gets a zero Y value, so
// it adds nothing (an entry of A only meets its own column's outputs, and
// outputs past n are not stored).
// row pairs per register set of the streaming form: 12 for two output tiles
// (k > 32: 3.73 against 4.12 ms for W^T A at 10^6 x 2400, k = 50, although
// one wavefront per SIMD then fits), 8 for one (no gain from more)
template <int NT>
constexpr int h_set_rows() {
  return NT == 1 ? 8 : 12;
}

template <int NT>
struct HSet {
  static constexpr int U = h_set_rows<NT>();
  float4 a[U];
  float y[U][NT];
};

template <int NT>
__device__ __forceinline__ void h_load(HSet<NT>& S, const float* __restrict__ A, int64_t lda,
                                       const float* __restrict__ Y, int64_t ldy, int64_t r, int64_t m, int64_t colc,
                                       int h, int j, int k) {
#pragma unroll
  for (int u = 0; u < HSet<NT>::U; ++u) {
    const int64_t rr = r + 2 * u + h;
    const int64_t rc = rr < m ? rr : m - 1;
    S.a[u] = load_stream(A + rc * lda + colc);
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      const int c = 32 * tt + j;
      S.y[u][tt] = Y[rc * ldy + (c < k ? c : k - 1)];
    }
  }
}

template <int NT>
__device__ __forceinline__ void h_compute(const HSet<NT>& S, v16f (&acc)[4][NT], int64_t r, int64_t r_end, int h,
                                          int j, int k) {
#pragma unroll
  for (int u = 0; u < HSet<NT>::U; ++u) {
    const bool rok = r + 2 * u + h < r_end;
    const float av[4] = {S.a[u].x, S.a[u].y, S.a[u].z, S.a[u].w};
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      const float yv = (rok && 32 * tt + j < k) ? S.y[u][tt] : 0.0f;
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q][tt] = mfma32(yv, av[q], acc[q][tt]);
    }
  }
}

template <int NT>
__global__ __launch_bounds__(64) void k_rhs_h_f32s(int64_t m, int64_t n, int k, const float* __restrict__ A,
                                                   int64_t lda, const float* __restrict__ Y, int64_t ldy,
                                                   float* __restrict__ P, int64_t ldp, int64_t rows_per_split,
                                                   int64_t split_stride, int64_t ngroups, int64_t nsplit) {
  const int64_t per_xcd = gridDim.x / 8;
  const int64_t lid = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (lid >= ngroups * nsplit) return;
  const int64_t gx = lid % ngroups, gy = lid / ngroups;
  const int lane = threadIdx.x;
  const int j = lane & 31, h = lane >> 5;
  const int64_t col = gx * kHCols + 4 * j;
  const int64_t colc = col < lda - 3 ? col : lda - 4;
  const int64_t r_begin = gy * rows_per_split;
  const int64_t r_end = (r_begin + rows_per_split < m) ? r_begin + rows_per_split : m;

  v16f acc[4][NT];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) acc[q][tt] = v16f{};

  constexpr int kG = 2 * HSet<NT>::U;  // rows per register set
  HSet<NT> S0, S1;
  h_load<NT>(S0, A, lda, Y, ldy, r_begin, m, colc, h, j, k);
  h_load<NT>(S1, A, lda, Y, ldy, r_begin + kG, m, colc, h, j, k);
  for (int64_t r = r_begin; r < r_end; r += 2 * kG) {
    h_compute<NT>(S0, acc, r, r_end, h, j, k);
    h_load<NT>(S0, A, lda, Y, ldy, r + 2 * kG, m, colc, h, j, k);
    h_compute<NT>(S1, acc, r + kG, r_end, h, j, k);
    h_load<NT>(S1, A, lda, Y, ldy, r + 3 * kG, m, colc, h, j, k);
  }
  float* out = P + gy * split_stride;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t row = col + q;
    if (row >= n) continue;
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int c = 32 * tt + (v & 3) + 8 * (v >> 2) + 4 * h;
        if (c < k) out[row * ldp + c] = acc[q][tt][v];
      }
  }
}

// R[row][c] = sum_s P[s][row][c], summed in FP64 in split order.
__global__ void k_split_reduce(int64_t n, int k, int S, const float* __restrict__ P, int64_t split_stride,
                               float* __restrict__ R, int64_t ldr) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int64_t row = e / k;
  const int c = (int)(e - row * k);
  double s = 0.0;
  for (int sp = 0; sp < S; ++sp) s += (double)P[sp * split_stride + e];
  R[row * ldr + c] = (float)s;
}

struct HSplit {
  int64_t colgroups;
  int S;
  int64_t rows_per_split;
};

HSplit h_split(int64_t m, int64_t n) {
  HSplit s;
  s.colgroups = nmf::cdiv(n, kHCols);
  const int64_t target_waves = 4096;
  int64_t S = nmf::cdiv(target_waves, s.colgroups);
  const int64_t max_s = m / 512 > 1 ? m / 512 : 1;
  if (S > max_s) S = max_s;
  if (S > 65535) S = 65535;
  if (S < 1) S = 1;
  int64_t rps = nmf::cdiv(m, S);
  rps = (rps + 2 * kHUnroll - 1) / (2 * kHUnroll) * (2 * kHUnroll);
  s.S = (int)nmf::cdiv(m, rps > 0 ? rps : 1);
  if (s.S < 1) s.S = 1;
  s.rows_per_split = rps > 0 ? rps : 2 * kHUnroll;
  return s;
}

// Leading dimension of the transposed, padded Y of the streaming side-W kernel:
// whole 64-column blocks of the transposition kernel, whole chunks of the product.
static_assert(64 % kSC == 0, "a transposition block covers whole chunks");
int64_t w_yt_ld(int64_t n) { return nmf::cdiv(n, 64) * 64; }

bool w_streaming(const float* A, int64_t lda) { return (lda % 4 == 0) && ((uintptr_t)A % 16 == 0); }

// Contraction split of the streaming side-W kernel: as many column ranges as
// fit row tiles x ranges into kWSplitBlocks workgroups (three resident per CU
// on 256 CUs: one whole round, since a second partial round of these
// long-lived workgroups would nearly double the time), each range at least
// kWSplitMinChunks chunks long.
constexpr int64_t kWSplitBlocks = 768;
constexpr int64_t kWSplitMinChunks = 64;
struct WSplit {
  int S;
  int64_t cps;  // columns per range, a multiple of the chunk
};
WSplit w_split(int64_t m, int64_t n) {
  const int64_t tiles = nmf::cdiv(m, kWTM);
  int64_t S = tiles > 0 ? kWSplitBlocks / tiles : 1;
  if (S <= 1 && n >= 1024 * kSC) {
    // at least a round of tiles and a long contraction: the split count up
    // to 8 whose workgroups fill their last round best
    double best = 0.0;
    for (int64_t q = 1; q <= 8; ++q) {
      const int64_t blocks = tiles * q;
      const double fill = (double)blocks / (double)(nmf::cdiv(blocks, kWSplitBlocks) * kWSplitBlocks);
      if (fill > best + 1e-9) {
        best = fill;
        S = q;
      }
    }
  }
  const int64_t max_s = n / (kWSplitMinChunks * kSC);
  if (S > max_s) S = max_s;
  if (S > 65535) S = 65535;
  if (S < 1) S = 1;
  int64_t cps = nmf::cdiv(nmf::cdiv(n, S), kSC) * kSC;
  if (cps < kSC) cps = kSC;
  WSplit w;
  w.S = (int)nmf::cdiv(n, cps);
  if (w.S < 1) w.S = 1;
  w.cps = w.S > 1 ? cps : (n > 0 ? n : 1);
  return w;
}
// floats of the side-W scratch: the transposed Y, then (split) the partials
size_t w_yt_floats(int64_t n, int k) { return (size_t)(k <= 32 ? 32 : 64) * w_yt_ld(n); }

template <int NT>
int launch_w_f32(int64_t m, int64_t n, int k, const float* A, int64_t lda, const float* Y, int64_t ldy,
                 float* R, int64_t ldr, float* yt, hipStream_t s) {
  const dim3 grid((unsigned)nmf::cdiv(m, kWTM));
  if (w_streaming(A, lda)) {
    const int64_t ldt = w_yt_ld(n);
    const WSplit sp = w_split(m, n);
    float* partial = yt + w_yt_floats(n, k);
    float* P = sp.S > 1 ? partial : R;
    const int64_t ldp = sp.S > 1 ? k : ldr;
    const int64_t stride = sp.S > 1 ? m * k : 0;
    hipLaunchKernelGGL(k_transpose_y, dim3((unsigned)(ldt / 64)), dim3(256), 0, s, n, k, 32 * NT, Y, ldy, yt, ldt);
    NMF_TRY(nmf::launch_status("rhs side W (fp32): transpose Y"));
    nmf::mark_begin(s);
    hipLaunchKernelGGL((k_rhs_w_f32s<NT>), dim3(grid.x, (unsigned)sp.S), dim3(256), 0, s, m, n, k, A, lda, yt, ldt,
                       P, ldp, sp.cps, stride);
    nmf::mark_end(s);
    NMF_TRY(nmf::launch_status("rhs side W (fp32)"));
    if (sp.S > 1) {
      hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)nmf::cdiv(m * k, 256)), dim3(256), 0, s, m, k, sp.S, partial,
                         stride, R, ldr);
      NMF_TRY(nmf::launch_status("rhs side W reduce"));
    }
    return NMF_OK;
  }
  nmf::mark_begin(s);
  hipLaunchKernelGGL((k_rhs_w_f32<NT, false>), grid, dim3(256), 0, s, m, n, k, A, lda, Y, ldy, R, ldr);
  nmf::mark_end(s);
  return nmf::launch_status("rhs side W (fp32)");
}

template <int NT>
int launch_h_f32(int64_t m, int64_t n, int k, const float* A, int64_t lda, const float* Y, int64_t ldy,
                 float* R, int64_t ldr, float* partial, hipStream_t s) {
  const HSplit sp = h_split(m, n);
  const bool vec = (lda % 4 == 0) && ((uintptr_t)A % 16 == 0);
  float* P = sp.S > 1 ? partial : R;
  const int64_t ldp = sp.S > 1 ? k : ldr;
  const int64_t stride = sp.S > 1 ? n * k : 0;
  const dim3 grid((unsigned)(nmf::cdiv(sp.colgroups * sp.S, 8) * 8));
  nmf::mark_begin(s);
  if (vec && n >= 4)
    hipLaunchKernelGGL((k_rhs_h_f32s<NT>), grid, dim3(64), 0, s, m, n, k, A, lda, Y, ldy, P, ldp,
                       sp.rows_per_split, stride, sp.colgroups, (int64_t)sp.S);
  else if (vec)
    hipLaunchKernelGGL((k_rhs_h_f32<NT, true>), grid, dim3(64), 0, s, m, n, k, A, lda, Y, ldy, P, ldp,
                       sp.rows_per_split, stride, sp.colgroups, (int64_t)sp.S);
  else
    hipLaunchKernelGGL((k_rhs_h_f32<NT, false>), grid, dim3(64), 0, s, m, n, k, A, lda, Y, ldy, P, ldp,
                       sp.rows_per_split, stride, sp.colgroups, (int64_t)sp.S);
  nmf::mark_end(s);
  NMF_TRY(nmf::launch_status("rhs side H (fp32)"));
  if (sp.S > 1) {
    hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)nmf::cdiv(n * k, 256)), dim3(256), 0, s, n, k, sp.S,
                       partial, stride, R, ldr);
    NMF_TRY(nmf::launch_status("rhs side H reduce"));
  }
  return NMF_OK;
}

}  // namespace

// BF16X3 entry points (rhs_bf16.hip)
namespace nmf {
int bf16x3_plan(int side, int64_t m, int64_t n, int k, Carver& c, void** scratch);
int bf16x3_launch(int side, int64_t m, int64_t n, int k, const void* Bt, const float* Y, int64_t ldy, float* R,
                  int64_t ldr, void* scratch, hipStream_t s, bool y_ready);
int64_t bf16x3_chain(int side, int64_t m, int64_t n, int k);
}

namespace nmf {

int rhs_dense_plan(int side, int64_t m, int64_t n, int k, int prec, Carver& c, void** scratch) {
  *scratch = nullptr;
  if (prec == NMF_BF16X3) return bf16x3_plan(side, m, n, k, c, scratch);
  if (side == NMF_SIDE_W) {
    // transposed, padded Y of the streaming kernel (whatever A's alignment),
    // then the partials of a split contraction
    const WSplit sp = w_split(m, n);
    *scratch = c.take<float>(w_yt_floats(n, k) + (sp.S > 1 ? (size_t)sp.S * m * k : 0));
  } else {
    const HSplit sp = h_split(m, n);
    if (sp.S > 1) *scratch = c.take<float>((size_t)sp.S * n * k);
  }
  return NMF_OK;
}

int rhs_dense_launch(int side, int64_t m, int64_t n, int k, const float* A, int64_t lda, const void* Bt,
                     const float* Y, int64_t ldy, float* R, int64_t ldr, int prec, void* scratch, hipStream_t s,
                     bool y_ready) {
  if (prec == NMF_BF16X3) return bf16x3_launch(side, m, n, k, Bt, Y, ldy, R, ldr, scratch, s, y_ready);
  if (side == NMF_SIDE_W) {
    if (m == 0) return NMF_OK;
    float* yt = static_cast<float*>(scratch);
    return k <= 32 ? launch_w_f32<1>(m, n, k, A, lda, Y, ldy, R, ldr, yt, s)
                   : launch_w_f32<2>(m, n, k, A, lda, Y, ldy, R, ldr, yt, s);
  }
  if (n == 0) return NMF_OK;
  return k <= 32 ? launch_h_f32<1>(m, n, k, A, lda, Y, ldy, R, ldr, static_cast<float*>(scratch), s)
                 : launch_h_f32<2>(m, n, k, A, lda, Y, ldy, R, ldr, static_cast<float*>(scratch), s);
}

}  // namespace nmf

namespace {
// out (cols x rows) = X^T through a 64 x 65 LDS tile (odd pitch: conflict-free
// column reads); block (bx, by) takes rows 64 bx .. and columns 64 by ..
__global__ __launch_bounds__(256) void k_transpose_f32(int64_t rows, int64_t cols, const float* __restrict__ X,
                                                       int64_t ldx, float* __restrict__ out, int64_t ldo) {
  __shared__ float tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i, c = c0 + tx;
    if (r < rows && c < cols) tile[i][tx] = X[r * ldx + c];
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < cols && r < rows) out[c * ldo + r] = tile[tx][i];
  }
}
}  // namespace

extern "C" int nmf_transpose_f32(int64_t rows, int64_t cols, const float* X, int64_t ldx, float* out, int64_t ldo,
                                 void* stream) {
  if (rows < 0 || cols < 0) return nmf::fail(NMF_EINVAL, "nmf_transpose_f32: negative size");
  if (rows == 0 || cols == 0) return NMF_OK;  // nothing is read or written
  if (ldx < cols || ldo < rows) return nmf::fail(NMF_EINVAL, "nmf_transpose_f32: short leading dimension");
  if (!X || !out) return nmf::fail(NMF_EINVAL, "nmf_transpose_f32: null pointer");
  const int64_t gx = nmf::cdiv(rows, 64), gy = nmf::cdiv(cols, 64);
  if (gy > 65535 || gx > 0x7fffffff)
    return nmf::fail(NMF_EINVAL, "nmf_transpose_f32: %lld x %lld exceeds the grid", (long long)rows, (long long)cols);
  hipLaunchKernelGGL(k_transpose_f32, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, nmf::as_stream(stream), rows,
                     cols, X, ldx, out, ldo);
  return nmf::launch_status("nmf_transpose_f32");
}

static int check_rhs_args(int side, int64_t m, int64_t n, int k, int prec, const float* A, int64_t lda,
                          const void* Bt, const float* Y, int64_t ldy, const float* R, int64_t ldr) {
  if (side != NMF_SIDE_W && side != NMF_SIDE_H) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense: bad side %d", side);
  if (prec != NMF_F32 && prec != NMF_BF16X3) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense: bad prec %d", prec);
  if (!nmf::valid_k(k)) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense: k=%d outside [1,64]", k);
  if (m < 0 || n < 0) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense: negative size");
  if (ldy < k || ldr < k) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense: ldy/ldr < k");
  const int64_t rows_out = side == NMF_SIDE_W ? m : n;
  if (rows_out > 0 && !R) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense: R is null");
  if (m > 0 && n > 0 && !Y) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense: Y is null");
  if (prec == NMF_F32) {
    if (lda < n) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense: lda < n");
    if (m > 0 && n > 0 && !A) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense: A is null");
  } else {
    if (m > 0 && n > 0 && !Bt) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense: the tiled BF16 operand is null");
  }
  return NMF_OK;
}

extern "C" int nmf_rhs_dense_chain(int side, int64_t m, int64_t n, int k, int prec, int64_t* terms) {
  if (!terms) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense_chain: terms is null");
  if (side != NMF_SIDE_W && side != NMF_SIDE_H) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense_chain: bad side");
  if (prec != NMF_F32 && prec != NMF_BF16X3) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense_chain: bad prec");
  if (!nmf::valid_k(k) || m < 0 || n < 0) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense_chain: bad sizes");
  if (prec == NMF_BF16X3) {
    *terms = nmf::bf16x3_chain(side, m, n, k);
  } else if (side == NMF_SIDE_W) {
    const WSplit sp = w_split(m, n);
    *terms = sp.S > 1 ? sp.cps : n;
  } else {
    const HSplit sp = h_split(m, n);
    *terms = sp.S > 1 ? sp.rows_per_split : m;
  }
  return NMF_OK;
}

extern "C" int nmf_rhs_dense_workspace_bytes(int side, int64_t m, int64_t n, int k, int prec, size_t* bytes) {
  if (!bytes) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense_workspace_bytes: bytes is null");
  if (side != NMF_SIDE_W && side != NMF_SIDE_H) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense_workspace_bytes: bad side");
  if (prec != NMF_F32 && prec != NMF_BF16X3) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense_workspace_bytes: bad prec");
  if (!nmf::valid_k(k) || m < 0 || n < 0) return nmf::fail(NMF_EINVAL, "nmf_rhs_dense_workspace_bytes: bad sizes");
  nmf::Carver c(nullptr, 0);
  void* scratch;
  NMF_TRY(nmf::rhs_dense_plan(side, m, n, k, prec, c, &scratch));
  *bytes = c.off;
  return NMF_OK;
}

extern "C" int nmf_rhs_dense(int side, int64_t m, int64_t n, int k, const float* A, int64_t lda, const void* B_bf16,
                             const float* Y, int64_t ldy, float* R, int64_t ldr, int prec, void* ws, size_t ws_bytes,
                             void* stream) {
  NMF_TRY(check_rhs_args(side, m, n, k, prec, A, lda, B_bf16, Y, ldy, R, ldr));
  nmf::Carver c(ws, ws_bytes);
  void* scratch;
  NMF_TRY(nmf::rhs_dense_plan(side, m, n, k, prec, c, &scratch));
  if (c.off > 0 && (!ws || !c.fits()))
    return nmf::fail(NMF_EWORKSPACE, "nmf_rhs_dense: workspace %zu < %zu bytes", ws_bytes, c.off);
  // an empty contraction gives R = 0
  if (n == 0 && side == NMF_SIDE_W) return nmf::zero_f32(R, m, k, ldr, nmf::as_stream(stream));
  if (m == 0 && side == NMF_SIDE_H) return nmf::zero_f32(R, n, k, ldr, nmf::as_stream(stream));
  return nmf::rhs_dense_launch(side, m, n, k, A, lda, B_bf16, Y, ldy, R, ldr, prec, scratch, nmf::as_stream(stream));
}
