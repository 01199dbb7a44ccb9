// Learned warm start for BPP: features, the passive-set network, its
// training (forward, backward, Adam) and its fused inference.
//
// The BPP method (Section "Block Principal Pivoting") searches for the
// passive set of each NNLS problem; a good starting set saves rounds.  The
// network maps a problem's data to a starting set:
//   phi = [ s / ||s||_2 , diag(G) / mean(diag(G)) ],  s_i = f_i / sqrt(G_ii)
//         (s_i = 0 for pinned indices, G_ii <= 1e-14 max G_ll)
//   h1 = relu(phi W1 + b1), h2 = relu(h1 W2 + b2), z = h2 W3 + b3   (2k -> 128 -> 128 -> k)
//   F0 = { i : z_i > 0 } minus pinned indices
// trained with the mean binary cross-entropy against the converged BPP
// passive sets.  Parameters are one FP32 vector: W1[2k][128], b1[128],
// W2[128][128], b2[128], W3[128][k], b3[k] (input-major).
//
// Training is FP32 and deterministic: per-sample activations and their
// gradients (one block per 8 samples), then all weight gradients as
// LDS-tiled act^T dact products summed over the batch in sample order, then
// Adam.  Inference fuses the features
// and the three layers on v_mfma_f32_16x16x32_bf16: a wavefront takes 16
// problems, the hidden activations stay in the MFMA accumulators and are
// fed back as the next layer's B operand (the next layer's weights are staged
// in LDS in the matching permuted order), so nothing but R and the mask
// touches memory per problem.
#include <math.h>

#include "nmf_common.h"

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

namespace {

constexpr int kH = 128;

struct Layout {
  int k, in, W1, b1, W2, b2, W3, b3, total;
};

__host__ __device__ inline Layout layout(int k) {
  Layout L;
  L.k = k;
  L.in = 2 * k;
  L.W1 = 0;
  L.b1 = L.W1 + L.in * kH;
  L.W2 = L.b1 + kH;
  L.b2 = L.W2 + kH * kH;
  L.W3 = L.b2 + kH;
  L.b3 = L.W3 + kH * k;
  L.total = L.b3 + k;
  return L;
}

// ------------------------------------------------------------- features --
__device__ inline void diag_stats(int k, const double* __restrict__ G, double* dmax, double* mean) {
  double mx = 0.0, sum = 0.0;
  for (int q = 0; q < k; ++q) {
    const double d = G[q * k + q];
    mx = fmax(mx, d);
    sum += d;
  }
  *dmax = mx;
  *mean = sum / k;
}

// One wavefront per sampled problem b = e * stride; lane i < k owns index i.
__global__ __launch_bounds__(256) void k_features(int k, int64_t batch, int64_t stride, const double* __restrict__ G,
                                                  const float* __restrict__ R, int64_t ldr, float* __restrict__ phi) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  double dmax, mean;
  diag_stats(k, G, &dmax, &mean);
  const bool ok = lane < k;
  const double d = ok ? G[lane * k + lane] : 0.0;
  const bool pinned = !ok || d <= 1e-14 * dmax;
  const int64_t ns = (batch + stride - 1) / stride;
  for (int64_t e = wave; e < ns; e += nwaves) {
    const int64_t b = e * stride;
    const double f = ok ? (double)R[b * ldr + lane] : 0.0;
    const double sv = pinned ? 0.0 : f / sqrt(d);
    const double nrm = sqrt(wave_sum_f64(sv * sv));
    if (ok) {
      phi[e * 2 * k + lane] = (float)(nrm > 0.0 ? sv / nrm : 0.0);
      phi[e * 2 * k + k + lane] = (float)(mean > 0.0 ? d / mean : 0.0);
    }
  }
}

// ------------------------------------------------------------- training --
constexpr int kSB = 4;  // samples per block in the activation pass (8: 1.54 ms per 20 steps, 4: 1.17 ms; same parameters)

__device__ __forceinline__ int64_t sample_index(int64_t step, int64_t pos, int64_t nsamp, int sequential,
                                                const int64_t* __restrict__ order, int batch) {
  if (order) return order[step * batch + pos];
  const uint64_t q = (uint64_t)(step * 1000003 + pos);
  if (sequential) return (int64_t)(q % (uint64_t)nsamp);
  // Fibonacci hashing of (step, position): a fixed pseudo-random draw
  return (int64_t)(((q + 1) * 0x9E3779B97F4A7C15ull >> 11) % (uint64_t)nsamp);
}

// Per-sample forward pass, loss and activation gradients for kSB samples.
// Writes the gathered features and the activations the weight gradients need.
__global__ __launch_bounds__(kH) void k_mlp_act(int k, int batch, int64_t nsamp, int64_t step, int sequential,
                                                const int64_t* __restrict__ order, const float* __restrict__ p, const float* __restrict__ phi_all,
                                                const uint64_t* __restrict__ mask_all, float* __restrict__ xg,
                                                float* __restrict__ h1g, float* __restrict__ h2g,
                                                float* __restrict__ dzg, float* __restrict__ dh1g,
                                                float* __restrict__ dh2g, double* __restrict__ lossg) {
  const Layout L = layout(k);
  __shared__ float xs[kSB][128];
  __shared__ float hs1[kSB][kH];
  __shared__ float hs2[kSB][kH];
  __shared__ float dzs[kSB][64];
  __shared__ float dh2s[kSB][kH];
  __shared__ uint64_t ms[kSB];
  __shared__ double ls[kSB][64];
  const int u = threadIdx.x;
  const int b0 = blockIdx.x * kSB;
  const int ns = (batch - b0) < kSB ? (batch - b0) : kSB;
  const float scale = 1.0f / ((float)batch * (float)k);
  for (int e = u; e < kSB * L.in; e += kH) {
    const int s = e / L.in, i = e - s * L.in;
    float v = 0.0f;
    if (s < ns) {
      const int64_t src = sample_index(step, b0 + s, nsamp, sequential, order, batch);
      v = phi_all[src * L.in + i];
      xg[(int64_t)(b0 + s) * L.in + i] = v;
    }
    xs[s][i] = v;
  }
  if (u < kSB) ms[u] = (u < ns) ? mask_all[sample_index(step, b0 + u, nsamp, sequential, order, batch)] : 0ull;
  __syncthreads();
  float acc[kSB];
  // layer 1
#pragma unroll
  for (int s = 0; s < kSB; ++s) acc[s] = p[L.b1 + u];
  for (int i = 0; i < L.in; ++i) {
    const float w = p[L.W1 + i * kH + u];
#pragma unroll
    for (int s = 0; s < kSB; ++s) acc[s] += xs[s][i] * w;
  }
#pragma unroll
  for (int s = 0; s < kSB; ++s) hs1[s][u] = fmaxf(acc[s], 0.0f);
  __syncthreads();
  // layer 2
#pragma unroll
  for (int s = 0; s < kSB; ++s) acc[s] = p[L.b2 + u];
  for (int v = 0; v < kH; ++v) {
    const float w = p[L.W2 + v * kH + u];
#pragma unroll
    for (int s = 0; s < kSB; ++s) acc[s] += hs1[s][v] * w;
  }
#pragma unroll
  for (int s = 0; s < kSB; ++s) hs2[s][u] = fmaxf(acc[s], 0.0f);
  __syncthreads();
  // layer 3, loss and dz
  if (u < k) {
#pragma unroll
    for (int s = 0; s < kSB; ++s) acc[s] = p[L.b3 + u];
    for (int v = 0; v < kH; ++v) {
      const float w = p[L.W3 + v * k + u];
#pragma unroll
      for (int s = 0; s < kSB; ++s) acc[s] += hs2[s][v] * w;
    }
#pragma unroll
    for (int s = 0; s < kSB; ++s) {
      const float z = acc[s];
      const float t = (float)((ms[s] >> u) & 1ull);
      const float sig = 1.0f / (1.0f + expf(-z));
      dzs[s][u] = (s < ns) ? (sig - t) * scale : 0.0f;
      const double zl = (double)z;
      ls[s][u] = (s < ns) ? (fmax(zl, 0.0) + log1p(exp(-fabs(zl))) - (double)t * zl) : 0.0;
    }
  }
  __syncthreads();
  // dh2 = (dz W3^T) * [h2 > 0]
#pragma unroll
  for (int s = 0; s < kSB; ++s) acc[s] = 0.0f;
  for (int c = 0; c < k; ++c) {
    const float w = p[L.W3 + u * k + c];
#pragma unroll
    for (int s = 0; s < kSB; ++s) acc[s] += dzs[s][c] * w;
  }
#pragma unroll
  for (int s = 0; s < kSB; ++s) dh2s[s][u] = hs2[s][u] > 0.0f ? acc[s] : 0.0f;
  __syncthreads();
  // dh1 = (dh2 W2^T) * [h1 > 0]
#pragma unroll
  for (int s = 0; s < kSB; ++s) acc[s] = 0.0f;
  for (int v = 0; v < kH; ++v) {
    const float w = p[L.W2 + u * kH + v];
#pragma unroll
    for (int s = 0; s < kSB; ++s) acc[s] += dh2s[s][v] * w;
  }
  for (int s = 0; s < ns; ++s) {
    const int64_t row = b0 + s;
    dh1g[row * kH + u] = hs1[s][u] > 0.0f ? acc[s] : 0.0f;
    dh2g[row * kH + u] = dh2s[s][u];
    h1g[row * kH + u] = hs1[s][u];
    h2g[row * kH + u] = hs2[s][u];
    if (u < k) dzg[row * k + u] = dzs[s][u];
  }
  // block loss partial (fixed order)
  __syncthreads();
  if (u == 0) {
    double tot = 0.0;
    for (int s = 0; s < ns; ++s)
      for (int c = 0; c < k; ++c) tot += ls[s][c];
    lossg[blockIdx.x] = tot;
  }
}

// Weight and bias gradients as act^T dact products over the batch, one
// launch for all three layers: the grid is the union of 64 x 64 output tiles
// of dW1 (2k x 128), dW2 (128 x 128), dW3 (128 x k) plus one row of bias
// tiles.  Each thread owns a 4 x 4 block and sums the batch in sample order
// through LDS chunks of 32 samples, so the result is deterministic.
constexpr int kGT = 64;   // output tile edge
constexpr int kGB = 32;   // samples per LDS chunk
constexpr int kGSplit = 128;  // samples per batch split (blockIdx.y); partials summed in split order

struct GradRegion {
  const float* act;  // nullptr: bias (act = 1)
  int lda;
  const float* dact;
  int ldd;
  int rows, cols;    // rows = input units (or 1 for a bias), cols = output units
  int off;           // parameter offset
};

__global__ __launch_bounds__(256) void k_mlp_wgrad(int k, int batch, const float* __restrict__ xg,
                                                   const float* __restrict__ h1g, const float* __restrict__ h2g,
                                                   const float* __restrict__ dzg, const float* __restrict__ dh1g,
                                                   const float* __restrict__ dh2g, float* __restrict__ gpart) {
  const Layout L = layout(k);
  auto region = [&](int r) -> GradRegion {
    switch (r) {
      case 0: return {xg, L.in, dh1g, kH, L.in, kH, L.W1};
      case 1: return {h1g, kH, dh2g, kH, kH, kH, L.W2};
      case 2: return {h2g, kH, dzg, k, kH, k, L.W3};
      case 3: return {nullptr, 0, dh1g, kH, 1, kH, L.b1};
      case 4: return {nullptr, 0, dh2g, kH, 1, kH, L.b2};
      default: return {nullptr, 0, dzg, k, 1, k, L.b3};
    }
  };
  // locate this block's tile
  int tile = blockIdx.x, r = 0;
  int tr = 0, tc = 0;
  for (r = 0; r < 6; ++r) {
    const GradRegion q = region(r);
    const int nt = ((q.rows + kGT - 1) / kGT) * ((q.cols + kGT - 1) / kGT);
    if (tile < nt) {
      const int ntc = (q.cols + kGT - 1) / kGT;
      tr = tile / ntc;
      tc = tile - tr * ntc;
      break;
    }
    tile -= nt;
  }
  if (r >= 6) return;
  const GradRegion g = region(r);
  __shared__ __align__(16) float as[kGB][kGT];
  __shared__ __align__(16) float ds[kGB][kGT];
  const int t = threadIdx.x;
  const int ti = (t >> 4) * 4, tj = (t & 15) * 4;
  const int i0 = tr * kGT, j0 = tc * kGT;
  float acc[4][4] = {};
  const int bs = blockIdx.y * kGSplit;
  const int be = (bs + kGSplit < batch) ? bs + kGSplit : batch;
  float* grad = gpart + (int64_t)blockIdx.y * L.total;
  for (int b0 = bs; b0 < be; b0 += kGB) {
    __syncthreads();
    for (int e = t; e < kGB * kGT; e += 256) {
      const int bb = e / kGT, c = e - bb * kGT;
      const int b = b0 + bb;
      const bool okb = b < be;
      as[bb][c] = (okb && i0 + c < g.rows) ? (g.act ? g.act[(int64_t)b * g.lda + i0 + c] : 1.0f) : 0.0f;
      ds[bb][c] = (okb && j0 + c < g.cols) ? g.dact[(int64_t)b * g.ldd + j0 + c] : 0.0f;
    }
    __syncthreads();
    for (int bb = 0; bb < kGB; ++bb) {
      const float4 av = *reinterpret_cast<const float4*>(&as[bb][ti]);
      const float4 dv = *reinterpret_cast<const float4*>(&ds[bb][tj]);
      const float a4[4] = {av.x, av.y, av.z, av.w};
      const float d4[4] = {dv.x, dv.y, dv.z, dv.w};
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] += a4[x] * d4[y];
    }
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = i0 + ti + x, jj = j0 + tj + y;
      if (i < g.rows && jj < g.cols) grad[g.off + i * g.cols + jj] = acc[x][y];
    }
}

int wgrad_blocks(int k) {
  const Layout L = layout(k);
  auto nt = [](int r, int c) { return ((r + kGT - 1) / kGT) * ((c + kGT - 1) / kGT); };
  return nt(L.in, kH) + nt(kH, kH) + nt(kH, k) + nt(1, kH) + nt(1, kH) + nt(1, k);
}

// grad[e] = sum of the batch-split partials in split order
__global__ void k_grad_reduce(int n, int S, const float* __restrict__ gpart, float* __restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float s = 0.0f;
  for (int sp = 0; sp < S; ++sp) s += gpart[(int64_t)sp * n + e];
  grad[e] = s;
}

__global__ void k_adam(int n, int S, float* __restrict__ p, const float* __restrict__ gpart, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float gi = 0.0f;
  for (int sp = 0; sp < S; ++sp) gi += gpart[(int64_t)sp * n + e];
  const float mi = b1 * m[e] + (1.0f - b1) * gi;
  const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void k_sum_f64(int n, const double* __restrict__ a, double scale, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i];
  out[0] = s * scale;
}

// ----------------------------------------------------------- inference --
__device__ __forceinline__ uint16_t to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma16(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

union Pack8 {
  uint16_t h[8];
  uint32_t u[4];
  v8bf v;
  uint4 q;
};

// (a, b) rounded to BF16 (nearest even) in one packed conversion; a in the low half
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
// max(x, 0) as one integer max on the bit pattern (every negative float,
// -0 included, has a negative pattern); fmaxf of an MFMA result would first
// quieten a possible signalling NaN, a second instruction
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

// 16 x 16 MFMA output layout: lane (j, g) = (lane & 15, lane >> 4) holds rows
// 4g + v (v = 0..3) of column j.  A layer's accumulators are re-used as the
// next layer's B operand: in K-step s (32 hidden units), slot e of lane group
// g carries hidden unit 32s + 16(e >> 2) + 4g + (e & 3), i.e. register
// (e & 3) of output tile 2s + (e >> 2).  The next layer's weights are staged
// in LDS in the same order.
__device__ __forceinline__ int chain_unit(int s, int g, int e) { return 32 * s + 16 * (e >> 2) + 4 * g + (e & 3); }

// KS1: 32-wide K-steps of layer 1 (2k <= 32 KS1); NT3: 16-wide output tiles of layer 3.
// The weights as BF16 A operands, in LDS order: w1 [tile_out 8][kstep KS1][i 16][g 4][8],
// w2 [8][4][16][4][8], w3 [NT3][4][16][4][8], then the biases b1[128], b2[128], b3[64] (FP32).
template <int KS1, int NT3>
struct PackedNet {
  static constexpr int n1 = 8 * KS1 * 16 * 4 * 8;
  static constexpr int n2 = 8 * 4 * 16 * 4 * 8;
  static constexpr int n3 = NT3 * 4 * 16 * 4 * 8;
  static constexpr int bytes = 2 * (n1 + n2 + n3) + 4 * (kH + kH + 64);
};

// Builds the packed weights (one thread per entry); used directly by each
// inference block when no packed copy is supplied.
template <int KS1, int NT3>
__device__ inline void pack_entry(int k, const float* __restrict__ p, int e, uint16_t* w, float* bias) {
  using PN = PackedNet<KS1, NT3>;
  const Layout L = layout(k);
  if (e < PN::n1) {
    const int el = e & 7, gg = (e >> 3) & 3, i = (e >> 5) & 15, s = (e >> 9) % KS1, to = (e >> 9) / KS1;
    const int in = 32 * s + 8 * gg + el;
    w[e] = in < L.in ? to_bf16(p[L.W1 + in * kH + 16 * to + i]) : (uint16_t)0;
  } else if (e < PN::n1 + PN::n2) {
    const int f = e - PN::n1;
    const int el = f & 7, gg = (f >> 3) & 3, i = (f >> 5) & 15, s = (f >> 9) & 3, to = f >> 11;
    w[e] = to_bf16(p[L.W2 + chain_unit(s, gg, el) * kH + 16 * to + i]);
  } else if (e < PN::n1 + PN::n2 + PN::n3) {
    const int f = e - PN::n1 - PN::n2;
    const int el = f & 7, gg = (f >> 3) & 3, i = (f >> 5) & 15, s = (f >> 9) & 3, to = f >> 11;
    const int c = 16 * to + i;
    w[e] = c < k ? to_bf16(p[L.W3 + chain_unit(s, gg, el) * k + c]) : (uint16_t)0;
  } else {
    const int f = e - PN::n1 - PN::n2 - PN::n3;
    if (f < kH) bias[f] = p[L.b1 + f];
    else if (f < 2 * kH) bias[f] = p[L.b2 + f - kH];
    else if (f < 2 * kH + 64) bias[f] = (f - 2 * kH) < k ? p[L.b3 + f - 2 * kH] : 0.0f;
  }
}

template <int KS1, int NT3>
__global__ void k_mlp_pack(int k, const float* __restrict__ p, uint16_t* __restrict__ packed) {
  using PN = PackedNet<KS1, NT3>;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < PN::n1 + PN::n2 + PN::n3 + 2 * kH + 64)
    pack_entry<KS1, NT3>(k, p, e, packed, reinterpret_cast<float*>(packed + PN::n1 + PN::n2 + PN::n3));
}

template <int KS1, int NT3>
__global__ __launch_bounds__(256) void k_mlp_infer(int k, int64_t batch, const double* __restrict__ G,
                                                   const float* __restrict__ R, int64_t ldr,
                                                   const float* __restrict__ p, const uint16_t* __restrict__ packed,
                                                   uint64_t* __restrict__ mask_out) {
  using PN = PackedNet<KS1, NT3>;
  const Layout L = layout(k);
  __shared__ __align__(16) uint4 netbuf[(PN::bytes + 15) / 16];
  __shared__ float isd[64], gft[64];
  __shared__ uint64_t pinned_s;
  uint16_t* w1s = reinterpret_cast<uint16_t*>(netbuf);
  uint16_t* w2s = w1s + PN::n1;
  uint16_t* w3s = w2s + PN::n2;
  float* bias1 = reinterpret_cast<float*>(w3s + PN::n3);
  float* bias2 = bias1 + kH;
  float* bias3 = bias2 + kH;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int j = lane & 15, g = lane >> 4;

  if (packed) {
    const uint4* src = reinterpret_cast<const uint4*>(packed);
    for (int e = t; e < PN::bytes / 16; e += 256) netbuf[e] = src[e];
  } else {
    for (int e = t; e < PN::n1 + PN::n2 + PN::n3 + 2 * kH + 64; e += 256) pack_entry<KS1, NT3>(k, p, e, w1s, bias1);
  }
  if (t == 0) {
    double dmax, mean;
    diag_stats(k, G, &dmax, &mean);
    uint64_t pin = 0;
    for (int q = 0; q < k; ++q) {
      const double d = G[q * k + q];
      const bool pn = d <= 1e-14 * dmax;
      if (pn) pin |= 1ull << q;
      isd[q] = pn ? 0.0f : (float)(1.0 / sqrt(d));
      gft[q] = mean > 0.0 ? (float)(d / mean) : 0.0f;
    }
    for (int q = k; q < 64; ++q) isd[q] = gft[q] = 0.0f;
    pinned_s = pin;
  }
  __syncthreads();
  const uint64_t all = (k == 64) ? ~0ull : ((1ull << k) - 1ull);
  const uint64_t pinned = pinned_s;

  const int64_t ntiles = (batch + 15) / 16;
  const int64_t tstride = (int64_t)gridDim.x * 4;
  int64_t tile = (int64_t)blockIdx.x * 4 + wave;
  // raw right-hand sides of the next tile, loaded while the current one runs
  float rv[KS1][8];
  auto load_rhs = [&](int64_t tl) {
    const int64_t bb = tl * 16 + j;
    const bool okb = tl < ntiles && bb < batch;
#pragma unroll
    for (int s = 0; s < KS1; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int in = 32 * s + 8 * g + e;
        rv[s][e] = (okb && in < k) ? R[bb * ldr + in] : 0.0f;
      }
  };
  // per-lane constants: the scale and offset of each feature slot (slot
  // (s, e) of lane group g is input 32s + 8g + e), and the biases of the
  // output rows the lane holds (row 16t + 4g + v of tile t), which start the
  // accumulation of each layer
  float sc[KS1][8], ad[KS1][8];
#pragma unroll
  for (int s = 0; s < KS1; ++s)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int in = 32 * s + 8 * g + e;
      sc[s][e] = in < k ? isd[in] : 0.0f;
      ad[s][e] = (in >= k && in < L.in) ? gft[in - k] : 0.0f;
    }
  v4f b1v[8], b2v[8], b3v[NT3];
#pragma unroll
  for (int to = 0; to < 8; ++to)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      b1v[to][v] = bias1[16 * to + 4 * g + v];
      b2v[to][v] = bias2[16 * to + 4 * g + v];
    }
#pragma unroll
  for (int to = 0; to < NT3; ++to)
#pragma unroll
    for (int v = 0; v < 4; ++v) b3v[to][v] = bias3[16 * to + 4 * g + v];

  load_rhs(tile);
  for (; tile < ntiles; tile += tstride) {
    const int64_t b = tile * 16 + j;
    const bool ok = b < batch;
    // scaled right-hand side f_i / sqrt(G_ii) of problem b (zero past k)
    float tv[KS1][8];
    float ss = 0.0f;
#pragma unroll
    for (int s = 0; s < KS1; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float v = rv[s][e] * sc[s][e];
        ss = fmaf(v, v, ss);
        tv[s][e] = v;
      }
    load_rhs(tile + tstride);
    __builtin_amdgcn_sched_barrier(0);
    ss += __shfl_xor(ss, 16, 64);
    ss += __shfl_xor(ss, 32, 64);
    const float inv = ss > 0.0f ? 1.0f / sqrtf(ss) : 0.0f;
    // layer 1 (features: the normalised scaled right-hand side, then the
    // diagonal ratios)
    v4f a1[8];
#pragma unroll
    for (int s = 0; s < KS1; ++s) {
      Pack8 bx;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        bx.u[e] = pk_bf16(fmaf(tv[s][2 * e], inv, ad[s][2 * e]), fmaf(tv[s][2 * e + 1], inv, ad[s][2 * e + 1]));
#pragma unroll
      for (int to = 0; to < 8; ++to) {
        Pack8 wa;
        wa.q = *reinterpret_cast<const uint4*>(&w1s[(((to * KS1 + s) * 16 + j) * 4 + g) * 8]);
        a1[to] = mfma16(wa.v, bx.v, s == 0 ? b1v[to] : a1[to]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // layer 2
    v4f a2[8];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      Pack8 bx;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int ti = 2 * s + (e >> 1), v = 2 * (e & 1);
        bx.u[e] = pk_bf16(relu(a1[ti][v]), relu(a1[ti][v + 1]));
      }
#pragma unroll
      for (int to = 0; to < 8; ++to) {
        Pack8 wa;
        wa.q = *reinterpret_cast<const uint4*>(&w2s[(((to * 4 + s) * 16 + j) * 4 + g) * 8]);
        a2[to] = mfma16(wa.v, bx.v, s == 0 ? b2v[to] : a2[to]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // layer 3
    v4f a3[NT3];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      Pack8 bx;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int ti = 2 * s + (e >> 1), v = 2 * (e & 1);
        bx.u[e] = pk_bf16(relu(a2[ti][v]), relu(a2[ti][v + 1]));
      }
#pragma unroll
      for (int to = 0; to < NT3; ++to) {
        Pack8 wa;
        wa.q = *reinterpret_cast<const uint4*>(&w3s[(((to * 4 + s) * 16 + j) * 4 + g) * 8]);
        a3[to] = mfma16(wa.v, bx.v, s == 0 ? b3v[to] : a3[to]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    uint64_t bits = 0;
#pragma unroll
    for (int to = 0; to < NT3; ++to)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * to + 4 * g + v;
        if (c < k && a3[to][v] > 0.0f) bits |= 1ull << c;
      }
    bits |= __shfl_xor(bits, 16, 64);
    bits |= __shfl_xor(bits, 32, 64);
    if (ok && g == 0) mask_out[b] = bits & all & ~pinned;
  }
}

struct TrainPlan {
  float* xg;
  float* h1g;
  float* h2g;
  float* dzg;
  float* dh1g;
  float* dh2g;
  float* gpart;
  double* loss;
  int nblk;
  int nsplit;
};

void plan_train(int k, int batch, nmf::Carver& c, TrainPlan* P) {
  const Layout L = layout(k);
  P->nblk = (batch + kSB - 1) / kSB;
  P->xg = c.take<float>((size_t)batch * L.in);
  P->h1g = c.take<float>((size_t)batch * kH);
  P->h2g = c.take<float>((size_t)batch * kH);
  P->dzg = c.take<float>((size_t)batch * k);
  P->dh1g = c.take<float>((size_t)batch * kH);
  P->dh2g = c.take<float>((size_t)batch * kH);
  P->nsplit = (batch + kGSplit - 1) / kGSplit;
  P->gpart = c.take<float>((size_t)P->nsplit * L.total);
  P->loss = c.take<double>((size_t)P->nblk);
}

int grad_step(int k, int batch, int64_t nsamp, int64_t step, int sequential, const int64_t* order, const float* params,
              const float* phi, const uint64_t* masks, const TrainPlan& P, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_act, dim3(P.nblk), dim3(kH), 0, s, k, batch, nsamp, step, sequential, order, params, phi,
                     masks,
                     P.xg, P.h1g, P.h2g, P.dzg, P.dh1g, P.dh2g, P.loss);
  NMF_TRY(nmf::launch_status("mlp activations"));
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(wgrad_blocks(k), P.nsplit), dim3(256), 0, s, k, batch, P.xg, P.h1g, P.h2g,
                     P.dzg, P.dh1g, P.dh2g, P.gpart);
  return nmf::launch_status("mlp weight gradients");
}

}  // namespace

namespace nmf {

int features_launch(int k, int64_t batch, int64_t stride, const double* G, const float* R, int64_t ldr, float* phi,
                    hipStream_t s) {
  if (batch <= 0) return NMF_OK;
  const int64_t ns = cdiv(batch, stride);
  int64_t blocks = cdiv(ns, 4);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_features, dim3((unsigned)blocks), dim3(256), 0, s, k, batch, stride, G, R, ldr, phi);
  return launch_status("features");
}

int packed_bytes(int k) {
  if (k <= 16) return PackedNet<1, 1>::bytes;
  if (k <= 32) return PackedNet<2, 2>::bytes;
  return PackedNet<4, 4>::bytes;
}

int mlp_infer_plan(int k, int64_t batch, Carver& c, void** scratch) {
  (void)batch;
  *scratch = c.take<uint16_t>((size_t)packed_bytes(k) / 2 + 8);
  return NMF_OK;
}

// Packs the network's weights into `scratch` (BF16, LDS operand order).
int mlp_pack_launch(int k, const float* params, void* scratch, hipStream_t s) {
  uint16_t* out = static_cast<uint16_t*>(scratch);
  const int n = packed_bytes(k);  // entries <= bytes
  const dim3 grid((n + 255) / 256);
  if (k <= 16)
    hipLaunchKernelGGL((k_mlp_pack<1, 1>), grid, dim3(256), 0, s, k, params, out);
  else if (k <= 32)
    hipLaunchKernelGGL((k_mlp_pack<2, 2>), grid, dim3(256), 0, s, k, params, out);
  else
    hipLaunchKernelGGL((k_mlp_pack<4, 4>), grid, dim3(256), 0, s, k, params, out);
  return launch_status("mlp pack");
}

// scratch: packed weights from mlp_pack_launch, or null to pack per block.
int mlp_infer_launch(int k, int64_t batch, const double* G, const float* R, int64_t ldr, const float* params,
                     uint64_t* mask_out, void* scratch, hipStream_t s) {
  if (batch <= 0) return NMF_OK;
  const uint16_t* packed = static_cast<const uint16_t*>(scratch);
  const int64_t tiles = cdiv(batch, 16);
  int64_t blocks = cdiv(tiles, 4);
  if (blocks > 512) blocks = 512;
  if (k <= 16)
    hipLaunchKernelGGL((k_mlp_infer<1, 1>), dim3((unsigned)blocks), dim3(256), 0, s, k, batch, G, R, ldr, params,
                       packed, mask_out);
  else if (k <= 32)
    hipLaunchKernelGGL((k_mlp_infer<2, 2>), dim3((unsigned)blocks), dim3(256), 0, s, k, batch, G, R, ldr, params,
                       packed, mask_out);
  else
    hipLaunchKernelGGL((k_mlp_infer<4, 4>), dim3((unsigned)blocks), dim3(256), 0, s, k, batch, G, R, ldr, params,
                       packed, mask_out);
  return launch_status("mlp inference");
}

}  // namespace nmf

extern "C" int nmf_mlp_param_count(int k) { return nmf::valid_k(k) ? layout(k).total : -1; }

extern "C" int nmf_features(int k, int64_t batch, const double* G, const float* R, int64_t ldr, float* phi,
                            void* stream) {
  if (!nmf::valid_k(k) || batch < 0 || ldr < k) return nmf::fail(NMF_EINVAL, "nmf_features: bad sizes");
  if (batch > 0 && (!G || !R || !phi)) return nmf::fail(NMF_EINVAL, "nmf_features: null pointer");
  return nmf::features_launch(k, batch, 1, G, R, ldr, phi, nmf::as_stream(stream));
}

extern "C" int nmf_mlp_predict(int k, int64_t batch, const double* G, const float* R, int64_t ldr,
                               const float* params, uint64_t* mask_out, void* stream) {
  if (!nmf::valid_k(k) || batch < 0 || ldr < k) return nmf::fail(NMF_EINVAL, "nmf_mlp_predict: bad sizes");
  if (batch > 0 && (!G || !R || !params || !mask_out)) return nmf::fail(NMF_EINVAL, "nmf_mlp_predict: null pointer");
  return nmf::mlp_infer_launch(k, batch, G, R, ldr, params, mask_out, nullptr, nmf::as_stream(stream));
}

extern "C" int nmf_mlp_train_workspace_bytes(int k, int batch, size_t* bytes) {
  if (!bytes || !nmf::valid_k(k) || batch < 1) return nmf::fail(NMF_EINVAL, "nmf_mlp_train_workspace_bytes: bad args");
  nmf::Carver c(nullptr, 0);
  TrainPlan P;
  plan_train(k, batch, c, &P);
  *bytes = c.off;
  return NMF_OK;
}

extern "C" int nmf_mlp_grad(int k, int batch, const float* params, const float* phi, const uint64_t* masks,
                            float* grad_out, double* loss_out, void* ws, size_t ws_bytes, void* stream) {
  if (!nmf::valid_k(k) || batch < 1) return nmf::fail(NMF_EINVAL, "nmf_mlp_grad: bad sizes");
  if (!params || !phi || !masks || !grad_out) return nmf::fail(NMF_EINVAL, "nmf_mlp_grad: null pointer");
  nmf::Carver c(ws, ws_bytes);
  TrainPlan P;
  plan_train(k, batch, c, &P);
  if (!ws || !c.fits()) return nmf::fail(NMF_EWORKSPACE, "nmf_mlp_grad: workspace too small");
  hipStream_t s = nmf::as_stream(stream);
  NMF_TRY(grad_step(k, batch, batch, 0, 1, nullptr, params, phi, masks, P, s));
  const int total = layout(k).total;
  hipLaunchKernelGGL(k_grad_reduce, dim3((total + 255) / 256), dim3(256), 0, s, total, P.nsplit, P.gpart, grad_out);
  NMF_TRY(nmf::launch_status("mlp gradient reduce"));
  if (loss_out) {
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(64), 0, s, P.nblk, P.loss, 1.0 / ((double)batch * k), loss_out);
    NMF_TRY(nmf::launch_status("mlp loss"));
  }
  return NMF_OK;
}

extern "C" int nmf_mlp_train(int k, float* params, float* adam_m, float* adam_v, const float* phi,
                             const uint64_t* masks, int64_t nsamples, const int64_t* order, int steps, int batch,
                             float lr, int64_t step0, double* loss_out, void* ws, size_t ws_bytes, void* stream) {
  if (!nmf::valid_k(k) || batch < 1 || steps < 0 || nsamples < 1 || step0 < 0 || !(lr > 0.0f))
    return nmf::fail(NMF_EINVAL, "nmf_mlp_train: bad sizes");
  if (!params || !adam_m || !adam_v || !phi || !masks) return nmf::fail(NMF_EINVAL, "nmf_mlp_train: null pointer");
  nmf::Carver c(ws, ws_bytes);
  TrainPlan P;
  plan_train(k, batch, c, &P);
  if (!ws || !c.fits()) return nmf::fail(NMF_EWORKSPACE, "nmf_mlp_train: workspace too small");
  hipStream_t s = nmf::as_stream(stream);
  const int total = layout(k).total;
  const double b1 = 0.9, b2 = 0.999;
  for (int it = 0; it < steps; ++it) {
    const int64_t step = step0 + it;
    // with an explicit order, step t reads order[(t - step0) * batch ...]
    NMF_TRY(grad_step(k, batch, nsamples, order ? it : step, 0, order, params, phi, masks, P, s));
    const double t = (double)(step + 1);
    const float c1 = (float)(1.0 / (1.0 - pow(b1, t)));
    const float c2 = (float)(1.0 / (1.0 - pow(b2, t)));
    hipLaunchKernelGGL(k_adam, dim3((total + 255) / 256), dim3(256), 0, s, total, P.nsplit, params, P.gpart, adam_m,
                       adam_v, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
    NMF_TRY(nmf::launch_status("adam"));
  }
  if (loss_out && steps > 0) {
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(64), 0, s, P.nblk, P.loss, 1.0 / ((double)batch * k), loss_out);
    NMF_TRY(nmf::launch_status("mlp loss"));
  }
  return NMF_OK;
}
