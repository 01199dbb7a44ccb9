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
// gradients (one block per 8 samples), then every weight gradient as a
// fixed-order sum over the batch, then Adam.  Inference fuses the features
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
constexpr int kSB = 8;  // samples per block in the activation pass

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

// grad[e] for every parameter e, each a sum over the batch in sample order.
__global__ __launch_bounds__(256) void k_mlp_wgrad(int k, int batch, const float* __restrict__ xg,
                                                   const float* __restrict__ h1g, const float* __restrict__ h2g,
                                                   const float* __restrict__ dzg, const float* __restrict__ dh1g,
                                                   const float* __restrict__ dh2g, float* __restrict__ grad) {
  const Layout L = layout(k);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= L.total) return;
  const float* a;  // activation column (stride sa) or null for a bias
  const float* g;  // gradient column (stride sg)
  int sa = 0, sg = 0;
  if (e < L.b1) {
    const int i = e / kH, u = e - i * kH;
    a = xg + i, sa = L.in, g = dh1g + u, sg = kH;
  } else if (e < L.W2) {
    a = nullptr, g = dh1g + (e - L.b1), sg = kH;
  } else if (e < L.b2) {
    const int v = (e - L.W2) / kH, u = (e - L.W2) - v * kH;
    a = h1g + v, sa = kH, g = dh2g + u, sg = kH;
  } else if (e < L.W3) {
    a = nullptr, g = dh2g + (e - L.b2), sg = kH;
  } else if (e < L.b3) {
    const int v = (e - L.W3) / k, c = (e - L.W3) - v * k;
    a = h2g + v, sa = kH, g = dzg + c, sg = k;
  } else {
    a = nullptr, g = dzg + (e - L.b3), sg = k;
  }
  float acc = 0.0f;
  if (a) {
    for (int b = 0; b < batch; ++b) acc += a[(int64_t)b * sa] * g[(int64_t)b * sg];
  } else {
    for (int b = 0; b < batch; ++b) acc += g[(int64_t)b * sg];
  }
  grad[e] = acc;
}

__global__ void k_adam(int n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
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
  v8bf v;
  uint4 q;
};

// 16 x 16 MFMA output layout: lane (j, g) = (lane & 15, lane >> 4) holds rows
// 4g + v (v = 0..3) of column j.  A layer's accumulators are re-used as the
// next layer's B operand: in K-step s (32 hidden units), slot e of lane group
// g carries hidden unit 32s + 16(e >> 2) + 4g + (e & 3), i.e. register
// (e & 3) of output tile 2s + (e >> 2).  The next layer's weights are staged
// in LDS in the same order.
__device__ __forceinline__ int chain_unit(int s, int g, int e) { return 32 * s + 16 * (e >> 2) + 4 * g + (e & 3); }

// KS1: 32-wide K-steps of layer 1 (2k <= 32 KS1); NT3: 16-wide output tiles of layer 3.
template <int KS1, int NT3>
__global__ __launch_bounds__(256) void k_mlp_infer(int k, int64_t batch, const double* __restrict__ G,
                                                   const float* __restrict__ R, int64_t ldr,
                                                   const float* __restrict__ p, uint64_t* __restrict__ mask_out) {
  const Layout L = layout(k);
  // weights as BF16 A operands: [tile_out][kstep][i (16)][g (4)][8]
  __shared__ __align__(16) uint16_t w1s[8 * KS1 * 16 * 4 * 8];
  __shared__ __align__(16) uint16_t w2s[8 * 4 * 16 * 4 * 8];
  __shared__ __align__(16) uint16_t w3s[NT3 * 4 * 16 * 4 * 8];
  __shared__ float bias1[kH], bias2[kH], bias3[64];
  __shared__ float isd[64], gft[64];
  __shared__ uint64_t pinned_s;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int j = lane & 15, g = lane >> 4;

  for (int e = t; e < 8 * KS1 * 16 * 4 * 8; e += 256) {
    const int el = e & 7, gg = (e >> 3) & 3, i = (e >> 5) & 15, s = (e >> 9) % KS1, to = (e >> 9) / KS1;
    const int in = 32 * s + 8 * gg + el;
    w1s[e] = in < L.in ? to_bf16(p[L.W1 + in * kH + 16 * to + i]) : (uint16_t)0;
  }
  for (int e = t; e < 8 * 4 * 16 * 4 * 8; e += 256) {
    const int el = e & 7, gg = (e >> 3) & 3, i = (e >> 5) & 15, s = (e >> 9) & 3, to = e >> 11;
    w2s[e] = to_bf16(p[L.W2 + chain_unit(s, gg, el) * kH + 16 * to + i]);
  }
  for (int e = t; e < NT3 * 4 * 16 * 4 * 8; e += 256) {
    const int el = e & 7, gg = (e >> 3) & 3, i = (e >> 5) & 15, s = (e >> 9) & 3, to = e >> 11;
    const int c = 16 * to + i;
    w3s[e] = c < k ? to_bf16(p[L.W3 + chain_unit(s, gg, el) * k + c]) : (uint16_t)0;
  }
  for (int e = t; e < kH; e += 256) {
    bias1[e] = p[L.b1 + e];
    bias2[e] = p[L.b2 + e];
  }
  if (t < 64) bias3[t] = t < k ? p[L.b3 + t] : 0.0f;
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
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t b = tile * 16 + j;
    const bool ok = b < batch;
    // features of problem b: slot (s, e) of lane group g <-> input 32s + 8g + e
    float fv[KS1][8];
    float ss = 0.0f;
#pragma unroll
    for (int s = 0; s < KS1; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int in = 32 * s + 8 * g + e;
        float v = 0.0f;
        if (in < k) {
          v = ok ? R[b * ldr + in] * isd[in] : 0.0f;
          ss += v * v;
        } else if (in < L.in) {
          v = gft[in - k];
        }
        fv[s][e] = v;
      }
    __builtin_amdgcn_sched_barrier(0);
    ss += __shfl_xor(ss, 16, 64);
    ss += __shfl_xor(ss, 32, 64);
    const float inv = ss > 0.0f ? 1.0f / sqrtf(ss) : 0.0f;
    // layer 1
    v4f a1[8];
#pragma unroll
    for (int to = 0; to < 8; ++to) a1[to] = v4f{};
#pragma unroll
    for (int s = 0; s < KS1; ++s) {
      Pack8 bx;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int in = 32 * s + 8 * g + e;
        bx.h[e] = to_bf16(in < k ? fv[s][e] * inv : fv[s][e]);
      }
#pragma unroll
      for (int to = 0; to < 8; ++to) {
        Pack8 wa;
        wa.q = *reinterpret_cast<const uint4*>(&w1s[(((to * KS1 + s) * 16 + j) * 4 + g) * 8]);
        a1[to] = mfma16(wa.v, bx.v, a1[to]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // layer 2
    v4f a2[8];
#pragma unroll
    for (int to = 0; to < 8; ++to) a2[to] = v4f{};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      Pack8 bx;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int ti = 2 * s + (e >> 2), v = e & 3;
        bx.h[e] = to_bf16(fmaxf(a1[ti][v] + bias1[16 * ti + 4 * g + v], 0.0f));
      }
#pragma unroll
      for (int to = 0; to < 8; ++to) {
        Pack8 wa;
        wa.q = *reinterpret_cast<const uint4*>(&w2s[(((to * 4 + s) * 16 + j) * 4 + g) * 8]);
        a2[to] = mfma16(wa.v, bx.v, a2[to]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // layer 3
    v4f a3[NT3];
#pragma unroll
    for (int to = 0; to < NT3; ++to) a3[to] = v4f{};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      Pack8 bx;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int ti = 2 * s + (e >> 2), v = e & 3;
        bx.h[e] = to_bf16(fmaxf(a2[ti][v] + bias2[16 * ti + 4 * g + v], 0.0f));
      }
#pragma unroll
      for (int to = 0; to < NT3; ++to) {
        Pack8 wa;
        wa.q = *reinterpret_cast<const uint4*>(&w3s[(((to * 4 + s) * 16 + j) * 4 + g) * 8]);
        a3[to] = mfma16(wa.v, bx.v, a3[to]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    uint64_t bits = 0;
#pragma unroll
    for (int to = 0; to < NT3; ++to)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * to + 4 * g + v;
        if (c < k && a3[to][v] + bias3[c] > 0.0f) bits |= 1ull << c;
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
  float* grad;
  double* loss;
  int nblk;
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
  P->grad = c.take<float>((size_t)L.total);
  P->loss = c.take<double>((size_t)P->nblk);
}

int grad_step(int k, int batch, int64_t nsamp, int64_t step, int sequential, const int64_t* order, const float* params,
              const float* phi, const uint64_t* masks, const TrainPlan& P, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_act, dim3(P.nblk), dim3(kH), 0, s, k, batch, nsamp, step, sequential, order, params, phi,
                     masks,
                     P.xg, P.h1g, P.h2g, P.dzg, P.dh1g, P.dh2g, P.loss);
  NMF_TRY(nmf::launch_status("mlp activations"));
  const int total = layout(k).total;
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((total + 255) / 256), dim3(256), 0, s, k, batch, P.xg, P.h1g, P.h2g, P.dzg,
                     P.dh1g, P.dh2g, P.grad);
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

int mlp_infer_plan(int k, int64_t batch, Carver& c, void** scratch) {
  (void)k;
  (void)batch;
  (void)c;
  *scratch = nullptr;
  return NMF_OK;
}

int mlp_infer_launch(int k, int64_t batch, const double* G, const float* R, int64_t ldr, const float* params,
                     uint64_t* mask_out, void* scratch, hipStream_t s) {
  (void)scratch;
  if (batch <= 0) return NMF_OK;
  const int64_t tiles = cdiv(batch, 16);
  int64_t blocks = cdiv(tiles, 4);
  if (blocks > 2048) blocks = 2048;
  if (k <= 16)
    hipLaunchKernelGGL((k_mlp_infer<1, 1>), dim3((unsigned)blocks), dim3(256), 0, s, k, batch, G, R, ldr, params,
                       mask_out);
  else if (k <= 32)
    hipLaunchKernelGGL((k_mlp_infer<2, 2>), dim3((unsigned)blocks), dim3(256), 0, s, k, batch, G, R, ldr, params,
                       mask_out);
  else
    hipLaunchKernelGGL((k_mlp_infer<4, 4>), dim3((unsigned)blocks), dim3(256), 0, s, k, batch, G, R, ldr, params,
                       mask_out);
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
  const hipError_t e = hipMemcpyAsync(grad_out, P.grad, sizeof(float) * total, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return nmf::fail(NMF_EHIP, "nmf_mlp_grad: %s", hipGetErrorString(e));
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
    hipLaunchKernelGGL(k_adam, dim3((total + 255) / 256), dim3(256), 0, s, total, params, P.grad, adam_m, adam_v, lr,
                       (float)b1, (float)b2, 1e-8f, c1, c2);
    NMF_TRY(nmf::launch_status("adam"));
  }
  if (loss_out && steps > 0) {
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(64), 0, s, P.nblk, P.loss, 1.0 / ((double)batch * k), loss_out);
    NMF_TRY(nmf::launch_status("mlp loss"));
  }
  return NMF_OK;
}
