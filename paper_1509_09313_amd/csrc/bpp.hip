// Batched NNLS by block principal pivoting (Section "Block Principal
// Pivoting"; Eq. single NLS, Eq. KKT).  For every row b of R:
//     x = argmin_{x >= 0} 1/2 x^T G x - R[b]^T x.
// The passive/active exchange follows Kim & Park's BPP (full exchange of the
// infeasible set while it shrinks, at most three non-improving full
// exchanges, then the single largest infeasible index), as the paper
// prescribes by citation.
//
// Mapping to the wavefront.  One problem per K lanes (K in {8,16,32}: 64/K
// problems per wavefront; K in {56,64}: one, lanes >= K idle); lane p owns
// index p: the row p of G, f_p, x_p.  G is padded to K x K with the identity,
// so indices k <= p < K never pivot and their updates are no-ops, which keeps
// every loop fully unrolled over the compile-time K (the row lives in
// registers).
// G (k x k FP64) sits in LDS, shared by the block.  Each round solves the
// passive subsystem G_FF x_F = f_F in FP64 by symmetric elimination in index
// order (LDL^T with the back-substitution folded into the sweep, i.e.
// Gauss-Jordan): at pivot j every lane writes its current G-row entry
// a_pj and its right-hand side to LDS, reads the pivot row from the column
// (the trailing matrix stays symmetric) and updates its own row.  Active
// lanes ride along as non-pivot rows, so after the sweep
//     x_p = rhs_p / pivot_p   (p in F)      y_p = -rhs_p   (p not in F)
// gives the primal solution and the dual y = G x - f without another pass.
// The infeasible set V = {p in F: x_p < 0} U {p not in F: y_p < 0} is a
// ballot; the exchange rule is evaluated identically by every lane.
//
// Degenerate indices: an index with G_ii <= 1e-14 max_l G_ll is pinned at 0
// from the start; a passive-subset pivot <= 1e-12 G_jj pins its index
// (removed from F, never made passive again).  Pinned indices are excluded
// from V.  These rules match the CPU reference.
#include "nmf_common.h"

namespace {

constexpr int kWaves = 4;

__device__ __forceinline__ uint64_t bit64(int i) { return 1ull << i; }

template <int K>
__global__ __launch_bounds__(256) void k_bpp(int k, int64_t batch, const double* __restrict__ G,
                                             const float* __restrict__ R, int64_t ldr, float* __restrict__ X,
                                             int64_t ldx, const uint64_t* mask_in,
                                             uint64_t* mask_out, uint8_t* __restrict__ rounds_out,
                                             uint8_t* __restrict__ status_out, int max_rounds, int warm_cap,
                                             unsigned long long* __restrict__ counters) {
  constexpr int P = 64 / K;
  __shared__ double Gs[K * K];
  __shared__ double colv[kWaves][64];
  __shared__ double rfv[kWaves][64];
  __shared__ unsigned long long cnt[kWaves][NMF_BPP_COUNTERS];

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const bool lane_in = lane < P * K;
  const int sub = lane_in ? lane / K : 0;
  const int p = lane_in ? lane % K : 0;
  const int base = sub * K;

  for (int idx = t; idx < K * K; idx += 256) {
    const int q = idx / K, pp = idx - q * K;
    Gs[idx] = (q < k && pp < k) ? G[q * k + pp] : (q == pp ? 1.0 : 0.0);
  }
  __syncthreads();

  const uint64_t all = (k == 64) ? ~0ull : (bit64(k) - 1ull);
  double dmax = 0.0;
  for (int q = 0; q < k; ++q) dmax = fmax(dmax, Gs[q * K + q]);
  uint64_t pinned0 = 0;
  for (int q = 0; q < k; ++q)
    if (Gs[q * K + q] <= 1e-14 * dmax) pinned0 |= bit64(q);

  unsigned long long c_rounds = 0, c_solves = 0, c_f1 = 0, c_f2 = 0, c_f3 = 0;

  for (int64_t g = (int64_t)blockIdx.x * kWaves + wave; g * P < batch; g += (int64_t)gridDim.x * kWaves) {
    const int64_t b = g * P + sub;
    const bool vprob = lane_in && b < batch;
    const bool valid = vprob && p < k;
    const double f = valid ? (double)R[b * ldr + p] : 0.0;
    uint64_t F = (vprob && mask_in) ? (mask_in[b] & all & ~pinned0) : 0ull;
    uint64_t pinned = pinned0;
    bool warm = F != 0;
    int alpha = 3, beta = k + 1, rounds = 0, since = 0;
    int st = 0;
    bool done = !vprob;
    double xfin = 0.0;

    while (__ballot(!done) != 0) {
      uint64_t Fe = done ? 0ull : F;
      double r[K];
#pragma unroll
      for (int q = 0; q < K; ++q) r[q] = Gs[q * K + p];
      double rf = f, mypiv = 1.0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const bool pj = (Fe >> j) & 1ull;
        if (__ballot(pj) == 0) continue;
        colv[wave][lane] = r[j];
        rfv[wave][lane] = rf;
        wave_lds_sync();
        const double piv = colv[wave][base + j];
        const double zj = rfv[wave][base + j];
        bool use = pj;
        if (pj && !(piv > 1e-12 * Gs[j * K + j])) {
          use = false;
          F &= ~bit64(j);
          Fe &= ~bit64(j);
          pinned |= bit64(j);
          st |= NMF_BPP_SINGULAR;
        }
        const double inv = use ? 1.0 / piv : 0.0;
        const double mlt = (use && p != j) ? r[j] * inv : 0.0;
        if (use && p == j) mypiv = piv;
#pragma unroll
        for (int q = j + 1; q < K; ++q) r[q] -= mlt * colv[wave][base + q];
        rf -= mlt * zj;
        wave_lds_sync();
      }
      const bool inF = (Fe >> p) & 1ull;
      const double x = inF ? rf / mypiv : 0.0;
      const double y = inF ? 0.0 : -rf;
      const bool viol = valid && !done && !((pinned >> p) & 1ull) && (inF ? (x < 0.0) : (y < 0.0));
      const uint64_t bal = __ballot(viol);
      uint64_t V;
      if constexpr (K == 64) {
        V = bal;
      } else {
        V = (bal >> base) & (bit64(K) - 1ull);
      }
      if (!done) {
        const unsigned long long nf = (unsigned long long)__popcll(Fe);
        if (p == 0 && lane_in) {
          ++c_rounds;
          if (nf) {
            ++c_solves;
            c_f1 += nf;
            c_f2 += nf * nf;
            c_f3 += nf * nf * nf;
          }
        }
        ++rounds;
        ++since;
        if (V == 0) {
          done = true;
          xfin = x;
        } else if (warm && since >= warm_cap) {
          st |= NMF_BPP_WARM_FALLBACK;
          warm = false;
          F = 0;
          alpha = 3;
          beta = k + 1;
          since = 0;
        } else if (rounds >= max_rounds) {
          st |= NMF_BPP_CAPPED;
          done = true;
          xfin = x > 0.0 ? x : 0.0;
        } else {
          const int nv = __popcll(V);
          uint64_t S;
          if (nv < beta) {
            beta = nv;
            alpha = 3;
            S = V;
          } else if (alpha >= 1) {
            alpha -= 1;
            S = V;
          } else {
            S = bit64(63 - __clzll((long long)V));
          }
          F ^= S;
        }
      }
    }
    if (valid) X[b * ldx + p] = (float)xfin;
    if (vprob && p == 0) {
      if (pinned) st |= NMF_BPP_PINNED;
      if (mask_out) mask_out[b] = F;
      if (rounds_out) rounds_out[b] = (uint8_t)(rounds < 255 ? rounds : 255);
      if (status_out) status_out[b] = (uint8_t)st;
    }
  }

  if (counters) {
    unsigned long long v[NMF_BPP_COUNTERS] = {c_rounds, c_solves, c_f1, c_f2, c_f3};
#pragma unroll
    for (int e = 0; e < NMF_BPP_COUNTERS; ++e) {
      unsigned long long s = v[e];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) cnt[wave][e] = s;
    }
    __syncthreads();
    if (t < NMF_BPP_COUNTERS) {
      unsigned long long s = 0;
      for (int w = 0; w < kWaves; ++w) s += cnt[w][t];
      if (s) atomicAdd(counters + t, s);
    }
  }
}

template <int K>
int launch(int k, int64_t batch, const double* G, const float* R, int64_t ldr, float* X, int64_t ldx,
           const uint64_t* mask_in, uint64_t* mask_out, uint8_t* rounds, uint8_t* status, int max_rounds,
           int warm_cap, uint64_t* counters, hipStream_t s) {
  constexpr int P = 64 / K;
  const int64_t waves = nmf::cdiv(batch, P);
  int64_t blocks = nmf::cdiv(waves, kWaves);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_bpp<K>, dim3((unsigned)blocks), dim3(256), 0, s, k, batch, G, R, ldr, X, ldx, mask_in,
                     mask_out, rounds, status, max_rounds, warm_cap,
                     reinterpret_cast<unsigned long long*>(counters));
  return nmf::launch_status("nnls_bpp_batched");
}

}  // namespace

namespace nmf {

int bpp_launch(int k, int64_t batch, const double* G, const float* R, int64_t ldr, float* X, int64_t ldx,
               const uint64_t* mask_in, uint64_t* mask_out, uint8_t* rounds, uint8_t* status, int max_rounds,
               int warm_cap, uint64_t* counters, hipStream_t s) {
  if (batch == 0) return NMF_OK;
  if (k <= 8) return launch<8>(k, batch, G, R, ldr, X, ldx, mask_in, mask_out, rounds, status, max_rounds, warm_cap, counters, s);
  if (k <= 16) return launch<16>(k, batch, G, R, ldr, X, ldx, mask_in, mask_out, rounds, status, max_rounds, warm_cap, counters, s);
  if (k <= 32) return launch<32>(k, batch, G, R, ldr, X, ldx, mask_in, mask_out, rounds, status, max_rounds, warm_cap, counters, s);
  if (k <= 56) return launch<56>(k, batch, G, R, ldr, X, ldx, mask_in, mask_out, rounds, status, max_rounds, warm_cap, counters, s);
  return launch<64>(k, batch, G, R, ldr, X, ldx, mask_in, mask_out, rounds, status, max_rounds, warm_cap, counters, s);
}

}  // namespace nmf

extern "C" int nnls_bpp_batched(int k, int64_t batch, const double* G, const float* R, int64_t ldr, float* X,
                                int64_t ldx, const uint64_t* mask_in, uint64_t* mask_out, uint8_t* rounds,
                                uint8_t* status, int max_rounds, int warm_cap, uint64_t* counters, void* stream) {
  if (!nmf::valid_k(k)) return nmf::fail(NMF_EINVAL, "nnls_bpp_batched: k=%d outside [1,64]", k);
  if (batch < 0 || ldr < k || ldx < k) return nmf::fail(NMF_EINVAL, "nnls_bpp_batched: bad sizes");
  if (max_rounds < 1 || warm_cap < 1) return nmf::fail(NMF_EINVAL, "nnls_bpp_batched: max_rounds/warm_cap < 1");
  if (batch > 0 && (!G || !R || !X)) return nmf::fail(NMF_EINVAL, "nnls_bpp_batched: null pointer");
  return nmf::bpp_launch(k, batch, G, R, ldr, X, ldx, mask_in, mask_out, rounds, status, max_rounds, warm_cap,
                         counters, nmf::as_stream(stream));
}
