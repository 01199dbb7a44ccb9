// Batched NNLS by block principal pivoting (Section "Block Principal
// Pivoting"; Eq. single NLS, Eq. KKT).  For every row b of R:
//     x = argmin_{x >= 0} 1/2 x^T G x - R[b]^T x.
// The passive/active exchange follows Kim & Park's BPP (full exchange of the
// infeasible set while it shrinks, at most three non-improving full
// exchanges, then the single largest infeasible index), as the paper
// prescribes by citation.
//
// The passive subsystem G_FF x_F = f_F is solved in FP64 by symmetric
// elimination in index order (LDL^T with the back-substitution folded into
// the sweep, i.e. Gauss-Jordan): at pivot j each row subtracts its multiple of
// the pivot row (the trailing matrix stays symmetric, so the pivot row is read
// from the column), and after the sweep x_p = rhs_p / pivot_p.  The
// infeasible set V = {p in F: x_p < 0} U {p not in F: y_p < 0}, y = G x - f,
// is a ballot; the exchange rule is evaluated identically by every lane of a
// problem.
//
// Two kernels.  k_bpp_pair (below, every k) holds only the pivot rows, a
// problem per 4 to 32 lanes, and forms the other entries from one product
// with the solved pivots.  bpp_block, the one-row-per-lane form (one problem
// per wavefront, K in {56, 64}, lane p owns row p of G, f_p and x_p, G
// identity-padded to K x K so every loop unrolls over the compile-time K),
// finishes the problems k_bpp_pair defers: its non-pivot rows ride along
// through the elimination and come out as y_p = -rhs_p, and its pivot
// columns are packed at the end of the row (see the elimination), so a step
// touches only later pivots.
//
// Two forms of the same passive-set solve.  Each block also sweeps each G it
// serves once (symmetric sweep operator over the unpinned indices U, FP64,
// index order) to get G_U^{-1} in LDS, and each problem forms z = G_U^{-1} f.  When the
// active part A = U \ F is smaller than F, the round eliminates over A on
// (G^{-1}, z) instead of over F on (G, f): with v = ((G^{-1})_AA)^{-1} z_A,
//     x_F = z_F - (G^{-1})_FA v       y_A = -v
// (block inverse identities), so the common rounds with F = U or nearly so
// cost |A| pivot steps instead of |F|.  This form is used only if every
// sweep pivot of G exceeds 1e-6 G_jj (G well conditioned); otherwise, and
// whenever a pivot of it fails, the round eliminates over F on G.
//
// Degenerate indices: an index with G_ii <= 1e-14 max_l G_ll is pinned at 0
// from the start; a passive-subset pivot <= 1e-12 G_jj pins its index
// (removed from F, never made passive again).  Pinned indices are excluded
// from V.  These rules match the CPU reference.
#include "batched.h"
#include "nmf_common.h"

namespace {

constexpr int kWaves = 4;
constexpr int kSmall = 4;  // pivot-set size handled by the small-system path

__device__ __forceinline__ uint64_t bit64(int i) { return 1ull << i; }

// Per-lane sums a caller may want from the solutions without reading them
// again: sum over solved entries of f_i x_i (x rounded to FP32 as stored;
// the cross term of the trace-form objective), and the problems that ended
// capped or fell back from their start set.
struct BppExtras {
  double dot = 0.0;
  unsigned long long capped = 0, fallback = 0;
};

// Mark of a problem that the pivot-row kernel left to the one-row-per-lane
// kernel: a signalling NaN with a fixed payload in x_0 (arithmetic never
// produces a signalling NaN, so no solution can carry it).
constexpr uint32_t kDeferMark = 0xFFBADA55u;

// The one-row-per-lane kernel (K in {56, 64}, one problem per wavefront):
// solves the problems of [b0, b1) of one Gram matrix G whose x_0 holds
// kDeferMark (every problem of the range with `every`), found 64 at a time
// (chunk g_first, g_first + g_step, ... of 64 problems per wavefront) by a
// ballot, each from its start set.  Loads G into
// LDS first (after a barrier, so a persistent loop may call it again with
// another G).  Round and solve statistics are added to cacc (per lane; summed
// by the caller).
template <int K>
__device__ __forceinline__ void bpp_block(int k, const double* __restrict__ G, const float* __restrict__ R,
                                          int64_t ldr, float* __restrict__ X, int64_t ldx, const uint64_t* mask_in,
                                          uint64_t* mask_out, uint8_t* __restrict__ rounds_out,
                                          uint8_t* __restrict__ status_out, int max_rounds, int warm_cap, int64_t b0,
                                          int64_t b1, int64_t g_first, int64_t g_step,
                                          unsigned long long (&cacc)[NMF_BPP_COUNTERS], BppExtras& ex,
                                          bool every = false) {
  static_assert(K >= 56, "one problem per wavefront");
  constexpr int P = 1;
  __shared__ double Gs[K * K];
  __shared__ double Gi[K * K];
  __shared__ int inv_ok_s;
  // one slot per lane, plus a spare slot 64 for the packed form's non-pivot
  // lanes
  __shared__ double colv[kWaves][65];
  __shared__ double rfv[kWaves][65];
  __shared__ double dgv[kWaves][65];
  __shared__ int pix[kWaves][65];

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const bool lane_in = lane < P * K;
  const int sub = lane_in ? lane / K : 0;
  const int p = lane_in ? lane % K : 0;
  const int base = sub * K;

  __syncthreads();
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

  // G_U^{-1} by the symmetric sweep operator (one wavefront): sweeping index j
  // maps a_jj -> -1/d, a_ij -> a_ij/d, a_il -> a_il - a_ij a_jl/d (d = a_jj);
  // after sweeping all of U the U block holds -G_U^{-1}.  Lane i keeps row i,
  // rotated left by one entry per step so that column j sits in r[0] at step
  // j (the step loop then needs no register indexing by j).
  if (wave == 0) {
    const int pl = lane % K;
    double r[K];
#pragma unroll
    for (int q = 0; q < K; ++q) r[q] = Gs[q * K + pl];
    bool ok = true;
#pragma unroll 1
    for (int j = 0; j < K; ++j) {
      const bool sweep = j < k && !((pinned0 >> j) & 1ull);
      if (sweep) {
        colv[0][lane] = r[0];
        wave_lds_sync();
        const double d = colv[0][j];
        if (!(d > 1e-6 * Gs[j * K + j])) ok = false;
        const double inv = 1.0 / d;
        const bool pivot_lane = pl == j;
        const double m = r[0] * inv;
#pragma unroll
        for (int q = 1; q < K; ++q) {
          const int col = (j + q) % K;
          r[q] = pivot_lane ? r[q] * inv : r[q] - m * colv[0][col];
        }
        r[0] = pivot_lane ? -inv : m;
        wave_lds_sync();
      }
      const double first = r[0];
#pragma unroll
      for (int q = 0; q < K - 1; ++q) r[q] = r[q + 1];
      r[K - 1] = first;
    }
    if (lane < K) {
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const bool inU = q < k && pl < k && !((pinned0 >> q) & 1ull) && !((pinned0 >> pl) & 1ull);
        Gi[q * K + pl] = inU ? -r[q] : 0.0;
      }
    }
    if (lane == 0) inv_ok_s = ok ? 1 : 0;
  }
  __syncthreads();
  const bool inv_ok = inv_ok_s != 0;

  unsigned long long c_rounds = 0, c_solves = 0, c_f1 = 0, c_f2 = 0, c_f3 = 0, c_steps = 0;

  // the marked problems: sbits holds the unvisited marks of chunk sc0
  int64_t sc0 = b0 + g_first * 64;
  auto marks = [&](int64_t c0) {
    const int64_t bb = c0 + lane;
    return __ballot(bb < b1 && (every || __float_as_uint(X[bb * ldx]) == kDeferMark));
  };
  uint64_t sbits = sc0 < b1 ? marks(sc0) : 0ull;
  auto next_mark = [&]() {
    while (sbits == 0ull) {
      sc0 += g_step * 64;
      if (sc0 >= b1) break;
      sbits = marks(sc0);
    }
  };
  next_mark();
  while (sbits != 0ull) {
    const int64_t b = sc0 + (__ffsll((unsigned long long)sbits) - 1);
    sbits &= sbits - 1ull;
    next_mark();
    const bool vprob = lane_in;
    const double f = (vprob && p < k) ? (double)R[b * ldr + p] : 0.0;
    uint64_t F = (vprob && mask_in) ? (mask_in[b] & all & ~pinned0) : 0ull;
    const bool valid = vprob && p < k;
    uint64_t pinned = pinned0;
    bool warm = F != 0;
    int alpha = 3, beta = k + 1, rounds = 0, since = 0;
    int st = 0;
    bool done = !vprob;
    bool forceG = false;
    double xfin = 0.0;
    // unconstrained solution z = G_U^{-1} f
    double z = 0.0;
    if (inv_ok) {
      rfv[wave][lane] = f;
      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < K; ++q) z += Gi[q * K + p] * rfv[wave][base + q];
      wave_lds_sync();
    }

    while (__ballot(!done) != 0) {
      uint64_t Fe = done ? 0ull : F;
      const uint64_t Ae = done ? 0ull : (all & ~pinned & ~F);
      const bool useInv = inv_ok && !forceG && __popcll(Ae) < __popcll(Fe);
      uint64_t Pv = useInv ? Ae : Fe;
      const double* Mrow = useInv ? Gi : Gs;
      const double rf0 = useInv ? z : f;
      bool retry = false;
      double x, y;
      const int sp = __popcll(Pv);
      if (__ballot(sp != 0) == 0) {
        // No pivots anywhere in the wavefront: the solve is a read-out
        // (inverse form: x_F = z, y = 0; direct form: x = 0, y = -f).
        const bool inF = (Fe >> p) & 1ull;
        if (useInv) {
          x = inF ? z : 0.0;
          y = 0.0;
        } else {
          x = 0.0;
          y = inF ? 0.0 : -f;
        }
      } else if (__ballot(sp > kSmall) == 0) {
        // Small pivot sets (every problem of the wavefront): each lane reads
        // the entries it needs, M[p][j] for the pivots j, and solves the
        // s x s system M_PP u = rhs_P redundantly by LDL^T in index order
        // (the same pivots and pivot tests as the elimination below).
        // The largest pivot set of the wavefront bounds the (uniform) steps.
        int smax = 0;
#pragma unroll
        for (int t = 1; t <= kSmall; ++t)
          if (__ballot(sp >= t) != 0) smax = t;
        int jj[kSmall];
        bool vt[kSmall];
        uint64_t rem = Pv;
#pragma unroll
        for (int t = 0; t < kSmall; ++t) {
          vt[t] = false;
          jj[t] = 0;
          if (t < smax) {
            vt[t] = rem != 0ull;
            jj[t] = rem != 0ull ? (__ffsll((unsigned long long)rem) - 1) : 0;
            rem &= rem - 1ull;
          }
        }
        rfv[wave][lane] = rf0;
        wave_lds_sync();
        double bt[kSmall], mc[kSmall], dg[kSmall];
#pragma unroll
        for (int t = 0; t < kSmall; ++t) {
          bt[t] = 0.0;
          mc[t] = 0.0;
          dg[t] = 1.0;
          if (t < smax) {
            bt[t] = vt[t] ? rfv[wave][base + jj[t]] : 0.0;
            mc[t] = vt[t] ? Mrow[jj[t] * K + p] : 0.0;
            dg[t] = vt[t] ? Mrow[jj[t] * K + jj[t]] : 1.0;
          }
        }
        wave_lds_sync();
        double Lm[kSmall][kSmall], rinv[kSmall], dd[kSmall], u[kSmall];
#pragma unroll
        for (int a = 0; a < kSmall; ++a) {
#pragma unroll
          for (int b = 0; b < kSmall; ++b) Lm[b][a] = 0.0;
          rinv[a] = 0.0;
          dd[a] = 0.0;
          u[a] = 0.0;
        }
#pragma unroll
        for (int a = 0; a < kSmall; ++a) {
          if (a < smax) {
            double col[kSmall];
#pragma unroll
            for (int b = a; b < kSmall; ++b) {
              double v = 0.0;
              if (b < smax) {
                v = (vt[a] && vt[b]) ? Mrow[jj[b] * K + jj[a]] : 0.0;
#pragma unroll
                for (int c = 0; c < a; ++c) v -= Lm[b][c] * Lm[a][c] * dd[c];
              }
              col[b] = v;
            }
            const bool ok = vt[a] && col[a] > 1e-12 * dg[a];
            if (vt[a] && !ok) {
              if (useInv) {
                retry = true;
              } else {
                const uint64_t bj = bit64(jj[a]);
                F &= ~bj;
                Fe &= ~bj;
                pinned |= bj;
                st |= NMF_BPP_SINGULAR;
              }
              vt[a] = false;
            }
            // 1 / pivot: hardware estimate and two Newton steps, as in the
            // elimination below (W side at 10^6 x 2400, k = 30: 0.919 -> 0.902 ms
            // against the IEEE division)
            double ra = __builtin_amdgcn_rcp(col[a]);
            ra = fma(ra, fma(-col[a], ra, 1.0), ra);
            ra = fma(ra, fma(-col[a], ra, 1.0), ra);
            ra = ok ? ra : 0.0;
            rinv[a] = ra;
            dd[a] = ok ? col[a] : 0.0;
#pragma unroll
            for (int b = a + 1; b < kSmall; ++b) Lm[b][a] = col[b] * ra;
          }
        }
        // L w = rhs, then u = D^-1 w - L^T u (back)
#pragma unroll
        for (int a = 0; a < kSmall; ++a) {
          if (a < smax) {
            double v = vt[a] ? bt[a] : 0.0;
#pragma unroll
            for (int c = 0; c < a; ++c) v -= Lm[a][c] * u[c];
            u[a] = v;
          }
        }
#pragma unroll
        for (int a = kSmall - 1; a >= 0; --a) {
          if (a < smax) {
            double v = u[a] * rinv[a];
#pragma unroll
            for (int b = a + 1; b < kSmall; ++b) v -= Lm[b][a] * u[b];
            u[a] = vt[a] ? v : 0.0;
          }
        }
        double own = 0.0, corr = 0.0;
#pragma unroll
        for (int t = 0; t < kSmall; ++t) {
          if (vt[t] && jj[t] == p) own = u[t];
          corr += mc[t] * u[t];
        }
        const bool inF = (Fe >> p) & 1ull;
        const bool isPinned = (pinned >> p) & 1ull;
        if (useInv) {
          x = inF ? z - corr : 0.0;
          y = (inF || isPinned) ? 0.0 : -own;
        } else {
          x = inF ? own : 0.0;
          y = inF ? 0.0 : corr - f;
        }
      } else {
        // One problem per wavefront, so the pivot set is uniform.  The n_p
        // pivots are packed, in index order, at the end of a K-wide register
        // row (pivot c at position K - n_p + c): each step then updates only
        // the positions of the later pivots, about n_p^2 / 2 updates per
        // round instead of n_p K / 2, and the non-pivot columns are never
        // gathered.  A pivot lane publishes its entries at its own packed
        // slot, so every read of a step has a compile-time offset.  The
        // arithmetic on the pivot columns, and its order, is that of the
        // unpacked elimination below.
        const int np = __popcll(Pv);
        const int off = K - np;
        const bool inP = (Pv >> p) & 1ull;
        const int slot = inP ? off + __popcll(Pv & (bit64(p) - 1ull)) : 64;
        double* colw = &colv[wave][0];
        double* rfw = &rfv[wave][0];
        double* dgw = &dgv[wave][0];
        double r[K];
        {
          // each pivot lane enters its index at its packed slot, so the
          // gather's addresses need no serial scan of the pivot set
          int* pw = &pix[wave][0];
          pw[slot] = p;
          wave_lds_sync();
#pragma unroll
          for (int c = 0; c < K; ++c) {
            // positions before the pivots are never read; they load row 0
            const int jc = c >= off ? pw[c] : 0;
            r[c] = Mrow[jc * K + p];
          }
        }
        dgw[slot] = Mrow[p * K + p];
        double rf = rf0, mypiv = 1.0;
        {
          uint64_t rem = Pv;
#pragma unroll
          for (int c = 0; c < K; ++c) {
            if (c < off) continue;
            const int j = __ffsll((unsigned long long)rem) - 1;
            rem &= rem - 1ull;
            colw[slot] = r[c];
            rfw[slot] = rf;
            wave_lds_sync();
            const double piv = colw[c];
            const double zj = rfw[c];
            bool use = true;
            if (!(piv > 1e-12 * dgw[c])) {
              use = false;
              if (useInv) {
                retry = true;
              } else {
                F &= ~bit64(j);
                Fe &= ~bit64(j);
                pinned |= bit64(j);
                st |= NMF_BPP_SINGULAR;
              }
            }
            double inv = __builtin_amdgcn_rcp(piv);
            inv = fma(inv, fma(-piv, inv, 1.0), inv);
            inv = fma(inv, fma(-piv, inv, 1.0), inv);
            inv = use ? inv : 0.0;
            const double mlt = (use && p != j) ? r[c] * inv : 0.0;
            if (use && p == j) mypiv = piv;
#pragma unroll
            for (int q = c + 1; q < K; ++q) r[q] -= mlt * colw[q];
            rf -= mlt * zj;
            wave_lds_sync();
          }
        }
        const bool inF = (Fe >> p) & 1ull;
        const bool isPinned = (pinned >> p) & 1ull;
        if (useInv) {
          x = inF ? rf : 0.0;
          y = (inF || isPinned) ? 0.0 : -rf / mypiv;
        } else {
          x = inF ? rf / mypiv : 0.0;
          y = inF ? 0.0 : -rf;
        }
      }
      const bool isPinned = (pinned >> p) & 1ull;
      const bool inF = (Fe >> p) & 1ull;
      const bool viol = valid && !done && !retry && !isPinned && (inF ? (x < 0.0) : (y < 0.0));
      const uint64_t bal = __ballot(viol);
      uint64_t V;
      if constexpr (K == 64) {
        V = bal;
      } else {
        V = (bal >> base) & (bit64(K) - 1ull);
      }
      if (retry) forceG = true;
      if (!done && !retry) {
        const unsigned long long nf = (unsigned long long)__popcll(Fe);
        if (p == 0 && lane_in) {
          ++c_rounds;
          c_steps += (unsigned long long)__popcll(Pv);
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
    if (valid) {
      const float xs = (float)xfin;
      X[b * ldx + p] = xs;
      ex.dot += (double)xs * f;
    }
    if (vprob && p == 0) {
      ex.capped += (st & NMF_BPP_CAPPED) ? 1 : 0;
      ex.fallback += (st & NMF_BPP_WARM_FALLBACK) ? 1 : 0;
      if (pinned) st |= NMF_BPP_PINNED;
      if (mask_out) mask_out[b] = F;
      if (rounds_out) rounds_out[b] = (uint8_t)(rounds < 255 ? rounds : 255);
      if (status_out) status_out[b] = (uint8_t)st;
    }
  }

  cacc[0] += c_rounds;
  cacc[1] += c_solves;
  cacc[2] += c_f1;
  cacc[3] += c_f2;
  cacc[4] += c_f3;
  cacc[5] += c_steps;
}

// Sums the per-lane statistics of the block (NW wavefronts) and adds them to
// counters.
template <int NW = kWaves>
__device__ __forceinline__ void flush_counters(const unsigned long long (&cacc)[NMF_BPP_COUNTERS],
                                               unsigned long long* __restrict__ counters) {
  __shared__ unsigned long long cnt[NW][NMF_BPP_COUNTERS];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int e = 0; e < NMF_BPP_COUNTERS; ++e) {
    unsigned long long s = cacc[e];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) cnt[wave][e] = s;
  }
  __syncthreads();
  if (t < NMF_BPP_COUNTERS) {
    unsigned long long s = 0;
    for (int w = 0; w < NW; ++w) s += cnt[w][t];
    if (s) atomicAdd(counters + t, s);
  }
}

// Block sums of the extras: the dot sum to dot_partial[blockIdx.x] (summed
// in a fixed order, so the result does not depend on timing), the status
// counts added to status_counts[0] (capped) and [1] (fell back).
template <int NW = kWaves>
__device__ __forceinline__ void flush_extras(const BppExtras& ex, double* __restrict__ dot_partial,
                                             unsigned long long* __restrict__ status_counts) {
  __shared__ double sd[NW];
  __shared__ unsigned long long sc[NW][2];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double d = ex.dot;
  unsigned long long c = ex.capped, f = ex.fallback;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    d += __shfl_xor(d, off, 64);
    c += __shfl_xor(c, off, 64);
    f += __shfl_xor(f, off, 64);
  }
  if (lane == 0) {
    sd[wave] = d;
    sc[wave][0] = c;
    sc[wave][1] = f;
  }
  __syncthreads();
  if (t == 0) {
    double bd = 0.0;
    unsigned long long bc = 0, bf = 0;
    for (int w = 0; w < NW; ++w) {
      bd += sd[w];
      bc += sc[w][0];
      bf += sc[w][1];
    }
    if (dot_partial) dot_partial[blockIdx.x] = bd;
    if (status_counts) {
      if (bc) atomicAdd(status_counts, bc);
      if (bf) atomicAdd(status_counts + 1, bf);
    }
  }
}

// ---- The pivot-row kernel (every k) ------------------------------------------
// Whenever G_U^{-1} is available, a round eliminates over the smaller of F
// and its complement in U, so it has at most floor(k / 2) pivots: at most
// KK / 2 for the class KK in {8, 16, 32, 56, 64}.  The elimination needs only
// the pivot rows, so L lanes per problem (KK / 2, or 32 for KK >= 56) hold
// them, pivot c of n_p (in index order) at position KK / 2 - n_p + c, and a
// wavefront carries 64 / L problems (16, 8, 4, 2, 2).  Lane h of a problem
// owns indices h and h + L (f, z, x, the dual y and the KKT test).  The
// non-pivot entries come after the elimination from one product with the
// solved pivots:
//     direct form  (pivots F):  y_i = sum_c G_{i,j_c} x_c - f_i
//     inverse form (pivots A):  x_i = z_i - sum_c (G_U^{-1})_{i,j_c} v_c,
// instead of riding along in the elimination as the one-row-per-lane form's
// non-pivot rows do.  The pivot rows' arithmetic, and its order, is that of
// the one-row-per-lane form; only the non-pivot entries round differently.
// A round with more than KK / 2 pivots (G_U^{-1} unavailable, or a failed
// pivot of the inverse form forcing the direct form with a large F) cannot
// be held: the problem is left untouched except for kDeferMark in x_0, and
// the one-row-per-lane form solves it from its start afterwards.
// Blocks of 16 wavefronts (KK = 56: one block per CU, 4 per SIMD within 128
// VGPRs and 155 KB of LDS), 12 (KK = 64: one per CU at 3 per SIMD, the most
// that its 135-137 VGPRs allow) or 8 (KK <= 32: two per CU at 4 per SIMD)
// share G and G_U^{-1} in LDS; G_U^{-1} comes from the symmetric sweep run by
// the whole block.
constexpr int kPairBlocks = 256;
// wavefronts per block of the class KK (one block per CU for KK >= 56; two
// for KK <= 32, whose blocks are smaller in LDS)
constexpr int pair_waves(int KK) { return KK == 64 ? 12 : KK == 56 ? 16 : 8; }
// lanes per problem: indices h and h + L belong to lane h of a group
constexpr int pair_lanes(int KK) { return KK >= 56 ? 32 : KK / 2; }

// LDS of a pivot-row block: G and G_U^{-1}, and per problem group its
// exchange arrays, right-hand side, unconstrained solution and statistics in
// one struct, so that a single per-lane base address serves them all (and f,
// z and the statistics need no registers, the scarce resource here).
template <int KK>
struct PairShared {
  static constexpr int L = pair_lanes(KK);
  static constexpr int P = 64 / L;
  static constexpr int NW = pair_waves(KK);
  struct alignas(16) Grp {
    double colv[L];
    double rfv[L + 1];
    double dgv[L + 1];
    double vv[L];
    double fv[2 * L];  // the problem's right-hand side f
    double zv[2 * L];  // z = G_U^{-1} f
    double dotv[L];    // per lane: sum of f_i x_i over its finished problems
    // the group's totals: the NMF_BPP_COUNTERS in order, then the capped and
    // fell-back counts
    unsigned long long tot[NMF_BPP_COUNTERS + 2];
    int pix[L + 1];
    uint32_t pcnt[5];  // this problem's solves, sum |F|, |F|^2, |F|^3, pivot steps
  };
  // row stride of G and G_U^{-1}: one more than KK, so that the problem
  // groups of a wavefront, reading different rows at the same columns, do
  // not meet in one LDS bank
  static constexpr int KS = KK + 1;
  double Gs[KK * KS];
  double Gi[KK * KS];
  // G_U^{-1} again, transposed (row p holds column p) with an even pitch, so
  // that z = G_U^{-1} f reads two entries of a lane's row per 16-byte load;
  // kept where the LDS allows (the 64-lane class reads Gi instead)
  static constexpr bool kT = KK <= 56;
  static constexpr int KT = KK + 2;
  alignas(16) double GiT[kT ? KK * KT : 2];
  Grp grps[NW][P];
  double dsum[NW];
  int inv_ok_s;  // every sweep pivot passed the test (G_U^{-1} usable)
  // the sweep's pivot column, in two alternating buffers
  double colbuf[2][KK];

  __device__ void clear_stats() {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    Grp& gs = grps[wave][lane / L];
    if (lane % L == 0)
      for (int e = 0; e < NMF_BPP_COUNTERS + 2; ++e) gs.tot[e] = 0;
    gs.dotv[lane % L] = 0.0;
  }
  // block sums: the dot partial in a fixed order, the counts by atomics
  __device__ void flush(unsigned long long* counters, double* dot_partial, unsigned long long* status_counts) {
    // (an opaque copy of the thread index: the addresses below are formed
    // here, not kept alive from the kernel's start)
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const int lane = t & 63, wave = t >> 6;
    double dot = grps[wave][lane / L].dotv[lane % L];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) dot += __shfl_xor(dot, o, 64);
    if (lane == 0) dsum[wave] = dot;
    __syncthreads();
    if (t == 0 && dot_partial) {
      double bd = 0.0;
      for (int w = 0; w < NW; ++w) bd += dsum[w];
      dot_partial[blockIdx.x] = bd;
    }
    if (t < NMF_BPP_COUNTERS + 2) {
      unsigned long long v = 0;
      for (int w = 0; w < NW; ++w)
        for (int q = 0; q < P; ++q) v += grps[w][q].tot[t];
      if (t < NMF_BPP_COUNTERS) {
        if (counters && v) atomicAdd(counters + t, v);
      } else if (status_counts && v) {
        atomicAdd(status_counts + (t - NMF_BPP_COUNTERS), v);
      }
    }
  }
};

// Solves problems [b0, b1) of one G: problem group g (P problems, one per
// L lanes) for g = g_first, g_first + g_step, ...  Loads G and runs the sweep
// first (after a barrier, so a persistent loop may call it again with
// another G), unless `reuse` says that sh already holds this G, its
// G_U^{-1} and its pivot test from the block's previous call; adds its
// statistics to sh.
template <int KK>
__device__ __forceinline__ void pair_block(PairShared<KK>& sh, int k, const double* __restrict__ G,
                                           const float* __restrict__ R, int64_t ldr, float* __restrict__ X,
                                           int64_t ldx, const uint64_t* mask_in, uint64_t* mask_out,
                                           uint8_t* __restrict__ rounds_out, uint8_t* __restrict__ status_out,
                                           int max_rounds, int warm_cap, int64_t b0, int64_t b1, int64_t g_first,
                                           int64_t g_step, bool reuse = false) {
  constexpr int L = pair_lanes(KK);  // lanes per problem
  constexpr int P = 64 / L;          // problems per wavefront
  constexpr int NP = KK / 2;         // pivot positions: k <= KK, so at most KK / 2 pivots
  constexpr int NW = pair_waves(KK);
  constexpr int NT = NW * 64;
  constexpr int kPer = (KK * KK + NT - 1) / NT;  // sweep entries per thread
  using Grp = typename PairShared<KK>::Grp;
  constexpr int KS = PairShared<KK>::KS;
  double* Gs = sh.Gs;
  double* Gi = sh.Gi;

  // the thread index through an opaque copy: a persistent caller would
  // otherwise have the sweep's per-thread addresses hoisted out of its item
  // loop and kept alive through every solve
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  const int lane = t & 63, wave = t >> 6;
  const int grp = lane / L, h = lane % L;
  Grp& gs = sh.grps[wave][grp];
  const int i0 = h, i1 = h + L;
  // LDS column of an owned index (indices >= KK exist only as padding lanes)
  const int c1 = i1 < KK ? i1 : KK - 1;

  __syncthreads();
  if (!reuse) {
    for (int idx = t; idx < KK * KK; idx += NT) {
      const int q = idx / KK, pp = idx - q * KK;
      const double v = (q < k && pp < k) ? G[q * k + pp] : (q == pp ? 1.0 : 0.0);
      Gs[q * KS + pp] = v;
    }
    __syncthreads();
  }
  const uint64_t all = (k == 64) ? ~0ull : (bit64(k) - 1ull);
  double dmax = 0.0;
  for (int q = 0; q < k; ++q) dmax = fmax(dmax, Gs[q * KS + q]);
  uint64_t pinned0 = 0;
  for (int q = 0; q < k; ++q)
    if (Gs[q * KS + q] <= 1e-14 * dmax) pinned0 |= bit64(q);

  // G_U^{-1} by the symmetric sweep over the unpinned indices in index order,
  // on a row-major working copy W of the leading k x k block of G (the
  // identity padding never mixes with it): sweeping j maps W_jj -> -1/d,
  // W_jl -> W_jl / d, W_ij -> W_ij / d and W_il -> W_il - (W_ij / d) W_lj
  // (d = W_jj), as the one-row-per-lane form does with one row per lane;
  // then (G_U^{-1})_{q,p} = -W[p][q] on U x U.  Thread t keeps the entries
  // (i, l) = (t / k + e sr, t % k), e < kPer, in registers through the whole
  // sweep; a step needs only the old column j, which its owners publish in
  // one of two LDS buffers (alternating, so one barrier per step suffices).
  // Wavefronts without entries only keep the barriers.
  static_assert(KK * ((KK + kPer - 1) / kPer) <= NT, "every entry of W has an owner");
  if (!reuse) {
    bool inv_ok = true;
    const int sr = (k + kPer - 1) / kPer;  // row groups: k * sr <= NT
    const int wl = t % k, wr = t / k;
    const bool wown = t < k * sr;
    const bool wave_own = __builtin_amdgcn_readfirstlane(t >> 6) * 64 < k * sr;
    double w[kPer];
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int i = wr + e * sr;
      w[e] = (wown && i < k) ? Gs[i * KS + wl] : 0.0;
    }
    int par = 0;
    for (int j = 0; j < k; ++j) {
      if ((pinned0 >> j) & 1ull) continue;
      double* cb = sh.colbuf[par];
      par ^= 1;
      if (wown && wl == j) {
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
          const int i = wr + e * sr;
          if (i < k) cb[i] = w[e];
        }
      }
      __syncthreads();
      // every thread takes the pivot test (the same in all of them)
      const double d = cb[j];
      if (!(d > 1e-6 * Gs[j * KS + j])) inv_ok = false;
      if (wave_own) {
        // (every read of the step is issued here, and the update is
        // branch-free; entries past k and lanes without entries compute values
        // that are never stored)
        const double wlj = cb[wown ? wl : 0];
        double wij[kPer];
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
          const int i = wr + e * sr;
          wij[e] = cb[(wown && i < k) ? i : 0];
        }
        const double inv = 1.0 / d;
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
          const int i = wr + e * sr;
          const double m = wij[e] * inv;
          const double off_row = wl == j ? m : w[e] - m * wlj;
          const double piv_row = wl == j ? -inv : w[e] * inv;
          w[e] = i == j ? piv_row : off_row;
        }
      }
    }
    // Gi[q][p] = -W[p][q] on U x U, zero elsewhere (and the transposed copy)
    if (wown) {
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int i = wr + e * sr;
        if (i < k) {
          const bool inU = !((pinned0 >> wl) & 1ull) && !((pinned0 >> i) & 1ull);
          const double v = inU ? -w[e] : 0.0;
          Gi[wl * KS + i] = v;
          if constexpr (PairShared<KK>::kT) sh.GiT[i * PairShared<KK>::KT + wl] = v;
        }
      }
    }
    for (int idx = t; idx < KK * KK; idx += NT) {
      const int q = idx / KK, pp = idx - q * KK;
      if (q >= k || pp >= k) {
        Gi[q * KS + pp] = 0.0;
        if constexpr (PairShared<KK>::kT) sh.GiT[pp * PairShared<KK>::KT + q] = 0.0;
      }
    }
    if (t == 0) sh.inv_ok_s = inv_ok ? 1 : 0;
  }
  __syncthreads();
  const bool inv_ok = sh.inv_ok_s != 0;

  uint32_t* pc = gs.pcnt;
  unsigned long long* tg = gs.tot;
  int* pw = gs.pix;
  double* colw = gs.colv;
  double* rfw = gs.rfv;
  double* dgw = gs.dgv;
  double* vw = gs.vv;

  const int64_t npair = (b1 - b0 + P - 1) / P;  // problem groups, one per wavefront
  const int64_t gstride = g_step;
  int64_t g = g_first;
  // the next problem's right-hand side and start set are loaded during this
  // one's solve, except in the 56-lane class, whose 16-wavefront blocks leave
  // no registers for them
  constexpr bool kPrefetch = KK <= 32;
  float fn0 = 0.0f, fn1 = 0.0f;
  uint64_t mn = 0;
  if constexpr (kPrefetch) {
    const int64_t b = b0 + P * g + grp;
    if (g < npair && b < b1) {
      if (i0 < k) fn0 = R[b * ldr + i0];
      if (i1 < k) fn1 = R[b * ldr + i1];
      if (mask_in) mn = mask_in[b];
    }
  }
  for (; g < npair; g += gstride) {
    const int64_t b = b0 + P * g + grp;
    const bool vprob = b < b1;
    const bool val0 = vprob && i0 < k, val1 = vprob && i1 < k;
    double* fw = gs.fv;
    double* zw = gs.zv;
    uint64_t F;
    if constexpr (kPrefetch) {
      fw[i0] = (double)fn0;
      fw[i1] = (double)fn1;
      F = vprob ? (mn & all & ~pinned0) : 0ull;
      const int64_t bn = b0 + P * (g + gstride) + grp;
      const bool vn = g + gstride < npair && bn < b1;
      fn0 = (vn && i0 < k) ? R[bn * ldr + i0] : 0.0f;
      fn1 = (vn && i1 < k) ? R[bn * ldr + i1] : 0.0f;
      mn = (vn && mask_in) ? mask_in[bn] : 0ull;
    } else {
      // (opaque copies of the owned indices, so that the per-lane addresses
      // are formed here rather than kept through the problem loop)
      int o0 = i0, o1 = i1;
      asm volatile("" : "+v"(o0), "+v"(o1));
      fw[i0] = val0 ? (double)R[b * ldr + o0] : 0.0;
      fw[i1] = val1 ? (double)R[b * ldr + o1] : 0.0;
      F = (vprob && mask_in) ? (mask_in[b] & all & ~pinned0) : 0ull;
    }
    uint64_t pinned = pinned0;
    bool warm = F != 0;
    int alpha = 3, beta = k + 1, rounds = 0, since = 0;
    int st = 0;
    bool done = !vprob, defer = false;
    bool forceG = false;
    if (h == 0)
      for (int e = 0; e < 5; ++e) pc[e] = 0;
    // stores a finished problem's x (as FP32) and its share of the dot sum
    auto finish = [&](double x0, double x1) {
      double d = gs.dotv[h];
      int o0 = i0, o1 = i1;
      asm volatile("" : "+v"(o0), "+v"(o1));
      if (val0) {
        const float xs = (float)x0;
        X[b * ldx + o0] = xs;
        d += (double)xs * fw[i0];
      }
      if (val1) {
        const float xs = (float)x1;
        X[b * ldx + o1] = xs;
        d += (double)xs * fw[i1];
      }
      gs.dotv[h] = d;
    };
    // unconstrained solution z = G_U^{-1} f at the owned indices
    wave_lds_sync();
    if (inv_ok) {
      double z0 = 0.0, z1 = 0.0;
      if constexpr (PairShared<KK>::kT) {
        // two contraction indices per step, in the same order (entries past
        // k are zero in both operands)
        constexpr int KT = PairShared<KK>::KT;
        const double2* g0 = reinterpret_cast<const double2*>(&sh.GiT[i0 * KT]);
        const double2* g1 = reinterpret_cast<const double2*>(&sh.GiT[c1 * KT]);
        const double2* f2 = reinterpret_cast<const double2*>(fw);
        for (int q2 = 0; q2 < (k + 1) / 2; ++q2) {
          const double2 fq = f2[q2], a = g0[q2], c = g1[q2];
          z0 += a.x * fq.x;
          z0 += a.y * fq.y;
          z1 += c.x * fq.x;
          z1 += c.y * fq.y;
        }
      } else {
        for (int q = 0; q < k; ++q) {
          const double fq = fw[q];
          z0 += Gi[q * KS + i0] * fq;
          z1 += Gi[q * KS + c1] * fq;
        }
      }
      zw[i0] = z0;
      zw[i1] = z1;
    }

    while (__ballot(!done) != 0) {
      const uint64_t Ae = done ? 0ull : (all & ~pinned & ~F);
      const bool useInv = inv_ok && !forceG && __popcll(Ae) < __popcll(done ? 0ull : F);
      uint64_t Pv = useInv ? Ae : (done ? 0ull : F);
      if (__popcll(Pv) > NP) {
        // more pivots than lanes: left to the one-row-per-lane form
        defer = true;
        done = true;
        Pv = 0;
      }
      const double* Mrow = useInv ? Gi : Gs;
      const int np = __popcll(Pv);
      const int off = NP - np;
      // the first position that any problem of the wavefront uses, made
      // wave-uniform for the classes with up to four problems per wavefront:
      // a position before it then costs one scalar compare instead of a
      // ballot (the smaller classes, with four or eight positions, ballot)
      constexpr bool kFirst = P <= 4;
      int first = 0;
      if constexpr (kFirst) {
        int npw = 0;
#pragma unroll
        for (int q = 0; q < P; ++q) npw = max(npw, __builtin_amdgcn_readlane(np, q * L));
        first = NP - npw;
      }
      bool retry = false;
      // each owned pivot enters its index, right-hand side and diagonal at
      // its packed position
      const bool pv0 = (Pv >> i0) & 1ull, pv1 = (Pv >> i1) & 1ull;
      const int s0 = pv0 ? off + __popcll(Pv & (bit64(i0) - 1ull)) : L;
      const int s1 = pv1 ? off + __popcll(Pv & (bit64(i1) - 1ull)) : L;
      pw[s0] = i0;
      rfw[s0] = useInv ? zw[i0] : fw[i0];
      dgw[s0] = 1e-12 * Mrow[i0 * KS + i0];
      pw[s1] = i1;
      rfw[s1] = useInv ? zw[i1] : fw[i1];
      dgw[s1] = 1e-12 * Mrow[c1 * KS + c1];
      wave_lds_sync();
      const bool mine = h >= off && h < NP;
      const int jh = mine ? pw[h] : 0;
      double r[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        if (c % 8 == 0) __builtin_amdgcn_sched_barrier(0);
        // positions before every problem's first pivot are skipped (zero, so
        // that no value is carried between rounds)
        if constexpr (kFirst) {
          if (c < first) {
            r[c] = 0.0;
            continue;
          }
        }
        // positions before a problem's own pivots are never read; they load
        // row 0.  (The position tests of the three loops use an opaque copy of
        // c, so the compiler does not keep NP lane masks alive through the
        // round.)
        int cs = c;
        asm volatile("" : "+s"(cs));
        const bool act = cs >= off;
        if constexpr (!kFirst) {
          if (__ballot(act) == 0ull) {
            r[c] = 0.0;
            continue;
          }
        }
        const int jc = act ? pw[c] : 0;
        r[c] = Mrow[jc * KS + jh];
      }
      double rf = mine ? rfw[h] : 0.0, mypiv = 1.0;
      bool myok = mine;
      wave_lds_sync();
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        if constexpr (kFirst) {
          if (c < first) continue;
        }
        int cs = c;
        asm volatile("" : "+s"(cs));
        const bool act = cs >= off;
        if constexpr (!kFirst) {
          if (__ballot(act) == 0ull) continue;
        }
        const bool pl = h == cs;  // this step's pivot lane
        colw[h] = r[c];
        rfw[h] = rf;
        wave_lds_sync();
        const double piv = colw[c];
        const double zj = rfw[c];
        // a failed pivot (rare) is handled behind a wave-uniform branch, so
        // that the common step carries no divergent control flow
        const bool bad = (!(piv > dgw[c])) & act;
        const bool use = act & !bad;
        if (__ballot(bad) != 0ull) {
          // (selects rather than branches: the compiler would otherwise fold
          // this test into divergent control flow around every step)
          const int j = pw[c];
          myok = myok & !(bad & pl);
          retry = retry | (bad & useInv);
          const bool pin = bad & !useInv;
          const uint64_t drop = pin ? bit64(j) : 0ull;
          F &= ~drop;
          pinned |= drop;
          st |= pin ? NMF_BPP_SINGULAR : 0;
        }
        double inv = __builtin_amdgcn_rcp(piv);
        inv = fma(inv, fma(-piv, inv, 1.0), inv);
        inv = fma(inv, fma(-piv, inv, 1.0), inv);
        inv = use ? inv : 0.0;
        const double mlt = (use && !pl) ? r[c] * inv : 0.0;
        if (use && pl) mypiv = piv;
        // (the pivot row is read four entries at a time, so that its loads
        // do not all stay in flight beside the row)
#pragma unroll
        for (int q = c + 1; q < NP; ++q) {
          if ((q - c) % 4 == 0) __builtin_amdgcn_sched_barrier(0);
          r[q] -= mlt * colw[q];
        }
        rf -= mlt * zj;
        wave_lds_sync();
      }
      // the solved pivots by position (zero before the pivots and for a
      // failed pivot), then the owned entries
      vw[h] = myok ? rf / mypiv : 0.0;
      wave_lds_sync();
      double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        if constexpr (kFirst) {
          if (c < first) continue;
        }
        int cs = c;
        asm volatile("" : "+s"(cs));
        const bool act = cs >= off;
        if constexpr (!kFirst) {
          if (__ballot(act) == 0ull) continue;
        }
        if (c % 8 == 0) __builtin_amdgcn_sched_barrier(0);
        const int jc = act ? pw[c] : 0;
        const double vc = vw[c];
        acc0 += Mrow[jc * KS + i0] * vc;
        acc1 += Mrow[jc * KS + c1] * vc;
      }
      const double own0 = vw[s0 < L ? s0 : 0], own1 = vw[s1 < L ? s1 : 0];
      wave_lds_sync();
      const bool inF0 = !done && ((F >> i0) & 1ull), inF1 = !done && ((F >> i1) & 1ull);
      const bool pin0 = (pinned >> i0) & 1ull, pin1 = (pinned >> i1) & 1ull;
      double x0, y0, x1, y1;
      if (useInv) {
        x0 = inF0 ? zw[i0] - acc0 : 0.0;
        y0 = (inF0 || pin0) ? 0.0 : -own0;
        x1 = inF1 ? zw[i1] - acc1 : 0.0;
        y1 = (inF1 || pin1) ? 0.0 : -own1;
      } else {
        x0 = inF0 ? own0 : 0.0;
        y0 = inF0 ? 0.0 : acc0 - fw[i0];
        x1 = inF1 ? own1 : 0.0;
        y1 = inF1 ? 0.0 : acc1 - fw[i1];
      }
      const bool live = !done && !retry;
      const bool viol0 = val0 && live && !pin0 && (inF0 ? (x0 < 0.0) : (y0 < 0.0));
      const bool viol1 = val1 && live && !pin1 && (inF1 ? (x1 < 0.0) : (y1 < 0.0));
      const uint64_t bal0 = __ballot(viol0), bal1 = __ballot(viol1);
      const int sh = grp * L;
      constexpr uint64_t mL = (1ull << L) - 1ull;
      const uint64_t V = ((bal0 >> sh) & mL) | (((bal1 >> sh) & mL) << L);
      if (retry) forceG = true;
      if (live) {
        if (h == 0) {
          const uint32_t nf = (uint32_t)__popcll(F);
          pc[4] += (uint32_t)np;
          if (nf) {
            pc[0] += 1;
            pc[1] += nf;
            pc[2] += nf * nf;
            pc[3] += nf * nf * nf;
          }
        }
        ++rounds;
        ++since;
        if (V == 0) {
          done = true;
          finish(x0, x1);
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
          finish(x0 > 0.0 ? x0 : 0.0, x1 > 0.0 ? x1 : 0.0);
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
    if (vprob && defer) {
      if (h == 0) X[b * ldx] = __uint_as_float(kDeferMark);
    } else if (vprob) {
      if (h == 0) {
        tg[0] += (unsigned long long)rounds;
        for (int e = 0; e < 5; ++e) tg[1 + e] += pc[e];
        tg[6] += (st & NMF_BPP_CAPPED) ? 1 : 0;
        tg[7] += (st & NMF_BPP_WARM_FALLBACK) ? 1 : 0;
        if (pinned) st |= NMF_BPP_PINNED;
        if (mask_out) mask_out[b] = F;
        if (rounds_out) rounds_out[b] = (uint8_t)(rounds < 255 ? rounds : 255);
        if (status_out) status_out[b] = (uint8_t)st;
      }
    }
  }
}

template <int KK>
__global__ __launch_bounds__(pair_waves(KK) * 64) __attribute__((amdgpu_waves_per_eu(KK == 64 ? 3 : 4))) void k_bpp_pair(
    int k, int64_t batch, const double* __restrict__ G, const float* __restrict__ R, int64_t ldr,
    float* __restrict__ X, int64_t ldx, const uint64_t* mask_in, uint64_t* mask_out, uint8_t* __restrict__ rounds_out,
    uint8_t* __restrict__ status_out, int max_rounds, int warm_cap, unsigned long long* __restrict__ counters,
    double* __restrict__ dot_partial, unsigned long long* __restrict__ status_counts) {
  __shared__ PairShared<KK> sh;
  constexpr int NW = pair_waves(KK);
  sh.clear_stats();
  pair_block<KK>(sh, k, G, R, ldr, X, ldx, mask_in, mask_out, rounds_out, status_out, max_rounds, warm_cap, 0, batch,
                 (int64_t)blockIdx.x * NW + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), (int64_t)gridDim.x * NW);
  sh.flush(counters, dot_partial, status_counts);
}

// Grouped form: a persistent walk over items (ranges of problems of one G),
// each block taking whole items.
template <int KK>
__global__ __launch_bounds__(pair_waves(KK) * 64) __attribute__((amdgpu_waves_per_eu(KK == 64 ? 3 : 4))) void
k_bpp_pair_grouped(const nmf::BppItem* __restrict__ items, int64_t n, int max_rounds, int warm_cap,
                   unsigned long long* __restrict__ counters) {
  __shared__ PairShared<KK> sh;
  constexpr int NW = pair_waves(KK);
  sh.clear_stats();
  // a contiguous range of items per block: the items of one instance are
  // adjacent, so most calls find their G already loaded and swept
  const int64_t i0 = (int64_t)blockIdx.x * n / gridDim.x, i1 = ((int64_t)blockIdx.x + 1) * n / gridDim.x;
  const double* prevG = nullptr;
  int prevk = 0;
  for (int64_t i = i0; i < i1; ++i) {
    const nmf::BppItem it = items[i];
    const bool reuse = it.G == prevG && it.k == prevk;
    pair_block<KK>(sh, it.k, it.G, it.R, it.ldr, it.X, it.ldx, it.mask, it.mask, nullptr, it.status, max_rounds,
                   warm_cap, it.b0, it.b1, __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), NW, reuse);
    prevG = it.G;
    prevk = it.k;
  }
  sh.flush(counters, nullptr, nullptr);
}

// The one-row-per-lane form: solves the problems that k_bpp_pair marked, from
// their start sets, or with `every` all of them (when X overlaps R, so that
// no mark may be written).  dot_partial: one entry per block at
// dot_partial[dot_skip + block]; with `every` block 0 also zeros the
// dot_skip entries before them (the pivot-row kernel's, which did not run).
template <int K>
__global__ __launch_bounds__(256) void k_bpp_deferred(int k, int64_t batch, const double* __restrict__ G,
                                                      const float* __restrict__ R, int64_t ldr, float* X,
                                                      int64_t ldx, const uint64_t* mask_in, uint64_t* mask_out,
                                                      uint8_t* __restrict__ rounds_out,
                                                      uint8_t* __restrict__ status_out, int max_rounds, int warm_cap,
                                                      unsigned long long* __restrict__ counters,
                                                      double* __restrict__ dot_partial, int64_t dot_skip,
                                                      unsigned long long* __restrict__ status_counts, int every) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t w0 = (int64_t)blockIdx.x * kWaves + wave, ws = (int64_t)gridDim.x * kWaves;
  if (every && blockIdx.x == 0 && dot_partial)
    for (int64_t e = threadIdx.x; e < dot_skip; e += 256) dot_partial[e] = 0.0;
  double* dp = dot_partial ? dot_partial + dot_skip : nullptr;
  bool any = false;
  for (int64_t c0 = w0 * 64; c0 < batch; c0 += ws * 64) {
    const int64_t bb = c0 + lane;
    any |= bb < batch && (every || __float_as_uint(X[bb * ldx]) == kDeferMark);
  }
  if (!__syncthreads_or(any)) {
    if (threadIdx.x == 0 && dp) dp[blockIdx.x] = 0.0;
    return;
  }
  unsigned long long cacc[NMF_BPP_COUNTERS] = {0, 0, 0, 0, 0, 0};
  BppExtras ex;
  bpp_block<K>(k, G, R, ldr, X, ldx, mask_in, mask_out, rounds_out, status_out, max_rounds, warm_cap, 0, batch, w0,
               ws, cacc, ex, every != 0);
  if (counters) flush_counters(cacc, counters);
  if (dp || status_counts) flush_extras(ex, dp, status_counts);
}

// Grouped form of the same: for each item with marked problems, the
// one-row-per-lane form solves them (items without marks are skipped before G
// is loaded).
template <int K>
__global__ __launch_bounds__(256) void k_bpp_deferred_grouped(const nmf::BppItem* __restrict__ items, int64_t n,
                                                              int max_rounds, int warm_cap,
                                                              unsigned long long* __restrict__ counters) {
  unsigned long long cacc[NMF_BPP_COUNTERS] = {0, 0, 0, 0, 0, 0};
  BppExtras ex;  // not used here
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const nmf::BppItem it = items[i];
    bool any = false;
    for (int64_t c0 = it.b0 + wave * 64; c0 < it.b1; c0 += kWaves * 64) {
      const int64_t bb = c0 + lane;
      any |= bb < it.b1 && __float_as_uint(it.X[bb * it.ldx]) == kDeferMark;
    }
    if (!__syncthreads_or(any)) continue;
    bpp_block<K>(it.k, it.G, it.R, it.ldr, it.X, it.ldx, it.mask, it.mask, nullptr, it.status,
                              max_rounds, warm_cap, it.b0, it.b1, wave, kWaves, cacc, ex);
  }
  if (counters) flush_counters(cacc, counters);
}

constexpr int64_t kMaxBppBlocks = 1024;

// the pivot-row kernel's blocks, then the scan's (a chunk
// of 64 problems per wavefront)
int64_t pair_blocks(int K, int64_t batch) {
  const int64_t per_block = (int64_t)(64 / pair_lanes(K)) * pair_waves(K);
  const int64_t cap = K >= 56 ? kPairBlocks : 2 * kPairBlocks;
  const int64_t b = nmf::cdiv(batch, per_block);
  return b < cap ? b : cap;
}
int64_t scan_blocks(int64_t batch) {
  const int64_t b = nmf::cdiv(nmf::cdiv(batch, 64), kWaves);
  return b < kMaxBppBlocks ? b : kMaxBppBlocks;
}
int64_t launch_blocks(int K, int64_t batch) {
  return pair_blocks(K, batch) + scan_blocks(batch);
}

template <int K>
int launch(int k, int64_t batch, const double* G, const float* R, int64_t ldr, float* X, int64_t ldx,
           const uint64_t* mask_in, uint64_t* mask_out, uint8_t* rounds, uint8_t* status, int max_rounds,
           int warm_cap, uint64_t* counters, double* dot_partial, uint64_t* status_counts, hipStream_t s) {
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(counters);
  unsigned long long* sc = reinterpret_cast<unsigned long long*>(status_counts);
  const int64_t pb = pair_blocks(K, batch), db = scan_blocks(batch);
  // X overlapping R (allowed with ldx == ldr) leaves no room for a deferral
  // mark: then the one-row-per-lane form solves every problem instead
  const uintptr_t xb = (uintptr_t)X, xe = (uintptr_t)(X + (batch - 1) * ldx + k);
  const uintptr_t rb = (uintptr_t)R, re = (uintptr_t)(R + (batch - 1) * ldr + k);
  const int every = xb < re && rb < xe;
  if (!every) {
    hipLaunchKernelGGL(k_bpp_pair<K>, dim3((unsigned)pb), dim3(pair_waves(K) * 64), 0, s, k, batch, G, R, ldr, X,
                       ldx, mask_in, mask_out, rounds, status, max_rounds, warm_cap, cnt, dot_partial, sc);
    NMF_TRY(nmf::launch_status("nnls_bpp_batched (pivot rows only)"));
  }
  // deferred problems (or all): one per wavefront, in the class that holds every k <= K
  constexpr int KD = K == 64 ? 64 : 56;
  hipLaunchKernelGGL(k_bpp_deferred<KD>, dim3((unsigned)db), dim3(256), 0, s, k, batch, G, R, ldr, X, ldx, mask_in,
                     mask_out, rounds, status, max_rounds, warm_cap, cnt, dot_partial, pb, sc, every);
  return nmf::launch_status("nnls_bpp_batched (one row per lane)");
}

}  // namespace

namespace nmf {

int64_t bpp_blocks(int k, int64_t batch) { return batch > 0 ? launch_blocks(bpp_class(k), batch) : 0; }

int bpp_launch(int k, int64_t batch, const double* G, const float* R, int64_t ldr, float* X, int64_t ldx,
               const uint64_t* mask_in, uint64_t* mask_out, uint8_t* rounds, uint8_t* status, int max_rounds,
               int warm_cap, uint64_t* counters, hipStream_t s, double* dot_partial, uint64_t* status_counts) {
  if (batch == 0) return NMF_OK;
#define NMF_BPP_LAUNCH(KK)                                                                                   \
  return launch<KK>(k, batch, G, R, ldr, X, ldx, mask_in, mask_out, rounds, status, max_rounds, warm_cap, counters, \
                    dot_partial, status_counts, s)
  if (k <= 8) NMF_BPP_LAUNCH(8);
  if (k <= 16) NMF_BPP_LAUNCH(16);
  if (k <= 32) NMF_BPP_LAUNCH(32);
  if (k <= 56) NMF_BPP_LAUNCH(56);
  NMF_BPP_LAUNCH(64);
#undef NMF_BPP_LAUNCH
}

// The pivot-row classes: the grouped kernel, then the scan of its deferred
// problems (grid of the scan: one block per item up to the pivot-row grid's
// wavefront count).
template <int K>
int pair_grouped_launch(const BppItem* items, int64_t n, int grid, int max_rounds, int warm_cap,
                        unsigned long long* c, hipStream_t s) {
  hipLaunchKernelGGL(k_bpp_pair_grouped<K>, dim3((unsigned)grid), dim3(pair_waves(K) * 64), 0, s, items, n,
                     max_rounds, warm_cap, c);
  NMF_TRY(launch_status("nnls bpp (grouped, pivot rows only)"));
  constexpr int KD = K == 64 ? 64 : 56;
  const int64_t sg = n < (int64_t)grid * pair_waves(K) ? n : (int64_t)grid * pair_waves(K);
  hipLaunchKernelGGL(k_bpp_deferred_grouped<KD>, dim3((unsigned)sg), dim3(256), 0, s, items, n, max_rounds, warm_cap,
                     c);
  return launch_status("nnls bpp (grouped, deferred problems)");
}

int bpp_grouped_launch(int K, const BppItem* items, int64_t n, int grid, int max_rounds, int warm_cap,
                       uint64_t* counters, hipStream_t s) {
  if (n == 0) return NMF_OK;
  unsigned long long* c = reinterpret_cast<unsigned long long*>(counters);
  switch (K) {
    case 8: return pair_grouped_launch<8>(items, n, grid, max_rounds, warm_cap, c, s);
    case 16: return pair_grouped_launch<16>(items, n, grid, max_rounds, warm_cap, c, s);
    case 32: return pair_grouped_launch<32>(items, n, grid, max_rounds, warm_cap, c, s);
    case 56: return pair_grouped_launch<56>(items, n, grid, max_rounds, warm_cap, c, s);
    case 64: return pair_grouped_launch<64>(items, n, grid, max_rounds, warm_cap, c, s);
    default: return fail(NMF_EINVAL, "bpp (grouped): K=%d", K);
  }
  return launch_status("nnls bpp (grouped)");
}

int bpp_class(int k) { return k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : k <= 56 ? 56 : 64; }

int bpp_grouped_occupancy(int K, int* per_cu) {
  hipError_t e = hipErrorInvalidValue;
  switch (K) {
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_bpp_pair_grouped<8>, pair_waves(8) * 64, 0); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_bpp_pair_grouped<16>, pair_waves(16) * 64, 0); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_bpp_pair_grouped<32>, pair_waves(32) * 64, 0); break;
    case 56: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_bpp_pair_grouped<56>, pair_waves(56) * 64, 0); break;
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_bpp_pair_grouped<64>, pair_waves(64) * 64, 0); break;
    default: break;
  }
  return e == hipSuccess ? NMF_OK : NMF_EHIP;
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
