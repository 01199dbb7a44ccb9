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
// ballot; the exchange rule is evaluated identically by every lane.  In the
// one-problem classes the pivot columns are first packed at the end of the
// row (see the elimination), so a step touches only later pivots.
//
// Two forms of the same passive-set solve.  Each block also sweeps G once
// (symmetric sweep operator over the unpinned indices U, FP64, index order)
// to get G_U^{-1} in LDS, and each problem forms z = G_U^{-1} f.  When the
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

// Solves problems b0 + g * P + sub (g = g_first, g_first + g_step, ... while
// b0 + g * P < b1) of one Gram matrix G; P = 64 / K problems per wavefront,
// sub selects the lane group.  Loads G into LDS first (after a barrier, so a
// persistent loop may call it again with another G).  Round and solve
// statistics are added to cacc (per lane; summed by the caller).
template <int K, bool kRegGi = false>
__device__ __forceinline__ void bpp_block(int k, const double* __restrict__ G, const float* __restrict__ R,
                                          int64_t ldr, float* __restrict__ X, int64_t ldx, const uint64_t* mask_in,
                                          uint64_t* mask_out, uint8_t* __restrict__ rounds_out,
                                          uint8_t* __restrict__ status_out, int max_rounds, int warm_cap, int64_t b0,
                                          int64_t b1, int64_t g_first, int64_t g_step,
                                          unsigned long long (&cacc)[NMF_BPP_COUNTERS], BppExtras& ex) {
  constexpr int P = 64 / K;
  __shared__ double Gs[K * K];
  __shared__ double Gi[K * K];
  __shared__ int inv_ok_s;
  // one slot per lane, plus (one-problem classes) a spare slot 64 for the
  // packed form's non-pivot lanes
  constexpr int kSlots = P == 1 ? 65 : 64;
  __shared__ double colv[kWaves][kSlots];
  __shared__ double rfv[kWaves][kSlots];
  __shared__ double dgv[kWaves][P == 1 ? 65 : 1];
  __shared__ int pix[kWaves][P == 1 ? 65 : 1];

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
  // kRegGi (the single-matrix kernel's 32-lane class) keeps this lane's
  // column of G_U^{-1} in registers for every problem's z (W side at
  // 10^6 x 2400, k = 30: 0.920 -> 0.896 ms); elsewhere it would cost a
  // wavefront per SIMD
  double gic[kRegGi ? K : 1];
  if constexpr (kRegGi) {
#pragma unroll
    for (int q = 0; q < K; ++q) gic[q] = Gi[q * K + p];
  }

  // the next problem's right-hand side and start set are loaded while the
  // current one is solved
  const int64_t gstride = g_step;
  int64_t g = g_first;
  float f_next = 0.0f;
  uint64_t m_next = 0;
  {
    const int64_t b = b0 + g * P + sub;
    if (lane_in && b < b1 && p < k) f_next = R[b * ldr + p];
    if (lane_in && b < b1 && mask_in) m_next = mask_in[b];
  }
  for (; b0 + g * P < b1; g += gstride) {
    const int64_t b = b0 + g * P + sub;
    const bool vprob = lane_in && b < b1;
    const bool valid = vprob && p < k;
    const double f = (double)f_next;
    uint64_t F = vprob ? (m_next & all & ~pinned0) : 0ull;
    {
      const int64_t bn = b0 + (g + gstride) * P + sub;
      f_next = (lane_in && bn < b1 && p < k) ? R[bn * ldr + p] : 0.0f;
      m_next = (lane_in && bn < b1 && mask_in) ? mask_in[bn] : 0ull;
    }
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
      for (int q = 0; q < K; ++q) {
        double gq;
        if constexpr (kRegGi) {
          gq = gic[q];
        } else {
          gq = Gi[q * K + p];
        }
        z += gq * rfv[wave][base + q];
      }
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
      } else if constexpr (P == 1) {
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
      } else {
        double r[K];
#pragma unroll
        for (int q = 0; q < K; ++q) r[q] = Mrow[q * K + p];
        double rf = rf0, mypiv = 1.0;
        // The lanes of a problem hold the same pivot set, so the union over
        // the wavefront's problems is the OR of lanes 0, K, 2K, ... (read into
        // SGPRs), and the per-index skip test is a scalar branch.
        uint64_t PU = 0;
#pragma unroll
        for (int sp = 0; sp < P; ++sp)
          PU |= ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(Pv >> 32), sp * K) << 32) |
                (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)Pv, sp * K);
        {
#pragma unroll
          for (int j = 0; j < K; ++j) {
            const bool pj = (Pv >> j) & 1ull;
            if (!((PU >> j) & 1ull)) continue;
            colv[wave][lane] = r[j];
            rfv[wave][lane] = rf;
            wave_lds_sync();
            const double piv = colv[wave][base + j];
            const double zj = rfv[wave][base + j];
            bool use = pj;
            if (pj && !(piv > 1e-12 * Mrow[j * K + j])) {
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
            // 1 / piv: hardware estimate and two Newton steps y <- y (2 - piv y)
            double inv = __builtin_amdgcn_rcp(piv);
            inv = fma(inv, fma(-piv, inv, 1.0), inv);
            inv = fma(inv, fma(-piv, inv, 1.0), inv);
            inv = use ? inv : 0.0;
            const double mlt = (use && p != j) ? r[j] * inv : 0.0;
            if (use && p == j) mypiv = piv;
#pragma unroll
            for (int q = j + 1; q < K; ++q) r[q] -= mlt * colv[wave][base + q];
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

// Sums the per-lane statistics of the block and adds them to counters.
__device__ __forceinline__ void flush_counters(const unsigned long long (&cacc)[NMF_BPP_COUNTERS],
                                               unsigned long long* __restrict__ counters) {
  __shared__ unsigned long long cnt[kWaves][NMF_BPP_COUNTERS];
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
    for (int w = 0; w < kWaves; ++w) s += cnt[w][t];
    if (s) atomicAdd(counters + t, s);
  }
}

// Block sums of the extras: the dot sum to dot_partial[blockIdx.x] (summed
// in a fixed order, so the result does not depend on timing), the status
// counts added to status_counts[0] (capped) and [1] (fell back).
__device__ __forceinline__ void flush_extras(const BppExtras& ex, double* __restrict__ dot_partial,
                                             unsigned long long* __restrict__ status_counts) {
  __shared__ double sd[kWaves];
  __shared__ unsigned long long sc[kWaves][2];
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
    for (int w = 0; w < kWaves; ++w) {
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

template <int K>
__global__ __launch_bounds__(256) void k_bpp(int k, int64_t batch, const double* __restrict__ G,
                                             const float* __restrict__ R, int64_t ldr, float* __restrict__ X,
                                             int64_t ldx, const uint64_t* mask_in,
                                             uint64_t* mask_out, uint8_t* __restrict__ rounds_out,
                                             uint8_t* __restrict__ status_out, int max_rounds, int warm_cap,
                                             unsigned long long* __restrict__ counters,
                                             double* __restrict__ dot_partial,
                                             unsigned long long* __restrict__ status_counts) {
  unsigned long long cacc[NMF_BPP_COUNTERS] = {0, 0, 0, 0, 0, 0};
  BppExtras ex;
  const int wave = threadIdx.x >> 6;
  bpp_block<K, K == 32>(k, G, R, ldr, X, ldx, mask_in, mask_out, rounds_out, status_out, max_rounds, warm_cap, 0,
                        batch, (int64_t)blockIdx.x * kWaves + wave, (int64_t)gridDim.x * kWaves, cacc, ex);
  if (counters) flush_counters(cacc, counters);
  if (dot_partial || status_counts) flush_extras(ex, dot_partial, status_counts);
}

// Grouped form: a persistent walk over items, each a range of problems of
// one Gram matrix (start sets from, and final sets to, the item's masks when
// it has them; cold starts otherwise).
template <int K>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(K >= 56 ? 2 : 1))) void k_bpp_grouped(const nmf::BppItem* __restrict__ items, int64_t n,
                                                     int max_rounds, int warm_cap,
                                                     unsigned long long* __restrict__ counters) {
  unsigned long long cacc[NMF_BPP_COUNTERS] = {0, 0, 0, 0, 0, 0};
  BppExtras ex;  // not used here
  const int wave = threadIdx.x >> 6;
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const nmf::BppItem it = items[i];
    bpp_block<K>(it.k, it.G, it.R, it.ldr, it.X, it.ldx, it.mask, it.mask, nullptr, it.status, max_rounds, warm_cap,
                 it.b0, it.b1, wave, kWaves, cacc, ex);
  }
  if (counters) flush_counters(cacc, counters);
}

constexpr int64_t kMaxBppBlocks = 1024;

int64_t grid_blocks(int K, int64_t batch) {
  const int64_t waves = nmf::cdiv(batch, 64 / K);
  const int64_t blocks = nmf::cdiv(waves, kWaves);
  return blocks < kMaxBppBlocks ? blocks : kMaxBppBlocks;
}

template <int K>
int launch(int k, int64_t batch, const double* G, const float* R, int64_t ldr, float* X, int64_t ldx,
           const uint64_t* mask_in, uint64_t* mask_out, uint8_t* rounds, uint8_t* status, int max_rounds,
           int warm_cap, uint64_t* counters, double* dot_partial, uint64_t* status_counts, hipStream_t s) {
  const int64_t blocks = grid_blocks(K, batch);
  hipLaunchKernelGGL(k_bpp<K>, dim3((unsigned)blocks), dim3(256), 0, s, k, batch, G, R, ldr, X, ldx, mask_in,
                     mask_out, rounds, status, max_rounds, warm_cap,
                     reinterpret_cast<unsigned long long*>(counters), dot_partial,
                     reinterpret_cast<unsigned long long*>(status_counts));
  return nmf::launch_status("nnls_bpp_batched");
}

}  // namespace

namespace nmf {

int64_t bpp_blocks(int k, int64_t batch) { return batch > 0 ? grid_blocks(bpp_class(k), batch) : 0; }

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

int bpp_grouped_launch(int K, const BppItem* items, int64_t n, int grid, int max_rounds, int warm_cap,
                       uint64_t* counters, hipStream_t s) {
  if (n == 0) return NMF_OK;
  unsigned long long* c = reinterpret_cast<unsigned long long*>(counters);
  switch (K) {
    case 8: hipLaunchKernelGGL(k_bpp_grouped<8>, dim3((unsigned)grid), dim3(256), 0, s, items, n, max_rounds, warm_cap, c); break;
    case 16: hipLaunchKernelGGL(k_bpp_grouped<16>, dim3((unsigned)grid), dim3(256), 0, s, items, n, max_rounds, warm_cap, c); break;
    case 32: hipLaunchKernelGGL(k_bpp_grouped<32>, dim3((unsigned)grid), dim3(256), 0, s, items, n, max_rounds, warm_cap, c); break;
    case 56: hipLaunchKernelGGL(k_bpp_grouped<56>, dim3((unsigned)grid), dim3(256), 0, s, items, n, max_rounds, warm_cap, c); break;
    case 64: hipLaunchKernelGGL(k_bpp_grouped<64>, dim3((unsigned)grid), dim3(256), 0, s, items, n, max_rounds, warm_cap, c); break;
    default: return fail(NMF_EINVAL, "bpp (grouped): K=%d", K);
  }
  return launch_status("nnls bpp (grouped)");
}

int bpp_class(int k) { return k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : k <= 56 ? 56 : 64; }

int bpp_grouped_occupancy(int K, int* per_cu) {
  hipError_t e = hipErrorInvalidValue;
  switch (K) {
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_bpp_grouped<8>, 256, 0); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_bpp_grouped<16>, 256, 0); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_bpp_grouped<32>, 256, 0); break;
    case 56: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_bpp_grouped<56>, 256, 0); break;
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_bpp_grouped<64>, 256, 0); break;
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
