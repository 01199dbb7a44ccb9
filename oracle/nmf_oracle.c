/*
 * FP64 CPU oracle for ANLS-BPP nonnegative matrix factorisation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU path and is deliberately plain: loops in index order, float64
 * throughout (the data matrix A is held as its float32 values, promoted
 * exactly), OpenMP only across independent rows / columns so that the order
 * of every individual sum is fixed and written out here.
 *
 * What it computes (Kannan, Ballard & Park, "A High-Performance Parallel
 * Algorithm for Nonnegative Matrix Factorization"):
 *   - the NMF objective ||A - W H||_F^2 of the problem statement (Eq. NMF);
 *   - the alternating scheme of Eq. two-block / Algorithm 1 (ANLS): W from
 *     H H^T and A H^T, then H from W^T W and W^T A;
 *   - each row of W / column of H as an independent NNLS problem
 *     min_{x>=0} ||C x - b||^2 (Eq. single NLS), used only through
 *     G = C^T C and f = C^T b, solved by block principal pivoting (Section
 *     "Block Principal Pivoting"; the pivoting rules are those of Kim & Park,
 *     SIAM J. Sci. Comput. 33(6) 2011, with the Judice & Pires single-index
 *     backup rule, which the paper cites for the method's details);
 *   - the KKT conditions (Eq. KKT) used as the acceptance test of each BPP
 *     round.
 *
 * Readings where the paper is silent (the same rules hold on the GPU path):
 *   - index i is "pinned" (kept at x_i = 0, never made passive) when
 *     G_ii <= 1e-14 * max_l G_ll, or when its Cholesky pivot on the passive
 *     subset is <= 1e-12 * G_ii;
 *   - a problem that still violates KKT after `max_rounds` rounds stops with
 *     status CAPPED and returns its last iterate clamped to x >= 0;
 *   - a warm start that has not converged within `warm_cap` rounds restarts
 *     from the empty passive set (status WARM_FALLBACK).
 */
#include <omp.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXK 64

enum {
  ORC_ST_WARM_FALLBACK = 1,
  ORC_ST_CAPPED = 2,
  ORC_ST_PINNED = 4,
  ORC_ST_SINGULAR = 8,
};

/* ------------------------------------------------------------------------- */
/* Local products of Algorithm 1: Gram matrices and right-hand sides.         */
/* ------------------------------------------------------------------------- */

/* G = X^T X for X (rows x k, row-major, leading dimension ldx).  Gives H H^T
 * from Ht = H^T and W^T W from W (Algorithm 1, "Update W using H H^T ...").
 * Each entry is summed over rows in ascending order. */
void orc_gram(int64_t rows, int k, const double* X, int64_t ldx, double* G) {
  #pragma omp parallel for schedule(static)
  for (int i = 0; i < k; ++i) {
    double acc[ORC_MAXK];
    for (int j = 0; j < k; ++j) acc[j] = 0.0;
    for (int64_t r = 0; r < rows; ++r) {
      const double xi = X[r * ldx + i];
      for (int j = 0; j < k; ++j) acc[j] += xi * X[r * ldx + j];
    }
    for (int j = 0; j < k; ++j) G[i * k + j] = acc[j];
  }
}

/* R = A * Y: A is dense m x n (float32 values, row-major, lda), Y is n x k.
 * With Y = H^T this is A H^T, the right-hand side of the W update. */
void orc_rhs_dense_w(int64_t m, int64_t n, int k, const float* A, int64_t lda, const double* Y,
                     double* R) {
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    double acc[ORC_MAXK];
    for (int l = 0; l < k; ++l) acc[l] = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      const double a = (double)A[i * lda + j];
      for (int l = 0; l < k; ++l) acc[l] += a * Y[j * k + l];
    }
    for (int l = 0; l < k; ++l) R[i * k + l] = acc[l];
  }
}

/* R = A^T * Y: Y is m x k (Y = W), R is n x k, i.e. (W^T A)^T, the right-hand
 * side of the H update.  Each entry is summed over i in ascending order. */
void orc_rhs_dense_h(int64_t m, int64_t n, int k, const float* A, int64_t lda, const double* Y,
                     double* R) {
  const int64_t cb = 64;
  #pragma omp parallel for schedule(dynamic, 1)
  for (int64_t j0 = 0; j0 < n; j0 += cb) {
    const int64_t j1 = (j0 + cb < n) ? j0 + cb : n;
    double* acc = (double*)calloc((size_t)(j1 - j0) * k, sizeof(double));
    for (int64_t i = 0; i < m; ++i) {
      const double* y = Y + i * k;
      for (int64_t j = j0; j < j1; ++j) {
        const double a = (double)A[i * lda + j];
        double* out = acc + (j - j0) * k;
        for (int l = 0; l < k; ++l) out[l] += a * y[l];
      }
    }
    memcpy(R + j0 * k, acc, sizeof(double) * (size_t)(j1 - j0) * k);
    free(acc);
  }
}

/* R = A * Y for A in CSR (rows x cols), Y cols x k; nonzeros summed in
 * storage order.  Passing CSR(A) with Ht gives A H^T; CSR(A^T) with W gives
 * (W^T A)^T (the sparse case of the local products). */
void orc_rhs_csr(int64_t rows, int k, const int64_t* rowptr, const int32_t* colidx, const float* vals,
                 const double* Y, double* R) {
  #pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < rows; ++i) {
    double acc[ORC_MAXK];
    for (int l = 0; l < k; ++l) acc[l] = 0.0;
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      const double a = (double)vals[p];
      const double* y = Y + (int64_t)colidx[p] * k;
      for (int l = 0; l < k; ++l) acc[l] += a * y[l];
    }
    for (int l = 0; l < k; ++l) R[i * k + l] = acc[l];
  }
}

/* ------------------------------------------------------------------------- */
/* NNLS by block principal pivoting (Eq. single NLS, Eq. KKT).                */
/* ------------------------------------------------------------------------- */

/* Pinned indices: columns of C that are (numerically) zero. */
uint64_t orc_pinned_set(int k, const double* G) {
  double mx = 0.0;
  for (int i = 0; i < k; ++i) mx = G[i * k + i] > mx ? G[i * k + i] : mx;
  uint64_t p = 0;
  for (int i = 0; i < k; ++i)
    if (G[i * k + i] <= 1e-14 * mx) p |= (1ull << i);
  return p;
}

/* Least squares restricted to the passive set F via the normal equations
 * G_FF x_F = f_F (Section "Block Principal Pivoting" and Eq. KKT: on the
 * passive set the gradient vanishes, so x_F solves the passive block of the
 * normal equations), by Cholesky G_FF = L L^T built
 * row by row in index order.  An index whose pivot is <= 1e-12 * G_jj is
 * pinned and left out.  Writes x (x_i = 0 off F); returns the status bits. */
static int solve_passive(int k, const double* G, const double* f, uint64_t* F, uint64_t* pinned,
                         double* x) {
  int idx[ORC_MAXK];
  double L[ORC_MAXK][ORC_MAXK];
  int nf = 0, st = 0;
  for (int i = 0; i < k; ++i) x[i] = 0.0;
  for (int j = 0; j < k; ++j) {
    if (!((*F >> j) & 1ull)) continue;
    /* candidate row a = nf of L */
    for (int b = 0; b < nf; ++b) {
      double s = G[j * k + idx[b]];
      for (int c = 0; c < b; ++c) s -= L[nf][c] * L[b][c];
      L[nf][b] = s / L[b][b];
    }
    double d = G[j * k + j];
    for (int c = 0; c < nf; ++c) d -= L[nf][c] * L[nf][c];
    if (!(d > 1e-12 * G[j * k + j])) {
      *F &= ~(1ull << j);
      *pinned |= (1ull << j);
      st |= ORC_ST_SINGULAR;
      continue;
    }
    L[nf][nf] = sqrt(d);
    idx[nf++] = j;
  }
  /* L z = f_F, then L^T x_F = z */
  double z[ORC_MAXK];
  for (int a = 0; a < nf; ++a) {
    double s = f[idx[a]];
    for (int c = 0; c < a; ++c) s -= L[a][c] * z[c];
    z[a] = s / L[a][a];
  }
  for (int a = nf - 1; a >= 0; --a) {
    double s = z[a];
    for (int c = a + 1; c < nf; ++c) s -= L[c][a] * x[idx[c]];
    x[idx[a]] = s / L[a][a];
  }
  return st;
}

/* One NNLS problem min_{x>=0} 1/2 x^T G x - f^T x by block principal pivoting.
 *   F_io     : in = initial passive set (0 = cold start), out = final one
 *   max_rounds, warm_cap : round limits (see header)
 *   rounds_out : number of KKT checks performed
 *   y_out (optional): the final dual vector y = G x - f with y_F = 0
 * Returns the status bits. */
int orc_bpp(int k, const double* G, const double* f, double* x, uint64_t* F_io, int max_rounds,
            int warm_cap, int* rounds_out, double* y_out) {
  const uint64_t all = (k == 64) ? ~0ull : ((1ull << k) - 1ull);
  uint64_t pinned = orc_pinned_set(k, G);
  int st = pinned ? ORC_ST_PINNED : 0;
  /* a warm start is an initial passive set that is nonempty once the
   * pinned indices are removed from it */
  uint64_t F = *F_io & all & ~pinned;
  int warm = F != 0;
  int alpha = 3, beta = k + 1, rounds = 0, since_start = 0;
  double y[ORC_MAXK];
  for (;;) {
    st |= solve_passive(k, G, f, &F, &pinned, x);
    /* y = G x - f off the passive set, 0 on it (Eq. KKT) */
    for (int i = 0; i < k; ++i) {
      if ((F >> i) & 1ull) { y[i] = 0.0; continue; }
      double s = 0.0;
      for (int j = 0; j < k; ++j) s += G[i * k + j] * x[j];
      y[i] = s - f[i];
    }
    /* infeasible set V: passive with x < 0, or active (not pinned) with y < 0 */
    uint64_t V = 0;
    for (int i = 0; i < k; ++i) {
      if ((pinned >> i) & 1ull) continue;
      if (((F >> i) & 1ull) ? (x[i] < 0.0) : (y[i] < 0.0)) V |= (1ull << i);
    }
    ++rounds;
    ++since_start;
    if (V == 0) break;
    if (warm && since_start >= warm_cap) {
      /* warm start did not converge in time: restart cold */
      st |= ORC_ST_WARM_FALLBACK;
      warm = 0;
      F = 0;
      alpha = 3;
      beta = k + 1;
      since_start = 0;
      continue;
    }
    if (rounds >= max_rounds) {
      st |= ORC_ST_CAPPED;
      for (int i = 0; i < k; ++i) x[i] = x[i] > 0.0 ? x[i] : 0.0;
      break;
    }
    /* exchange rule: full exchange while |V| keeps shrinking, up to three
     * non-improving full exchanges, then the single largest index */
    const int nv = __builtin_popcountll(V);
    uint64_t S;
    if (nv < beta) {
      beta = nv;
      alpha = 3;
      S = V;
    } else if (alpha >= 1) {
      alpha -= 1;
      S = V;
    } else {
      S = 1ull << (63 - __builtin_clzll(V));
    }
    F ^= S;
  }
  *F_io = F;
  if (rounds_out) *rounds_out = rounds;
  if (y_out) memcpy(y_out, y, sizeof(double) * (size_t)k);
  if (pinned) st |= ORC_ST_PINNED;
  return st;
}

/* Rows of R (batch x k) as independent problems sharing G (Section "Naive
 * Parallel NMF Algorithm": the right-hand sides are independent). */
void orc_bpp_batched(int k, int64_t batch, const double* G, const double* R, double* X,
                     const uint64_t* mask_in, uint64_t* mask_out, int32_t* rounds, int32_t* status,
                     int max_rounds, int warm_cap) {
  #pragma omp parallel for schedule(dynamic, 64)
  for (int64_t b = 0; b < batch; ++b) {
    uint64_t F = mask_in ? mask_in[b] : 0ull;
    int r = 0;
    const int st = orc_bpp(k, G, R + b * k, X + b * k, &F, max_rounds, warm_cap, &r, NULL);
    if (mask_out) mask_out[b] = F;
    if (rounds) rounds[b] = r;
    if (status) status[b] = st;
  }
}

/* ------------------------------------------------------------------------- */
/* Objective (Eq. NMF)                                                        */
/* ------------------------------------------------------------------------- */

/* ||A||_F^2 and ||A - W H||_F^2 for dense A, with H given as Ht (n x k). */
void orc_objective_dense(int64_t m, int64_t n, int k, const float* A, int64_t lda, const double* W,
                         const double* Ht, double* fro2_A, double* fro2_res) {
  double sa = 0.0, sr = 0.0;
  #pragma omp parallel for schedule(static) reduction(+ : sa, sr)
  for (int64_t i = 0; i < m; ++i) {
    double ra = 0.0, rr = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      double wh = 0.0;
      for (int l = 0; l < k; ++l) wh += W[i * k + l] * Ht[j * k + l];
      const double a = (double)A[i * lda + j];
      ra += a * a;
      rr += (a - wh) * (a - wh);
    }
    sa += ra;
    sr += rr;
  }
  *fro2_A = sa;
  *fro2_res = sr;
}

/* Sparse A: ||A - WH||^2 = ||A||^2 - 2 sum_nnz a_ij (WH)_ij + <W^T W, H H^T>,
 * the expansion of the Frobenius norm over the stored entries plus the
 * trace term <W^T W, H H^T> = ||W H||_F^2. */
void orc_objective_csr(int64_t m, int64_t n, int k, const int64_t* rowptr, const int32_t* colidx,
                       const float* vals, const double* W, const double* Ht, double* fro2_A,
                       double* fro2_res) {
  double sa = 0.0, cross = 0.0;
  #pragma omp parallel for schedule(dynamic, 256) reduction(+ : sa, cross)
  for (int64_t i = 0; i < m; ++i) {
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      const double a = (double)vals[p];
      double wh = 0.0;
      for (int l = 0; l < k; ++l) wh += W[i * k + l] * Ht[(int64_t)colidx[p] * k + l];
      sa += a * a;
      cross += a * wh;
    }
  }
  double GW[ORC_MAXK * ORC_MAXK], GH[ORC_MAXK * ORC_MAXK];
  orc_gram(m, k, W, k, GW);
  orc_gram(n, k, Ht, k, GH);
  double t = 0.0;
  for (int i = 0; i < k * k; ++i) t += GW[i] * GH[i];
  *fro2_A = sa;
  *fro2_res = sa - 2.0 * cross + t;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1 (ANLS) driver                                                  */
/* ------------------------------------------------------------------------- */

typedef struct {
  int kind; /* 0 = dense, 1 = CSR */
  int64_t m, n;
  const float* A;
  int64_t lda;
  const int64_t* rowptr;
  const int32_t* colidx;
  const float* vals;
  const int64_t* rowptr_t;
  const int32_t* colidx_t;
  const float* vals_t;
} orc_matrix;

static void rhs_w(const orc_matrix* A, int k, const double* Ht, double* R) {
  if (A->kind == 0) orc_rhs_dense_w(A->m, A->n, k, A->A, A->lda, Ht, R);
  else orc_rhs_csr(A->m, k, A->rowptr, A->colidx, A->vals, Ht, R);
}

static void rhs_h(const orc_matrix* A, int k, const double* W, double* R) {
  if (A->kind == 0) orc_rhs_dense_h(A->m, A->n, k, A->A, A->lda, W, R);
  else orc_rhs_csr(A->n, k, A->rowptr_t, A->colidx_t, A->vals_t, W, R);
}

static double dot(int64_t len, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t i = 0; i < len; ++i) s += a[i] * b[i];
  return s;
}

/* Runs T iterations of Algorithm 1 from the given W, Ht (both overwritten).
 * Per iteration t it records the relative objective ||A-WH||_F / ||A||_F
 * after the W update (r_half[t]) and after the H update (r_full[t]), using
 * the expansion ||A||^2 - 2 <R, X> + <W^T W, H H^T> with R the right-hand side
 * of the factor X just computed.  warm = 1 starts each BPP from the previous
 * iteration's passive set of the same row/column (same unique solution).
 * rounds_w / rounds_h (optional, T entries) receive the total BPP rounds per
 * half-step; masks_w / masks_h (optional) receive the final passive sets. */
/* Wall seconds of the last orc_anls call by phase (timing only):
 * [0] A H^T, [1] BPP for W, [2] both Gram products, [3] W^T A, [4] BPP for H,
 * [5] the objective sums. */
static double g_phase[6];
void orc_last_phase_seconds(double* out) {
  for (int i = 0; i < 6; ++i) out[i] = g_phase[i];
}

int orc_anls(const orc_matrix* A, int k, double* W, double* Ht, int T, int max_rounds, int warm,
             int warm_cap, double fro2_A, double* r_half, double* r_full, int64_t* rounds_w,
             int64_t* rounds_h, int64_t* capped, uint64_t* masks_w, uint64_t* masks_h) {
  const int64_t m = A->m, n = A->n;
  for (int i = 0; i < 6; ++i) g_phase[i] = 0.0;
  double tw = omp_get_wtime(), tn;
#define ORC_PHASE(i) (tn = omp_get_wtime(), g_phase[i] += tn - tw, tw = tn)
  double* RW = (double*)malloc(sizeof(double) * (size_t)m * k);
  double* RH = (double*)malloc(sizeof(double) * (size_t)n * k);
  uint64_t* MW = (uint64_t*)calloc((size_t)m, sizeof(uint64_t));
  uint64_t* MH = (uint64_t*)calloc((size_t)n, sizeof(uint64_t));
  int32_t* rnd = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > n ? m : n));
  int32_t* sts = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > n ? m : n));
  if (!RW || !RH || !MW || !MH || !rnd || !sts) return 1;
  double GH[ORC_MAXK * ORC_MAXK], GW[ORC_MAXK * ORC_MAXK];
  int64_t ncap = 0;
  for (int t = 0; t < T; ++t) {
    /* W <- argmin_{W>=0} ||A - W H||  via  H H^T and A H^T */
    orc_gram(n, k, Ht, k, GH);
    ORC_PHASE(2);
    rhs_w(A, k, Ht, RW);
    ORC_PHASE(0);
    orc_bpp_batched(k, m, GH, RW, W, warm ? MW : NULL, MW, rnd, sts, max_rounds, warm_cap);
    int64_t s = 0;
    for (int64_t i = 0; i < m; ++i) { s += rnd[i]; ncap += (sts[i] & ORC_ST_CAPPED) != 0; }
    if (rounds_w) rounds_w[t] = s;
    ORC_PHASE(1);
    orc_gram(m, k, W, k, GW);
    ORC_PHASE(2);
    if (r_half) {
      double r2 = fro2_A - 2.0 * dot(m * k, RW, W) + dot(k * k, GW, GH);
      r_half[t] = sqrt(r2 > 0.0 ? r2 : 0.0) / sqrt(fro2_A);
    }
    ORC_PHASE(5);
    /* H <- argmin_{H>=0} ||A - W H||  via  W^T W and W^T A */
    rhs_h(A, k, W, RH);
    ORC_PHASE(3);
    orc_bpp_batched(k, n, GW, RH, Ht, warm ? MH : NULL, MH, rnd, sts, max_rounds, warm_cap);
    s = 0;
    for (int64_t j = 0; j < n; ++j) { s += rnd[j]; ncap += (sts[j] & ORC_ST_CAPPED) != 0; }
    if (rounds_h) rounds_h[t] = s;
    ORC_PHASE(4);
    orc_gram(n, k, Ht, k, GH);
    ORC_PHASE(2);
    if (r_full) {
      double r2 = fro2_A - 2.0 * dot(n * k, RH, Ht) + dot(k * k, GW, GH);
      r_full[t] = sqrt(r2 > 0.0 ? r2 : 0.0) / sqrt(fro2_A);
    }
    ORC_PHASE(5);
  }
#undef ORC_PHASE
  if (capped) *capped = ncap;
  if (masks_w) memcpy(masks_w, MW, sizeof(uint64_t) * (size_t)m);
  if (masks_h) memcpy(masks_h, MH, sizeof(uint64_t) * (size_t)n);
  free(RW); free(RH); free(MW); free(MH); free(rnd); free(sts);
  return 0;
}

/* Threads the OpenMP loops above use (reported with the CPU baseline). */
int orc_max_threads(void) { return omp_get_max_threads(); }
/* Thread count of the parallel loops (for timing the oracle at 1 thread). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
