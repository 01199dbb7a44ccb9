/*
 * libnmf -- ANLS-BPP nonnegative matrix factorisation on one MI355X (gfx950).
 *
 * Problem (Kannan, Ballard & Park, Eq. NMF): given A (m x n), find W >= 0
 * (m x k) and H >= 0 (k x n) minimising ||A - W H||_F^2, by the alternating
 * scheme of Eq. two-block / Algorithm 1: W from (H H^T, A H^T), then H from
 * (W^T W, W^T A), each row of W and column of H being an independent
 * nonnegative least-squares problem (Eq. single NLS) solved by block principal
 * pivoting (Section "Block Principal Pivoting").
 *
 * Conventions for every entry point:
 *  - Pointers named as device pointers are device memory, owned and allocated
 *    by the caller; the library never allocates or frees device memory (its
 *    one static device array, the scratch of nmf_gram_noalloc, is part of the
 *    loaded code object).
 *  - Matrices are row-major with an explicit leading dimension (in elements).
 *    H is always passed transposed, as Ht (n x k), so that both factor
 *    updates are "one problem per row of an (rows x k) matrix".
 *  - Scratch space is a caller-provided device buffer `ws` of `ws_bytes`,
 *    sized by the matching *_workspace_bytes query (256-byte aligned).
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL means
 *    the default stream) and is complete only after the stream is
 *    synchronised.  No entry point synchronises the stream.
 *  - Return value: NMF_OK, or an error code; on error nothing has been
 *    enqueued unless the code is NMF_EHIP, and nmf_last_error() returns a
 *    message (thread-local).  Argument checks are done on the host before any
 *    device call.
 *  - k (the rank) must satisfy 1 <= k <= 64.
 */
#ifndef LIBNMF_H
#define LIBNMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------- */
#define NMF_OK 0
#define NMF_EINVAL 1        /* bad size, leading dimension, null pointer, k */
#define NMF_EUNSUPPORTED 2  /* a combination the library does not implement */
#define NMF_EHIP 3          /* a HIP runtime call or kernel launch failed */
#define NMF_EWORKSPACE 4    /* ws too small (query *_workspace_bytes) */

/* ---- enumerations --------------------------------------------------------- */
#define NMF_F32 0     /* right-hand sides in FP32 (MFMA / SpMM) */
#define NMF_BF16X3 1  /* right-hand sides as hi*hi + hi*lo + lo*hi BF16 MFMA, FP32 accumulate */

#define NMF_SIDE_W 0  /* R (m x k) = A  * Ht : right-hand side of the W update */
#define NMF_SIDE_H 1  /* R (n x k) = A^T * W : (W^T A)^T, right-hand side of the H update */

#define NMF_DENSE 0
#define NMF_CSR 1

#define NMF_OBJ_DIRECT 0  /* ||A - W H||_F from A itself (dense) or its nonzeros (CSR) */
#define NMF_OBJ_TRACE 1   /* ||A||^2 - 2 <A^T W, H^T> + <W^T W, H H^T>, FP64, monitoring */

#define NMF_WARM_COLD 0     /* every BPP starts from the empty passive set */
#define NMF_WARM_PREV 1     /* start from the previous iteration's passive set */
#define NMF_WARM_LEARNED 2  /* start from the warm-start network's prediction */
#define NMF_WARM_ALL 3      /* start from the full set (every unpinned index passive) */

/* local NLS solver of Algorithm 1 (nmf_opts.solver, nmf_local_update) */
#define NMF_SOLVER_BPP 0    /* block principal pivoting (the exact NNLS solution) */
#define NMF_SOLVER_HALS 1   /* one HALS sweep, Eq. halsupdate */
#define NMF_SOLVER_MU 2     /* one multiplicative update, Eq. muupdate */

/* per-problem BPP status bits */
#define NMF_BPP_WARM_FALLBACK 1  /* warm start restarted cold after warm_cap rounds */
#define NMF_BPP_CAPPED 2         /* KKT still violated after max_rounds; x clamped to >= 0 */
#define NMF_BPP_PINNED 4         /* an index with G_ii <= 1e-14 max G_ll was held at 0 */
#define NMF_BPP_SINGULAR 8       /* a passive-subset pivot <= 1e-12 G_jj; index held at 0 */

/* BPP counters (device array of NMF_BPP_COUNTERS uint64, accumulated, optional):
 * [0] KKT checks (rounds), [1] passive-set solves (rounds with F nonempty),
 * [2] sum |F|, [3] sum |F|^2, [4] sum |F|^3, each over the solves,
 * [5] elimination (pivot) steps executed. */
#define NMF_BPP_COUNTERS 6

const char* nmf_last_error(void);
const char* nmf_version(void);

/* ---- Gram matrix ----------------------------------------------------------
 * G = X^T X (k x k, FP64, both triangles, ld k) for X (rows x k, FP32,
 * leading dimension ldx >= k).  With X = Ht this is H H^T, with X = W it is
 * W^T W (Algorithm 1, both updates; the local Gram of Algorithm 3).  FP32
 * products are exact in FP64 and are summed in FP64 in a fixed order, so the
 * result is deterministic.  rows == 0 gives G = 0 (X and ldx unused). */
int nmf_gram_workspace_bytes(int64_t rows, int k, size_t* bytes);
int nmf_gram(int64_t rows, int k, const float* X, int64_t ldx, double* G, void* ws, size_t ws_bytes,
             void* stream);

/* The same Gram matrix, for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no workspace argument, and no allocation of any kind.  The block partials
 * go to a static device array of NMF_GRAM_NOALLOC_SCRATCH_BYTES (32 MiB),
 * which every device the library runs this on keeps until the process ends;
 * it holds the partials of every valid (rows, k), and a request beyond it
 * would return NMF_EINVAL.  Same kernels and summation order as nmf_gram, so
 * the result is bit-identical to it.  The first call on a device looks up the
 * array's address there (a runtime symbol query, no allocation).  All calls on
 * one device share the array: calls that overlap in time on one device (two
 * streams, two host threads) race and give wrong results; serialise them.
 * Nothing in the array needs to start at zero, so what an earlier call left
 * there is never read.  Errors: NMF_EINVAL as nmf_gram, NMF_EHIP if the
 * address lookup fails, NMF_EUNSUPPORTED for a device index >= 64. */
#define NMF_GRAM_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int nmf_gram_noalloc(int64_t rows, int k, const float* X, int64_t ldx, double* G, void* stream);

/* ---- dense right-hand sides -----------------------------------------------
 * side NMF_SIDE_W: R (m x k) = A (m x n) * Y with Y = Ht (n x k), i.e. A H^T.
 * side NMF_SIDE_H: R (n x k) = A^T * Y with Y = W (m x k), i.e. (W^T A)^T.
 * A: FP32 m x n, leading dimension lda >= n (device).
 * prec NMF_F32: FP32 MFMA with FP32 accumulation (side H: split over rows of
 *   A with a deterministic FP64 sum of the FP32 partials).
 * prec NMF_BF16X3: the operand whose rows are the output rows is given in the
 *   padded BF16 form of nmf_split_bf16: for side W that of A (transpose 0),
 *   for side H that of A^T (transpose 1).  Y is split in the workspace each
 *   call; R = hi*hi + hi*lo + lo*hi (lo*lo dropped), FP32 accumulation.  A
 *   itself is not read in this mode and may be NULL.
 * R: FP32, leading dimension ldr >= k (device). */
/* Error analysis: the longest FP32 accumulation (number of products added
 * into one FP32 accumulator) that nmf_rhs_dense uses for these arguments on
 * the current device (split-K partials are summed in FP64 afterwards), so
 * |R - R_exact(operands)| <= terms * 2^-24 * (|A| |Y|) entrywise, the
 * operands being FP32 A and Y, or for NMF_BF16X3 the three BF16 products. */
int nmf_rhs_dense_chain(int side, int64_t m, int64_t n, int k, int prec, int64_t* terms);
int nmf_rhs_dense_workspace_bytes(int side, int64_t m, int64_t n, int k, int prec, size_t* bytes);
int nmf_rhs_dense(int side, int64_t m, int64_t n, int k, const float* A, int64_t lda, const void* B_bf16,
                  const float* Y, int64_t ldy, float* R, int64_t ldr, int prec, void* ws, size_t ws_bytes,
                  void* stream);

/* One-time split of an FP32 matrix X (rows x cols, ldx) into the padded BF16
 * form: the operand B = X (transpose 0) or B = X^T (transpose 1), rows_B x
 * cols_B, is stored as two row-major planes of Rp x Cp BF16 values (Rp =
 * rows_B rounded up to 128, Cp = cols_B rounded up to 64, zero padding): the
 * hi plane, then the lo plane, hi = bf16_rne(x), lo = bf16_rne(x - hi)
 * (x - hi is exact in FP32).  The 4 bytes per entry of A are kept.
 * nmf_split_bf16_bytes gives the size of `out` (device). */
size_t nmf_split_bf16_bytes(int64_t rows, int64_t cols, int transpose);
int nmf_split_bf16(int64_t rows, int64_t cols, const float* X, int64_t ldx, int transpose, void* out, void* stream);

/* One-time FP32 transposed copy: out (cols x rows, leading dimension ldo >=
 * rows) = X^T for X rows x cols (ldx >= cols), all device pointers; exact.
 * Keeping both orientations of A resident is what the BF16 planes do for the
 * BF16X3 form; this gives the FP32 form the same (nmf_matrix.At).  X and out
 * may not overlap.  An empty matrix is a no-op.  NMF_EINVAL for negative
 * sizes, or for a non-empty matrix with short leading dimensions or a null
 * pointer. */
int nmf_transpose_f32(int64_t rows, int64_t cols, const float* X, int64_t ldx, float* out, int64_t ldo,
                      void* stream);

/* ---- sparse right-hand side -----------------------------------------------
 * R (rows x k) = A_csr (rows x cols) * Y (cols x k, ldy >= k).  Pass CSR(A)
 * with Y = Ht for A H^T, CSR(A^T) with Y = W for (W^T A)^T.  rowptr int64
 * (rows + 1), colidx int32 in [0, cols), vals FP32.  One wavefront per row,
 * products accumulated in FP64 in storage order, stored as FP32.  The cost is
 * gathering one row of Y per nonzero: an ldy whose rows never straddle a
 * 128-byte line (a power of two >= k for k <= 32, else a multiple of 32) is
 * markedly faster; nmf_anls_iter copies its factor to such a layout itself. */
int nmf_rhs_csr(int64_t rows, int64_t cols, int k, const int64_t* rowptr, const int32_t* colidx,
                const float* vals, const float* Y, int64_t ldy, float* R, int64_t ldr, void* stream);

/* ---- batched NNLS by block principal pivoting -----------------------------
 * For each row b < batch: X[b] = argmin_{x >= 0} 1/2 x^T G x - R[b]^T x,
 * i.e. min ||C x - c||^2 with C^T C = G, C^T c = R[b] (Eq. single NLS, KKT
 * conditions Eq. KKT).  G: k x k FP64, symmetric (device).  R: FP32 rows,
 * ldr >= k; X: FP32 rows, ldx >= k (X may alias R only if ldx == ldr; then
 * every problem is solved by the slower one-row-per-lane form).
 * mask_in (optional): initial passive sets (bit i = index i passive); NULL
 * or an all-zero mask is a cold start.  mask_out (optional): final passive
 * sets (may alias mask_in).  rounds (optional): KKT checks per problem
 * (saturating at 255).  status (optional): NMF_BPP_* bits per problem.
 * max_rounds >= 1 caps the KKT checks; warm_cap >= 1 is the number of rounds a
 * nonempty mask_in gets before the cold restart.  counters (optional): see
 * NMF_BPP_COUNTERS; accumulated (not cleared).  The passive-subset systems
 * are solved in FP64 (symmetric elimination in index order).  Returns
 * NMF_OK even when some problems are capped (see status). */
int nnls_bpp_batched(int k, int64_t batch, const double* G, const float* R, int64_t ldr, float* X,
                     int64_t ldx, const uint64_t* mask_in, uint64_t* mask_out, uint8_t* rounds,
                     uint8_t* status, int max_rounds, int warm_cap, uint64_t* counters, void* stream);

/* ---- learned warm start ---------------------------------------------------
 * A network predicts each problem's starting passive set for BPP (Section
 * "Block Principal Pivoting": BPP searches for this set; any start is
 * verified by the KKT test of Eq. KKT and a start that does not converge in
 * warm_cap rounds restarts cold).  Features of a problem (G, f):
 *   phi = [ s / ||s||_2 , diag(G) / mean(diag(G)) ]  (2k),  s_i = f_i / sqrt(G_ii)
 * (s_i = 0 for pinned indices); network 2k -> 128 -> 128 -> k with ReLU,
 * start set { i : logit_i > 0 } minus pinned indices.  Parameters: one FP32
 * device vector, W1[2k][128], b1[128], W2[128][128], b2[128], W3[128][k],
 * b3[k] (input-major); nmf_mlp_param_count(k) gives its length. */
int nmf_mlp_param_count(int k);

/* phi (batch x 2k FP32, device) of the rows of R (ldr >= k) against G. */
int nmf_features(int k, int64_t batch, const double* G, const float* R, int64_t ldr, float* phi, void* stream);

/* Start sets for every row of R: features and the three layers fused on BF16
 * MFMA (FP32 accumulation), written to mask_out (device uint64 per row). */
int nmf_mlp_predict(int k, int64_t batch, const double* G, const float* R, int64_t ldr, const float* params,
                    uint64_t* mask_out, void* stream);

/* Training in FP32 on (phi, final passive set) samples (device, nsamples of
 * each) by Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * mean binary cross-entropy.  Step t (t = step0 .. step0+steps-1) uses the
 * samples order[(t - step0) * batch + i], i < batch, when `order` (device
 * int64, steps * batch entries in [0, nsamples)) is given, else the fixed
 * draw ((t * 1000003 + i + 1) * 0x9E3779B97F4A7C15 >> 11) mod nsamples; the
 * bias correction uses t + 1.  params, adam_m, adam_v are updated in place.
 * loss_out (optional, device FP64): mean loss of the last step's batch.
 * nmf_mlp_grad: the gradient (FP32, param-count entries) and mean loss of the
 * first `batch` samples, for checking. */
int nmf_mlp_train_workspace_bytes(int k, int batch, size_t* bytes);
int nmf_mlp_grad(int k, int batch, const float* params, const float* phi, const uint64_t* masks, float* grad_out,
                 double* loss_out, void* ws, size_t ws_bytes, void* stream);
int nmf_mlp_train(int k, float* params, float* adam_m, float* adam_v, const float* phi, const uint64_t* masks,
                  int64_t nsamples, const int64_t* order, int steps, int batch, float lr, int64_t step0,
                  double* loss_out, void* ws, size_t ws_bytes, void* stream);

/* ---- other local updates (Section "Nonnegative Least Squares") ------------
 * One MU (Eq. muupdate) or HALS (Eq. halsupdate) update of every row x of X
 * (rows x k FP32, ldx >= k, device, in place) from G (k x k FP64, row-major,
 * device: the Gram matrix of the other factor, which must be symmetric; the
 * kernel reads column l of G as row l) and R (rows x k FP32, ldr >= k: A H^T rows for
 * the rows of W, (W^T A)^T rows for the rows of H^T):
 *   NMF_SOLVER_MU:   x_j <- x_j r_j / (x^T G)_j, all j from the old x;
 *                    x_j <- 0 where (x^T G)_j <= 0;
 *   NMF_SOLVER_HALS: for i = 0 .. k-1 in order,
 *                    x_i <- max(0, r_i - sum_{l != i} G_li x_l) / G_ii.
 * Indices with G_ii <= 1e-14 max_l G_ll are set to 0.  FP64 arithmetic, one
 * rounding to FP32 per entry (HALS divides by G_ii as a product with its
 * FP64 reciprocal, MU by (x^T G)_j as a product with a Newton-refined
 * reciprocal; partial sums in a fixed order of four).  Enqueued on
 * `stream`; X may not overlap R.  NMF_EINVAL for another solver, k outside
 * [1, 64], rows < 0, ldr or ldx < k, or a null pointer with rows > 0. */
int nmf_local_update(int solver, int k, int64_t rows, const double* G, const float* R, int64_t ldr, float* X,
                     int64_t ldx, void* stream);

/* ---- the data matrix ------------------------------------------------------- */
typedef struct nmf_matrix {
  int kind;                 /* NMF_DENSE or NMF_CSR */
  int64_t m, n;
  /* dense */
  const float* A;           /* m x n FP32, leading dimension lda (device) */
  int64_t lda;
  const void* A_bf16;       /* BF16X3 only: padded BF16 form of A   (nmf_split_bf16, transpose 0) */
  const void* At_bf16;      /* BF16X3 only: padded BF16 form of A^T (nmf_split_bf16, transpose 1) */
  const float* At;          /* FP32 only, optional: A^T (n x m, leading dimension ldat >= m, from
                               nmf_transpose_f32); when set, nmf_anls_iter forms the side-H
                               right-hand side A^T W as nmf_rhs_dense side W of A^T, whose
                               row-streaming kernel reads the resident copy */
  int64_t ldat;
  /* sparse */
  int64_t nnz;              /* number of stored entries (both CSR copies) */
  const int64_t* rowptr;    /* CSR(A):   m + 1 */
  const int32_t* colidx;
  const float* vals;
  const int64_t* rowptr_t;  /* CSR(A^T): n + 1 */
  const int32_t* colidx_t;
  const float* vals_t;
  /* ||A||_F^2 (device FP64 scalar, from nmf_fro2); needed by NMF_OBJ_TRACE and
   * by the per-iteration objective of nmf_anls_iter */
  const double* fro2;
} nmf_matrix;

/* ||A||_F^2 in FP64 into *out (device). */
int nmf_fro2_workspace_bytes(const nmf_matrix* A, size_t* bytes);
int nmf_fro2(const nmf_matrix* A, double* out, void* ws, size_t ws_bytes, void* stream);

/* ---- objective ----------------------------------------------------------------
 * r = ||A - W H||_F / ||A||_F (Eq. NMF), written to out[0] (device); out[1] =
 * ||A - W H||_F^2 and out[2] = ||A||_F^2.  W: m x k, Ht: n x k (FP32, ld k).
 * NMF_OBJ_DIRECT: dense A is read once and W H is formed tile by tile (FP32
 *   MFMA) with FP64 sums; CSR uses ||A||^2 - 2 sum_nnz a_ij (WH)_ij +
 *   <W^T W, H H^T> in FP64.  G_W, G_H, R_H are ignored (may be NULL).
 * NMF_OBJ_TRACE: uses A->fro2 and the FP64 Grams G_W = W^T W, G_H = H H^T
 *   and R_H = A^T W (n x k, ld k) of the current factors. */
int nmf_objective_workspace_bytes(const nmf_matrix* A, int k, int mode, size_t* bytes);
int nmf_objective(const nmf_matrix* A, int k, const float* W, const float* Ht, int mode,
                  const double* G_W, const double* G_H, const float* R_H, double* out, void* ws,
                  size_t ws_bytes, void* stream);

/* ---- the ANLS driver --------------------------------------------------------- */
typedef struct nmf_opts {
  int prec;             /* NMF_F32 or NMF_BF16X3 (dense only) */
  int warm;             /* NMF_WARM_COLD / NMF_WARM_PREV / NMF_WARM_LEARNED / NMF_WARM_ALL */
  int max_rounds;       /* BPP round cap (e.g. 100) */
  int warm_cap;         /* rounds a warm start gets before its cold restart */
  int trace_objective;  /* 1: record r after each half-step (TRACE, FP64) */
  int reset_masks;      /* 1: clear the stored passive sets before the first iteration */
  const float* net_w;   /* NMF_WARM_LEARNED: W-side network parameters (device) */
  const float* net_h;   /* NMF_WARM_LEARNED: H-side network parameters (device) */
  /* sample collection for training the network (optional, device buffers):
   * in every half-step the problems b with b % stride == 0 store their
   * features (2k FP32) and final passive set; the W-side samples of the
   * t-th iteration of this call go to positions
   * coll_off_w + t * ceil(m / collect_stride_w) + b / collect_stride_w
   * (H side likewise with n); positions >= the capacity are dropped. */
  int collect;
  int collect_stride_w;
  int collect_stride_h;
  float* coll_phi_w;
  uint64_t* coll_mask_w;
  int64_t coll_cap_w;
  int64_t coll_off_w;
  float* coll_phi_h;
  uint64_t* coll_mask_h;
  int64_t coll_cap_h;
  int64_t coll_off_h;
  /* optional phase timing: hipEvent_t handles (from nmf_events_create);
   * iteration t records events[2 * (t * NMF_PHASES + ph)] before phase ph and
   * the next entry after it; entries beyond phase_events_cap are skipped.
   * For the product phases the pair brackets the main product kernel only. */
  void** phase_events;
  int phase_events_cap;
  /* the local update of both half-steps: NMF_SOLVER_BPP (0, the default of a
   * zeroed struct), NMF_SOLVER_HALS or NMF_SOLVER_MU.  HALS and MU start from
   * the current W and Ht and need warm = NMF_WARM_COLD and collect = 0; the
   * BPP counters of nmf_iter_stats stay zero for them. */
  int solver;
} nmf_opts;

/* phases of one iteration, for nmf_opts.phase_events */
#define NMF_PH_RHS_W 0    /* A H^T (main kernel) */
#define NMF_PH_INFER_W 1  /* warm-start network, W side */
#define NMF_PH_BPP_W 2    /* NNLS for the rows of W */
#define NMF_PH_GRAM_W 3   /* W^T W */
#define NMF_PH_RHS_H 4    /* W^T A (main kernel) */
#define NMF_PH_INFER_H 5
#define NMF_PH_BPP_H 6
#define NMF_PH_GRAM_H 7   /* H H^T */
#define NMF_PH_OTHER 8    /* objective, statistics, sample collection */
#define NMF_PHASES 9

/* Host helpers for timing: create / destroy n hipEvent_t handles, and the
 * elapsed milliseconds between two recorded events (after they complete). */
int nmf_events_create(int n, void** events);
int nmf_events_destroy(int n, void** events);
int nmf_events_elapsed_ms(void* start, void* stop, float* ms);

/* Per-iteration statistics, written to a device array of `iters` entries. */
typedef struct nmf_iter_stats {
  double r_half;        /* relative objective after the W update (trace form) */
  double r_full;        /* relative objective after the H update (trace form) */
  uint64_t bpp_w[NMF_BPP_COUNTERS];  /* counters of the W half-step */
  uint64_t bpp_h[NMF_BPP_COUNTERS];  /* counters of the H half-step */
  uint64_t capped;      /* problems with NMF_BPP_CAPPED in this iteration */
  uint64_t fallback;    /* problems with NMF_BPP_WARM_FALLBACK */
} nmf_iter_stats;

/* Runs `iters` iterations of Algorithm 1 (W update, then H update) in place
 * on W (m x k) and Ht (n x k), FP32 device buffers with ld k.  The workspace
 * holds the Gram matrices, right-hand sides and the passive sets that carry
 * over between calls for NMF_WARM_PREV (keep ws alive and unchanged between
 * calls; set reset_masks on the first call).  stats: device array of `iters`
 * nmf_iter_stats (optional). */
int nmf_anls_workspace_bytes(const nmf_matrix* A, int k, const nmf_opts* o, size_t* bytes);
int nmf_anls_iter(const nmf_matrix* A, int k, float* W, float* Ht, int iters, const nmf_opts* o,
                  nmf_iter_stats* stats, void* ws, size_t ws_bytes, void* stream);

/* ---- many uneven instances: grouped persistent phases, graphs, tuning ------
 * Algorithm 1 run on a batch of independent dense NMF problems of different
 * m, n and k (each as nmf_anls_iter with NMF_BF16X3 right-hand sides, FP64
 * Gram matrices and FP64 BPP from cold starts).  Every phase of an iteration
 * is one persistent launch that walks a work list spanning all instances
 * (Gram tiles, Y splits, BF16x3 product tiles with split-K, split sums and
 * ranges of NNLS problems), so an iteration is a fixed sequence of launches
 * whatever the batch size, and a whole run can be captured as one graph.
 *
 * Problem i: A_i (m x n) is given by its padded BF16 planes in both
 * orientations (nmf_split_bf16 with transpose 0 and 1); W_i (m x k, ld ldw)
 * is overwritten; Ht_i (n x k, ld ldh) holds the initial H^T and receives
 * the result.  All pointers are device pointers owned by the caller. */
typedef struct nmf_batch_problem {
  int64_t m, n;
  int k, pad;
  const void* A_bf16;   /* nmf_split_bf16(m, n, A, lda, 0, ...) */
  const void* At_bf16;  /* nmf_split_bf16(m, n, A, lda, 1, ...) */
  float* W;
  int64_t ldw;
  float* Ht;
  int64_t ldh;
} nmf_batch_problem;

/* Work-item sizes and tile shapes of the grouped phases (what the autotuner
 * chooses). */
typedef struct nmf_batch_tune {
  int gram_tiles;    /* 64-row tiles per Gram work item (>= 1) */
  int rhs_w_chunks;  /* 64-column chunks of the contraction per A H^T item (>= 1; split-K) */
  int rhs_h_chunks;  /* 64-row chunks of the contraction per A^T W item (>= 1; split-K) */
  int bpp_problems;  /* NNLS problems per BPP item (>= 64) */
  int grid_scale;    /* persistent grid = grid_scale x resident workgroups (1..8) */
  int warm_prev;     /* 1: each NNLS starts from its own passive set of the previous
                      * iteration (kept in the workspace; cold after a reset, and a
                      * warm start still unsolved after 8 rounds restarts cold);
                      * the solutions are the same either way.  Not searched by the
                      * autotuner, which keeps the default (1). */
  int rhs_tile_rows; /* rows of R per product tile: 128 (four wavefronts) or 64 (two) */
  int bpp_wide;      /* 0: each instance's NNLS problems in the narrowest lane class
                      * that holds k (8, 16, 32, 56 or 64 lanes per problem); 1: the
                      * next wider class (more lanes per problem, fewer problems per
                      * wavefront).  Same solutions either way. */
} nmf_batch_tune;

#define NMF_BATCH_RESET 1  /* flag: clear the kept passive sets first (cold start) */

/* Fills a tuning that works everywhere (used when tune is NULL below). */
void nmf_batch_tune_default(nmf_batch_tune* t);

/* Workspace for a plan with tuning t; t == NULL gives a size that fits every
 * tuning nmf_batch_autotune tries (and the default). */
int nmf_batch_workspace_bytes(int count, const nmf_batch_problem* P, const nmf_batch_tune* t, size_t* bytes);

/* Lays out the per-instance buffers and builds the work lists in ws
 * (synchronous: the lists are copied to the device before it returns).  The
 * plan is a host object; ws and the problems' buffers must outlive it.
 * Errors: NMF_EINVAL (count < 1, a bad size or k, a null pointer),
 * NMF_EWORKSPACE, NMF_EHIP. */
int nmf_batch_plan_create(int count, const nmf_batch_problem* P, const nmf_batch_tune* t, void* ws,
                          size_t ws_bytes, void** plan);
int nmf_batch_plan_destroy(void* plan);

/* Enqueues `iters` iterations (W update then H update of every instance) on
 * stream; no host synchronisation and no allocation, so it may be captured.
 * flags: NMF_BATCH_RESET clears the kept passive sets first (with a fill
 * kernel).  counters: optional device array of 2 * NMF_BPP_COUNTERS uint64
 * (W side, then H side), added to (not cleared). */
int nmf_batch_iterate(void* plan, int iters, uint64_t* counters, int flags, void* stream);

/* Captures nmf_batch_iterate(plan, iters, counters, flags) on `stream` (a
 * non-null stream) into an executable graph; launch it any number of times
 * (with NMF_BATCH_RESET every launch starts cold). */
int nmf_batch_graph_create(void* plan, int iters, uint64_t* counters, int flags, void* stream, void** graph);
int nmf_batch_graph_launch(void* graph, void* stream);
int nmf_batch_graph_destroy(void* graph);

/* Chooses the work-item sizes, the product tile shape and the NNLS lane
 * classes by timing one iteration per candidate (coordinate search over each
 * field in turn, starting from the default).
 * The problems' W and Ht are saved to the workspace first and restored
 * afterwards, so the batch is left as it was.  ws must hold
 * nmf_batch_workspace_bytes(count, P, NULL).  best_ms: time of one iteration
 * with the chosen tuning (optional). */
int nmf_batch_autotune(int count, const nmf_batch_problem* P, void* ws, size_t ws_bytes, nmf_batch_tune* best,
                       double* best_ms, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LIBNMF_H */
