// Algorithm 1 (ANLS) on one GPU: for each iteration
//   G_H = H H^T (from Ht), R_W = A H^T, W = BPP(G_H, R_W)       (W update)
//   G_W = W^T W,           R_H = A^T W, Ht = BPP(G_W, R_H)      (H update)
// (or one HALS / MU update of W and Ht in place of BPP: nmf_opts.solver)
// with the optional trace-form objective after each half-step.  At p = 1 the
// collectives of Algorithm 3 vanish and these are exactly its local steps.
// Everything is enqueued on one stream; nothing synchronises with the host.
#include "nmf_common.h"

namespace nmf {
int trace_objective_launch(int64_t len, const float* a, const float* b, int k, const double* GW, const double* GH,
                           const double* fro2, double* partial, int nblocks, double* out, double* r_copy,
                           hipStream_t s);
int trace_finish_launch(int nblocks, const double* partial, int k, const double* GW, const double* GH,
                        const double* fro2, double* out, double* r_copy, hipStream_t s);
// warm-start network (mlp.hip)
int mlp_infer_plan(int k, int64_t batch, Carver& c, void** scratch);
int mlp_pack_launch(int k, const float* params, void* scratch, hipStream_t s);
int mlp_infer_launch(int k, int64_t batch, const double* G, const float* R, int64_t ldr, const float* params,
                     uint64_t* mask_out, void* scratch, hipStream_t s);
int features_launch(int k, int64_t batch, int64_t stride, const double* G, const float* R, int64_t ldr, float* phi,
                    hipStream_t s);
}  // namespace nmf

namespace {

__global__ void k_zero_u64(uint64_t* __restrict__ p, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = 0;
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, int64_t n, uint64_t v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

// NMF_WARM_ALL: every problem of the next BPP launch starts from the full set
int fill_full_sets(uint64_t* masks, int64_t n, int k, hipStream_t s) {
  const uint64_t full = k >= 64 ? ~0ull : ((1ull << k) - 1ull);
  int64_t blocks = nmf::cdiv(n, 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, s, masks, n, full);
  return nmf::launch_status("full start sets");
}

// Copies the sampled problems' final passive sets (b % stride == 0) to
// positions base + b / stride of the sample buffer.
__global__ void k_collect_masks(int64_t batch, int64_t stride, const uint64_t* __restrict__ masks,
                                uint64_t* __restrict__ out, int64_t cap, int64_t base) {
  const int64_t ns = (batch + stride - 1) / stride;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ns; e += (int64_t)gridDim.x * blockDim.x)
    if (base + e < cap) out[base + e] = masks[e * stride];
}

struct Plan {
  double* GH;
  double* GW;
  float* RW;
  float* RH;
  uint64_t* MW;
  uint64_t* MH;
  uint8_t* rounds;
  uint8_t* status;
  double* gpart;
  int gblocks;
  void* rhs_w;
  void* rhs_h;
  double* obj;
  double* dpart;
  int dblocks;
  double* bdot;  // per-block cross terms from the BPP kernel
  void* infer_w;
  void* infer_h;
};

int plan_anls(const nmf_matrix* A, int k, const nmf_opts* o, nmf::Carver& c, Plan* P) {
  const int64_t m = A->m, n = A->n, mx = m > n ? m : n;
  P->GH = c.take<double>((size_t)k * k);
  P->GW = c.take<double>((size_t)k * k);
  P->RW = c.take<float>((size_t)m * k);
  P->RH = c.take<float>((size_t)n * k);
  P->MW = c.take<uint64_t>((size_t)m);
  P->MH = c.take<uint64_t>((size_t)n);
  P->rounds = c.take<uint8_t>((size_t)mx);
  P->status = c.take<uint8_t>((size_t)mx);
  nmf::gram_plan(mx, k, c, &P->gpart, &P->gblocks);
  P->rhs_w = P->rhs_h = nullptr;
  if (A->kind == NMF_DENSE) {
    NMF_TRY(nmf::rhs_dense_plan(NMF_SIDE_W, m, n, k, o->prec, c, &P->rhs_w));
    if (o->prec == NMF_F32 && A->At)
      NMF_TRY(nmf::rhs_dense_plan(NMF_SIDE_W, n, m, k, o->prec, c, &P->rhs_h));  // A^T W as side W of A^T
    else
      NMF_TRY(nmf::rhs_dense_plan(NMF_SIDE_H, m, n, k, o->prec, c, &P->rhs_h));
  } else if (nmf::csr_pad_ld(k) != k) {
    // line-aligned copy of the SpMM's factor (Ht, then W: one after the other)
    P->rhs_w = P->rhs_h = c.take<float>((size_t)mx * nmf::csr_pad_ld(k));
  }
  P->obj = c.take<double>(4);
  nmf::dot_plan(mx * k, c, &P->dpart, &P->dblocks);
  {
    const int64_t bw = nmf::bpp_blocks(k, m), bh = nmf::bpp_blocks(k, n);
    P->bdot = c.take<double>((size_t)(bw > bh ? (bw > 1 ? bw : 1) : (bh > 1 ? bh : 1)));
  }
  P->infer_w = P->infer_h = nullptr;
  if (o->warm == NMF_WARM_LEARNED) {
    NMF_TRY(nmf::mlp_infer_plan(k, mx, c, &P->infer_w));
    NMF_TRY(nmf::mlp_infer_plan(k, mx, c, &P->infer_h));
  }
  return NMF_OK;
}

int check_opts(const nmf_matrix* A, const nmf_opts* o) {
  if (!o) return nmf::fail(NMF_EINVAL, "nmf_anls: opts is null");
  if (o->prec != NMF_F32 && o->prec != NMF_BF16X3) return nmf::fail(NMF_EINVAL, "nmf_anls: bad prec");
  if (o->prec == NMF_BF16X3 && A->kind != NMF_DENSE)
    return nmf::fail(NMF_EINVAL, "nmf_anls: BF16X3 needs a dense matrix");
  if (o->prec == NMF_BF16X3 && (!A->A_bf16 || !A->At_bf16))
    return nmf::fail(NMF_EINVAL, "nmf_anls: BF16X3 needs the tiled BF16 forms of A and A^T");
  if (o->warm < NMF_WARM_COLD || o->warm > NMF_WARM_ALL) return nmf::fail(NMF_EINVAL, "nmf_anls: bad warm mode");
  if (o->warm == NMF_WARM_LEARNED && (!o->net_w || !o->net_h))
    return nmf::fail(NMF_EINVAL, "nmf_anls: learned warm start needs both networks");
  if (o->max_rounds < 1 || o->warm_cap < 1) return nmf::fail(NMF_EINVAL, "nmf_anls: max_rounds/warm_cap < 1");
  if (o->solver != NMF_SOLVER_BPP && o->solver != NMF_SOLVER_HALS && o->solver != NMF_SOLVER_MU)
    return nmf::fail(NMF_EINVAL, "nmf_anls: bad solver");
  if (o->solver != NMF_SOLVER_BPP && (o->warm != NMF_WARM_COLD || o->collect))
    return nmf::fail(NMF_EINVAL, "nmf_anls: HALS and MU take no warm start and collect no samples");
  if (o->collect) {
    if (o->collect_stride_w < 1 || o->collect_stride_h < 1 || !o->coll_phi_w || !o->coll_mask_w ||
        !o->coll_phi_h || !o->coll_mask_h || o->coll_off_w < 0 || o->coll_off_h < 0)
      return nmf::fail(NMF_EINVAL, "nmf_anls: sample collection needs strides, offsets and buffers");
  }
  return NMF_OK;
}

int check_matrix(const nmf_matrix* A) {
  if (!A) return nmf::fail(NMF_EINVAL, "nmf_anls: matrix is null");
  if (A->m < 1 || A->n < 1) return nmf::fail(NMF_EINVAL, "nmf_anls: empty matrix");
  if (A->kind == NMF_DENSE) {
    if (A->lda < A->n || !A->A) return nmf::fail(NMF_EINVAL, "nmf_anls: bad dense matrix");
    if (A->At && A->ldat < A->m) return nmf::fail(NMF_EINVAL, "nmf_anls: ldat < m");
  } else if (A->kind == NMF_CSR) {
    if (!A->rowptr || !A->colidx || !A->vals || !A->rowptr_t || !A->colidx_t || !A->vals_t)
      return nmf::fail(NMF_EINVAL, "nmf_anls: CSR(A) and CSR(A^T) are both needed");
  } else {
    return nmf::fail(NMF_EINVAL, "nmf_anls: bad matrix kind");
  }
  return NMF_OK;
}

int rhs(const nmf_matrix* A, int side, int k, int prec, const float* Y, float* R, void* scratch, hipStream_t s,
        bool y_ready = false) {
  if (A->kind == NMF_CSR) {
    float* ypad = static_cast<float*>(scratch);
    if (side == NMF_SIDE_W)
      return nmf::rhs_csr_launch(A->m, A->n, k, A->rowptr, A->colidx, A->vals, Y, k, R, k, ypad, s);
    return nmf::rhs_csr_launch(A->n, A->m, k, A->rowptr_t, A->colidx_t, A->vals_t, Y, k, R, k, ypad, s);
  }
  if (side == NMF_SIDE_H && prec == NMF_F32 && A->At)  // the resident A^T: A^T W streams its rows
    return nmf::rhs_dense_launch(NMF_SIDE_W, A->n, A->m, k, A->At, A->ldat, nullptr, Y, k, R, k, prec, scratch, s);
  const void* bt = side == NMF_SIDE_W ? A->A_bf16 : A->At_bf16;
  return nmf::rhs_dense_launch(side, A->m, A->n, k, A->A, A->lda, bt, Y, k, R, k, prec, scratch, s, y_ready);
}

int collect(int k, int64_t batch, int64_t stride, const double* G, const float* R, const uint64_t* masks,
            float* phi, uint64_t* mout, int64_t cap, int64_t* host_count, hipStream_t s) {
  const int64_t ns = nmf::cdiv(batch, stride);
  const int64_t base = *host_count;
  if (base >= cap) return NMF_OK;
  const int64_t take = (base + ns <= cap) ? ns : cap - base;
  // features of sampled rows (b % stride == 0) straight into the sample buffer
  NMF_TRY(nmf::features_launch(k, (take - 1) * stride + 1, stride, G, R, k, phi + base * 2 * k, s));
  int64_t blocks = nmf::cdiv(take, 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_collect_masks, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, s,
                     (take - 1) * stride + 1, stride, masks, mout, cap, base);
  NMF_TRY(nmf::launch_status("collect masks"));
  *host_count = base + ns;
  return NMF_OK;
}

}  // namespace

extern "C" int nmf_anls_workspace_bytes(const nmf_matrix* A, int k, const nmf_opts* o, size_t* bytes) {
  if (!bytes) return nmf::fail(NMF_EINVAL, "nmf_anls_workspace_bytes: bytes is null");
  NMF_TRY(check_matrix(A));
  if (!nmf::valid_k(k)) return nmf::fail(NMF_EINVAL, "nmf_anls_workspace_bytes: k=%d outside [1,64]", k);
  NMF_TRY(check_opts(A, o));
  nmf::Carver c(nullptr, 0);
  Plan P;
  NMF_TRY(plan_anls(A, k, o, c, &P));
  *bytes = c.off;
  return NMF_OK;
}

extern "C" int nmf_anls_iter(const nmf_matrix* A, int k, float* W, float* Ht, int iters, const nmf_opts* o,
                             nmf_iter_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  NMF_TRY(check_matrix(A));
  if (!nmf::valid_k(k)) return nmf::fail(NMF_EINVAL, "nmf_anls_iter: k=%d outside [1,64]", k);
  if (!W || !Ht || iters < 0) return nmf::fail(NMF_EINVAL, "nmf_anls_iter: bad factors or iters");
  NMF_TRY(check_opts(A, o));
  if (o->trace_objective && !A->fro2) return nmf::fail(NMF_EINVAL, "nmf_anls_iter: trace objective needs A->fro2");
  nmf::Carver c(ws, ws_bytes);
  Plan P;
  NMF_TRY(plan_anls(A, k, o, c, &P));
  if (!ws || !c.fits()) return nmf::fail(NMF_EWORKSPACE, "nmf_anls_iter: workspace %zu < %zu bytes", ws_bytes, c.off);
  hipStream_t s = nmf::as_stream(stream);
  const int64_t m = A->m, n = A->n;

  if (o->reset_masks) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1024), dim3(256), 0, s, P.MW, m);
    hipLaunchKernelGGL(k_zero_u64, dim3(1024), dim3(256), 0, s, P.MH, n);
    NMF_TRY(nmf::launch_status("reset masks"));
  }
  // every half-step appends ceil(batch / stride) samples, so the positions
  // are known on the host
  int64_t hc[2] = {o->collect ? o->coll_off_w : 0, o->collect ? o->coll_off_h : 0};

  if (stats && iters > 0) {  // every iteration's record starts from zero
    const int64_t words = (int64_t)iters * (int64_t)(sizeof(nmf_iter_stats) / sizeof(uint64_t));
    const int64_t blocks = nmf::cdiv(words, 256);
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)(blocks > 1024 ? 1024 : blocks)), dim3(256), 0, s,
                       reinterpret_cast<uint64_t*>(stats), words);
    NMF_TRY(nmf::launch_status("zero stats"));
  }
  NMF_TRY(nmf::gram_launch(n, k, Ht, k, P.GH, P.gpart, P.gblocks, s));
  if (o->warm == NMF_WARM_LEARNED) {
    NMF_TRY(nmf::mlp_pack_launch(k, o->net_w, P.infer_w, s));
    NMF_TRY(nmf::mlp_pack_launch(k, o->net_h, P.infer_h, s));
  }
  const bool warm = o->warm != NMF_WARM_COLD;
  auto ev = [&](int t, int ph, int which) -> hipEvent_t {
    const int64_t idx = 2 * ((int64_t)t * NMF_PHASES + ph) + which;
    return (o->phase_events && idx < o->phase_events_cap) ? static_cast<hipEvent_t>(o->phase_events[idx]) : nullptr;
  };
  auto rec = [&](hipEvent_t e) {
    if (e) hipEventRecord(e, s);
  };
  struct MarkScope {  // brackets the main product kernel with the given events
    MarkScope(hipEvent_t a, hipEvent_t b) { nmf::kernel_mark() = {a, b}; }
    ~MarkScope() { nmf::kernel_mark() = {}; }
  };
  for (int t = 0; t < iters; ++t) {
    nmf_iter_stats* st = stats ? stats + t : nullptr;
    // ---- W update: W = argmin ||A - W H||, from H H^T and A H^T
    {
      MarkScope mark(ev(t, NMF_PH_RHS_W, 0), ev(t, NMF_PH_RHS_W, 1));
      NMF_TRY(rhs(A, NMF_SIDE_W, k, o->prec, Ht, P.RW, P.rhs_w, s));
    }
    rec(ev(t, NMF_PH_INFER_W, 0));
    if (o->warm == NMF_WARM_LEARNED)
      NMF_TRY(nmf::mlp_infer_launch(k, m, P.GH, P.RW, k, o->net_w, P.MW, P.infer_w, s));
    if (o->warm == NMF_WARM_ALL) NMF_TRY(fill_full_sets(P.MW, m, k, s));
    rec(ev(t, NMF_PH_INFER_W, 1));
    rec(ev(t, NMF_PH_BPP_W, 0));
    // with BPP the cross term <R_W, W> of the trace objective and the status
    // counts come out of the solve itself
    const bool bpp = o->solver == NMF_SOLVER_BPP;
    const bool trace = st && o->trace_objective;
    if (bpp) {
      NMF_TRY(nmf::bpp_launch(k, m, P.GH, P.RW, k, W, k, warm ? P.MW : nullptr, P.MW, nullptr, P.status,
                              o->max_rounds, o->warm_cap, st ? st->bpp_w : nullptr, s, trace ? P.bdot : nullptr,
                              st ? &st->capped : nullptr));
    } else {
      NMF_TRY(nmf::local_update_launch(o->solver, k, m, P.GH, P.RW, k, W, k, s));
    }
    rec(ev(t, NMF_PH_BPP_W, 1));
    if (o->collect)
      NMF_TRY(collect(k, m, o->collect_stride_w, P.GH, P.RW, P.MW, o->coll_phi_w, o->coll_mask_w, o->coll_cap_w,
                      &hc[0], s));
    // BF16x3: the Gram pass over W also writes W's transposed split, the Y
    // planes of the W^T A product that follows
    const bool split_in_gram = A->kind == NMF_DENSE && o->prec == NMF_BF16X3;
    uint16_t *yth = nullptr, *ytl = nullptr;
    int64_t ldt = 0;
    int KP = 0;
    if (split_in_gram) nmf::bf16x3_y_planes(NMF_SIDE_H, m, n, k, P.rhs_h, &yth, &ytl, &ldt, &KP);
    rec(ev(t, NMF_PH_GRAM_W, 0));
    NMF_TRY(nmf::gram_launch(m, k, W, k, P.GW, P.gpart, P.gblocks, s, yth, ytl, ldt, KP));
    rec(ev(t, NMF_PH_GRAM_W, 1));
    if (trace && bpp) {
      NMF_TRY(nmf::trace_finish_launch((int)nmf::bpp_blocks(k, m), P.bdot, k, P.GW, P.GH, A->fro2, P.obj,
                                       &st->r_half, s));
    } else if (trace) {
      NMF_TRY(nmf::trace_objective_launch(m * k, P.RW, W, k, P.GW, P.GH, A->fro2, P.dpart, P.dblocks, P.obj,
                                          &st->r_half, s));
    }
    // ---- H update: H = argmin ||A - W H||, from W^T W and W^T A
    {
      MarkScope mark(ev(t, NMF_PH_RHS_H, 0), ev(t, NMF_PH_RHS_H, 1));
      NMF_TRY(rhs(A, NMF_SIDE_H, k, o->prec, W, P.RH, P.rhs_h, s, split_in_gram));
    }
    rec(ev(t, NMF_PH_INFER_H, 0));
    if (o->warm == NMF_WARM_LEARNED)
      NMF_TRY(nmf::mlp_infer_launch(k, n, P.GW, P.RH, k, o->net_h, P.MH, P.infer_h, s));
    if (o->warm == NMF_WARM_ALL) NMF_TRY(fill_full_sets(P.MH, n, k, s));
    rec(ev(t, NMF_PH_INFER_H, 1));
    rec(ev(t, NMF_PH_BPP_H, 0));
    if (bpp) {
      NMF_TRY(nmf::bpp_launch(k, n, P.GW, P.RH, k, Ht, k, warm ? P.MH : nullptr, P.MH, nullptr, P.status,
                              o->max_rounds, o->warm_cap, st ? st->bpp_h : nullptr, s, trace ? P.bdot : nullptr,
                              st ? &st->capped : nullptr));
    } else {
      NMF_TRY(nmf::local_update_launch(o->solver, k, n, P.GW, P.RH, k, Ht, k, s));
    }
    rec(ev(t, NMF_PH_BPP_H, 1));
    if (o->collect)
      NMF_TRY(collect(k, n, o->collect_stride_h, P.GW, P.RH, P.MH, o->coll_phi_h, o->coll_mask_h, o->coll_cap_h,
                      &hc[1], s));
    rec(ev(t, NMF_PH_GRAM_H, 0));
    NMF_TRY(nmf::gram_launch(n, k, Ht, k, P.GH, P.gpart, P.gblocks, s));
    rec(ev(t, NMF_PH_GRAM_H, 1));
    rec(ev(t, NMF_PH_OTHER, 0));
    if (trace && bpp) {
      NMF_TRY(nmf::trace_finish_launch((int)nmf::bpp_blocks(k, n), P.bdot, k, P.GW, P.GH, A->fro2, P.obj,
                                       &st->r_full, s));
    } else if (trace) {
      NMF_TRY(nmf::trace_objective_launch(n * k, P.RH, Ht, k, P.GW, P.GH, A->fro2, P.dpart, P.dblocks, P.obj,
                                          &st->r_full, s));
    }
    rec(ev(t, NMF_PH_OTHER, 1));
  }
  return nmf::launch_status("nmf_anls_iter");
}
