// Many uneven NMF instances at once: Algorithm 1 for every instance of a
// batch, each phase of an iteration as one persistent launch over a work
// list that spans all instances, a graph of whole runs, and an autotuner for
// the work-item sizes, the product tile shape and the NNLS lane classes.
//
// An iteration is the fixed launch sequence
//   Gram H H^T (tiles, then per-instance sums)      -> G_H
//   split H^T into BF16 planes, A H^T (BF16x3 tiles, split-K sums) -> R_W
//   BPP for every row of every W, per K class       -> W
//   Gram W^T W, split W, A^T W, BPP for every column of every H -> Ht
// i.e. the local steps of Algorithm 1 / Algorithm 3 at p = 1 for each
// instance; the instances never interact.  Work items carry their own
// instance's pointers, so the kernels need no per-instance launches.
#include <vector>

#include "batched.h"
#include "nmf_common.h"

namespace {

using nmf::BppItem;
using nmf::Bf16Item;
using nmf::Carver;
using nmf::GramItem;
using nmf::GramReduceItem;
using nmf::SplitReduceItem;
using nmf::SplitYItem;

constexpr int kTR = 128;  // row padding of the BF16 planes and rows per product tile
constexpr int kTC = 64;   // column padding / contraction chunk
constexpr int kGramRows = 64;
constexpr int kClasses = 5;
constexpr int kClassK[kClasses] = {8, 16, 32, 56, 64};
constexpr int kNoSplit = 1 << 30;

int class_index(int K) {
  for (int c = 0; c < kClasses; ++c)
    if (kClassK[c] == K) return c;
  return kClasses - 1;
}

// candidate values searched by the autotuner (the first of each is the finest)
const int kCandGram[] = {2, 8, 32};
const int kCandRhsW[] = {8, 32, kNoSplit};
const int kCandRhsH[] = {8, 32, 128};
const int kCandBpp[] = {128, 256, 1024};
const int kCandGrid[] = {1, 2};
const int kCandTile[] = {64, 128};
const int kCandWide[] = {0, 1};

nmf_batch_tune finest_tune() {
  nmf_batch_tune t;
  t.gram_tiles = kCandGram[0];
  t.rhs_w_chunks = kCandRhsW[0];
  t.rhs_h_chunks = kCandRhsH[0];
  t.bpp_problems = kCandBpp[0];
  t.grid_scale = 1;
  t.warm_prev = 1;
  t.rhs_tile_rows = kCandTile[0];
  t.bpp_wide = 0;
  return t;
}

bool tune_ok(const nmf_batch_tune& t) {
  return t.gram_tiles >= 1 && t.rhs_w_chunks >= 1 && t.rhs_h_chunks >= 1 && t.bpp_problems >= 64 &&
         t.grid_scale >= 1 && t.grid_scale <= 8 && (t.warm_prev == 0 || t.warm_prev == 1) &&
         (t.rhs_tile_rows == 64 || t.rhs_tile_rows == 128) && (t.bpp_wide == 0 || t.bpp_wide == 1);
}

// NNLS lane class of an instance of rank k under tuning t
int lane_class(int k, const nmf_batch_tune& t) {
  const int K = nmf::bpp_class(k);
  if (!t.bpp_wide) return K;
  const int ci = class_index(K);
  return kClassK[ci + 1 < kClasses ? ci + 1 : ci];
}

template <class T>
struct List {
  std::vector<T> host;
  T* dev = nullptr;
  int64_t n() const { return (int64_t)host.size(); }
};

struct Plan {
  int count = 0;
  nmf_batch_tune tune{};
  List<GramItem> gh, gw;
  List<GramReduceItem> ghr, gwr;
  List<SplitYItem> syw, syh;
  List<Bf16Item> rw[2], rh[2];
  List<SplitReduceItem> srw, srh;
  List<BppItem> bw[kClasses], bh[kClasses];
  int grid_gram = 0, grid_reduce = 0, grid_split = 0, grid_bf16[2] = {0, 0}, grid_bpp[kClasses] = {0, 0, 0, 0, 0};
  int max_rounds = 200;
  int warm_cap = 8;
  uint64_t* masks = nullptr;  // kept passive sets (warm_prev), all problems
  int64_t nmasks = 0;
};

__global__ void k_zero_masks(uint64_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Everything the plan places in the workspace.  The backup of the factors
// (used only by the autotuner) comes first so that it has the same address
// under every tuning.
int layout(int count, const nmf_batch_problem* P, const nmf_batch_tune& t, Carver& c, Plan* plan) {
  int64_t nprob = 0;
  for (int i = 0; i < count; ++i) {
    c.take<float>((size_t)P[i].m * P[i].k);  // W backup
    c.take<float>((size_t)P[i].n * P[i].k);  // Ht backup
    nprob += P[i].m + P[i].n;
  }
  uint64_t* masks = t.warm_prev ? c.take<uint64_t>((size_t)nprob) : nullptr;
  if (plan) {
    plan->masks = masks;
    plan->nmasks = t.warm_prev ? nprob : 0;
  }
  int64_t moff = 0;
  for (int i = 0; i < count; ++i) {
    const nmf_batch_problem& p = P[i];
    const int64_t m = p.m, n = p.n;
    const int k = p.k;
    const int NT = k <= 32 ? 1 : 2;
    const int KP = 32 * NT;
    const int K = lane_class(k, t);
    const int ci = class_index(K);
    double* GH = c.take<double>((size_t)k * k);
    double* GW = c.take<double>((size_t)k * k);
    float* RW = c.take<float>((size_t)m * k);
    float* RH = c.take<float>((size_t)n * k);
    uint8_t* stw = c.take<uint8_t>((size_t)m);
    uint8_t* sth = c.take<uint8_t>((size_t)n);
    // BF16 planes of Y for the two products
    const int64_t nkc_w = nmf::cdiv(n, kTC), ldt_w = nkc_w * kTC;  // side W: Y = Ht, K = n
    const int64_t nkc_h = nmf::cdiv(m, kTC), ldt_h = nkc_h * kTC;  // side H: Y = W,  K = m
    uint16_t* yw = c.take<uint16_t>((size_t)2 * KP * ldt_w);
    uint16_t* yh = c.take<uint16_t>((size_t)2 * KP * ldt_h);
    // split-K partials
    const int64_t cw = t.rhs_w_chunks < nkc_w ? t.rhs_w_chunks : nkc_w;
    const int64_t ch = t.rhs_h_chunks < nkc_h ? t.rhs_h_chunks : nkc_h;
    const int64_t Sw = nmf::cdiv(nkc_w, cw), Sh = nmf::cdiv(nkc_h, ch);
    float* pw = Sw > 1 ? c.take<float>((size_t)Sw * m * k) : nullptr;
    float* ph = Sh > 1 ? c.take<float>((size_t)Sh * n * k) : nullptr;
    // Gram partial slots
    const int64_t tiles_h = nmf::cdiv(n, kGramRows), tiles_w = nmf::cdiv(m, kGramRows);
    const int64_t slots_h = nmf::cdiv(tiles_h, t.gram_tiles), slots_w = nmf::cdiv(tiles_w, t.gram_tiles);
    double* gph = c.take<double>((size_t)slots_h * k * k);
    double* gpw = c.take<double>((size_t)slots_w * k * k);
    uint64_t* mw = masks ? masks + moff : nullptr;
    uint64_t* mh = masks ? masks + moff + m : nullptr;
    moff += m + n;
    if (!plan) continue;

    // Gram items and their sums
    for (int64_t s = 0; s < slots_h; ++s) {
      const int64_t t0 = s * t.gram_tiles;
      const int64_t nt = (t0 + t.gram_tiles < tiles_h ? t0 + t.gram_tiles : tiles_h) - t0;
      plan->gh.host.push_back(GramItem{p.Ht, p.ldh, n, k, 0, t0, nt, gph ? gph + s * k * k : nullptr});
    }
    for (int64_t s = 0; s < slots_w; ++s) {
      const int64_t t0 = s * t.gram_tiles;
      const int64_t nt = (t0 + t.gram_tiles < tiles_w ? t0 + t.gram_tiles : tiles_w) - t0;
      plan->gw.host.push_back(GramItem{p.W, p.ldw, m, k, 0, t0, nt, gpw ? gpw + s * k * k : nullptr});
    }
    for (int64_t e0 = 0; e0 < (int64_t)k * k; e0 += 256) {
      plan->ghr.host.push_back(GramReduceItem{gph, GH, k, (int)slots_h, e0});
      plan->gwr.host.push_back(GramReduceItem{gpw, GW, k, (int)slots_w, e0});
    }
    // splits of Y
    for (int64_t K0 = 0; K0 < ldt_w; K0 += 64)
      plan->syw.host.push_back(SplitYItem{p.Ht, p.ldh, n, k, KP, yw, yw ? yw + (size_t)KP * ldt_w : nullptr, ldt_w, K0});
    for (int64_t K0 = 0; K0 < ldt_h; K0 += 64)
      plan->syh.host.push_back(SplitYItem{p.W, p.ldw, m, k, KP, yh, yh ? yh + (size_t)KP * ldt_h : nullptr, ldt_h, K0});
    // product tiles (A H^T: B = A planes, rows m; A^T W: B = A^T planes, rows n)
    const uint16_t* Ab = static_cast<const uint16_t*>(p.A_bf16);
    const uint16_t* Atb = static_cast<const uint16_t*>(p.At_bf16);
    const int64_t Rp_w = nmf::cdiv(m, kTR) * kTR, Rp_h = nmf::cdiv(n, kTR) * kTR;
    const int TR = t.rhs_tile_rows;
    for (int64_t s = 0; s < Sw; ++s)
      for (int64_t r0 = 0; r0 < m; r0 += TR) {
        const int64_t kc0 = s * cw, kc1 = (kc0 + cw < nkc_w ? kc0 + cw : nkc_w);
        float* out = Sw > 1 ? (pw ? pw + s * m * k : nullptr) : RW;
        plan->rw[NT - 1].host.push_back(Bf16Item{Ab, Rp_w, nkc_w, yw, yw ? yw + (size_t)KP * ldt_w : nullptr, ldt_w,
                                                 out, k, m, k, 0, r0, kc0, kc1});
      }
    for (int64_t s = 0; s < Sh; ++s)
      for (int64_t r0 = 0; r0 < n; r0 += TR) {
        const int64_t kc0 = s * ch, kc1 = (kc0 + ch < nkc_h ? kc0 + ch : nkc_h);
        float* out = Sh > 1 ? (ph ? ph + s * n * k : nullptr) : RH;
        plan->rh[NT - 1].host.push_back(Bf16Item{Atb, Rp_h, nkc_h, yh, yh ? yh + (size_t)KP * ldt_h : nullptr, ldt_h,
                                                 out, k, n, k, 0, r0, kc0, kc1});
      }
    if (Sw > 1)
      for (int64_t e0 = 0; e0 < m * k; e0 += 256)
        plan->srw.host.push_back(SplitReduceItem{pw, m * k, RW, k, m, k, (int)Sw, e0});
    if (Sh > 1)
      for (int64_t e0 = 0; e0 < n * k; e0 += 256)
        plan->srh.host.push_back(SplitReduceItem{ph, n * k, RH, k, n, k, (int)Sh, e0});
    // NNLS ranges
    for (int64_t b0 = 0; b0 < m; b0 += t.bpp_problems)
      plan->bw[ci].host.push_back(BppItem{GH, RW, k, p.W, p.ldw, stw, mw, k, 0, b0,
                                          b0 + t.bpp_problems < m ? b0 + t.bpp_problems : m});
    for (int64_t b0 = 0; b0 < n; b0 += t.bpp_problems)
      plan->bh[ci].host.push_back(BppItem{GW, RH, k, p.Ht, p.ldh, sth, mh, k, 0, b0,
                                          b0 + t.bpp_problems < n ? b0 + t.bpp_problems : n});
  }
  return NMF_OK;
}

// Item arrays are counted on a measuring pass (no plan), then carved.
struct Counts {
  int64_t gh = 0, gw = 0, ghr = 0, gwr = 0, syw = 0, syh = 0, rw[2] = {0, 0}, rh[2] = {0, 0}, srw = 0, srh = 0,
          bw[kClasses] = {0, 0, 0, 0, 0}, bh[kClasses] = {0, 0, 0, 0, 0};
};

Counts count_items(int count, const nmf_batch_problem* P, const nmf_batch_tune& t) {
  Plan tmp;
  Carver c(nullptr, 0);
  layout(count, P, t, c, &tmp);
  Counts n;
  n.gh = tmp.gh.n(); n.gw = tmp.gw.n(); n.ghr = tmp.ghr.n(); n.gwr = tmp.gwr.n();
  n.syw = tmp.syw.n(); n.syh = tmp.syh.n(); n.srw = tmp.srw.n(); n.srh = tmp.srh.n();
  for (int q = 0; q < 2; ++q) { n.rw[q] = tmp.rw[q].n(); n.rh[q] = tmp.rh[q].n(); }
  for (int q = 0; q < kClasses; ++q) { n.bw[q] = tmp.bw[q].n(); n.bh[q] = tmp.bh[q].n(); }
  return n;
}

template <class T>
void carve_list(Carver& c, List<T>& l, int64_t n) {
  l.dev = c.take<T>((size_t)(n > 0 ? n : 1));
}

size_t bytes_for(int count, const nmf_batch_problem* P, const nmf_batch_tune& t) {
  Carver c(nullptr, 0);
  layout(count, P, t, c, nullptr);
  const Counts n = count_items(count, P, t);
  Plan dummy;
  carve_list(c, dummy.gh, n.gh); carve_list(c, dummy.gw, n.gw);
  carve_list(c, dummy.ghr, n.ghr); carve_list(c, dummy.gwr, n.gwr);
  carve_list(c, dummy.syw, n.syw); carve_list(c, dummy.syh, n.syh);
  for (int q = 0; q < 2; ++q) { carve_list(c, dummy.rw[q], n.rw[q]); carve_list(c, dummy.rh[q], n.rh[q]); }
  carve_list(c, dummy.srw, n.srw); carve_list(c, dummy.srh, n.srh);
  for (int q = 0; q < kClasses; ++q) { carve_list(c, dummy.bw[q], n.bw[q]); carve_list(c, dummy.bh[q], n.bh[q]); }
  return c.off;
}

int validate(int count, const nmf_batch_problem* P) {
  if (count < 1 || !P) return nmf::fail(NMF_EINVAL, "nmf_batch: count=%d", count);
  for (int i = 0; i < count; ++i) {
    const nmf_batch_problem& p = P[i];
    if (p.m < 1 || p.n < 1 || !nmf::valid_k(p.k) || p.ldw < p.k || p.ldh < p.k)
      return nmf::fail(NMF_EINVAL, "nmf_batch: problem %d has bad sizes (m=%lld n=%lld k=%d)", i, (long long)p.m,
                       (long long)p.n, p.k);
    if (!p.A_bf16 || !p.At_bf16 || !p.W || !p.Ht) return nmf::fail(NMF_EINVAL, "nmf_batch: problem %d null pointer", i);
  }
  return NMF_OK;
}

// Resident workgroups of a grouped kernel on the current device.
int capacity(int per_cu_rc, int per_cu) {
  int dev = 0, cus = 0;
  if (per_cu_rc != NMF_OK || per_cu <= 0 || hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
    (void)hipGetLastError();
    return 1024;
  }
  return per_cu * cus;
}

int grid_for(int cap, int scale, int64_t items) {
  int64_t g = (int64_t)cap * scale;
  if (g > items) g = items;
  return (int)(g < 1 ? 1 : g);
}

template <class T>
int upload(List<T>& l, hipStream_t s) {
  if (l.host.empty()) return NMF_OK;
  if (hipMemcpyAsync(l.dev, l.host.data(), l.host.size() * sizeof(T), hipMemcpyHostToDevice, s) != hipSuccess)
    return nmf::fail(NMF_EHIP, "nmf_batch_plan_create: uploading work lists failed");
  return NMF_OK;
}

int plan_build(int count, const nmf_batch_problem* P, const nmf_batch_tune& t, void* ws, size_t ws_bytes,
               Plan* plan, hipStream_t s) {
  plan->count = count;
  plan->tune = t;
  Carver c(ws, ws_bytes);
  layout(count, P, t, c, plan);
  carve_list(c, plan->gh, plan->gh.n()); carve_list(c, plan->gw, plan->gw.n());
  carve_list(c, plan->ghr, plan->ghr.n()); carve_list(c, plan->gwr, plan->gwr.n());
  carve_list(c, plan->syw, plan->syw.n()); carve_list(c, plan->syh, plan->syh.n());
  for (int q = 0; q < 2; ++q) { carve_list(c, plan->rw[q], plan->rw[q].n()); carve_list(c, plan->rh[q], plan->rh[q].n()); }
  carve_list(c, plan->srw, plan->srw.n()); carve_list(c, plan->srh, plan->srh.n());
  for (int q = 0; q < kClasses; ++q) { carve_list(c, plan->bw[q], plan->bw[q].n()); carve_list(c, plan->bh[q], plan->bh[q].n()); }
  if (!ws || !c.fits()) return nmf::fail(NMF_EWORKSPACE, "nmf_batch_plan_create: workspace %zu < %zu bytes", ws_bytes, c.off);

  NMF_TRY(upload(plan->gh, s)); NMF_TRY(upload(plan->gw, s));
  NMF_TRY(upload(plan->ghr, s)); NMF_TRY(upload(plan->gwr, s));
  NMF_TRY(upload(plan->syw, s)); NMF_TRY(upload(plan->syh, s));
  for (int q = 0; q < 2; ++q) { NMF_TRY(upload(plan->rw[q], s)); NMF_TRY(upload(plan->rh[q], s)); }
  NMF_TRY(upload(plan->srw, s)); NMF_TRY(upload(plan->srh, s));
  for (int q = 0; q < kClasses; ++q) { NMF_TRY(upload(plan->bw[q], s)); NMF_TRY(upload(plan->bh[q], s)); }
  if (hipStreamSynchronize(s) != hipSuccess) return nmf::fail(NMF_EHIP, "nmf_batch_plan_create: synchronize failed");

  int pc = 0;
  int rc = nmf::gram_grouped_occupancy(nmf::kCapGram, &pc);
  plan->grid_gram = capacity(rc, pc) * t.grid_scale;
  rc = nmf::bf16_grouped_occupancy(nmf::kCapReduce, &pc);
  plan->grid_reduce = capacity(rc, pc) * t.grid_scale;
  rc = nmf::bf16_grouped_occupancy(nmf::kCapSplitY, &pc);
  plan->grid_split = capacity(rc, pc) * t.grid_scale;
  const bool t64 = t.rhs_tile_rows == 64;
  rc = nmf::bf16_grouped_occupancy(t64 ? nmf::kCapBf16NT1T64 : nmf::kCapBf16NT1, &pc);
  plan->grid_bf16[0] = capacity(rc, pc) * t.grid_scale;
  rc = nmf::bf16_grouped_occupancy(t64 ? nmf::kCapBf16NT2T64 : nmf::kCapBf16NT2, &pc);
  plan->grid_bf16[1] = capacity(rc, pc) * t.grid_scale;
  for (int q = 0; q < kClasses; ++q) {
    rc = nmf::bpp_grouped_occupancy(kClassK[q], &pc);
    plan->grid_bpp[q] = capacity(rc, pc) * t.grid_scale;
  }
  return NMF_OK;
}

int enqueue(const Plan& p, int iters, uint64_t* counters, int flags, hipStream_t s) {
  uint64_t* cw = counters;
  uint64_t* ch = counters ? counters + NMF_BPP_COUNTERS : nullptr;
  if ((flags & NMF_BATCH_RESET) && p.masks && p.nmasks > 0) {
    int64_t blocks = nmf::cdiv(p.nmasks, 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero_masks, dim3((unsigned)blocks), dim3(256), 0, s, p.masks, p.nmasks);
    NMF_TRY(nmf::launch_status("nmf_batch: clearing passive sets"));
  }
  for (int it = 0; it < iters; ++it) {
    // W update: G_H, R_W = A H^T, BPP
    NMF_TRY(nmf::gram_grouped_launch(p.gh.dev, p.gh.n(), grid_for(p.grid_gram, 1, p.gh.n()), s));
    NMF_TRY(nmf::gram_reduce_grouped_launch(p.ghr.dev, p.ghr.n(), grid_for(p.grid_reduce, 1, p.ghr.n()), s));
    NMF_TRY(nmf::split_y_grouped_launch(p.syw.dev, p.syw.n(), grid_for(p.grid_split, 1, p.syw.n()), s));
    for (int q = 0; q < 2; ++q)
      NMF_TRY(nmf::bf16x3_grouped_launch(q + 1, p.tune.rhs_tile_rows, p.rw[q].dev, p.rw[q].n(),
                                         grid_for(p.grid_bf16[q], 1, p.rw[q].n()), s));
    NMF_TRY(nmf::split_reduce_grouped_launch(p.srw.dev, p.srw.n(), grid_for(p.grid_reduce, 1, p.srw.n()), s));
    for (int q = 0; q < kClasses; ++q)
      NMF_TRY(nmf::bpp_grouped_launch(kClassK[q], p.bw[q].dev, p.bw[q].n(), grid_for(p.grid_bpp[q], 1, p.bw[q].n()),
                                      p.max_rounds, p.warm_cap, cw, s));
    // H update: G_W, R_H = A^T W, BPP
    NMF_TRY(nmf::gram_grouped_launch(p.gw.dev, p.gw.n(), grid_for(p.grid_gram, 1, p.gw.n()), s));
    NMF_TRY(nmf::gram_reduce_grouped_launch(p.gwr.dev, p.gwr.n(), grid_for(p.grid_reduce, 1, p.gwr.n()), s));
    NMF_TRY(nmf::split_y_grouped_launch(p.syh.dev, p.syh.n(), grid_for(p.grid_split, 1, p.syh.n()), s));
    for (int q = 0; q < 2; ++q)
      NMF_TRY(nmf::bf16x3_grouped_launch(q + 1, p.tune.rhs_tile_rows, p.rh[q].dev, p.rh[q].n(),
                                         grid_for(p.grid_bf16[q], 1, p.rh[q].n()), s));
    NMF_TRY(nmf::split_reduce_grouped_launch(p.srh.dev, p.srh.n(), grid_for(p.grid_reduce, 1, p.srh.n()), s));
    for (int q = 0; q < kClasses; ++q)
      NMF_TRY(nmf::bpp_grouped_launch(kClassK[q], p.bh[q].dev, p.bh[q].n(), grid_for(p.grid_bpp[q], 1, p.bh[q].n()),
                                      p.max_rounds, p.warm_cap, ch, s));
  }
  return NMF_OK;
}

struct Graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Copies rows x k FP32 between a strided factor and its dense backup.
int copy_factor(float* dst, int64_t ldd, const float* src, int64_t lds, int64_t rows, int k, hipStream_t s) {
  if (hipMemcpy2DAsync(dst, (size_t)ldd * sizeof(float), src, (size_t)lds * sizeof(float), (size_t)k * sizeof(float),
                       (size_t)rows, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return nmf::fail(NMF_EHIP, "nmf_batch_autotune: factor copy failed");
  return NMF_OK;
}

int backup_factors(int count, const nmf_batch_problem* P, void* ws, bool save, hipStream_t s) {
  Carver c(ws, ~size_t(0));
  for (int i = 0; i < count; ++i) {
    float* bw = c.take<float>((size_t)P[i].m * P[i].k);
    float* bh = c.take<float>((size_t)P[i].n * P[i].k);
    if (save) {
      NMF_TRY(copy_factor(bw, P[i].k, P[i].W, P[i].ldw, P[i].m, P[i].k, s));
      NMF_TRY(copy_factor(bh, P[i].k, P[i].Ht, P[i].ldh, P[i].n, P[i].k, s));
    } else {
      NMF_TRY(copy_factor(P[i].W, P[i].ldw, bw, P[i].k, P[i].m, P[i].k, s));
      NMF_TRY(copy_factor(P[i].Ht, P[i].ldh, bh, P[i].k, P[i].n, P[i].k, s));
    }
  }
  return NMF_OK;
}

// One timed iteration of a candidate tuning, from the saved factors.
int time_tuning(int count, const nmf_batch_problem* P, const nmf_batch_tune& t, void* ws, size_t ws_bytes,
                hipStream_t s, double* ms) {
  Plan plan;
  NMF_TRY(plan_build(count, P, t, ws, ws_bytes, &plan, s));
  NMF_TRY(backup_factors(count, P, ws, false, s));
  NMF_TRY(enqueue(plan, 1, nullptr, NMF_BATCH_RESET, s));  // warm-up
  NMF_TRY(backup_factors(count, P, ws, false, s));
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return nmf::fail(NMF_EHIP, "nmf_batch_autotune: event");
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return nmf::fail(NMF_EHIP, "nmf_batch_autotune: event");
  }
  int rc = NMF_OK;
  if (hipEventRecord(e0, s) != hipSuccess) rc = nmf::fail(NMF_EHIP, "nmf_batch_autotune: record");
  if (rc == NMF_OK) rc = enqueue(plan, 2, nullptr, NMF_BATCH_RESET, s);
  if (rc == NMF_OK && hipEventRecord(e1, s) != hipSuccess) rc = nmf::fail(NMF_EHIP, "nmf_batch_autotune: record");
  if (rc == NMF_OK && hipEventSynchronize(e1) != hipSuccess) rc = nmf::fail(NMF_EHIP, "nmf_batch_autotune: sync");
  float f = 0.0f;
  if (rc == NMF_OK && hipEventElapsedTime(&f, e0, e1) != hipSuccess) rc = nmf::fail(NMF_EHIP, "nmf_batch_autotune: time");
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *ms = f / 2.0;
  return rc;
}

}  // namespace

extern "C" void nmf_batch_tune_default(nmf_batch_tune* t) {
  if (!t) return;
  t->gram_tiles = 8;
  t->rhs_w_chunks = kNoSplit;
  t->rhs_h_chunks = 32;
  t->bpp_problems = 256;
  t->grid_scale = 1;
  t->warm_prev = 1;
  t->rhs_tile_rows = 128;
  t->bpp_wide = 0;
}

extern "C" int nmf_batch_workspace_bytes(int count, const nmf_batch_problem* P, const nmf_batch_tune* t,
                                         size_t* bytes) {
  if (!bytes) return nmf::fail(NMF_EINVAL, "nmf_batch_workspace_bytes: null bytes");
  NMF_TRY(validate(count, P));
  if (t && !tune_ok(*t)) return nmf::fail(NMF_EINVAL, "nmf_batch_workspace_bytes: bad tuning");
  if (t) {
    *bytes = bytes_for(count, P, *t);
  } else {
    // the finest candidates bound every tuning the autotuner builds, up to
    // the 256-byte alignment of each item list (the lane-class choice moves
    // items between the per-class lists): a 16 KiB margin covers it
    nmf_batch_tune d;
    nmf_batch_tune_default(&d);
    size_t mx = 0;
    for (int wide = 0; wide < 2; ++wide) {
      nmf_batch_tune f = finest_tune(), e = d;
      f.bpp_wide = e.bpp_wide = wide;
      const size_t a = bytes_for(count, P, f), b = bytes_for(count, P, e);
      mx = a > mx ? a : mx;
      mx = b > mx ? b : mx;
    }
    *bytes = mx + ((size_t)16 << 10);
  }
  return NMF_OK;
}

extern "C" int nmf_batch_plan_create(int count, const nmf_batch_problem* P, const nmf_batch_tune* t, void* ws,
                                     size_t ws_bytes, void** plan) {
  if (!plan) return nmf::fail(NMF_EINVAL, "nmf_batch_plan_create: null plan");
  *plan = nullptr;
  NMF_TRY(validate(count, P));
  nmf_batch_tune tune;
  if (t) {
    if (!tune_ok(*t)) return nmf::fail(NMF_EINVAL, "nmf_batch_plan_create: bad tuning");
    tune = *t;
  } else {
    nmf_batch_tune_default(&tune);
  }
  Plan* p = new Plan();
  const int rc = plan_build(count, P, tune, ws, ws_bytes, p, nullptr);
  if (rc != NMF_OK) {
    delete p;
    return rc;
  }
  *plan = p;
  return NMF_OK;
}

extern "C" int nmf_batch_plan_destroy(void* plan) {
  delete static_cast<Plan*>(plan);
  return NMF_OK;
}

extern "C" int nmf_batch_iterate(void* plan, int iters, uint64_t* counters, int flags, void* stream) {
  if (!plan || iters < 0) return nmf::fail(NMF_EINVAL, "nmf_batch_iterate: bad arguments");
  return enqueue(*static_cast<Plan*>(plan), iters, counters, flags, nmf::as_stream(stream));
}

extern "C" int nmf_batch_graph_create(void* plan, int iters, uint64_t* counters, int flags, void* stream,
                                      void** graph) {
  if (!plan || !graph || iters < 1) return nmf::fail(NMF_EINVAL, "nmf_batch_graph_create: bad arguments");
  if (!stream) return nmf::fail(NMF_EINVAL, "nmf_batch_graph_create: capture needs a non-null stream");
  *graph = nullptr;
  hipStream_t s = nmf::as_stream(stream);
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return nmf::fail(NMF_EHIP, "nmf_batch_graph_create: begin capture failed");
  const int rc = enqueue(*static_cast<Plan*>(plan), iters, counters, flags, s);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (rc != NMF_OK || e != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return rc != NMF_OK ? rc : nmf::fail(NMF_EHIP, "nmf_batch_graph_create: end capture failed");
  }
  Graph* gr = new Graph();
  gr->graph = g;
  if (hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(g);
    delete gr;
    return nmf::fail(NMF_EHIP, "nmf_batch_graph_create: instantiate failed");
  }
  *graph = gr;
  return NMF_OK;
}

extern "C" int nmf_batch_graph_launch(void* graph, void* stream) {
  if (!graph) return nmf::fail(NMF_EINVAL, "nmf_batch_graph_launch: null graph");
  if (hipGraphLaunch(static_cast<Graph*>(graph)->exec, nmf::as_stream(stream)) != hipSuccess)
    return nmf::fail(NMF_EHIP, "nmf_batch_graph_launch: launch failed");
  return NMF_OK;
}

extern "C" int nmf_batch_graph_destroy(void* graph) {
  Graph* g = static_cast<Graph*>(graph);
  if (!g) return NMF_OK;
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
  return NMF_OK;
}

extern "C" int nmf_batch_autotune(int count, const nmf_batch_problem* P, void* ws, size_t ws_bytes,
                                  nmf_batch_tune* best, double* best_ms, void* stream) {
  if (!best) return nmf::fail(NMF_EINVAL, "nmf_batch_autotune: null best");
  size_t need = 0;
  NMF_TRY(nmf_batch_workspace_bytes(count, P, nullptr, &need));
  if (!ws || ws_bytes < need) return nmf::fail(NMF_EWORKSPACE, "nmf_batch_autotune: workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t s = nmf::as_stream(stream);
  NMF_TRY(backup_factors(count, P, ws, true, s));
  nmf_batch_tune cur;
  nmf_batch_tune_default(&cur);
  double cur_ms = 0.0;
  int rc = time_tuning(count, P, cur, ws, ws_bytes, s, &cur_ms);
  // coordinate search: each field in turn over its candidates (the NNLS lane
  // classes and the product tile shape first, then the work-item sizes)
  struct Field {
    const int* cand;
    int nc;
    int nmf_batch_tune::*slot;
  };
  const Field fields[] = {{kCandWide, 2, &nmf_batch_tune::bpp_wide},
                          {kCandTile, 2, &nmf_batch_tune::rhs_tile_rows},
                          {kCandBpp, 3, &nmf_batch_tune::bpp_problems},
                          {kCandRhsH, 3, &nmf_batch_tune::rhs_h_chunks},
                          {kCandRhsW, 3, &nmf_batch_tune::rhs_w_chunks},
                          {kCandGram, 3, &nmf_batch_tune::gram_tiles},
                          {kCandGrid, 2, &nmf_batch_tune::grid_scale}};
  for (const Field& f : fields) {
    if (rc != NMF_OK) break;
    const int* cand = f.cand;
    const int nc = f.nc;
    for (int q = 0; q < nc && rc == NMF_OK; ++q) {
      nmf_batch_tune t = cur;
      int* slot = &(t.*f.slot);
      if (*slot == cand[q]) continue;
      *slot = cand[q];
      double ms = 0.0;
      rc = time_tuning(count, P, t, ws, ws_bytes, s, &ms);
      if (rc == NMF_OK && ms < cur_ms) {
        cur = t;
        cur_ms = ms;
      }
    }
  }
  const int rr = backup_factors(count, P, ws, false, s);
  if (hipStreamSynchronize(s) != hipSuccess && rc == NMF_OK) rc = nmf::fail(NMF_EHIP, "nmf_batch_autotune: sync");
  if (rc != NMF_OK) return rc;
  if (rr != NMF_OK) return rr;
  *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return NMF_OK;
}
