// Learned warm start for BPP: features and the passive-set network.
//
// Features of one problem (G, f): phi = [s / ||s||_2, diag(G) / mean(diag(G))]
// with s_i = f_i / sqrt(G_ii) (0 for pinned indices, G_ii <= 1e-14 max G_ll).
// They are invariant to scaling the least-squares problem (C, b) -> (cC, cb).
#include <math.h>

#include "nmf_common.h"

namespace {

// One wavefront per sampled problem b = e * stride; lane i < k owns index i.
__global__ __launch_bounds__(256) void k_features(int k, int64_t batch, int64_t stride, const double* __restrict__ G,
                                                  const float* __restrict__ R, int64_t ldr, float* __restrict__ phi) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  double dmax = 0.0, dsum = 0.0;
  for (int q = 0; q < k; ++q) {
    const double d = G[q * k + q];
    dmax = fmax(dmax, d);
    dsum += d;
  }
  const double mean = dsum / k;
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
  (void)k; (void)batch; (void)c;
  *scratch = nullptr;
  return NMF_OK;
}

int mlp_infer_launch(int k, int64_t batch, const double* G, const float* R, int64_t ldr, const float* params,
                     uint64_t* mask_out, void* scratch, hipStream_t s) {
  (void)k; (void)batch; (void)G; (void)R; (void)ldr; (void)params; (void)mask_out; (void)scratch; (void)s;
  return fail(NMF_EUNSUPPORTED, "learned warm start is not built yet");
}

}  // namespace nmf
