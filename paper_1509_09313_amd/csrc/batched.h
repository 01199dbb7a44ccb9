// Work items of the grouped (many-instance) phase kernels.  Each item is
// self-contained: it carries the pointers and sizes of the instance it
// belongs to, so a persistent kernel walks one flat array of items that spans
// every instance of a batch.  Items are built on the host once per plan and
// uploaded into the caller's workspace.
#pragma once

#include "nmf_common.h"

namespace nmf {

// G partial = X[tile0*64 .. (tile0+ntiles)*64)^T X[...] (k x k, row-major)
struct GramItem {
  const float* X;
  int64_t ldx, rows;
  int k, pad;
  int64_t tile0, ntiles;
  double* partial;
};

// G[e] = sum_{s < nslots} partial[s * k * k + e] for e in [e0, e0 + 256)
struct GramReduceItem {
  const double* partial;
  double* G;
  int k, nslots;
  int64_t e0;
};

// 64 rows of Y (K x k) -> columns [K0, K0 + 64) of the transposed BF16 planes
struct SplitYItem {
  const float* Y;
  int64_t ldy, K;
  int k, KP;
  uint16_t *Yth, *Ytl;
  int64_t ldt, K0;
};

// one tile (64 or 128 rows from row0) of R = B * Y over 64-column chunks [kc0, kc1)
struct Bf16Item {
  const uint16_t* B;
  int64_t Rp, nkc;
  const uint16_t *Yth, *Ytl;
  int64_t ldt;
  float* out;
  int64_t ldp, rows;
  int k, pad;
  int64_t row0, kc0, kc1;
};

// R[e] = sum_{s < S} P[s * stride + e] (FP64 sum in s order) for entries
// [e0, e0 + 256) of a rows x k block
struct SplitReduceItem {
  const float* P;
  int64_t stride;
  float* R;
  int64_t ldr, rows;
  int k, S;
  int64_t e0;
};

// NNLS problems [b0, b1) sharing one Gram matrix; mask (optional, indexed
// like X) holds each problem's passive set: read as its start set and
// overwritten with the final one
struct BppItem {
  const double* G;
  const float* R;
  int64_t ldr;
  float* X;
  int64_t ldx;
  uint8_t* status;
  uint64_t* mask;
  int k, pad;
  int64_t b0, b1;
};

// grouped launchers (persistent: `grid` workgroups walk the item array)
int gram_grouped_launch(const GramItem* items, int64_t n, int grid, hipStream_t s);
int gram_reduce_grouped_launch(const GramReduceItem* items, int64_t n, int grid, hipStream_t s);
int split_y_grouped_launch(const SplitYItem* items, int64_t n, int grid, hipStream_t s);
int bf16x3_grouped_launch(int NT, int tile_rows, const Bf16Item* items, int64_t n, int grid, hipStream_t s);
int split_reduce_grouped_launch(const SplitReduceItem* items, int64_t n, int grid, hipStream_t s);
int bpp_grouped_launch(int K, const BppItem* items, int64_t n, int grid, int max_rounds, int warm_cap,
                       uint64_t* counters, hipStream_t s);
// resident workgroups of each grouped kernel on the current device (0 if unknown)
int grouped_capacity(int which);
int gram_grouped_occupancy(int which, int* per_cu);
int bf16_grouped_occupancy(int which, int* per_cu);
int bpp_grouped_occupancy(int K, int* per_cu);
int bpp_class(int k);
enum { kCapGram = 0, kCapSplitY, kCapBf16NT1, kCapBf16NT2, kCapReduce, kCapBpp16, kCapBpp32, kCapBpp56,
       kCapBpp64, kCapBpp8, kCapBf16NT1T64, kCapBf16NT2T64, kCapCount };

}  // namespace nmf
