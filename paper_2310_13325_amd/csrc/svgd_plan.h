// Workspace layout of the SVGD / sSVGD step.
#pragma once

#include <algorithm>
#include <cstdint>

#include "vip_internal.h"

namespace vip {

struct SvgdPlan {
  uint32_t *status = nullptr;
  float *xbar = nullptr, *xc = nullptr;
  float *sq = nullptr, *vq = nullptr;   // diagonal kernel: sqrt(q_a), 1 / q_a per coordinate
  uint16_t *xc16 = nullptr;
  float *part = nullptr, *D = nullptr, *K = nullptr, *s = nullptr;
  uint32_t *hist = nullptr, *sel = nullptr;
  uint32_t *chol = nullptr;   // blocked Cholesky: [0] attempt failed, [1] every retry failed
  double *h2 = nullptr, *L = nullptr;
  float *Lf = nullptr;   // FP32 copy of L, transposed (Lf[j][i] = L[i][j])
  float *xi = nullptr, *phi = nullptr;
  uint16_t *khi = nullptr;                   // K in BF16, rows of ldk
  uint32_t *bph = nullptr, *bpl = nullptr;   // B split: pairs of rows, 4 pairs of a column together
  int ldk = 0;
  long long dp = 0;
  int nbt = 0;
  int splits = 0, splits16 = 0;        // k splits of the FP32 and of the BF16 Gram
  long long kspan = 0, kspan16 = 0;    // coordinates per split, same order
  int nbt2 = 0, splits2 = 0;           // BF16 Gram in 256 x 256 blocks (LDS ring): blocks a side, k splits
  long long kspan2 = 0;
  size_t bytes = 0;
};

// Gram blocks are 128 x 128 (upper triangle only); the contraction over d is
// split so that about 512 workgroups run, each over at least 256 coordinates.
// Each Gram takes more splits when they spread its blocks more evenly over the
// 256 compute units (all of them are resident at once, so a unit that holds
// one block more than the others sets the kernel's time): the FP32 Gram up to
// four times the base count, the BF16 Gram, six times shorter, up to one and a
// half times, since every extra partial costs the distance pass a read of n x n.
inline void plan_svgd(int n, long long d, char *base, SvgdPlan *P) {
  P->nbt = (n + 127) / 128;
  const int nup = P->nbt * (P->nbt + 1) / 2;
  const int s0 = std::max(1, std::min(64, (512 + nup - 1) / nup));
  auto balanced = [nup, s0](int smax) {
    int sb = s0;
    double best = 0.0;
    for (int s = s0; s <= std::min(64, smax); ++s) {
      const long long b = (long long)nup * s;
      const double even = double(b) / double(256 * ((b + 255) / 256));
      if (even > best + 0.02) best = even, sb = s;
    }
    return sb;
  };
  const int sb = balanced(4 * s0), sb16 = balanced((3 * s0 + 1) / 2);
  auto span_of = [d](int splits) {
    long long span = (d + splits - 1) / splits;
    span = (span + 15) / 16 * 16;   // k ranges start on 16-element boundaries (vector loads)
    return std::max<long long>(256, (span + 63) / 64 * 64);
  };
  P->kspan = span_of(sb);
  P->splits = int((d + P->kspan - 1) / P->kspan);
  P->kspan16 = span_of(sb16);
  P->splits16 = int((d + P->kspan16 - 1) / P->kspan16);
  // 256 x 256 blocks, one per compute unit: as many splits as keep the blocks
  // within one round of the 256 units and spread them most evenly
  P->nbt2 = (n + 255) / 256;
  {
    const int nup2 = P->nbt2 * (P->nbt2 + 1) / 2;
    int sb2 = 1;
    double best = 0.0;
    for (int s = 1; s <= 64; ++s) {
      const long long b = (long long)nup2 * s;
      if (b > 256 && s > 1) break;
      const double even = double(b) / 256.0;
      if (even > best) best = even, sb2 = s;
    }
    P->kspan2 = span_of(sb2);
    P->splits2 = int((d + P->kspan2 - 1) / P->kspan2);
  }
  const size_t nn = size_t(n) * size_t(n), nd = size_t(n) * size_t(d);
  Arena A;
  A.base = base;
  P->status = reinterpret_cast<uint32_t *>(base);
  P->xbar = A.take<float>(size_t(d));
  P->sq = A.take<float>(size_t(d));
  P->vq = A.take<float>(size_t(d));
  P->xc = A.take<float>(nd);
  P->xc16 = A.take<uint16_t>(nd);
  P->part = A.take<float>(size_t(std::max(std::max(P->splits, P->splits16), P->splits2)) * nn);
  P->D = A.take<float>(nn);
  P->K = A.take<float>(nn);
  P->s = A.take<float>(size_t(n));
  P->hist = A.take<uint32_t>(2 * 2048);   // two radix histograms of up to 2048 bins
  P->sel = A.take<uint32_t>(8);
  P->chol = A.take<uint32_t>(2);
  P->h2 = A.take<double>(1);
  P->L = A.take<double>(nn);
  P->Lf = A.take<float>(nn);
  P->xi = A.take<float>(nd);
  P->phi = A.take<float>(nd);
  P->ldk = (n + 31) / 32 * 32;
  P->khi = A.take<uint16_t>(size_t(n) * size_t(P->ldk));
  P->dp = (d + 7) / 8 * 8;
  P->bph = A.take<uint32_t>(size_t(P->ldk / 2) * size_t(P->dp));
  P->bpl = A.take<uint32_t>(size_t(P->ldk / 2) * size_t(P->dp));
  P->bytes = A.bytes();
}

}  // namespace vip
