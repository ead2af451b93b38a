// SVGD and stochastic SVGD particle updates (paper section 2.3-2.4).
//
//   RBF kernel (eq:rbf)       K_ij = exp(-|x_i - x_j|^2 / (2 h^2))
//   SVGD (eq:phi_mean)        phi_i = 1/n sum_j [K_ij g_j + K_ij (x_i - x_j) / h^2]
//                                   = 1/n [ (K G)_i + (s_i x_i - (K X)_i) / h^2 ],  s_i = sum_j K_ij
//   sSVGD (eq:stochastic_svgd, eq:matrixDK, eq:noise_term)
//                             x_i <- x_i + eps phi_i + sqrt(2 eps) (L Xi)_i,  L L^T = K / n
//   uniform prior, strategy 1 (section 3): clip to [lo, hi] after the update
//   (the other prior kinds act through the gradient only).
//
// Kernel sequence for one step:
//   centre      xbar = mean_i x_i (FP64 sums); Xc = X - xbar in FP32 and BF16
//   gram        partial Gram blocks of Xc Xc^T over split ranges of d:
//               BF16 on matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation)
//               or FP32 on matrix cores (v_mfma_f32_32x32x2_f32)
//   distances   D_ij = G_ii + G_jj - 2 G_ij straight from the partials, G summed
//               over them in a fixed order (G itself is not stored)
//   median      exact k-th order statistics of the D values by 4-pass radix
//               select on their IEEE bits (non-negative floats order like
//               unsigned integers), then h^2 = med / (2 ln(n+1)) (1 if med = 0)
//   rbf         K = exp(-D / (2 h^2)), row sums s (FP64 sums)
//   cholesky    (sSVGD) L = chol(K / n) in FP64 in LDS, jitter retries
//   update      one GEMM pass computing K (G - Xc / h^2), then phi, the
//               update and the clip in its epilogue: on the FP32 matrix cores
//               for the FP32 path, on the BF16 matrix cores with both operands
//               split into BF16 pairs for the BF16 path, on the vector units
//               (with L Xi) for sSVGD.
// Distances come from centred particles: D is translation invariant, and
// centring removes the large common velocity that BF16 could not resolve.
#include <cmath>
#include <mutex>
#include <cstring>

#include "vip_internal.h"
#include "philox.h"
#include "svgd_plan.h"
#include "opt_rules.h"

namespace vip {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// ---- centre ----------------------------------------------------------------
// Block of 32 coordinates x 32 row groups: each thread sums every 32nd
// particle of its coordinate (FP64), the 32 partial sums are added in a fixed
// order, and the block then writes the centred columns.  For the diagonal
// matrix-valued kernel (sq != null) a second pass forms the variance across
// particles (FP64, ddof 0), q = 1 / var (1 where var = 0), and the BF16 copy
// used by the Gram is scaled by sqrt(q).
//
// With CACHE > 0 (X under 4 GiB) a thread keeps its first CACHE values in
// registers, so that for n <= 32 CACHE the later passes do not read X again.
// Those values move through raw buffer loads and stores over X, Xc and the
// BF16 copy: a 32-bit lane offset plus a row offset that is the same for the
// whole block, and the range check returns 0 for rows past n (and drops
// their stores).
constexpr int CENTRE_COLS = 32, CENTRE_GROUPS = 32, CENTRE_CACHE = 64;
using SvgdRsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ SvgdRsrc svgd_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, int(bytes), 0x00020000);
}
template <int CACHE>
__global__ __launch_bounds__(CENTRE_COLS *CENTRE_GROUPS) void centre_kernel(
    const float *x, float *xbar, float *xc, uint16_t *xc16, float *sq, float *vq, int n,
    long long d, uint32_t *status) {
  __shared__ double part[CENTRE_GROUPS][CENTRE_COLS];
  __shared__ float mean[CENTRE_COLS], scale[CENTRE_COLS];
  const int tx = threadIdx.x % CENTRE_COLS, ty = threadIdx.x / CENTRE_COLS;
  const long long a = (long long)blockIdx.x * CENTRE_COLS + tx;
  const bool in = a < d;
  const float *xa = x + (in ? a : 0);   // column a (in range even for idle threads)
  constexpr int NV = CACHE > 0 ? CACHE : 1;
  float v[NV];
  const int rest0 = ty + CACHE * CENTRE_GROUPS;   // first row not cached
  // byte offsets: my element of cached row k is at lb + k rb
  const uint32_t nbytes = CACHE > 0 ? uint32_t(n) * uint32_t(d) * 4u : 0u;
  const uint32_t lb = CACHE > 0 ? (uint32_t(ty) * uint32_t(d) + uint32_t(in ? a : 0)) * 4u : 0u;
  const uint32_t rb = uint32_t(CENTRE_GROUPS) * uint32_t(d) * 4u;
  if constexpr (CACHE > 0) {
    const SvgdRsrc rx = svgd_rsrc(x, nbytes);
#pragma unroll
    for (int k = 0; k < CACHE; ++k)
      v[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, int(lb), int(k * rb), 0));
#pragma unroll
    for (int k = 0; k < CACHE; ++k) v[k] = in ? v[k] : 0.0f;
  }
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < CACHE; ++k) sum += double(v[k]);
  if (in)
    for (int i = rest0; i < n; i += CENTRE_GROUPS) sum += double(xa[(long long)i * d]);
  part[ty][tx] = sum;
  __syncthreads();
  if (ty == 0) {
    double t = 0.0;
    for (int g = 0; g < CENTRE_GROUPS; ++g) t += part[g][tx];
    const float m = float(t / double(n));
    mean[tx] = m;
    scale[tx] = 1.0f;
    if (in) {
      xbar[a] = m;
      if (!isfinite(m)) atomicOr(status, VIP_FLAG_NONFINITE);
    }
  }
  __syncthreads();
  const float m = mean[tx];
  if (sq) {
    double ss = 0.0;
#pragma unroll
    for (int k = 0; k < CACHE; ++k) {
      // an opaque copy, so the FP64 conversions of the first pass are not
      // kept alive in registers for this one
      float vk = v[k];
      asm volatile("" : "+v"(vk));
      const double dv = double(vk) - double(m);
      if (ty + k * CENTRE_GROUPS < n) ss += dv * dv;
    }
    if (in)
      for (int i = rest0; i < n; i += CENTRE_GROUPS) {
        const double dv = double(xa[(long long)i * d]) - double(m);
        ss += dv * dv;
      }
    __syncthreads();   // every thread has read the means and sums before part is reused
    part[ty][tx] = ss;
    __syncthreads();
    if (ty == 0 && in) {
      double t = 0.0;
      for (int g = 0; g < CENTRE_GROUPS; ++g) t += part[g][tx];
      const double var = t / double(n);
      const double qv = var > 0.0 ? 1.0 / var : 1.0;
      scale[tx] = float(sqrt(qv));
      sq[a] = float(sqrt(qv));
      vq[a] = float(1.0 / qv);
    }
    __syncthreads();
  }
  if (!in) return;
  const float sc = scale[tx];
  if constexpr (CACHE > 0) {
    const SvgdRsrc r16 = svgd_rsrc(xc16, nbytes / 2u);
#pragma unroll
    for (int k = 0; k < CACHE; ++k) {
      const float c = v[k] - m;
      __builtin_amdgcn_raw_buffer_store_b16(f32_to_bf16_rne(sq ? c * sc : c), r16, int(lb / 2u),
                                            int(k * (rb / 2u)), 0);
    }
    if (xc) {
      const SvgdRsrc rc = svgd_rsrc(xc, nbytes);
#pragma unroll
      for (int k = 0; k < CACHE; ++k)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v[k] - m), rc, int(lb),
                                              int(k * rb), 0);
    }
  }
  for (int i = rest0; i < n; i += CENTRE_GROUPS) {
    const long long e = (long long)i * d + a;
    const float c = x[e] - m;
    if (xc) xc[e] = c;
    xc16[e] = f32_to_bf16_rne(sq ? c * sc : c);
  }
}

// Upper-triangular block index u -> (bi, bj), bi <= bj, row-major over bi.
__device__ __forceinline__ void upper_block(int u, int nb, int &bi, int &bj) {
  int row = 0, rem = u;
  while (rem >= nb - row) {
    rem -= nb - row;
    ++row;
  }
  bi = row;
  bj = row + rem;
}

// ---- Gram, BF16 matrix cores -------------------------------------------------
// Block 128x128 of Xc Xc^T over k in [s*kspan, (s+1)*kspan); 4 waves, each a
// 64x64 sub-block as 2x2 MFMA 32x32 tiles.  Operand layout of
// v_mfma_f32_32x32x16_bf16: lane l holds row (l % 32) and k = 8 (l / 32) .. +7
// of each operand; result register r of lane l is row 8 (r / 4) + 4 (l / 32) + r % 4,
// column l % 32.
constexpr int GB = 128;   // block edge
constexpr int GK = 64;    // k per LDS stage
constexpr int GKP = GK + 8;
constexpr int GIT = GB * GK / 8 / 256;   // 16-byte chunks per thread and operand per stage

// One stage of Gram operands into registers: chunk it of thread t is row
// (t + 256 it) / (GK / 8), k chunk (t + 256 it) % (GK / 8), from rows i0 + row
// (A) and j0 + row (B; on a diagonal block B is A and is not loaded).  No
// loaded value is used here, so the loads stay in flight during the stage.
__device__ __forceinline__ void gram_load(const uint16_t *xc16, int n, long long d, long long k1,
                                          int i0, int j0, bool diag, bool vec_ok, long long kb,
                                          uint4 (&pa)[GIT], uint4 (&pb)[GIT]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int it = 0; it < GIT; ++it) {
    const int idx = t + it * 256;
    const int row = idx / (GK / 8), ch = idx % (GK / 8);
    const long long kc = kb + ch * 8;
    uint4 va = make_uint4(0, 0, 0, 0), vbv = make_uint4(0, 0, 0, 0);
    if (vec_ok && kc + 8 <= k1) {
      if (i0 + row < n) va = *reinterpret_cast<const uint4 *>(xc16 + (long long)(i0 + row) * d + kc);
      if (!diag && j0 + row < n)
        vbv = *reinterpret_cast<const uint4 *>(xc16 + (long long)(j0 + row) * d + kc);
    } else {
      uint32_t ta[4] = {0, 0, 0, 0}, tb[4] = {0, 0, 0, 0};
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const long long k = kc + e;
        const uint32_t a16 = (i0 + row < n && k < k1) ? xc16[(long long)(i0 + row) * d + k] : 0u;
        const uint32_t b16 = (!diag && j0 + row < n && k < k1) ? xc16[(long long)(j0 + row) * d + k] : 0u;
        ta[e >> 1] |= a16 << (16 * (e & 1));
        tb[e >> 1] |= b16 << (16 * (e & 1));
      }
      va = make_uint4(ta[0], ta[1], ta[2], ta[3]);
      vbv = make_uint4(tb[0], tb[1], tb[2], tb[3]);
    }
    pa[it] = va;
    pb[it] = vbv;   // not loaded on a diagonal block: the store takes pa there
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 4))) void gram_bf16_kernel(
    const uint16_t *xc16, float *part, int n, long long d, long long kspan, int nbt) {
  __shared__ __attribute__((aligned(16))) uint16_t As[GB][GKP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GB][GKP];
  const int nup = nbt * (nbt + 1) / 2;
  // tile index, contiguous per XCD (blocks are dealt round-robin over 8 XCDs),
  // so that blocks of one k range that share rows meet in one L2
  const int per = int(gridDim.x) >> 3;
  const int tb = (int(blockIdx.x) & 7) * per + (int(blockIdx.x) >> 3);
  if (tb >= nup * int((d + kspan - 1) / kspan)) return;
  const int split = tb / nup;
  int bi, bj;
  upper_block(tb - split * nup, nbt, bi, bj);
  const int i0 = bi * GB, j0 = bj * GB;
  const bool diag = bi == bj;   // A and B are the same rows
  const long long k0 = (long long)split * kspan;
  const long long k1 = min(d, k0 + kspan);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;
  f32x16_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
  const bool vec_ok = (d % 8) == 0;
  // the next stage is prefetched into registers while this one is computed
  uint4 pa[GIT], pb[GIT];
  gram_load(xc16, n, d, k1, i0, j0, diag, vec_ok, k0, pa, pb);
  for (long long kb = k0; kb < k1; kb += GK) {
#pragma unroll
    for (int it = 0; it < GIT; ++it) {
      const int idx = t + it * 256;
      const int row = idx / (GK / 8), ch = idx % (GK / 8);
      *reinterpret_cast<uint4 *>(&As[row][ch * 8]) = pa[it];
      const uint4 a = pa[it], b = pb[it];   // component-wise select (a value, not an address)
      *reinterpret_cast<uint4 *>(&Bs[row][ch * 8]) =
          make_uint4(diag ? a.x : b.x, diag ? a.y : b.y, diag ? a.z : b.z, diag ? a.w : b.w);
    }
    __syncthreads();
    if (kb + GK < k1) gram_load(xc16, n, d, k1, i0, j0, diag, vec_ok, kb + GK, pa, pb);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 16) {
      bf16x8_t fa[2], fb[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        uint4 ra = *reinterpret_cast<const uint4 *>(&As[wi * 64 + m * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
        uint4 rb = *reinterpret_cast<const uint4 *>(&Bs[wj * 64 + m * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
        __builtin_memcpy(&fa[m], &ra, 16);
        __builtin_memcpy(&fb[m], &rb, 16);
      }
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[m], fb[q], acc[m][q], 0, 0, 0);
    }
    __syncthreads();
  }
  float *P = part + (long long)split * n * n;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        int row = i0 + wi * 64 + m * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        int col = j0 + wj * 64 + q * 32 + (lane & 31);
        if (row < n && col < n) P[(long long)row * n + col] = acc[m][q][r];
      }
}

// The BF16 Gram in 256 x 256 blocks of the upper triangle, one block per
// compute unit, 8 waves (4 x 2) of 64 x 128 (2 x 4 tiles of 32 x 32).  The
// operands stream through a ring of four LDS stages of 32 coordinates (A and
// B rows: 16 KB each; a diagonal block loads A only and reads it for both) by
// 16-byte loads that write LDS directly, three stages ahead of the matrix
// instructions, with one barrier per stage.  Chunk c (8 coordinates) of row r
// sits in slot c ^ ((r >> 2) & 3) of the row's four, so that the fragment
// reads of 16 consecutive rows meet distinct banks.  Rows past n and
// coordinates past the split's end read as zeros (offsets beyond the range).
// The loads are inline assembly with explicit counter waits, for the reason
// given at update_bf16x2_ring_kernel.  Needs rows of a multiple of 8
// coordinates (16-byte aligned) and n d 2 bytes below 2^31.
constexpr int G2B = 256, G2K = 32, G2S = 4, G2T = 512;
constexpr bool kGramRing = true;
constexpr int G2_OP = G2B * G2K * 2, G2_STAGE = 2 * G2_OP;
__global__ __launch_bounds__(G2T) __attribute__((amdgpu_waves_per_eu(2, 2))) void gram_bf16_ring_kernel(
    const uint16_t *xc16, float *part, int n, long long d, long long kspan, int nbt) {
  __shared__ __attribute__((aligned(16))) unsigned char ring[G2S][G2_STAGE];
  const int nup = nbt * (nbt + 1) / 2;
  const int per = int(gridDim.x) >> 3;
  const int tb = (int(blockIdx.x) & 7) * per + (int(blockIdx.x) >> 3);
  if (tb >= nup * int((d + kspan - 1) / kspan)) return;
  const int split = tb / nup;
  int bi, bj;
  upper_block(tb - split * nup, nbt, bi, bj);
  const int i0 = bi * G2B, j0 = bj * G2B;
  const bool diag = bi == bj;
  const long long k0 = (long long)split * kspan;
  const long long k1 = min(d, k0 + kspan);
  const int nst = int((k1 - k0 + G2K - 1) / G2K);
  const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wi = w >> 1, wj = w & 1;

  typedef uint32_t U32x4 __attribute__((ext_vector_type(4)));
  U32x4 rx;
  {
    const uint64_t b = reinterpret_cast<uint64_t>(xc16);
    rx.x = __builtin_amdgcn_readfirstlane(uint32_t(b));
    rx.y = __builtin_amdgcn_readfirstlane(uint32_t(b >> 32)) & 0xffffu;
    rx.z = __builtin_amdgcn_readfirstlane(uint32_t(n) * uint32_t(d) * 2u);
    rx.w = 0x00020000u;
  }
  const uint32_t ring0 = uint32_t(reinterpret_cast<uintptr_t>(
      (__attribute__((address_space(3))) unsigned char *)&ring[0][0]));
  // My loads of a stage: A loads w and w + 8 of the 16 (rows 16 q + lane / 4),
  // then (off the diagonal) B loads w and w + 8.
  auto issue = [&](int st) {
    const long long kb = k0 + (long long)st * G2K;
    const uint32_t base = ring0 + uint32_t((st % G2S) * G2_STAGE);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k >= 2 && diag) break;
      const int q = w + 8 * (k & 1);
      const int row = 16 * q + (lane >> 2);
      const int chunk = (lane & 3) ^ ((row >> 2) & 3);
      const int grow = (k < 2 ? i0 : j0) + row;
      const long long kc = kb + chunk * 8;
      const uint32_t m0 = base + uint32_t((k >= 2 ? G2_OP : 0) + q * 16 * 64);
      const uint32_t off = (grow < n && kc < k1) ? uint32_t(((long long)grow * d + kc) * 2)
                                                 : 0x80000000u;
      uint32_t keep;
      asm volatile(
          "s_mov_b32 %0, m0\n\ts_mov_b32 m0, %1\n\ts_nop 0\n\t"
          "buffer_load_dwordx4 %2, %3, 0 offen lds\n\ts_mov_b32 m0, %0"
          : "=&s"(keep)
          : "s"(m0), "v"(off), "s"(rx)
          : "memory");
    }
  };

  f32x16_t acc[2][4];
  for (int m = 0; m < 2; ++m)
    for (int q = 0; q < 4; ++q)
      for (int r = 0; r < 16; ++r) acc[m][q][r] = 0.0f;
  for (int st = 0; st < 3 && st < nst; ++st) issue(st);
  for (int st = 0; st < nst; ++st) {
    // this stage has landed once only the later stages' loads may fly (two
    // loads a stage on the diagonal, four off it)
    const int newer = min(nst - 1 - st, 2);
    if (diag) {
      if (newer == 2) __builtin_amdgcn_s_waitcnt(0x0F74);        // vmcnt(4)
      else if (newer == 1) __builtin_amdgcn_s_waitcnt(0x0F72);   // vmcnt(2)
      else __builtin_amdgcn_s_waitcnt(0x0F70);
    } else {
      if (newer == 2) __builtin_amdgcn_s_waitcnt(0x0F78);        // vmcnt(8)
      else if (newer == 1) __builtin_amdgcn_s_waitcnt(0x0F74);   // vmcnt(4)
      else __builtin_amdgcn_s_waitcnt(0x0F70);
    }
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (st + 3 < nst) issue(st + 3);
    const unsigned char *sa = &ring[st % G2S][0];
    const unsigned char *sb = diag ? sa : sa + G2_OP;
#pragma unroll
    for (int kk = 0; kk < G2K; kk += 16) {
      const int c = (kk + 8 * (lane >> 5)) >> 3;   // my chunk of 8 coordinates
      bf16x8_t fa[2], fb[4];
      for (int m = 0; m < 2; ++m) {
        const int row = wi * 64 + m * 32 + (lane & 31);
        const uint4 v = *reinterpret_cast<const uint4 *>(sa + (row * 4 + (c ^ ((row >> 2) & 3))) * 16);
        __builtin_memcpy(&fa[m], &v, 16);
      }
      for (int q = 0; q < 4; ++q) {
        const int row = wj * 128 + q * 32 + (lane & 31);
        const uint4 v = *reinterpret_cast<const uint4 *>(sb + (row * 4 + (c ^ ((row >> 2) & 3))) * 16);
        __builtin_memcpy(&fb[q], &v, 16);
      }
      for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 4; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[m], fb[q], acc[m][q], 0, 0, 0);
    }
  }
  float *P = part + (long long)split * n * n;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = i0 + wi * 64 + m * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = j0 + wj * 128 + q * 32 + (lane & 31);
        if (row < n && col < n) P[(long long)row * n + col] = acc[m][q][r];
      }
}

// ---- Gram, FP32 matrix cores -------------------------------------------------
// Same 128x128 blocks and k splits; 4 waves, each a 64x64 sub-block as 2x2
// tiles of v_mfma_f32_32x32x2_f32 (lane l holds A[l % 32][l / 32] and
// B[l / 32][l % 32]; result register r of lane l is C[8 (r / 4) + 4 (l / 32) +
// r % 4][l % 32]).  k is staged 16 at a time, stored k-major in LDS so that
// each half-wave reads 32 consecutive rows.
constexpr int GF_K = 16, GF_P = 4;
__global__ __launch_bounds__(256) void gram_f32_kernel(const float *xc, const float *sq,
                                                       float *part, int n, long long d,
                                                       long long kspan, int nbt) {
  __shared__ __attribute__((aligned(16))) float As[GF_K][GB + GF_P];
  __shared__ __attribute__((aligned(16))) float Bs[GF_K][GB + GF_P];
  const int nup = nbt * (nbt + 1) / 2;
  // tile index, contiguous per XCD (blocks are dealt round-robin over 8 XCDs),
  // so that blocks of one k range that share rows meet in one L2
  const int per = int(gridDim.x) >> 3;
  const int tb = (int(blockIdx.x) & 7) * per + (int(blockIdx.x) >> 3);
  if (tb >= nup * int((d + kspan - 1) / kspan)) return;
  const int split = tb / nup;
  int bi, bj;
  upper_block(tb - split * nup, nbt, bi, bj);
  const int i0 = bi * GB, j0 = bj * GB;
  const long long k0 = (long long)split * kspan;
  const long long k1 = min(d, k0 + kspan);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;
  const bool vec = (d % 4) == 0 && (kspan % 4) == 0;
  f32x16_t acc[2][2];
  for (int m = 0; m < 2; ++m)
    for (int q = 0; q < 2; ++q)
      for (int r = 0; r < 16; ++r) acc[m][q][r] = 0.0f;
  for (long long kb = k0; kb < k1; kb += GF_K) {
    // 128 rows x 16 k per operand: 4 threads per row, a float4 each, two rows per thread
    for (int it = 0; it < 2; ++it) {
      const int idx = t + it * 256;
      const int row = idx >> 2, kq = (idx & 3) * 4;
      const long long k = kb + kq;
      float va[4], vb[4];
      if (vec && k + 3 < k1) {
        const float4 fa = i0 + row < n ? *reinterpret_cast<const float4 *>(xc + (long long)(i0 + row) * d + k)
                                       : make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 fb = j0 + row < n ? *reinterpret_cast<const float4 *>(xc + (long long)(j0 + row) * d + k)
                                       : make_float4(0.f, 0.f, 0.f, 0.f);
        va[0] = fa.x; va[1] = fa.y; va[2] = fa.z; va[3] = fa.w;
        vb[0] = fb.x; vb[1] = fb.y; vb[2] = fb.z; vb[3] = fb.w;
      } else {
        for (int c = 0; c < 4; ++c) {
          va[c] = (i0 + row < n && k + c < k1) ? xc[(long long)(i0 + row) * d + k + c] : 0.0f;
          vb[c] = (j0 + row < n && k + c < k1) ? xc[(long long)(j0 + row) * d + k + c] : 0.0f;
        }
      }
      if (sq)   // diagonal kernel: columns scaled by sqrt(q)
        for (int c = 0; c < 4; ++c) {
          const float w = k + c < k1 ? sq[k + c] : 0.0f;
          va[c] *= w;
          vb[c] *= w;
        }
      for (int c = 0; c < 4; ++c) {
        As[kq + c][row] = va[c];
        Bs[kq + c][row] = vb[c];
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GF_K; kk += 2) {
      const int k = kk + (lane >> 5);
      float fa[2], fb[2];
      for (int m = 0; m < 2; ++m) fa[m] = As[k][wi * 64 + m * 32 + (lane & 31)];
      for (int q = 0; q < 2; ++q) fb[q] = Bs[k][wj * 64 + q * 32 + (lane & 31)];
      for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 2; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[m], fb[q], acc[m][q], 0, 0, 0);
    }
    __syncthreads();
  }
  float *P = part + (long long)split * n * n;
  for (int m = 0; m < 2; ++m)
    for (int q = 0; q < 2; ++q)
      for (int r = 0; r < 16; ++r) {
        int row = i0 + wi * 64 + m * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        int col = j0 + wj * 64 + q * 32 + (lane & 31);
        if (row < n && col < n) P[(long long)row * n + col] = acc[m][q][r];
      }
}

// Squared distances D_ij = G_ii + G_jj - 2 G_ij (0 on the diagonal, clamped at
// 0) straight from the Gram partials, G = sum of part[s] in split order.  A
// block takes a 32 x 32 tile (ti, tj), ti <= tj, which lies in an upper
// 128 x 128 Gram block, reads its partial rows coalesced, writes its tile of
// D and, off the diagonal, the mirrored tile through LDS; D is exactly
// symmetric.
constexpr int DT = 32;
__global__ __launch_bounds__(256) void gram_dist_kernel(const float *part, float *D, int n,
                                                        int splits, int ntile, uint32_t *status) {
  __shared__ float tile[DT][DT + 1];
  __shared__ float dg[2][DT];   // G_ii of my rows, G_jj of my columns
  int ti, tj;
  upper_block(int(blockIdx.x), ntile, ti, tj);
  const int i0 = ti * DT, j0 = tj * DT;
  const long long nn = (long long)n * n;
  const int t = threadIdx.x;
  if (t < 2 * DT) {
    const int k = (t < DT ? i0 : j0) + t % DT;
    float g = 0.0f;
    if (k < n) {
#pragma unroll 8
      for (int p = 0; p < splits; ++p) g += part[p * nn + (long long)k * n + k];
    }
    dg[t / DT][t % DT] = g;
  }
  __syncthreads();
  const int c = t % DT, r0 = t / DT;
  bool bad = false;
#pragma unroll
  for (int r = r0; r < DT; r += 256 / DT) {
    const int i = i0 + r, j = j0 + c;
    float v = 0.0f;
    if (i < n && j < n) {
      float g = 0.0f;
      // unrolled so that the partials' loads are in flight together (the sum
      // keeps its order)
#pragma unroll 8
      for (int p = 0; p < splits; ++p) g += part[p * nn + (long long)i * n + j];
      v = (i == j) ? 0.0f : fmaxf(dg[0][r] + dg[1][c] - 2.0f * g, 0.0f);
      bad |= !isfinite(v);
      D[(long long)i * n + j] = v;
    }
    tile[r][c] = v;
  }
  if (ti != tj) {
    __syncthreads();
#pragma unroll
    for (int r = r0; r < DT; r += 256 / DT) {
      const int j = j0 + r, i = i0 + c;
      if (i < n && j < n) D[(long long)j * n + i] = tile[c][r];
    }
  }
  if (bad) atomicOr(status, VIP_FLAG_NONFINITE);
}

// ---- exact median by radix select -------------------------------------------
// sel[0..2] = (prefix, mask, rank) for target 0, sel[3..5] for target 1.
// Counts one element of the wave into a 256-bin LDS histogram: the digit of
// the first counting lane is added once with the number of lanes sharing it
// (in the first passes most keys share their leading bits, and 64 lanes
// adding to one bin would serialise), every other counting lane adds its own.
// Must be reached by the whole wave.
__device__ __forceinline__ void wave_count(uint32_t *h, bool act, uint32_t digit) {
  const unsigned long long am = __ballot(act);
  if (!am) return;
  const int lane = int(threadIdx.x & 63);
  const int leader = __ffsll(am) - 1;
  const uint32_t ld = uint32_t(__builtin_amdgcn_readlane(int(digit), leader));   // leader is uniform
  const bool same = act && digit == ld;
  const unsigned long long sm = __ballot(same);
  if (lane == leader) atomicAdd(&h[ld], uint32_t(__popcll(sm)));
  if (act && !same) atomicAdd(&h[digit], 1u);
}

// One pass of the radix select: histogram of the `bits`-wide digit at `shift`
// over the keys (float bits of D >= 0) that match each target's prefix so far
// (three passes of 11, 11 and 10 bits).  While the two targets still share
// their prefix, one histogram serves both.
// Sixteen keys per thread and trip, as four 16-byte loads (when D is
// aligned) issued before any of them is counted; the loop runs the same
// number of times on every lane.
constexpr int RADIX_V = 4;       // 4-key groups per thread and trip
constexpr int RADIX_BINS = 2048;  // bins of the widest digit
__global__ __launch_bounds__(256) void radix_hist_kernel(const float *D, int n, int offdiag,
                                                         int vec, int shift, int bits,
                                                         const uint32_t *sel, uint32_t *hist) {
  __shared__ uint32_t h[2][RADIX_BINS];
  for (int b = threadIdx.x; b < 2 * RADIX_BINS; b += 256) (&h[0][0])[b] = 0;
  __syncthreads();
  const uint32_t p0 = sel[0], m0 = sel[1], p1 = sel[3], m1 = sel[4];
  const bool one = p0 == p1 && m0 == m1;
  const long long total = (long long)n * n;
  const long long groups = (total + 3) / 4;
  const long long stride = (long long)gridDim.x * blockDim.x * RADIX_V;
  for (long long base = (long long)blockIdx.x * blockDim.x * RADIX_V; base < groups; base += stride) {
    float v[RADIX_V][4];
#pragma unroll
    for (int u = 0; u < RADIX_V; ++u) {
      const long long e0 = 4 * (base + u * (long long)blockDim.x + threadIdx.x);
      if (vec && e0 + 3 < total) {
        const float4 f = *reinterpret_cast<const float4 *>(D + e0);
        v[u][0] = f.x, v[u][1] = f.y, v[u][2] = f.z, v[u][3] = f.w;
      } else {
        for (int q = 0; q < 4; ++q) v[u][q] = e0 + q < total ? D[e0 + q] : 0.0f;
      }
    }
#pragma unroll
    for (int u = 0; u < RADIX_V; ++u) {
      const long long e0 = 4 * (base + u * (long long)blockDim.x + threadIdx.x);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const long long e = e0 + q;
        bool in = e < total;
        if (offdiag && in) {
          const int i = int(e / n), j = int(e - (long long)i * n);
          in = i < j;
        }
        const uint32_t key = __float_as_uint(v[u][q]);
        const uint32_t digit = (key >> shift) & ((1u << bits) - 1u);
        wave_count(h[0], in && (key & m0) == p0, digit);
        if (!one) wave_count(h[1], in && (key & m1) == p1, digit);
      }
    }
  }
  __syncthreads();
  const int nb = 1 << bits;
  for (int b = threadIdx.x; b < 2 * RADIX_BINS; b += 256) {
    const int bb = b & (RADIX_BINS - 1);
    if (bb >= nb) continue;
    const uint32_t v = one ? h[0][bb] : (&h[0][0])[b];
    if (v) atomicAdd(&hist[b], v);
  }
}

// One wave per target: each lane holds RADIX_BINS / 64 consecutive bins, a
// wave prefix sum of the lanes' totals finds the lane whose bins contain the
// rank, that lane resolves the bin; the histogram is then cleared for the
// next pass.
__global__ __launch_bounds__(128) void radix_select_kernel(uint32_t *sel, uint32_t *hist,
                                                           int shift, int bits) {
  constexpr int PL = RADIX_BINS / 64;
  const int t = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t *s = sel + 3 * t;
  uint32_t *h = hist + RADIX_BINS * t + PL * lane;
  const uint32_t k = s[2];
  uint32_t bins[PL];
  uint32_t own = 0;
#pragma unroll
  for (int e = 0; e < PL; ++e) own += (bins[e] = h[e]);
  uint32_t incl = own;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  const unsigned long long hit = __ballot(incl > k);
  const int first = hit ? __ffsll(hit) - 1 : 63;
  if (lane == first) {
    uint32_t r = k - (incl - own);
    int e = 0;
    for (; e < PL - 1; ++e) {
      if (r < bins[e]) break;
      r -= bins[e];
    }
    const uint32_t b = uint32_t(PL * lane + e);
    s[0] |= b << shift;
    s[1] |= ((1u << bits) - 1u) << shift;
    s[2] = r;
  }
#pragma unroll
  for (int e = 0; e < PL; ++e) h[e] = 0;
}

__global__ void bandwidth_kernel(const uint32_t *sel, long long count, int n, int mode,
                                 double h_fixed, double *h2, double *h2_out) {
  double v;
  if (mode == VIP_BW_FIXED) {
    v = h_fixed * h_fixed;
  } else {
    double med = 0.0;
    if (count > 0) {
      double a = double(__uint_as_float(sel[0])), b = double(__uint_as_float(sel[3]));
      med = (count % 2 == 1) ? b : 0.5 * (a + b);
    }
    v = (med == 0.0) ? 1.0 : med / (2.0 * log(double(n) + 1.0));
  }
  h2[0] = v;
  if (h2_out) h2_out[0] = v;
}

// ---- kernel matrix and row sums ---------------------------------------------
// With khi non-null the row is also written in BF16 (bf16(k), rounded to
// nearest even) in rows of ldk, zero past column n.
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
__global__ __launch_bounds__(256) void rbf_kernel(const float *D, const double *h2, float *K,
                                                  float *s, int n, uint16_t *khi, int ldk) {
  __shared__ double part[4];
  const int i = blockIdx.x;
  const float inv = float(1.0 / (2.0 * h2[0]));
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    float k = expf(-D[(long long)i * n + j] * inv);
    K[(long long)i * n + j] = k;
    acc += double(k);
    if (khi) khi[(long long)i * ldk + j] = f32_to_bf16_rne(k);
  }
  if (khi)
    for (int j = n + int(threadIdx.x); j < ldk; j += 256) khi[(long long)i * ldk + j] = 0;
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) s[i] = float((part[0] + part[1]) + (part[2] + part[3]));
}

// ---- Cholesky of K/n in FP64, one workgroup, matrix in LDS ---------------------
// Right-looking: for each column k, sqrt of the pivot, scale the column below,
// rank-1 update of the trailing lower triangle.  On a non-positive pivot, start
// again from K/n + delta I, delta = 1e-12 trace(K/n)/n, x10 per retry.
constexpr int kCholMax = 128;

__global__ __launch_bounds__(1024) void cholesky_kernel(const float *D, const double *h2, double *L,
                                                        float *LfT, int n, int max_retries,
                                                        uint32_t *status) {
  __shared__ double A[kCholMax][kCholMax + 1];
  __shared__ int fail;
  const int t = threadIdx.x, nt = blockDim.x;
  const double inv2h2 = 1.0 / (2.0 * h2[0]);
  const double invn = 1.0 / double(n);
  double delta = 1e-12 * (double(n) * invn) / double(n);   // trace(K/n)/n with K_ii = 1
  int attempt = 0;
  for (; attempt <= max_retries; ++attempt) {
    const double jit = attempt == 0 ? 0.0 : delta;
    for (int e = t; e < n * n; e += nt) {
      int i = e / n, j = e - (e / n) * n;
      double v = exp(-double(D[e]) * inv2h2) * invn;
      A[i][j] = (i == j) ? v + jit : v;
    }
    if (t == 0) fail = 0;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
      if (t == 0) {
        double p = A[k][k];
        if (!(p > 0.0)) fail = 1;
        A[k][k] = p > 0.0 ? sqrt(p) : 1.0;
      }
      __syncthreads();
      if (fail) break;
      const double piv = A[k][k];
      for (int i = k + 1 + t; i < n; i += nt) A[i][k] /= piv;
      __syncthreads();
      const int m = n - k - 1;
      for (int e = t; e < m * m; e += nt) {
        int i = k + 1 + e / m, j = k + 1 + e % m;
        if (j <= i) A[i][j] -= A[i][k] * A[j][k];
      }
      __syncthreads();
    }
    __syncthreads();
    if (!fail) break;
    if (attempt > 0) delta *= 10.0;
    __syncthreads();
  }
  const bool ok = !fail;
  if (t == 0) {
    if (!ok) atomicOr(status, VIP_FLAG_NOT_PD);
    else if (attempt > 0) atomicOr(status, VIP_FLAG_JITTER);
  }
  for (int e = t; e < n * n; e += nt) {
    int i = e / n, j = e - (e / n) * n;
    double v = (ok && j <= i) ? A[i][j] : 0.0;
    L[e] = v;
    LfT[(long long)j * n + i] = float(v);
  }
}

// ---- blocked Cholesky of K/n in FP64 for n > kCholMax --------------------------
// Right-looking over panels of CB columns.  Per panel k0, chol_panel_kernel:
// wave 0 of every block factors the CB x CB diagonal block with one row per
// lane in registers (column k's entries broadcast with readlane, no barriers),
// then inverts it (one column of L11^-1 per lane, L11 read from LDS); block 0
// writes L11 back, the other blocks each form 64 rows of the panel below,
// L21 = A21 L11^-T, as a small product.  chol_update_kernel then subtracts
// L21 L21^T from the trailing lower triangle in 64 x 64 tiles.  A
// non-positive pivot sets state[0], after which every later kernel of the
// attempt returns at once; chol_retry_kernel then repeats the factorisation
// with the jitter protocol of the one-workgroup kernel (delta = 1e-12
// trace(K/n)/n, x10 per retry) in a single workgroup over the matrix in global
// memory -- the path of (numerically) coincident particles, which trades speed
// for simplicity.  chol_output_kernel writes L (zero above the diagonal, all
// zero if every retry failed) and its FP32 copy.
constexpr int CB = 32;        // panel width
constexpr int CR = 64;        // panel rows per block below the diagonal block

// A = K/n + jit I on and below the diagonal, 0 above; state[0..1] cleared.
__global__ void chol_init_kernel(const float *D, const double *h2, double *A, int n, double jit,
                                 uint32_t *state) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) state[0] = state[1] = 0u;
  if (e >= (long long)n * n) return;
  const int i = int(e / n), j = int(e - (e / n) * n);
  double v = 0.0;
  if (j <= i) {   // the same FP64 K/n as the one-workgroup kernel
    v = exp(-double(D[e]) * (1.0 / (2.0 * h2[0]))) * (1.0 / double(n));
    if (i == j) v += jit;
  }
  A[e] = v;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane(unsigned(b), lane);
  const unsigned hi = __builtin_amdgcn_readlane(unsigned(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__global__ __launch_bounds__(256) void chol_panel_kernel(double *A, int n, int k0,
                                                         uint32_t *state) {
  __shared__ double Ls[CB][CB + 1];   // L11
  __shared__ double Li[CB][CB + 1];   // L11^-1 (lower)
  __shared__ double As[CR][CB + 1];   // this block's rows of A21
  __shared__ int bad;
  const int t = threadIdx.x;
  const int b = min(CB, n - k0);
  const int r0 = k0 + CB + (int(blockIdx.x) - 1) * CR;   // first A21 row (blocks >= 1)
  // the failure flag is read together with the block's first loads (all of
  // them read A only), so that the two latencies overlap
  const uint32_t failed = state[0];
  // lane i < CB of wave 0 holds row i of the diagonal block (identity beyond
  // the matrix); lanes CB.. repeat row CB - 1 and are never read
  const int i = t < CB ? t : CB - 1;
  double r[CB];
  if (t < 64) {
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      double v = i == j ? 1.0 : 0.0;
      if (i < b && j < b && j <= i) v = A[(long long)(k0 + i) * n + k0 + j];
      r[j] = v;
    }
  }
  if (blockIdx.x > 0) {   // stage A21 while wave 0 factors (unrolled: all loads in flight at once)
    constexpr int SE = CR * CB / 256;
    double v[SE];
#pragma unroll
    for (int q = 0; q < SE; ++q) {
      const int e = t + 256 * q, r = e / CB, k = e - (e / CB) * CB;
      v[q] = r0 + r < n ? A[(long long)(r0 + r) * n + k0 + k] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < SE; ++q) {
      const int e = t + 256 * q, r = e / CB, k = e - (e / CB) * CB;
      As[r][k] = v[q];
    }
  }
  if (failed) return;   // uniform over the block
  if (t < 64) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < CB; ++k) {
      const double p = readlane_f64(r[k], k);   // the pivot, uniform
      ok = ok && p > 0.0;
      // sqrt(p) and the column's division by it both through 1/sqrt(p), the
      // hardware estimate refined by two Newton steps, so that the step's
      // dependency chain holds no square root or division
      const double pp = p > 0.0 ? p : 1.0;
      double rs = __builtin_amdgcn_rsq(pp);
#pragma unroll
      for (int it = 0; it < 2; ++it) rs = fma(0.5 * rs, fma(-pp * rs, rs, 1.0), rs);
      const double piv = pp * rs;
      const double l = r[k] * rs;
      r[k] = i == k ? piv : (i > k ? l : r[k]);
#pragma unroll
      for (int j = k + 1; j < CB; ++j) r[j] = fma(-r[k], readlane_f64(r[k], j), r[j]);
    }
    if (t < CB) {
#pragma unroll
      for (int j = 0; j < CB; ++j) Ls[t][j] = j <= t ? r[j] : 0.0;
    }
    if (t == 0) bad = ok ? 0 : 1;
    if (blockIdx.x == 0 && ok && t < b) {
#pragma unroll
      for (int j = 0; j < CB; ++j)
        if (j <= t && j < b) A[(long long)(k0 + t) * n + k0 + j] = r[j];
    }
  }
  __syncthreads();
  if (bad) {
    if (blockIdx.x == 0 && t == 0) atomicOr(state, 1u);
    return;
  }
  if (blockIdx.x == 0) return;
  if (t < CB) {
    // column j = t of L11^-1: L11 x = e_j by forward substitution, each
    // diagonal reciprocal formed outside the chain from x[0] to x[CB - 1]
    double x[CB];
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      const double rdq = 1.0 / Ls[q][q];
      double v = q == t ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < q; ++m) v = fma(-Ls[q][m], x[m], v);
      x[q] = v * rdq;
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) Li[q][t] = x[q];
  }
  __syncthreads();
  // X = A21 L11^-T: thread t gives row t / 4, columns 8 (t % 4) .. + 7
  const int rr = t >> 2, c0 = (t & 3) * 8;
  double acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = 0.0;
#pragma unroll 8
  for (int m = 0; m < CB; ++m) {
    const double a = As[rr][m];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = fma(a, Li[c0 + c][m], acc[c]);
  }
  if (r0 + rr < n) {
#pragma unroll
    for (int c = 0; c < 8; ++c) A[(long long)(r0 + rr) * n + k0 + c0 + c] = acc[c];
  }
}

// Trailing update A22 -= L21 L21^T on the lower triangle, 64 x 64 tiles (tile
// (ti, tj) with tj <= ti), 256 threads with 4 x 4 outputs each.
__global__ __launch_bounds__(256) void chol_update_kernel(double *A, int n, int k0,
                                                          uint32_t *state) {
  __shared__ double Li[64][CB + 1], Lj[64][CB + 1];
  const int r0 = k0 + CB;
  const int b = CB;   // update panels are always full: a short last panel has no trailing part
  // lower-triangle tile of this block: tb = ti (ti + 1) / 2 + tj
  const int tb = blockIdx.x;
  int ti = int((sqrt(8.0 * tb + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= tb) ++ti;
  while (ti * (ti + 1) / 2 > tb) --ti;
  const int tj = tb - ti * (ti + 1) / 2;
  const int i0 = r0 + 64 * ti, j0 = r0 + 64 * tj;
  const int t = threadIdx.x;
  const int ty = t >> 4, tx = t & 15;
  // the failure flag, the panel columns and this thread's old trailing
  // entries are all read up front (the staging loop unrolled), so that their
  // latencies overlap
  const uint32_t failed = state[0];
  constexpr int SE = 64 * CB / 256;   // staged elements per thread and operand
  double vi[SE], vj[SE];
#pragma unroll
  for (int q = 0; q < SE; ++q) {
    const int e = t + 256 * q, r = e / CB, k = e - (e / CB) * CB;
    vi[q] = i0 + r < n ? A[(long long)(i0 + r) * n + k0 + k] : 0.0;
    vj[q] = j0 + r < n ? A[(long long)(j0 + r) * n + k0 + k] : 0.0;
  }
  double old[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + ty + 16 * r;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + tx + 16 * c;
      old[r][c] = (i < n && j <= i) ? A[(long long)i * n + j] : 0.0;
    }
  }
  if (failed) return;   // uniform over the block
#pragma unroll
  for (int q = 0; q < SE; ++q) {
    const int e = t + 256 * q, r = e / CB, k = e - (e / CB) * CB;
    Li[r][k] = vi[q];
    Lj[r][k] = vj[q];
  }
  __syncthreads();
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
#pragma unroll 4
  for (int k = 0; k < b; ++k) {
    double a[4], bb[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[r] = Li[ty + 16 * r][k];
      bb[r] = Lj[tx + 16 * r][k];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], bb[c], acc[r][c]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + ty + 16 * r;
    if (i >= n) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + tx + 16 * c;
      if (j <= i && j < n) A[(long long)i * n + j] = old[r][c] - acc[r][c];
    }
  }
}

// After a failed blocked attempt: the jitter retries in one workgroup over the
// matrix in global memory (right-looking, column by column).  state[1] = 1
// when every retry failed.
__global__ __launch_bounds__(1024) void chol_retry_kernel(const float *D, const double *h2,
                                                          double *A, int n, int max_retries,
                                                          uint32_t *state, uint32_t *status) {
  __shared__ int fail;
  if (!state[0]) return;   // the blocked attempt succeeded
  const int t = threadIdx.x, nt = blockDim.x;
  const double inv2h2 = 1.0 / (2.0 * h2[0]);
  const double invn = 1.0 / double(n);
  double delta = 1e-12 * (double(n) * invn) / double(n);   // trace(K/n)/n with K_ii = 1
  bool ok = false;
  int attempt = 1;
  for (; attempt <= max_retries; ++attempt) {
    for (long long e = t; e < (long long)n * n; e += nt) {
      const int i = int(e / n), j = int(e - (e / n) * n);
      double v = 0.0;
      if (j <= i) v = exp(-double(D[e]) * inv2h2) * invn + (i == j ? delta : 0.0);
      A[e] = v;
    }
    if (t == 0) fail = 0;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
      if (t == 0) {
        const double p = A[(long long)k * n + k];
        if (!(p > 0.0)) fail = 1;
        A[(long long)k * n + k] = p > 0.0 ? sqrt(p) : 1.0;
      }
      __syncthreads();
      if (fail) break;
      const double piv = A[(long long)k * n + k];
      for (int i = k + 1 + t; i < n; i += nt) A[(long long)i * n + k] /= piv;
      __syncthreads();
      const long long m = n - k - 1;
      for (long long e = t; e < m * m; e += nt) {
        const int i = k + 1 + int(e / m), j = k + 1 + int(e % m);
        if (j <= i) A[(long long)i * n + j] -= A[(long long)i * n + k] * A[(long long)j * n + k];
      }
      __syncthreads();
    }
    __syncthreads();
    if (!fail) {
      ok = true;
      break;
    }
    delta *= 10.0;
    __syncthreads();
  }
  if (t == 0) {
    if (ok) atomicOr(status, VIP_FLAG_JITTER);
    else atomicOr(status, VIP_FLAG_NOT_PD);
    state[1] = ok ? 0u : 1u;
  }
}

// L = the factor (lower part; all zero after a failure) in FP64, and its FP32
// copy transposed (LfT[j][i] = L[i][j], the layout the noise product stages).
// Each element of A is read and rewritten by the thread that writes its
// transposed copy.
// With L16 set (the BF16 noise product) it writes instead the row-major BF16
// pair of L: L16[i n + j] = hi = bf16(L[i][j]), L16[n^2 + i n + j] =
// bf16(L[i][j] - hi), each thread on one element in row-major order.
__global__ void chol_output_kernel(double *A, float *LfT, uint16_t *L16, int n,
                                   const uint32_t *state) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nn = (long long)n * n;
  if (e >= nn) return;
  if (L16) {
    const int i = int(e / n), j = int(e - (e / n) * n);   // e = i n + j
    const double v = (j <= i && !state[1]) ? A[e] : 0.0;
    A[e] = v;
    const uint16_t h = f32_to_bf16_rne(float(v));
    L16[e] = h;
    L16[nn + e] = f32_to_bf16_rne(float(v - double(bf16_to_f32(h))));
    return;
  }
  const int j = int(e / n), i = int(e - (e / n) * n);   // e = j n + i
  double *a = A + (long long)i * n + j;
  const double v = (j <= i && !state[1]) ? *a : 0.0;
  *a = v;
  LfT[e] = float(v);
}

__global__ void philox_fill_kernel(float *out, long long count, uint32_t k0, uint32_t k1,
                                   uint32_t s0, uint32_t s1) {
  long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (4 * q >= count) return;
  float z[4];
  philox_normals4(uint64_t(q), k0, k1, s0, s1, z);
  for (int k = 0; k < 4; ++k)
    if (4 * q + k < count) out[4 * q + k] = z[k];
}

// The same update (without noise) with the product on the FP32 matrix cores
// (v_mfma_f32_32x32x2_f32: lane l holds A[l % 32][l / 32] and B[l / 32][l % 32];
// result register r of lane l is C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]).
// Block: 256 particles x 128 coordinates, 8 waves (4 x 2) of 2 x 2 tiles of
// 32 x 32; the particle index j of the product runs in stages of 16 through
// LDS, the next stage's tiles prefetched into registers during the current
// one.  K is symmetric (bitwise: G is mirrored and D_ij, D_ji add the same two
// diagonal terms), so the A tile K[i][j0 + k] is read as rows j0 + k of K.
// Blocks that share a column range are consecutive per XCD, so its B tiles
// meet in one L2.
constexpr int UM = 256, UN = 128, UK = 16, UP = 4, UT = 512;
template <bool RULE>
__global__ __launch_bounds__(UT) void update_mfma_kernel(const float *K, const float *g,
                                                         const float *xc, const float *vq,
                                                         const float *s,
                                                         const double *h2, float *x, float *phi,
                                                         const float *lo, const float *hi, int n,
                                                         long long d, int mblocks, int vec,
                                                         float eps, OptArgs opt, uint32_t *status) {
  __shared__ __attribute__((aligned(16))) float As[UK][UM + UP];   // As[k][i] = K[i][j0 + k]
  __shared__ __attribute__((aligned(16))) float Bs[UK][UN + UP];   // Bs[k][a] = B[j0 + k][a0 + a]
  // tile index, contiguous per XCD (blocks are dealt round-robin over 8 XCDs)
  const int per = int(gridDim.x) >> 3;
  const int tb = (int(blockIdx.x) & 7) * per + (int(blockIdx.x) >> 3);
  const int nt = mblocks * int((d + UN - 1) / UN);
  if (tb >= nt) return;
  const int i0 = (tb % mblocks) * UM;
  const long long a0 = (long long)(tb / mblocks) * UN;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;
  const float inv_h2 = float(1.0 / h2[0]);

  // staging: A rows k = t / 64 + 8 e (e = 0, 1), columns 4 (t % 64); B row
  // k = t / 32, columns 4 (t % 32)
  const int ak = t >> 6, ac = (t & 63) * 4;
  const int bk = t >> 5, bc = (t & 31) * 4;
  float4 pa[2], pg, px;
  auto load4 = [&](const float *base, long long off, long long lim) {
    if (vec && off + 3 < lim) return *reinterpret_cast<const float4 *>(base + off);
    float tmp[4];
    for (int q = 0; q < 4; ++q) tmp[q] = (off + q < lim) ? base[off + q] : 0.f;
    return make_float4(tmp[0], tmp[1], tmp[2], tmp[3]);
  };
  auto load_stage = [&](int j0) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int j = j0 + ak + 8 * e;
      pa[e] = j < n ? load4(K + (long long)j * n, i0 + ac, n) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const int j = j0 + bk;
    pg = px = make_float4(0.f, 0.f, 0.f, 0.f);
    if (j < n) {
      pg = load4(g + (long long)j * d, a0 + bc, d);
      px = load4(xc + (long long)j * d, a0 + bc, d);
      if (vq) {   // diagonal kernel: Q^-1 g
        const float4 w = load4(vq, a0 + bc, d);
        pg.x *= w.x;
        pg.y *= w.y;
        pg.z *= w.z;
        pg.w *= w.w;
      }
    }
  };
  auto store_stage = [&]() {
#pragma unroll
    for (int e = 0; e < 2; ++e) *reinterpret_cast<float4 *>(&As[ak + 8 * e][ac]) = pa[e];
    float4 bv;
    bv.x = fmaf(-px.x, inv_h2, pg.x);
    bv.y = fmaf(-px.y, inv_h2, pg.y);
    bv.z = fmaf(-px.z, inv_h2, pg.z);
    bv.w = fmaf(-px.w, inv_h2, pg.w);
    *reinterpret_cast<float4 *>(&Bs[bk][bc]) = bv;
  };

  f32x16_t acc[2][2];
  for (int m = 0; m < 2; ++m)
    for (int q = 0; q < 2; ++q)
      for (int r = 0; r < 16; ++r) acc[m][q][r] = 0.0f;
  load_stage(0);
  for (int j0 = 0; j0 < n; j0 += UK) {
    __syncthreads();               // the previous stage's tiles are no longer read
    store_stage();
    __syncthreads();
    if (j0 + UK < n) load_stage(j0 + UK);
#pragma unroll
    for (int kk = 0; kk < UK; kk += 2) {
      const int k = kk + (lane >> 5);
      float fa[2], fb[2];
      for (int m = 0; m < 2; ++m) fa[m] = As[k][wi * 64 + m * 32 + (lane & 31)];
      for (int q = 0; q < 2; ++q) fb[q] = Bs[k][wj * 64 + q * 32 + (lane & 31)];
      for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 2; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[m], fb[q], acc[m][q], 0, 0, 0);
    }
  }

  const float inv_n = 1.0f / float(n);
  bool bad = false;
  if constexpr (RULE) {
    // a step rule with per-coordinate state: one element at a time
    for (int m = 0; m < 2; ++m)
      for (int r = 0; r < 16; ++r) {
        const int i = i0 + wi * 64 + m * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (i >= n) continue;
        const float si = s[i] * inv_h2;
        for (int q = 0; q < 2; ++q) {
          const long long a = a0 + wj * 64 + q * 32 + (lane & 31);
          if (a >= d) continue;
          const long long e = (long long)i * d + a;
          const float p = fmaf(si, xc[e], acc[m][q][r]) * inv_n;
          phi[e] = p;
          float v = x[e] + opt_step(opt, e, p, eps);
          if (lo) v = fminf(fmaxf(v, lo[a]), hi[a]);
          bad |= !isfinite(v);
          x[e] = v;
        }
      }
  } else {
    // Plain steps, four result registers (eight elements) at a time: the
    // batch's loads of xc and x are all issued before its stores (which could
    // alias them as far as the compiler knows).  Register r of sub-tile m is
    // row 8 (r / 4) + r % 4 + m 32 past my first.
    const int lrow = wi * 64 + 4 * (lane >> 5);
    const int lcol = wj * 64 + (lane & 31);
    const long long el = (long long)(i0 + lrow) * d + a0 + lcol;
    float lov[2], hiv[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const long long a = a0 + lcol + q * 32;
      lov[q] = (lo && a < d) ? lo[a] : 0.0f;
      hiv[q] = (lo && a < d) ? hi[a] : 0.0f;
    }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int rb = 0; rb < 16; rb += 4) {
        float xv[4][2], cv[4][2], si[4];
        // unconditional loads (elements outside the ensemble read element 0
        // and are never used), so no branch separates them
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int r = rb + rr, lr = m * 32 + 8 * (r >> 2) + (r & 3);
          const int i = i0 + lrow + lr;
          si[rr] = s[i < n ? i : 0];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const bool in = i < n && a0 + lcol + q * 32 < d;
            const long long e = in ? el + (long long)lr * d + q * 32 : 0;
            xv[rr][q] = x[e];
            cv[rr][q] = xc[e];
          }
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int r = rb + rr, lr = m * 32 + 8 * (r >> 2) + (r & 3);
          if (i0 + lrow + lr >= n) continue;
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            if (a0 + lcol + q * 32 >= d) continue;
            const long long e = el + (long long)lr * d + q * 32;
            const float p = fmaf(si[rr] * inv_h2, cv[rr][q], acc[m][q][r]) * inv_n;
            phi[e] = p;
            float v = xv[rr][q] + eps * p;
            if (lo) v = fminf(fmaxf(v, lov[q]), hiv[q]);
            bad |= !isfinite(v);
            x[e] = v;
          }
        }
      }
  }
  if (bad) atomicOr(status, VIP_FLAG_NONFINITE);
}

// Noise epilogue shared by the noise kernels: x <- clip(x + scale sqrt(vq) acc)
// for the block's 256 x 128 results (wave (wi, wj) holds rows wi 64 .., columns
// wj 64 .. as 2 x 2 tiles of 32 x 32 in the matrix-core result layout), in
// batches of four result registers, loads before stores.
__device__ __forceinline__ void noise_epilogue(const f32x16_t (&acc)[2][2], int i0, long long a0,
                                               int wi, int wj, int lane, const float *vq,
                                               float *x, const float *lo, const float *hi, int n,
                                               long long d, float scale, uint32_t *status) {
  const int lrow = wi * 64 + 4 * (lane >> 5);
  const int lcol = wj * 64 + (lane & 31);
  const long long el = (long long)(i0 + lrow) * d + a0 + lcol;
  float sc[2], lov[2], hiv[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const long long a = a0 + lcol + q * 32;
    sc[q] = (vq && a < d) ? scale * sqrtf(vq[a]) : scale;
    lov[q] = (lo && a < d) ? lo[a] : 0.0f;
    hiv[q] = (lo && a < d) ? hi[a] : 0.0f;
  }
  bool bad = false;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int rb = 0; rb < 16; rb += 4) {
      float xv[4][2];
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int r = rb + rr, lr = m * 32 + 8 * (r >> 2) + (r & 3);
        const int i = i0 + lrow + lr;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const bool in = i < n && a0 + lcol + q * 32 < d;
          xv[rr][q] = x[in ? el + (long long)lr * d + q * 32 : 0];
        }
      }
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int r = rb + rr, lr = m * 32 + 8 * (r >> 2) + (r & 3);
        if (i0 + lrow + lr >= n) continue;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (a0 + lcol + q * 32 >= d) continue;
          float v = fmaf(sc[q], acc[m][q][r], xv[rr][q]);
          if (lo) v = fminf(fmaxf(v, lov[q]), hiv[q]);
          bad |= !isfinite(v);
          x[el + (long long)lr * d + q * 32] = v;
        }
      }
    }
  if (bad) atomicOr(status, VIP_FLAG_NONFINITE);
}

// The sSVGD noise on the FP32 matrix cores, after the update has added eps phi
// (without the clip): x <- clip(x + sqrt(2 eps) sqrt(vq) (L Xi)) per element,
// vq = 1 / q of the diagonal matrix kernel (or 1).  Same blocks, staging and
// layouts as update_mfma_kernel, with A = L and B = Xi: the A tile
// As[k][i] = L[i0 + i][j0 + k] is a row segment of the transposed FP32 copy
// LfT, and since L is lower triangular a block of rows i0 .. i0 + UM - 1 takes
// j < i0 + UM only (about half the product overall).  A block's work grows
// with its row block, so the blocks go out longest first: XCD x = blockIdx % 8
// owns the column blocks [x nc / 8, (x + 1) nc / 8), and its k-th block takes
// row block mblocks - 1 - k / ncx, column block k % ncx of that range (the
// grid is 8 mblocks ceil(nc / 8) blocks).
__global__ __launch_bounds__(UT) void noise_mfma_kernel(const float *LfT, const float *xi,
                                                        const float *vq, float *x,
                                                        const float *lo, const float *hi, int n,
                                                        long long d, int mblocks, int vec,
                                                        float scale, uint32_t *status) {
  __shared__ __attribute__((aligned(16))) float As[UK][UM + UP];   // As[k][i] = L[i0 + i][j0 + k]
  __shared__ __attribute__((aligned(16))) float Bs[UK][UN + UP];   // Bs[k][a] = Xi[j0 + k][a0 + a]
  const long long nc = (d + UN - 1) / UN;
  const int xcd = int(blockIdx.x) & 7, kb = int(blockIdx.x) >> 3;
  const long long cb0 = xcd * nc / 8;
  const int ncx = int((xcd + 1) * nc / 8 - cb0);
  if (kb >= mblocks * ncx) return;
  const int i0 = (mblocks - 1 - kb / ncx) * UM;
  const long long a0 = (cb0 + kb % ncx) * UN;
  const int jend = min(n, i0 + UM);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;
  const int ak = t >> 6, ac = (t & 63) * 4;
  const int bk = t >> 5, bc = (t & 31) * 4;
  float4 pa[2], pb;
  auto load4 = [&](const float *base, long long off, long long lim) {
    if (vec && off + 3 < lim) return *reinterpret_cast<const float4 *>(base + off);
    float tmp[4];
    for (int q = 0; q < 4; ++q) tmp[q] = (off + q < lim) ? base[off + q] : 0.f;
    return make_float4(tmp[0], tmp[1], tmp[2], tmp[3]);
  };
  auto load_stage = [&](int j0) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int j = j0 + ak + 8 * e;
      pa[e] = j < jend ? load4(LfT + (long long)j * n, i0 + ac, n) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const int j = j0 + bk;
    pb = j < jend ? load4(xi + (long long)j * d, a0 + bc, d) : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  auto store_stage = [&]() {
#pragma unroll
    for (int e = 0; e < 2; ++e) *reinterpret_cast<float4 *>(&As[ak + 8 * e][ac]) = pa[e];
    *reinterpret_cast<float4 *>(&Bs[bk][bc]) = pb;
  };
  f32x16_t acc[2][2];
  for (int m = 0; m < 2; ++m)
    for (int q = 0; q < 2; ++q)
      for (int r = 0; r < 16; ++r) acc[m][q][r] = 0.0f;
  load_stage(0);
  for (int j0 = 0; j0 < jend; j0 += UK) {
    __syncthreads();
    store_stage();
    __syncthreads();
    if (j0 + UK < jend) load_stage(j0 + UK);
#pragma unroll
    for (int kk = 0; kk < UK; kk += 2) {
      const int k = kk + (lane >> 5);
      float fa[2], fb[2];
      for (int m = 0; m < 2; ++m) fa[m] = As[k][wi * 64 + m * 32 + (lane & 31)];
      for (int q = 0; q < 2; ++q) fb[q] = Bs[k][wj * 64 + q * 32 + (lane & 31)];
      for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 2; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[m], fb[q], acc[m][q], 0, 0, 0);
    }
  }
  noise_epilogue(acc, i0, a0, wi, wj, lane, vq, x, lo, hi, n, d, scale, status);
}

// The same noise on the BF16 matrix cores, for the BF16 path beyond one
// workgroup's Cholesky: L and Xi are each split into a BF16 pair (v = hi + lo,
// hi = bf16(v), lo = bf16(v - hi)) and L Xi ~ Lh Xh + Lh Xl + Ll Xh, three
// products with FP32 accumulation (the dropped Ll Xl and the rounding of the
// pairs leave about 2^-16 relative per term).  L comes as its row-major BF16
// pair (Lh[i][j], then Ll), written by the Cholesky's output kernel; Xi is
// FP32 and split while it is staged.  Blocks, their order (longest first) and
// the epilogue are those of noise_mfma_kernel.  Per stage of NK = 32 steps of
// j both operands sit in LDS with k contiguous, in rows of NAP ushorts (16-byte
// fragment reads at a pitch of 20 dwords hit every bank once per 16 lanes):
// the A rows are copied as 16-byte chunks, and a thread loads 4 consecutive j
// of one Xi column (each load one coalesced row segment over the wave), splits
// them and writes them as one 8-byte run of its column's row.
constexpr int NK = 32, NAP = NK + 8;
__global__ __launch_bounds__(UT) __attribute__((amdgpu_waves_per_eu(4, 4))) void noise_bf16x3_kernel(const uint16_t *L16, const float *xi,
                                                          const float *vq, float *x,
                                                          const float *lo, const float *hi, int n,
                                                          long long d, int mblocks, int vec,
                                                          float scale, uint32_t *status) {
  __shared__ __attribute__((aligned(16))) uint16_t Ah[UM][NAP], Al[UM][NAP];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[UN][NAP], Bl[UN][NAP];
  const long long nc = (d + UN - 1) / UN;
  const int xcd = int(blockIdx.x) & 7, kb = int(blockIdx.x) >> 3;
  const long long cb0 = xcd * nc / 8;
  const int ncx = int((xcd + 1) * nc / 8 - cb0);
  if (kb >= mblocks * ncx) return;
  const int i0 = (mblocks - 1 - kb / ncx) * UM;
  const long long a0 = (cb0 + kb % ncx) * UN;
  const int jend = min(n, i0 + UM);
  const long long nn = (long long)n * n;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;
  // staging: A chunk c = t + UT it (it < 4) is part c / 1024 (0: hi, 1: lo),
  // row (c % 1024) / 4, 8 values from j0 + 8 (c % 4); B group it (< 2) of
  // thread t is column t % 128, steps 16 it + 4 (t / 128) .. + 3
  uint4 pa[4];
  float4 pb[2];
  auto load_a = [&](int j0) {
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int c = t + UT * it, part = c >> 10, row = (c & 1023) >> 2, j = j0 + 8 * (c & 3);
      const int i = i0 + row;
      const uint16_t *src = L16 + part * nn + (long long)i * n + j;
      if (vec && i < n && j + 7 < n) {
        pa[it] = *reinterpret_cast<const uint4 *>(src);
      } else {
        uint32_t v[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (i < n && j + e < n) v[e >> 1] |= uint32_t(src[e]) << (16 * (e & 1));
        pa[it] = make_uint4(v[0], v[1], v[2], v[3]);
      }
    }
  };
  auto load_b = [&](int j0) {
    const long long a = a0 + (t & (UN - 1));
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int jb = j0 + 16 * it + 4 * (t >> 7);
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = (jb + e < n && a < d) ? xi[(long long)(jb + e) * d + a] : 0.0f;
      pb[it] = make_float4(v[0], v[1], v[2], v[3]);
    }
  };
  auto store_a = [&]() {
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int c = t + UT * it, part = c >> 10, row = (c & 1023) >> 2, ch = c & 3;
      uint16_t *dst = part ? &Al[row][8 * ch] : &Ah[row][8 * ch];
      *reinterpret_cast<uint4 *>(dst) = pa[it];
    }
  };
  auto store_b = [&]() {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int col = t & (UN - 1), k = 16 * it + 4 * (t >> 7);
      const float v[4] = {pb[it].x, pb[it].y, pb[it].z, pb[it].w};
      uint32_t h[2] = {0u, 0u}, l[2] = {0u, 0u};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint16_t hb = f32_to_bf16_rne(v[e]);
        const uint16_t lb = f32_to_bf16_rne(v[e] - bf16_to_f32(hb));
        h[e >> 1] |= uint32_t(hb) << (16 * (e & 1));
        l[e >> 1] |= uint32_t(lb) << (16 * (e & 1));
      }
      *reinterpret_cast<uint2 *>(&Bh[col][k]) = make_uint2(h[0], h[1]);
      *reinterpret_cast<uint2 *>(&Bl[col][k]) = make_uint2(l[0], l[1]);
    }
  };
  f32x16_t acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[m][q][r] = 0.0f;
  for (int j0 = 0; j0 < jend; j0 += NK) {
    // no prefetch into registers: two blocks share a compute unit, and one
    // block's staging overlaps the other's products
    load_a(j0);
    __syncthreads();
    store_a();
    load_b(j0);
    store_b();
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < NK; ks += 16) {
      const int kq = ks + 8 * (lane >> 5);
      // fragments as the products need them (24 registers live, not 32): the
      // three products in turns over the four tiles, so that no product waits
      // on the one just issued into the same accumulator
      bf16x8_t fa[2], fbh[2], fbl[2];
      auto afrag = [&](const uint16_t (*A)[NAP], int m) {
        const uint4 r = *reinterpret_cast<const uint4 *>(&A[wi * 64 + m * 32 + (lane & 31)][kq]);
        bf16x8_t f;
        __builtin_memcpy(&f, &r, 16);
        return f;
      };
      auto bfrag = [&](const uint16_t (*B)[NAP], int q) {
        const uint4 r = *reinterpret_cast<const uint4 *>(&B[wj * 64 + q * 32 + (lane & 31)][kq]);
        bf16x8_t f;
        __builtin_memcpy(&f, &r, 16);
        return f;
      };
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        fa[e] = afrag(Al, e);
        fbh[e] = bfrag(Bh, e);
      }
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[m], fbh[q], acc[m][q], 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        fa[e] = afrag(Ah, e);
        fbl[e] = bfrag(Bl, e);
      }
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[m], fbl[q], acc[m][q], 0, 0, 0);
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[m], fbh[q], acc[m][q], 0, 0, 0);
    }
  }
  noise_epilogue(acc, i0, a0, wi, wj, lane, vq, x, lo, hi, n, d, scale, status);
}

// The same update with the product K B on the BF16 matrix cores: K rounded to
// BF16 (the precision its distances come from on this path), and the FP32 B
// split into a BF16 pair B = hi + lo (hi = bf16(B), lo = bf16(B - hi)), the
// product taken as K hi + K lo.  The rounding of K alone contributes about
// 4e-5 relative L2 to phi at n = 2048 (an FP64 emulation on the c5 inputs
// with the exact K: 2.4e-6 with K split as well, 1.6e-3 with B not split), a
// fraction of what the BF16 Gram already puts into K through the distances;
// this is the update of the BF16 path.
//
// bpair_kernel forms B = G Q^-1 - Xc / h^2 once (Xc = x - xbar recomputed, the
// centring kernel does not store it on this path) and splits it.  Rows j and
// j + 1 are packed into one 32-bit pair (the k order of a matrix-core
// operand), and four consecutive pairs of one column are stored together:
// word r of column a in group q (rows 8q .. 8q + 7) sits at (q dp + a) 4 + r,
// so that a 16-byte load gives one lane's fragment of 8 k.  Rows are padded
// with zeros to ldk and columns to dp.
// Grid: y = group q, x = 256 columns per block, one per thread (each load
// instruction of a wave reads 256 contiguous bytes of a row, each store
// writes 1 KB contiguous).
__global__ __launch_bounds__(256) void bpair_kernel(const float *g, const float *x,
                                                    const float *xbar, const float *vq,
                                                    const double *h2,
                                                    uint32_t *bph, uint32_t *bpl, int n,
                                                    long long d, long long dp) {
  const int q = int(blockIdx.y);
  const long long a = (long long)blockIdx.x * 256 + threadIdx.x;   // my column
  if (a >= dp) return;
  uint32_t hw[4] = {0u, 0u, 0u, 0u}, lw[4] = {0u, 0u, 0u, 0u};
  if (a < d) {
    const float inv_h2 = float(1.0 / h2[0]);
    const float xb = xbar[a], sc = vq ? vq[a] : 1.0f;
    float gv[8], xv[8];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int j = 8 * q + jj;
      const long long e = (long long)(j < n ? j : 0) * d + a;   // rows past n are not used
      gv[jj] = g[e];
      xv[jj] = x[e];
    }
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      if (8 * q + jj >= n) break;
      const float gs = vq ? gv[jj] * sc : gv[jj];
      const float b = fmaf(-(xv[jj] - xb), inv_h2, gs);   // x - xbar: the centring kernel's Xc
      const uint16_t hb = f32_to_bf16_rne(b);
      const uint16_t lb = f32_to_bf16_rne(b - bf16_to_f32(hb));
      hw[jj >> 1] |= uint32_t(hb) << (16 * (jj & 1));
      lw[jj >> 1] |= uint32_t(lb) << (16 * (jj & 1));
    }
  }
  const long long o = ((long long)q * dp + a) * 4;
  *reinterpret_cast<uint4 *>(bph + o) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
  *reinterpret_cast<uint4 *>(bpl + o) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
}

// Block: 128 particles x 256 coordinates, 4 waves (2 x 2) of 2 x 4 tiles of
// 32 x 32 (v_mfma_f32_32x32x16_bf16, operand and result layout as in the Gram
// kernel), 50 KB of LDS and at most 256 registers, so that two blocks share a
// compute unit: one block's epilogue (HBM-bound) and barriers then overlap
// the other's matrix instructions.  The particle index j runs in stages of
// 32 through LDS, the next stage prefetched into registers.  A = K rows i (K
// is symmetric) with 32 consecutive j from the BF16 copy; a B fragment is
// the four 32-bit pairs of one column and group, stored as such by
// bpair_kernel and kept column by column in LDS (16 pairs and 4 cells of
// padding per column, so that the 16-byte accesses of 8 consecutive lanes
// meet distinct banks).  The two products go over all eight tiles in turn,
// so that consecutive matrix instructions accumulate into different tiles.
constexpr int VM = 128, VN = 256, VK = 32, VKP = VK + 8, VBT = VK / 2 + 4, VT = 256;
template <bool RULE>
__global__ __launch_bounds__(VT) __attribute__((amdgpu_waves_per_eu(2, 2))) void update_bf16x2_kernel(
    const uint16_t *khi, int ldk, const uint32_t *bph, const uint32_t *bpl,
    long long dp, const float *xbar, const float *s, const double *h2, float *x, float *phi,
    const float *lo, const float *hi, int n, long long d, int mblocks, float eps, OptArgs opt,
    uint32_t *status) {
  __shared__ __attribute__((aligned(16))) uint16_t Ah[VM][VKP];   // Ah[i][k] = bf16(K[i0 + i][j0 + k])
  __shared__ __attribute__((aligned(16))) uint32_t Bh[VN][VBT];   // Bh[a][p] = pair j0 / 2 + p
  __shared__ __attribute__((aligned(16))) uint32_t Bl[VN][VBT];
  const int per = int(gridDim.x) >> 3;
  const int tb = (int(blockIdx.x) & 7) * per + (int(blockIdx.x) >> 3);
  const int nt = mblocks * int((d + VN - 1) / VN);
  if (tb >= nt) return;
  const int i0 = (tb % mblocks) * VM;
  const long long a0 = (long long)(tb / mblocks) * VN;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;

  // staging: A row t / 2, k half 16 (t % 2); B column t, all four groups
  const int ar = t >> 1, ak = (t & 1) * 16;
  const bool bin = a0 + t < dp;   // dp is a multiple of 8: zero columns beyond it
  uint4 pah[2], pbh[4], pbl[4];
  auto load_stage = [&](int j0) {
    const int i = i0 + ar;
    if (i < n) {
      const uint16_t *ph = khi + (long long)i * ldk + j0 + ak;
      pah[0] = *reinterpret_cast<const uint4 *>(ph);
      pah[1] = *reinterpret_cast<const uint4 *>(ph + 8);
    } else {
      pah[0] = pah[1] = make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const long long off = ((long long)(j0 / 8 + h) * dp + a0 + t) * 4;
      pbh[h] = bin ? *reinterpret_cast<const uint4 *>(bph + off) : make_uint4(0, 0, 0, 0);
      pbl[h] = bin ? *reinterpret_cast<const uint4 *>(bpl + off) : make_uint4(0, 0, 0, 0);
    }
  };
  auto store_stage = [&]() {
    *reinterpret_cast<uint4 *>(&Ah[ar][ak]) = pah[0];
    *reinterpret_cast<uint4 *>(&Ah[ar][ak + 8]) = pah[1];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      *reinterpret_cast<uint4 *>(&Bh[t][4 * h]) = pbh[h];
      *reinterpret_cast<uint4 *>(&Bl[t][4 * h]) = pbl[h];
    }
  };

  f32x16_t acc[2][4];
  for (int m = 0; m < 2; ++m)
    for (int q = 0; q < 4; ++q)
      for (int r = 0; r < 16; ++r) acc[m][q][r] = 0.0f;
  load_stage(0);
  for (int j0 = 0; j0 < n; j0 += VK) {
    __syncthreads();               // the previous stage's tiles are no longer read
    store_stage();
    __syncthreads();
    if (j0 + VK < n) load_stage(j0 + VK);
#pragma unroll
    for (int kk = 0; kk < VK; kk += 16) {
      const int kq = kk + 8 * (lane >> 5);   // first of my 8 k
      bf16x8_t fah[2], fbh[4], fbl[4];
      for (int m = 0; m < 2; ++m) {
        const int row = wi * 64 + m * 32 + (lane & 31);
        const uint4 rh = *reinterpret_cast<const uint4 *>(&Ah[row][kq]);
        __builtin_memcpy(&fah[m], &rh, 16);
      }
      for (int q = 0; q < 4; ++q) {
        const int col = wj * 128 + q * 32 + (lane & 31);
        const uint4 uh = *reinterpret_cast<const uint4 *>(&Bh[col][kq / 2]);
        const uint4 ul = *reinterpret_cast<const uint4 *>(&Bl[col][kq / 2]);
        __builtin_memcpy(&fbh[q], &uh, 16);
        __builtin_memcpy(&fbl[q], &ul, 16);
      }
      for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 4; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[m], fbl[q], acc[m][q], 0, 0, 0);
      for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 4; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[m], fbh[q], acc[m][q], 0, 0, 0);
    }
  }

  const float inv_n = 1.0f / float(n);
  const float inv_h2 = float(1.0 / h2[0]);
  bool bad = false;
  if constexpr (RULE) {
    // a step rule with per-coordinate state: one element at a time
    for (int m = 0; m < 2; ++m)
      for (int r = 0; r < 16; ++r) {
        const int i = i0 + wi * 64 + m * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (i >= n) continue;
        const float si = s[i] * inv_h2;
        for (int q = 0; q < 4; ++q) {
          const long long a = a0 + wj * 128 + q * 32 + (lane & 31);
          if (a >= d) continue;
          const long long e = (long long)i * d + a;
          const float xe = x[e];
          const float p = fmaf(si, xe - xbar[a], acc[m][q][r]) * inv_n;
          phi[e] = p;
          float v = xe + opt_step(opt, e, p, eps);
          if (lo) v = fminf(fmaxf(v, lo[a]), hi[a]);
          bad |= !isfinite(v);
          x[e] = v;
        }
      }
  } else {
    // Plain steps in four batches of eight result registers (32 elements):
    // every x of a batch is loaded before any store (the stores to phi and x
    // could alias them as far as the compiler knows, which would otherwise
    // serialise each load behind the previous element's stores), and the next
    // batch's loads go out before this batch's stores, since loads and stores
    // retire through one in-order counter: waiting for loads issued after the
    // stores would wait for the stores too.  Batch b covers sub-tile b / 2,
    // registers 8 (b % 2) .. + 7; element (r, q) of sub-tile m sits at
    // el + (m 32 + 8 (r / 4) + r % 4) d + 32 q.
    const int lrow = wi * 64 + 4 * (lane >> 5);      // my first local row
    const int lcol = wj * 128 + (lane & 31);         // my first local column
    const long long el = (long long)(i0 + lrow) * d + a0 + lcol;
    float xb[4], lov[4], hiv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long long a = a0 + lcol + q * 32;
      xb[q] = a < d ? xbar[a] : 0.0f;
      lov[q] = (lo && a < d) ? lo[a] : 0.0f;
      hiv[q] = (lo && a < d) ? hi[a] : 0.0f;
    }
    // local row (relative to my first) of register r of sub-tile m
    auto lrow_of = [](int m, int r) { return m * 32 + 8 * (r >> 2) + (r & 3); };
    float xv[2][8][4], si[2][8];
    // Loads are unconditional (elements outside the ensemble read x[0] and
    // s[0] and are never used), so no branch separates them from each other.
    auto load_batch = [&](int b, float (&xvb)[8][4], float (&sib)[8]) {
      const int m = b >> 1, rb = (b & 1) * 8;
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        const int lr = lrow_of(m, rb + rr);
        const int i = i0 + lrow + lr;
        sib[rr] = s[i < n ? i : 0];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool in = i < n && a0 + lcol + q * 32 < d;
          xvb[rr][q] = x[in ? el + (long long)lr * d + q * 32 : 0];
        }
      }
    };
    load_batch(0, xv[0], si[0]);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (b + 1 < 4) load_batch(b + 1, xv[(b + 1) & 1], si[(b + 1) & 1]);
      const int m = b >> 1, rb = (b & 1) * 8;
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        const int lr = lrow_of(m, rb + rr);
        if (i0 + lrow + lr >= n) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (a0 + lcol + q * 32 >= d) continue;
          const long long e = el + (long long)lr * d + q * 32;
          const float xe = xv[b & 1][rr][q];
          const float p = fmaf(si[b & 1][rr] * inv_h2, xe - xb[q], acc[m][q][rb + rr]) * inv_n;
          phi[e] = p;
          float v = xe + eps * p;
          if (lo) v = fminf(fmaxf(v, lov[q]), hiv[q]);
          bad |= !isfinite(v);
          x[e] = v;
        }
      }
    }
  }
  if (bad) atomicOr(status, VIP_FLAG_NONFINITE);
}

// The same update with the operands streamed through a ring of three LDS
// stages by 16-byte loads that write LDS directly (no registers held while
// they fly), two stages ahead of the matrix instructions.  Block: 256
// particles x 256 coordinates, 8 waves (4 x 2) of 64 x 128 (2 x 4 tiles of
// 32 x 32, the same fragments and the same order of matrix instructions per
// tile as update_bf16x2_kernel, so phi is bitwise the same), one block per
// compute unit (147 KB of LDS), two waves per SIMD.  A stage is 32 j:
//  * A: rows i0 .. i0 + 255 of K in BF16, 64 bytes a row in four 16-byte
//    chunks; chunk c of row r sits in slot c ^ ((r >> 2) & 3) of the row, so
//    that the fragment reads of 16 consecutive rows meet distinct banks;
//  * B: for each of the four groups of 8 j and each of the 256 columns, the
//    16-byte pair words of bpair_kernel, hi and lo in two arrays.
// Rows past n, and columns past dp, read as zeros (the loads' range check and
// an offset beyond it).  The loads are written as inline assembly: a compiler
// that sees loads writing LDS waits for them before any LDS access it cannot
// prove disjoint, which would drain the ring at every stage; here the waits
// are explicit (each wave issues 6 loads a stage, so waiting for all but the
// newest 6 completes the stage to be read) and a barrier then makes every
// wave's loads visible to all.
constexpr int RM = 256, RN = 256, RK = 32, RS = 3, RT = 512;
constexpr bool kUpdateRing = true;
constexpr int R_A = RM * RK * 2, R_B = 4 * RN * 16, R_STAGE = R_A + 2 * R_B;
template <bool RULE>
__global__ __launch_bounds__(RT) __attribute__((amdgpu_waves_per_eu(2, 2))) void update_bf16x2_ring_kernel(
    const uint16_t *khi, int ldk, const uint32_t *bph, const uint32_t *bpl,
    long long dp, const float *xbar, const float *s, const double *h2, float *x, float *phi,
    const float *lo, const float *hi, int n, long long d, int mblocks, float eps, OptArgs opt,
    uint32_t *status) {
  __shared__ __attribute__((aligned(16))) unsigned char ring[RS][R_STAGE];
  const int per = int(gridDim.x) >> 3;
  const int tb = (int(blockIdx.x) & 7) * per + (int(blockIdx.x) >> 3);
  const int nt = mblocks * int((d + RN - 1) / RN);
  if (tb >= nt) return;
  const int i0 = (tb % mblocks) * RM;
  const long long a0 = (long long)(tb / mblocks) * RN;
  // (the wave index as a scalar: the LDS addresses of the loads derive from it)
  const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wi = w >> 1, wj = w & 1;

  // descriptors of K (rows past n out of range) and of the B pairs
  typedef uint32_t U32x4 __attribute__((ext_vector_type(4)));
  auto rsrc = [](const void *base, uint32_t bytes) {
    const uint64_t b = reinterpret_cast<uint64_t>(base);
    U32x4 r;
    r.x = __builtin_amdgcn_readfirstlane(uint32_t(b));
    r.y = __builtin_amdgcn_readfirstlane(uint32_t(b >> 32)) & 0xffffu;
    r.z = __builtin_amdgcn_readfirstlane(bytes);
    r.w = 0x00020000u;
    return r;
  };
  const U32x4 rk = rsrc(khi, uint32_t(n) * uint32_t(ldk) * 2u);
  const uint32_t bbytes = uint32_t(ldk / 2) * uint32_t(dp) * 4u;
  const U32x4 rbh = rsrc(bph, bbytes), rbl = rsrc(bpl, bbytes);
  const uint32_t ring0 = uint32_t(reinterpret_cast<uintptr_t>(
      (__attribute__((address_space(3))) unsigned char *)&ring[0][0]));
  // My six loads of a stage: numbers w + 8 k of the stage's 48 (16 of A,
  // 16 of B hi, 16 of B lo), each 64 lanes x 16 bytes.
  //   A load q (0..15): rows 16 q + lane / 4, chunk (lane % 4) ^ ((row >> 2) & 3)
  //   B load q (0..15): group q / 4, columns 64 (q % 4) + lane
  auto issue = [&](int st) {
    const int j0 = st * RK;
    const uint32_t base = ring0 + uint32_t((st % RS) * R_STAGE);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int q = (w + 8 * k) & 15;
      uint32_t m0, off;
      U32x4 r;
      if (k < 2) {
        const int row = 16 * q + (lane >> 2);
        const int chunk = (lane & 3) ^ ((row >> 2) & 3);
        m0 = base + uint32_t(q * 16 * 64);
        off = (uint32_t(i0 + row) * uint32_t(ldk) + uint32_t(j0)) * 2u + uint32_t(chunk) * 16u;
        if (i0 + row >= n) off = 0x80000000u;
        r = rk;
      } else {
        const int h = q >> 2;
        const long long a = a0 + 64 * (q & 3) + lane;
        m0 = base + uint32_t(R_A + (k >= 4 ? R_B : 0) + (h * RN + 64 * (q & 3)) * 16);
        off = a < dp ? uint32_t(((long long)(j0 / 8 + h) * dp + a) * 16) : 0x80000000u;
        r = k >= 4 ? rbl : rbh;
      }
      uint32_t keep;
      asm volatile(
          "s_mov_b32 %0, m0\n\ts_mov_b32 m0, %1\n\ts_nop 0\n\t"
          "buffer_load_dwordx4 %2, %3, 0 offen lds\n\ts_mov_b32 m0, %0"
          : "=&s"(keep)
          : "s"(m0), "v"(off), "s"(r)
          : "memory");
    }
  };

  f32x16_t acc[2][4];
  for (int m = 0; m < 2; ++m)
    for (int q = 0; q < 4; ++q)
      for (int r = 0; r < 16; ++r) acc[m][q][r] = 0.0f;
  const int nst = (n + RK - 1) / RK;
  issue(0);
  if (nst > 1) issue(1);
  for (int st = 0; st < nst; ++st) {
    // this stage's loads have landed (only the next stage's six may fly), in
    // every wave once all have passed the barrier; that barrier also ends
    // every wave's reads of the slot the stage after next overwrites
    if (st + 1 < nst) __builtin_amdgcn_s_waitcnt(0x0F76);   // vmcnt(6)
    else __builtin_amdgcn_s_waitcnt(0x0F70);                // vmcnt(0)
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (st + 2 < nst) issue(st + 2);
    const unsigned char *sa = &ring[st % RS][0];
    const unsigned char *sbh = sa + R_A, *sbl = sa + R_A + R_B;
#pragma unroll
    for (int kk = 0; kk < RK; kk += 16) {
      const int kq = kk + 8 * (lane >> 5);   // first of my 8 j
      bf16x8_t fah[2], fbh[4], fbl[4];
      for (int m = 0; m < 2; ++m) {
        const int row = wi * 64 + m * 32 + (lane & 31);
        const int slot = (kq >> 3) ^ ((row >> 2) & 3);
        const uint4 rh = *reinterpret_cast<const uint4 *>(sa + (row * 4 + slot) * 16);
        __builtin_memcpy(&fah[m], &rh, 16);
      }
      for (int q = 0; q < 4; ++q) {
        const int col = wj * 128 + q * 32 + (lane & 31);
        const int o = ((kq >> 3) * RN + col) * 16;
        const uint4 uh = *reinterpret_cast<const uint4 *>(sbh + o);
        const uint4 ul = *reinterpret_cast<const uint4 *>(sbl + o);
        __builtin_memcpy(&fbh[q], &uh, 16);
        __builtin_memcpy(&fbl[q], &ul, 16);
      }
      for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 4; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[m], fbl[q], acc[m][q], 0, 0, 0);
      for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 4; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[m], fbh[q], acc[m][q], 0, 0, 0);
    }
  }

  const float inv_n = 1.0f / float(n);
  const float inv_h2 = float(1.0 / h2[0]);
  bool bad = false;
  if constexpr (RULE) {
    // a step rule with per-coordinate state: one element at a time
    for (int m = 0; m < 2; ++m)
      for (int r = 0; r < 16; ++r) {
        const int i = i0 + wi * 64 + m * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (i >= n) continue;
        const float si = s[i] * inv_h2;
        for (int q = 0; q < 4; ++q) {
          const long long a = a0 + wj * 128 + q * 32 + (lane & 31);
          if (a >= d) continue;
          const long long e = (long long)i * d + a;
          const float xe = x[e];
          const float p = fmaf(si, xe - xbar[a], acc[m][q][r]) * inv_n;
          phi[e] = p;
          float v = xe + opt_step(opt, e, p, eps);
          if (lo) v = fminf(fmaxf(v, lo[a]), hi[a]);
          bad |= !isfinite(v);
          x[e] = v;
        }
      }
  } else {
    // Plain steps in four batches of eight result registers (32 elements):
    // every x of a batch is loaded before any store (the stores to phi and x
    // could alias them as far as the compiler knows, which would otherwise
    // serialise each load behind the previous element's stores), and the next
    // batch's loads go out before this batch's stores, since loads and stores
    // retire through one in-order counter: waiting for loads issued after the
    // stores would wait for the stores too.  Batch b covers sub-tile b / 2,
    // registers 8 (b % 2) .. + 7; element (r, q) of sub-tile m sits at
    // el + (m 32 + 8 (r / 4) + r % 4) d + 32 q.
    const int lrow = wi * 64 + 4 * (lane >> 5);      // my first local row
    const int lcol = wj * 128 + (lane & 31);         // my first local column
    const long long el = (long long)(i0 + lrow) * d + a0 + lcol;
    float xb[4], lov[4], hiv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long long a = a0 + lcol + q * 32;
      xb[q] = a < d ? xbar[a] : 0.0f;
      lov[q] = (lo && a < d) ? lo[a] : 0.0f;
      hiv[q] = (lo && a < d) ? hi[a] : 0.0f;
    }
    // local row (relative to my first) of register r of sub-tile m
    auto lrow_of = [](int m, int r) { return m * 32 + 8 * (r >> 2) + (r & 3); };
    float xv[2][8][4], si[2][8];
    // Loads are unconditional (elements outside the ensemble read x[0] and
    // s[0] and are never used), so no branch separates them from each other.
    auto load_batch = [&](int b, float (&xvb)[8][4], float (&sib)[8]) {
      const int m = b >> 1, rb = (b & 1) * 8;
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        const int lr = lrow_of(m, rb + rr);
        const int i = i0 + lrow + lr;
        sib[rr] = s[i < n ? i : 0];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool in = i < n && a0 + lcol + q * 32 < d;
          xvb[rr][q] = x[in ? el + (long long)lr * d + q * 32 : 0];
        }
      }
    };
    load_batch(0, xv[0], si[0]);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (b + 1 < 4) load_batch(b + 1, xv[(b + 1) & 1], si[(b + 1) & 1]);
      const int m = b >> 1, rb = (b & 1) * 8;
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        const int lr = lrow_of(m, rb + rr);
        if (i0 + lrow + lr >= n) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (a0 + lcol + q * 32 >= d) continue;
          const long long e = el + (long long)lr * d + q * 32;
          const float xe = xv[b & 1][rr][q];
          const float p = fmaf(si[b & 1][rr] * inv_h2, xe - xb[q], acc[m][q][rb + rr]) * inv_n;
          phi[e] = p;
          float v = xe + eps * p;
          if (lo) v = fminf(fmaxf(v, lov[q]), hiv[q]);
          bad |= !isfinite(v);
          x[e] = v;
        }
      }
    }
  }
  if (bad) atomicOr(status, VIP_FLAG_NONFINITE);
}

// ---- host ---------------------------------------------------------------------

// Host-side validation of one step (everything that can fail before a launch).
static vip_status svgd_check(int32_t n, int64_t d, const float *x, const float *g, double eps,
                             int32_t bw_mode, double h_fixed, int32_t gram_prec,
                             const vip_prior *prior, bool noise, const vip_optimizer *opt,
                             int32_t kernel) {
  if (!x || !g) return VIP_E_ARG;
  if (kernel != VIP_KERNEL_RBF && kernel != VIP_KERNEL_DIAG_VAR) return VIP_E_ARG;
  OptArgs oa;
  if (opt && noise) return VIP_E_ARG;
  if (const vip_status st = make_opt_args(opt, &oa); st != VIP_OK) return st;
  if (n < 1 || d < 1 || !(eps >= 0.0) || !std::isfinite(eps)) return VIP_E_ARG;
  if (bw_mode < VIP_BW_MEDIAN_ALL || bw_mode > VIP_BW_FIXED) return VIP_E_ARG;
  if (bw_mode == VIP_BW_FIXED && !(h_fixed > 0.0)) return VIP_E_ARG;
  if (gram_prec != VIP_GRAM_BF16 && gram_prec != VIP_GRAM_FP32) return VIP_E_ARG;
  if (prior && prior->kind != VIP_PRIOR_NONE) {
    // only the clip strategy acts on the update; the transform and Gaussian
    // priors enter through the gradient
    if (prior->kind == VIP_PRIOR_UNIFORM_CLIP) {
      if (!prior->lo || !prior->hi) return VIP_E_ARG;
    } else if (prior->kind != VIP_PRIOR_UNIFORM_TRANSFORM && prior->kind != VIP_PRIOR_GAUSSIAN) {
      return VIP_E_ARG;
    }
  }
  const bool split_update = gram_prec == VIP_GRAM_BF16;
  if (split_update && (n + 31) / 32 * 16 > 65535) return VIP_E_UNSUPPORTED;   // a grid row per j pair
  {
    const long long ntiles = (long long)((n + UM - 1) / UM) * ((d + UN - 1) / UN);
    if (ntiles >= (1LL << 30)) return VIP_E_UNSUPPORTED;
  }
  return VIP_OK;
}

static vip_status svgd_common(vip_ctx *ctx, int32_t n, int64_t d, float *x, const float *g,
                              double eps, int32_t bw_mode, double h_fixed, int32_t gram_prec,
                              const vip_prior *prior, bool noise, const float *xi, uint64_t seed,
                              uint64_t stream, double *h2_out, void *ws, size_t ws_bytes,
                              uint32_t *status_ptr = nullptr,
                              const vip_optimizer *opt = nullptr, int32_t kernel = VIP_KERNEL_RBF) {
  if (!ctx || !ws) return VIP_E_ARG;
  VIP_TRY(svgd_check(n, d, x, g, eps, bw_mode, h_fixed, gram_prec, prior, noise, opt, kernel));
  OptArgs oa;
  (void)make_opt_args(opt, &oa);
  const float *lo = nullptr, *hi = nullptr;
  if (prior && prior->kind == VIP_PRIOR_UNIFORM_CLIP) {
    lo = prior->lo;
    hi = prior->hi;
  }
  SvgdPlan P;
  plan_svgd(n, d, static_cast<char *>(ws), &P);
  if (ws_bytes < P.bytes || !aligned(ws)) return VIP_E_WORKSPACE;
  if (status_ptr) P.status = status_ptr;
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  ctx->active = ctx->user;
  hipStream_t s = ctx->user;
  const long long nn = (long long)n * n;

  const bool diag = kernel == VIP_KERNEL_DIAG_VAR;
  float *sq = diag ? P.sq : nullptr, *vq = diag ? P.vq : nullptr;
  // the BF16 path never reads the FP32 Xc (it recomputes x - xbar); with
  // noise the update leaves the clip to the noise pass, as on the FP32 path
  const bool split_update = gram_prec == VIP_GRAM_BF16;
  // the register cache addresses X with 32-bit byte offsets, up to row 32 CACHE
  const unsigned long long rows = (unsigned long long)std::max(n, CENTRE_GROUPS * CENTRE_CACHE);
  auto *centre = rows * (unsigned long long)d * 4ull < (1ull << 31)
                     ? centre_kernel<CENTRE_CACHE>
                     : centre_kernel<0>;
  centre<<<dim3(unsigned((d + CENTRE_COLS - 1) / CENTRE_COLS)),
           dim3(CENTRE_COLS * CENTRE_GROUPS), 0, s>>>(
      x, P.xbar, split_update ? nullptr : P.xc, P.xc16, sq, vq, n, d, P.status);
  VIP_LAUNCH_CHECK();
  const int nup = P.nbt * (P.nbt + 1) / 2;
  const bool g16 = gram_prec == VIP_GRAM_BF16;
  // the ring Gram reads 16-byte chunks of rows (a multiple of 8 coordinates)
  // at 32-bit byte offsets
  const bool gring = g16 && kGramRing && d % 8 == 0 && (long long)n * d * 2 < (1LL << 31);
  const int gsplits = gring ? P.splits2 : g16 ? P.splits16 : P.splits;
  if (gring) {
    const int nup2 = P.nbt2 * (P.nbt2 + 1) / 2;
    gram_bf16_ring_kernel<<<dim3(unsigned((nup2 * gsplits + 7) / 8 * 8)), dim3(G2T), 0, s>>>(
        P.xc16, P.part, n, d, P.kspan2, P.nbt2);
  } else {
    dim3 ggrid(unsigned((nup * gsplits + 7) / 8 * 8));
    if (g16)
      gram_bf16_kernel<<<ggrid, dim3(256), 0, s>>>(P.xc16, P.part, n, d, P.kspan16, P.nbt);
    else
      gram_f32_kernel<<<ggrid, dim3(256), 0, s>>>(P.xc, sq, P.part, n, d, P.kspan, P.nbt);
  }
  VIP_LAUNCH_CHECK();
  {
    const int ntile = (n + DT - 1) / DT;
    gram_dist_kernel<<<dim3(unsigned(ntile * (ntile + 1) / 2)), dim3(256), 0, s>>>(
        P.part, P.D, n, gsplits, ntile, P.status);
    VIP_LAUNCH_CHECK();
  }

  long long count = 0;
  if (bw_mode != VIP_BW_FIXED) {
    count = bw_mode == VIP_BW_MEDIAN_ALL ? nn : (long long)n * (n - 1) / 2;
    // 0-based ranks of the middle values: m/2 - 1 and m/2 for even m, m/2 twice for odd m
    const long long r1 = count / 2, r0 = (count % 2 == 0) ? count / 2 - 1 : count / 2;
    int32_t sel_init[6] = {0, 0, int32_t(r0), 0, 0, int32_t(r1)};
    VIP_TRY(upload_i32(s, reinterpret_cast<int32_t *>(P.sel), sel_init, 6));
    if (count > 0) {
      unsigned hb = unsigned(std::min<long long>((nn + 4095) / 4096, 1024));
      const int vec = reinterpret_cast<uintptr_t>(P.D) % 16 == 0;
      // each select clears it for the next pass
      VIP_TRY(fill_u32(s, P.hist, 2 * RADIX_BINS, 0u));
      constexpr int kShift[3] = {21, 10, 0}, kBits[3] = {11, 11, 10};   // 32 bits in 3 digits
      for (int ps = 0; ps < 3; ++ps) {
        radix_hist_kernel<<<dim3(hb), dim3(256), 0, s>>>(P.D, n, bw_mode == VIP_BW_MEDIAN_OFFDIAG,
                                                         vec, kShift[ps], kBits[ps], P.sel,
                                                         P.hist);
        VIP_LAUNCH_CHECK();
        radix_select_kernel<<<dim3(1), dim3(128), 0, s>>>(P.sel, P.hist, kShift[ps], kBits[ps]);
        VIP_LAUNCH_CHECK();
      }
    }
  }
  bandwidth_kernel<<<dim3(1), dim3(1), 0, s>>>(P.sel, count, n, bw_mode, h_fixed, P.h2, h2_out);
  VIP_LAUNCH_CHECK();
  rbf_kernel<<<dim3(n), dim3(256), 0, s>>>(P.D, P.h2, P.K, P.s, n,
                                           split_update ? P.khi : nullptr, P.ldk);
  VIP_LAUNCH_CHECK();

  // phi and x + eps phi (or a step rule); with noise the prior clip waits for
  // the noise pass, which adds the noise to the updated x and then clips
  const float *ulo = noise ? nullptr : lo, *uhi = noise ? nullptr : hi;
  const int mblocks = (n + UM - 1) / UM;
  const long long ntiles = (long long)mblocks * ((d + UN - 1) / UN);
  // float4 staging needs rows of a multiple of 4 floats and 16-byte aligned bases
  const int vec = (d % 4 == 0) && (n % 4 == 0) && (reinterpret_cast<uintptr_t>(g) % 16 == 0) &&
                  (reinterpret_cast<uintptr_t>(P.xc) % 16 == 0) &&
                  (reinterpret_cast<uintptr_t>(P.K) % 16 == 0);
  if (split_update) {
    const int ngroups = P.ldk / 8;
    bpair_kernel<<<dim3(unsigned((P.dp + 255) / 256), unsigned(ngroups)), dim3(256), 0, s>>>(
        g, x, P.xbar, vq, P.h2, P.bph, P.bpl, n, d, P.dp);
    VIP_LAUNCH_CHECK();
    // the ring kernel addresses K and the B pairs with 32-bit byte offsets
    const bool ring = kUpdateRing && (long long)n * P.ldk * 2 < (1LL << 31) &&
                      (long long)(P.ldk / 2) * P.dp * 4 < (1LL << 31);
    if (ring) {
      const int rblocks = (n + RM - 1) / RM;
      const long long rtiles = (long long)rblocks * ((d + RN - 1) / RN);
      auto *kern = oa.kind == VIP_OPT_SGD ? update_bf16x2_ring_kernel<false>
                                          : update_bf16x2_ring_kernel<true>;
      kern<<<dim3(unsigned((rtiles + 7) / 8 * 8)), dim3(RT), 0, s>>>(
          P.khi, P.ldk, P.bph, P.bpl, P.dp, P.xbar, P.s, P.h2, x, P.phi, ulo, uhi, n, d,
          rblocks, float(eps), oa, P.status);
    } else {
      const int vblocks = (n + VM - 1) / VM;
      const long long vtiles = (long long)vblocks * ((d + VN - 1) / VN);
      auto *kern = oa.kind == VIP_OPT_SGD ? update_bf16x2_kernel<false> : update_bf16x2_kernel<true>;
      kern<<<dim3(unsigned((vtiles + 7) / 8 * 8)), dim3(VT), 0, s>>>(
          P.khi, P.ldk, P.bph, P.bpl, P.dp, P.xbar, P.s, P.h2, x, P.phi, ulo, uhi, n, d,
          vblocks, float(eps), oa, P.status);
    }
  } else {
    auto *kern = oa.kind == VIP_OPT_SGD ? update_mfma_kernel<false> : update_mfma_kernel<true>;
    kern<<<dim3(unsigned((ntiles + 7) / 8 * 8)), dim3(UT), 0, s>>>(
        P.K, g, P.xc, vq, P.s, P.h2, x, P.phi, ulo, uhi, n, d, mblocks, vec, float(eps), oa,
        P.status);
  }
  VIP_LAUNCH_CHECK();
  if (noise) {
    // BF16 path beyond one workgroup's Cholesky: the noise product on the BF16
    // matrix cores, L as a BF16 pair in the space of its FP32 copy (4 n^2 bytes)
    const bool noise16 = g16 && n > kCholMax;
    uint16_t *L16 = noise16 ? reinterpret_cast<uint16_t *>(P.Lf) : nullptr;
    if (n <= kCholMax) {
      cholesky_kernel<<<dim3(1), dim3(1024), 0, s>>>(P.D, P.h2, P.L, P.Lf, n, 6, P.status);
      VIP_LAUNCH_CHECK();
    } else {
      const unsigned nn_blocks = unsigned((nn + 255) / 256);
      chol_init_kernel<<<dim3(nn_blocks), dim3(256), 0, s>>>(P.D, P.h2, P.L, n, 0.0, P.chol);
      VIP_LAUNCH_CHECK();
      for (int k0 = 0; k0 < n; k0 += CB) {
        const int below = std::max(0, n - k0 - CB);
        chol_panel_kernel<<<dim3(unsigned(1 + (below + CR - 1) / CR)), dim3(256), 0, s>>>(
            P.L, n, k0, P.chol);
        VIP_LAUNCH_CHECK();
        if (below > 0) {
          const int m = (below + 63) / 64;
          chol_update_kernel<<<dim3(unsigned(m * (m + 1) / 2)), dim3(256), 0, s>>>(P.L, n, k0,
                                                                                  P.chol);
          VIP_LAUNCH_CHECK();
        }
      }
      chol_retry_kernel<<<dim3(1), dim3(1024), 0, s>>>(P.D, P.h2, P.L, n, 6, P.chol, P.status);
      VIP_LAUNCH_CHECK();
      chol_output_kernel<<<dim3(nn_blocks), dim3(256), 0, s>>>(P.L, P.Lf, L16, n, P.chol);
      VIP_LAUNCH_CHECK();
    }
    const float *xin = xi;
    if (!xin) {
      long long count_xi = (long long)n * d;
      philox_fill_kernel<<<dim3(unsigned(((count_xi + 3) / 4 + 255) / 256)), dim3(256), 0, s>>>(
          P.xi, count_xi, uint32_t(seed), uint32_t(seed >> 32), uint32_t(stream),
          uint32_t(stream >> 32));
      VIP_LAUNCH_CHECK();
      xin = P.xi;
    }
    const long long nxcd = (((d + UN - 1) / UN) + 7) / 8;   // column blocks per XCD, at most
    if (noise16) {
      const int v16 = (d % 4 == 0) && (n % 8 == 0) &&
                      (reinterpret_cast<uintptr_t>(xin) % 16 == 0) &&
                      (reinterpret_cast<uintptr_t>(L16) % 16 == 0);
      noise_bf16x3_kernel<<<dim3(unsigned(8 * mblocks * nxcd)), dim3(UT), 0, s>>>(
          L16, xin, vq, x, lo, hi, n, d, mblocks, v16, float(std::sqrt(2.0 * eps)), P.status);
    } else {
      const int nvec = (d % 4 == 0) && (n % 4 == 0) &&
                       (reinterpret_cast<uintptr_t>(xin) % 16 == 0) &&
                       (reinterpret_cast<uintptr_t>(P.Lf) % 16 == 0);
      noise_mfma_kernel<<<dim3(unsigned(8 * mblocks * nxcd)), dim3(UT), 0, s>>>(
          P.Lf, xin, vq, x, lo, hi, n, d, mblocks, nvec, float(std::sqrt(2.0 * eps)), P.status);
    }
  }
  VIP_LAUNCH_CHECK();
  return VIP_OK;
}

}  // namespace vip

using namespace vip;

extern "C" {

vip_status vip_svgd_workspace(int32_t n, int64_t d, size_t *bytes) {
  if (!bytes || n < 1 || d < 1) return VIP_E_ARG;
  SvgdPlan P;
  plan_svgd(n, d, nullptr, &P);
  *bytes = P.bytes;
  return VIP_OK;
}

vip_status vip_svgd_layout_of(int32_t n, int64_t d, vip_svgd_layout *out) {
  if (!out || n < 1 || d < 1) return VIP_E_ARG;
  SvgdPlan P;
  char *base = reinterpret_cast<char *>(kAlign);   // any aligned base; offsets only
  plan_svgd(n, d, base, &P);
  auto off = [&](const void *p) { return size_t(reinterpret_cast<const char *>(p) - base); };
  out->D = off(P.D);
  out->K = off(P.K);
  out->h2 = off(P.h2);
  out->L = off(P.L);
  out->phi = off(P.phi);
  return VIP_OK;
}

vip_status vip_svgd_step(vip_ctx *ctx, int32_t n, int64_t d, float *x, const float *g, double eps,
                         int32_t bw_mode, double h_fixed, int32_t gram_prec,
                         const vip_prior *prior, double *h2_out, void *ws, size_t ws_bytes) {
  return svgd_common(ctx, n, d, x, g, eps, bw_mode, h_fixed, gram_prec, prior, false, nullptr, 0, 0,
                     h2_out, ws, ws_bytes);
}

vip_status vip_svgd_step_ex(vip_ctx *ctx, int32_t n, int64_t d, float *x, const float *g,
                            double eps, const vip_svgd_config *cfg, const vip_prior *prior,
                            double *h2_out, void *ws, size_t ws_bytes) {
  if (!cfg) return VIP_E_ARG;
  if (cfg->noise != 0 && cfg->noise != 1) return VIP_E_ARG;
  return svgd_common(ctx, n, d, x, g, eps, cfg->bw_mode, cfg->h_fixed, cfg->gram_prec, prior,
                     cfg->noise != 0, cfg->xi, cfg->seed, cfg->stream, h2_out, ws, ws_bytes,
                     nullptr, cfg->opt, cfg->kernel);
}

vip_status vip_svgd_step_opt(vip_ctx *ctx, int32_t n, int64_t d, float *x, const float *g,
                             double eps, int32_t bw_mode, double h_fixed, int32_t gram_prec,
                             const vip_prior *prior, const vip_optimizer *opt, double *h2_out,
                             void *ws, size_t ws_bytes) {
  if (!opt) return VIP_E_ARG;
  return svgd_common(ctx, n, d, x, g, eps, bw_mode, h_fixed, gram_prec, prior, false, nullptr, 0, 0,
                     h2_out, ws, ws_bytes, nullptr, opt);
}

}  // extern "C"

namespace vip {

static size_t plan_svgd_multi(int32_t nens, const vip_ensemble *ens, std::vector<size_t> *offs) {
  size_t off = kStatusBytes;
  offs->clear();
  for (int e = 0; e < nens; ++e) {
    SvgdPlan P;
    plan_svgd(ens[e].n, ens[e].d, nullptr, &P);
    offs->push_back(off);
    off = align_up(off + P.bytes);
  }
  return off;
}

static vip_status svgd_multi(vip_ctx *ctx, int32_t nens, const vip_ensemble *ens, int32_t bw_mode,
                             double h_fixed, int32_t gram_prec, bool noise, uint64_t seed,
                             uint64_t stream, void *ws, size_t ws_bytes) {
  if (!ctx || !ens || !ws || nens < 1) return VIP_E_ARG;
  // every ensemble is checked before the first is updated in place
  for (int e = 0; e < nens; ++e)
    VIP_TRY(svgd_check(ens[e].n, ens[e].d, ens[e].x, ens[e].g, ens[e].eps, bw_mode, h_fixed,
                       gram_prec, &ens[e].prior, noise, nullptr, VIP_KERNEL_RBF));
  std::vector<size_t> offs;
  const size_t need = plan_svgd_multi(nens, ens, &offs);
  if (ws_bytes < need || !aligned(ws)) return VIP_E_WORKSPACE;
  char *base = static_cast<char *>(ws);
  for (int e = 0; e < nens; ++e) {
    const vip_ensemble &E = ens[e];
    VIP_TRY(svgd_common(ctx, E.n, E.d, E.x, E.g, E.eps, bw_mode, h_fixed, gram_prec, &E.prior, noise,
                        E.xi, seed, stream + uint64_t(e), E.h2_out, base + offs[size_t(e)],
                        ws_bytes - offs[size_t(e)], reinterpret_cast<uint32_t *>(base)));
  }
  return VIP_OK;
}

}  // namespace vip

extern "C" {

vip_status vip_svgd_multi_workspace(int32_t nens, const vip_ensemble *ens, size_t *bytes) {
  if (!bytes || !ens || nens < 1) return VIP_E_ARG;
  for (int e = 0; e < nens; ++e)
    if (ens[e].n < 1 || ens[e].d < 1) return VIP_E_ARG;
  std::vector<size_t> offs;
  *bytes = vip::plan_svgd_multi(nens, ens, &offs);
  return VIP_OK;
}

vip_status vip_svgd_step_multi(vip_ctx *ctx, int32_t nens, const vip_ensemble *ens, int32_t bw_mode,
                               double h_fixed, int32_t gram_prec, void *ws, size_t ws_bytes) {
  return vip::svgd_multi(ctx, nens, ens, bw_mode, h_fixed, gram_prec, false, 0, 0, ws, ws_bytes);
}

vip_status vip_ssvgd_step_multi(vip_ctx *ctx, int32_t nens, const vip_ensemble *ens,
                                int32_t bw_mode, double h_fixed, int32_t gram_prec, uint64_t seed,
                                uint64_t stream, void *ws, size_t ws_bytes) {
  return vip::svgd_multi(ctx, nens, ens, bw_mode, h_fixed, gram_prec, true, seed, stream, ws,
                         ws_bytes);
}

vip_status vip_ssvgd_step(vip_ctx *ctx, int32_t n, int64_t d, float *x, const float *g, double eps,
                          int32_t bw_mode, double h_fixed, int32_t gram_prec,
                          const vip_prior *prior, const float *xi, uint64_t seed, uint64_t stream,
                          double *h2_out, void *ws, size_t ws_bytes) {
  return svgd_common(ctx, n, d, x, g, eps, bw_mode, h_fixed, gram_prec, prior, true, xi, seed,
                     stream, h2_out, ws, ws_bytes);
}

}  // extern "C"

// ---- allocation-free variant of the SVGD step --------------------------------
// For callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid it): vip_svgd_step_noalloc runs
// the same kernels as vip_svgd_step with the step's workspace in a fixed
// array of the library, `scratch`, instead of a caller workspace.  In host
// code `scratch` names a host-side stand-in, so kernels and fills are given
// its device address, taken once per device by vip_noalloc_setup.

namespace vip {

static __device__ __align__(256) unsigned char scratch[VIP_NOALLOC_SCRATCH_BYTES];

constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kScratchDevices];

// Device address of `scratch` on `device`; vip_create calls it with `device`
// current, so every context has it before its first step.
vip_status vip_noalloc_setup(int device) {
  if (device < 0 || device >= kScratchDevices) return VIP_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return VIP_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    set_last_hip_error(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
    return VIP_E_HIP;
  }
  g_scratch_ptr[device] = ptr;
  return VIP_OK;
}

static void *scratch_of(int device) {
  if (device < 0 || device >= kScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace vip

extern "C" vip_status vip_svgd_step_noalloc(vip_ctx *ctx, int32_t n, int64_t d, float *x,
                                            const float *g, double eps, int32_t bw_mode,
                                            double h_fixed, int32_t gram_prec,
                                            const vip_prior *prior, double *h2_out,
                                            uint32_t *status) {
  if (!ctx) return VIP_E_ARG;
  VIP_TRY(svgd_check(n, d, x, g, eps, bw_mode, h_fixed, gram_prec, prior, false, nullptr,
                     VIP_KERNEL_RBF));
  SvgdPlan P;
  plan_svgd(n, d, nullptr, &P);
  if (P.bytes > size_t(VIP_NOALLOC_SCRATCH_BYTES)) return VIP_E_SCRATCH;
  void *ws = scratch_of(ctx->device);
  if (!ws) return VIP_E_HIP;   // vip_create could not take the array's address
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  // the array keeps the previous call's contents: the status word that the
  // kernels latch flags into starts at zero (every other buffer the step reads
  // is written earlier in the same step)
  if (!status) VIP_TRY(fill_u32(ctx->user, static_cast<uint32_t *>(ws), 1, 0u));
  return svgd_common(ctx, n, d, x, g, eps, bw_mode, h_fixed, gram_prec, prior, false, nullptr, 0,
                     0, h2_out, ws, size_t(VIP_NOALLOC_SCRATCH_BYTES), status);
}
