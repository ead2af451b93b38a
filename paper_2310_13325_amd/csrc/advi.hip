// Automatic differentiation variational inference (section 2.2: eq:normal,
// eq:gradient_mu, eq:gradient_L; the mean-field family of section 5).
//
//   sample  theta_s = mu + L eta_s                        (reparameterised eq:normal)
//   step    grad_mu = 1/S sum_s g_s                       (eq:gradient_mu)
//           grad_L  = 1/S sum_s g_s eta_s^T + (L^-1)^T    (eq:gradient_L)
//           on the free entries of L: its lower triangle (full rank) or its
//           diagonal (mean field).  L^-1 of a lower-triangular L is lower
//           triangular with diagonal 1/L_ii, so the lower part of (L^-1)^T
//           is diag(1/L_ii): no inverse is formed.
//           mu and L then move uphill by a step rule (SGD, AdaGrad, AdaDelta,
//           Adam) with caller-owned state.
//   elbo    1/S sum_s log p(theta_s, d) + sum_i log|L_ii| + d/2 (1 + log 2 pi)
//
// The full-rank L is dense row-major with leading dimension ldl; only entries
// j <= i are read or written.  Both full-rank kernels stream the lower
// triangle once and are bound by HBM bandwidth: the sample reads 4 B per entry
// (per group of up to 8 samples), the step reads and writes L and the rule's
// state, 8 / 16 / 24 / 24 B per entry for SGD / AdaGrad / AdaDelta / Adam.
#include <cmath>

#include "vip_internal.h"
#include "opt_rules.h"

namespace vip {

constexpr int kAdviThreads = 256;
constexpr int kSampleRows = 8;      // rows per block of the full-rank sample
constexpr int kSampleGroup = 8;     // samples per pass over L
constexpr int kStepRows = 64;       // tile of the full-rank step: rows ...
constexpr int kStepCols = 256;      // ... and columns (one per thread; 4 kStepRows)
constexpr int kStepBatch = 8;       // rows whose loads a thread issues together

// ---- full-rank sample ----------------------------------------------------------
// A block owns kSampleRows consecutive rows and walks their columns up to the
// last row's diagonal, four columns per thread per pass (16-byte loads, with
// the columns past each row's diagonal masked; one column per pass when L or
// eta rows are not 16-byte aligned), holding the SG samples' eta of those
// columns in registers, so each L entry is read once per SG samples.  Blocks are numbered from the bottom of the triangle up, so the
// longest rows are dispatched first and the short ones fill in behind them.
// The rows x samples partial sums are reduced across the block in a fixed
// order.
template <int SG>
__global__ __launch_bounds__(kAdviThreads) void advi_sample_full_kernel(
    const float *__restrict__ mu, const float *__restrict__ L, long long ldl,
    const float *__restrict__ eta, float *__restrict__ theta, long long d, int S, int vec) {
  __shared__ float red[kAdviThreads / 64][kSampleRows * SG];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s0 = blockIdx.y * SG;
  const long long nb = (d + kSampleRows - 1) / kSampleRows;
  const long long r0 = (nb - 1 - (long long)blockIdx.x) * kSampleRows;
  const long long rlast = (r0 + kSampleRows < d ? r0 + kSampleRows : d) - 1;
  float acc[kSampleRows][SG];
#pragma unroll
  for (int r = 0; r < kSampleRows; ++r)
#pragma unroll
    for (int s = 0; s < SG; ++s) acc[r][s] = 0.f;
  if (vec) {
    // d and ldl are multiples of 4, so a 4-column group starting at c <= rlast
    // lies inside every row of L and of eta
    for (long long c = 4 * tid; c <= rlast; c += 4 * kAdviThreads) {
      float4 e[SG];
#pragma unroll
      for (int s = 0; s < SG; ++s)
        e[s] = s0 + s < S ? *reinterpret_cast<const float4 *>(eta + (long long)(s0 + s) * d + c)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int r = 0; r < kSampleRows; ++r) {
        const long long row = r0 + r;
        float4 v = (row <= rlast && c <= row) ? *reinterpret_cast<const float4 *>(L + row * ldl + c)
                                              : make_float4(0.f, 0.f, 0.f, 0.f);
        v.y = c + 1 <= row ? v.y : 0.f;   // past the diagonal
        v.z = c + 2 <= row ? v.z : 0.f;
        v.w = c + 3 <= row ? v.w : 0.f;
#pragma unroll
        for (int s = 0; s < SG; ++s) {
          float a = acc[r][s];
          a = fmaf(v.x, e[s].x, a);
          a = fmaf(v.y, e[s].y, a);
          a = fmaf(v.z, e[s].z, a);
          acc[r][s] = fmaf(v.w, e[s].w, a);
        }
      }
    }
  } else {
    for (long long c = tid; c <= rlast; c += kAdviThreads) {
      float e[SG];
#pragma unroll
      for (int s = 0; s < SG; ++s) e[s] = s0 + s < S ? eta[(long long)(s0 + s) * d + c] : 0.f;
      float v[kSampleRows];
#pragma unroll
      for (int r = 0; r < kSampleRows; ++r) {
        const long long row = r0 + r;
        v[r] = (row <= rlast && c <= row) ? L[row * ldl + c] : 0.f;
      }
#pragma unroll
      for (int r = 0; r < kSampleRows; ++r)
#pragma unroll
        for (int s = 0; s < SG; ++s) acc[r][s] = fmaf(v[r], e[s], acc[r][s]);
    }
  }
#pragma unroll
  for (int r = 0; r < kSampleRows; ++r)
#pragma unroll
    for (int s = 0; s < SG; ++s) {
      float t = acc[r][s];
      for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
      if (lane == 0) red[wave][r * SG + s] = t;
    }
  __syncthreads();
  if (tid < kSampleRows * SG) {
    const int r = tid / SG, s = tid % SG;
    const long long row = r0 + r;
    if (row <= rlast && s0 + s < S) {
      const float t = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
      theta[(long long)(s0 + s) * d + row] = mu[row] + t;
    }
  }
}

// ---- full-rank step --------------------------------------------------------------
// Tiles of kStepRows rows x kStepCols columns over the lower triangle.  Row
// block rb has floor(rb / 4) + 1 column tiles (kStepCols = 4 kStepRows), so
// the row blocks come in quads q of 4 (q + 1) tiles and tile t decodes to
// (rb, tc) through the quad's prefix 2 q (q + 1).  A thread owns one column
// of its tile: it keeps eta_s of that column in registers and walks the
// tile's rows kStepBatch at a time (loads of L and state first, then the
// arithmetic, then the stores); the tile's rows of g sit in LDS and are read
// as broadcasts.  The last column tile of each row block holds its diagonal
// and also steps mu for those rows.
template <int SG>
__global__ __launch_bounds__(kAdviThreads) void advi_step_full_kernel(
    float *__restrict__ mu, float *__restrict__ L, long long ldl, const float *__restrict__ eta,
    const float *__restrict__ g, long long d, int S, float inv_s, float eps, OptArgs om,
    OptArgs ol, float *__restrict__ grad_mu, float *__restrict__ grad_L) {
  __shared__ float gt[SG][kStepRows];
  const long long t = blockIdx.x;
  long long q = (long long)((sqrt(2.0 * double(t) + 1.0) - 1.0) * 0.5);
  while (2 * q * (q + 1) > t) --q;
  while (2 * (q + 1) * (q + 2) <= t) ++q;
  const long long u = t - 2 * q * (q + 1);
  const long long rb = 4 * q + u / (q + 1), tc = u % (q + 1);
  const long long r0 = rb * kStepRows, c0 = tc * kStepCols;
  const int tid = threadIdx.x;
  for (int e = tid; e < SG * kStepRows; e += kAdviThreads) {
    const int s = e / kStepRows, r = e % kStepRows;
    const long long row = r0 + r;
    gt[s][r] = (s < S && row < d) ? g[(long long)s * d + row] : 0.f;
  }
  __syncthreads();
  if (tc == q && tid < kStepRows) {
    const long long row = r0 + tid;
    if (row < d) {
      float sum = 0.f;
#pragma unroll
      for (int s = 0; s < SG; ++s) sum += gt[s][tid];
      const float gm = sum * inv_s;
      if (grad_mu) grad_mu[row] = gm;
      mu[row] += opt_step(om, row, gm, eps);
    }
  }
  const long long c = c0 + tid;
  if (c >= d) return;
  float e[SG];
#pragma unroll
  for (int s = 0; s < SG; ++s) e[s] = s < S ? eta[(long long)s * d + c] : 0.f;
  const long long rbeg = r0 > c ? r0 : c;
  const long long rend = r0 + kStepRows < d ? r0 + kStepRows : d;
  for (long long row = rbeg; row < rend; row += kStepBatch) {
    float l[kStepBatch];
    OptState st[kStepBatch];
#pragma unroll
    for (int k = 0; k < kStepBatch; ++k) {
      if (row + k < rend) {
        const long long idx = (row + k) * ldl + c;
        l[k] = L[idx];
        st[k] = opt_load(ol, idx);
      }
    }
#pragma unroll
    for (int k = 0; k < kStepBatch; ++k) {
      if (row + k < rend) {
        const int r = int(row + k - r0);
        float sum = 0.f;
#pragma unroll
        for (int s = 0; s < SG; ++s) sum = fmaf(gt[s][r], e[s], sum);
        float gl = sum * inv_s;
        if (row + k == c) gl += 1.0f / l[k];
        const long long idx = (row + k) * ldl + c;
        if (grad_L) grad_L[idx] = gl;
        L[idx] = l[k] + opt_apply(ol, st[k], gl, eps);
        opt_store(ol, idx, st[k]);
      }
    }
  }
}

// Number of tiles of advi_step_full_kernel for dimension d.
static long long step_tiles(long long d) {
  const long long nrb = (d + kStepRows - 1) / kStepRows;
  const long long Q = nrb / 4;
  return 2 * Q * (Q + 1) + (nrb - 4 * Q) * (Q + 1);
}

// ---- mean field ------------------------------------------------------------------
__global__ __launch_bounds__(kAdviThreads) void advi_sample_diag_kernel(
    const float *__restrict__ mu, const float *__restrict__ l, const float *__restrict__ eta,
    float *__restrict__ theta, long long d, long long total) {
  const long long e = (long long)blockIdx.x * kAdviThreads + threadIdx.x;
  if (e >= total) return;
  const long long i = e % d;
  theta[e] = fmaf(l[i], eta[e], mu[i]);
}

__global__ __launch_bounds__(kAdviThreads) void advi_step_diag_kernel(
    float *__restrict__ mu, float *__restrict__ l, const float *__restrict__ eta,
    const float *__restrict__ g, long long d, int S, float inv_s, float eps, OptArgs om,
    OptArgs ol, float *__restrict__ grad_mu, float *__restrict__ grad_l) {
  const long long i = (long long)blockIdx.x * kAdviThreads + threadIdx.x;
  if (i >= d) return;
  float sg = 0.f, sge = 0.f;
  for (int s = 0; s < S; ++s) {
    const float gs = g[(long long)s * d + i];
    sg += gs;
    sge = fmaf(gs, eta[(long long)s * d + i], sge);
  }
  const float li = l[i];
  const float gm = sg * inv_s;
  const float gl = sge * inv_s + 1.0f / li;
  if (grad_mu) grad_mu[i] = gm;
  if (grad_l) grad_l[i] = gl;
  mu[i] += opt_step(om, i, gm, eps);
  l[i] = li + opt_step(ol, i, gl, eps);
}

// ---- ELBO estimate ---------------------------------------------------------------
// One block: FP64 sum of log|L_ii| (diagonal at stride ldiag), the mean of the
// samples' log p, and the Gaussian entropy constant.
__global__ __launch_bounds__(kAdviThreads) void advi_elbo_kernel(
    const float *__restrict__ L, long long ldiag, long long d, const double *__restrict__ logp,
    int S, double *__restrict__ elbo) {
  __shared__ double part[kAdviThreads / 64];
  double t = 0.0;
  for (long long i = threadIdx.x; i < d; i += kAdviThreads) t += log(fabs(double(L[i * ldiag])));
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double lp = 0.0;
    for (int s = 0; s < S; ++s) lp += logp[s];
    const double two_pi = 6.283185307179586476925286766559;
    elbo[0] = lp / double(S) + ((part[0] + part[1]) + (part[2] + part[3])) +
              0.5 * double(d) * (1.0 + log(two_pi));
  }
}

static int pow2_at_least(int s) {
  int p = 1;
  while (p < s) p <<= 1;
  return p;
}

static vip_status check_family(int32_t family, int64_t d, int32_t S, int64_t ldl) {
  if (family != VIP_ADVI_FULL_RANK && family != VIP_ADVI_MEAN_FIELD) return VIP_E_ARG;
  if (d < 1 || S < 1 || S > VIP_ADVI_MAX_SAMPLES) return VIP_E_ARG;
  if (family == VIP_ADVI_FULL_RANK && ldl < d) return VIP_E_ARG;
  return VIP_OK;
}

}  // namespace vip

using namespace vip;

extern "C" vip_status vip_advi_sample(vip_ctx *ctx, int32_t family, int64_t d, int32_t S,
                                      const float *mu, const float *L, int64_t ldl,
                                      const float *eta, float *theta) {
  if (!ctx || !mu || !L || !eta || !theta) return VIP_E_ARG;
  VIP_TRY(check_family(family, d, S, ldl));
  hipStream_t s = ctx->user;
  if (family == VIP_ADVI_MEAN_FIELD) {
    const long long total = (long long)S * d;
    advi_sample_diag_kernel<<<dim3(unsigned((total + kAdviThreads - 1) / kAdviThreads)),
                              dim3(kAdviThreads), 0, s>>>(mu, L, eta, theta, d, total);
    VIP_LAUNCH_CHECK();
    return VIP_OK;
  }
  const long long nb = (d + kSampleRows - 1) / kSampleRows;
  const int sg = S <= kSampleGroup ? pow2_at_least(S) : kSampleGroup;
  const dim3 grid(unsigned(nb), unsigned((S + sg - 1) / sg));
  const int vec = d % 4 == 0 && ldl % 4 == 0 && reinterpret_cast<uintptr_t>(L) % 16 == 0 &&
                  reinterpret_cast<uintptr_t>(eta) % 16 == 0;
  switch (sg) {
    case 1: advi_sample_full_kernel<1><<<grid, dim3(kAdviThreads), 0, s>>>(mu, L, ldl, eta, theta, d, S, vec); break;
    case 2: advi_sample_full_kernel<2><<<grid, dim3(kAdviThreads), 0, s>>>(mu, L, ldl, eta, theta, d, S, vec); break;
    case 4: advi_sample_full_kernel<4><<<grid, dim3(kAdviThreads), 0, s>>>(mu, L, ldl, eta, theta, d, S, vec); break;
    default: advi_sample_full_kernel<8><<<grid, dim3(kAdviThreads), 0, s>>>(mu, L, ldl, eta, theta, d, S, vec); break;
  }
  VIP_LAUNCH_CHECK();
  return VIP_OK;
}

extern "C" vip_status vip_advi_step(vip_ctx *ctx, int32_t family, int64_t d, int32_t S, float *mu,
                                    float *L, int64_t ldl, const float *eta, const float *g,
                                    double eps, const vip_optimizer *opt_mu,
                                    const vip_optimizer *opt_L, float *grad_mu, float *grad_L,
                                    const double *logpost, double *elbo) {
  if (!ctx || !mu || !L || !eta || !g) return VIP_E_ARG;
  VIP_TRY(check_family(family, d, S, ldl));
  if (!(eps >= 0.0) || !std::isfinite(eps)) return VIP_E_ARG;
  if (elbo && !logpost) return VIP_E_ARG;
  OptArgs om, ol;
  VIP_TRY(make_opt_args(opt_mu, &om));
  VIP_TRY(make_opt_args(opt_L, &ol));
  hipStream_t s = ctx->user;
  const bool full = family == VIP_ADVI_FULL_RANK;
  if (elbo) {
    advi_elbo_kernel<<<dim3(1), dim3(kAdviThreads), 0, s>>>(L, full ? ldl + 1 : 1, d, logpost,
                                                             S, elbo);
    VIP_LAUNCH_CHECK();
  }
  const float inv_s = float(1.0 / double(S));
  const float e = float(eps);
  if (!full) {
    advi_step_diag_kernel<<<dim3(unsigned((d + kAdviThreads - 1) / kAdviThreads)),
                            dim3(kAdviThreads), 0, s>>>(mu, L, eta, g, d, S, inv_s, e, om, ol,
                                                        grad_mu, grad_L);
    VIP_LAUNCH_CHECK();
    return VIP_OK;
  }
  const dim3 grid(unsigned(step_tiles(d)));
  const dim3 block(kAdviThreads);
  switch (pow2_at_least(S)) {
    case 1: advi_step_full_kernel<1><<<grid, block, 0, s>>>(mu, L, ldl, eta, g, d, S, inv_s, e, om, ol, grad_mu, grad_L); break;
    case 2: advi_step_full_kernel<2><<<grid, block, 0, s>>>(mu, L, ldl, eta, g, d, S, inv_s, e, om, ol, grad_mu, grad_L); break;
    case 4: advi_step_full_kernel<4><<<grid, block, 0, s>>>(mu, L, ldl, eta, g, d, S, inv_s, e, om, ol, grad_mu, grad_L); break;
    case 8: advi_step_full_kernel<8><<<grid, block, 0, s>>>(mu, L, ldl, eta, g, d, S, inv_s, e, om, ol, grad_mu, grad_L); break;
    case 16: advi_step_full_kernel<16><<<grid, block, 0, s>>>(mu, L, ldl, eta, g, d, S, inv_s, e, om, ol, grad_mu, grad_L); break;
    default: advi_step_full_kernel<32><<<grid, block, 0, s>>>(mu, L, ldl, eta, g, d, S, inv_s, e, om, ol, grad_mu, grad_L); break;
  }
  VIP_LAUNCH_CHECK();
  return VIP_OK;
}
