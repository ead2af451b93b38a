// 2-D acoustic finite-difference modelling, its exact discrete adjoint and
// the adjoint-state gradient of the log-posterior (paper section 4.2; adjoint
// method of section 3), batched over every (particle, shot) pair.
//
// Scheme (second order in time, fourth in space, Cerjan sponge g):
//   q^{n+1} = g (q^n + c (L u^n + f^n)),  u^{n+1} = g u^n + q^{n+1},  c = v^2 dt^2
// which is u^{n+1} = g (2u^n + c (L u^n + f^n) - g u^{n-1}) carried in increment
// form (q = u^{n+1} - g u^n) so FP32 keeps the small per-step change exactly
// instead of recovering it from the difference of two large fields; the
// Laplacian is evaluated as sum_o w_o (u_{i+o} - u_i) (the weights sum to 0),
// which keeps the same property inside the stencil.
//
// Adjoint (scaled multiplier z = g c lambda) obeys the same recurrence run
// backwards with the residual injected at the receivers:
//   Q^j = g (Q^{j+1} + c (L z^{j+1} + R^T rho^j)),  z^j = g z^{j+1} + Q^j,
// and the gradient is dJ/dv_pad = (2/v_pad) sum_n z^{n+1} (L u^n + f^n),
// folded back onto the model by the transpose of the edge padding.
//
// Time stepping launches one kernel per step over all live pairs; each block
// owns a 64-column x 4*RZ-row tile, stages u (the only field read at
// neighbours) with its two-cell halo in LDS, and fuses the source injection,
// the receiver gather (forward), the residual injection and the imaging sum
// (adjoint), and the checkpoint writes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "vip_internal.h"
#include "fwi_plan.h"
#include "fd_block.h"
#include "fd_pipe.h"

namespace vip {

// step-kernel kinds (also the timing kinds; MODE_FWS: forward that stores a^n)
enum { MODE_FWD = 0, MODE_REC = 1, MODE_ADJ = 2, MODE_FWS = 3 };

struct StepArgs {
  int NX, NZ, N;
  int tiles_x, tiles_per_pair, total_tiles;
  int pair0, ns, nt, nr;
  float cx, cz, inv_area;
  const float *gx, *gz, *c;
  const int *src_idx, *rrow, *rmap;
  const float *wavelet;
  uint32_t *status;
  int n;          // FWD/REC: index of the input state u^n; ADJ: produces z^{n+1}
  int zero_in;    // input state is identically zero (nothing read)
  const float *u_in, *q_in;
  long long in_stride;
  float *u_out, *q_out;   // null: do not advance
  long long out_stride;
  float *data;            // FWD: receiver traces [pair][nt][nr]
  long long data_stride;
  float *seg;             // REC: a^n slot written; ADJ: a^n slot read
  long long seg_stride;
  const float *rho;       // ADJ: residual [pair][nt][nr]
  long long rho_stride;
  double *acc64;          // ADJ: FP64 imaging sum [pair][N]
  long long acc64_stride;
};

__device__ __forceinline__ int tile_of_block(int total_tiles) {
  // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of tiles so that neighbouring tiles (shared halos) and
  // the shots of one particle (shared coefficients) meet in the same L2.
  int per = int(gridDim.x) >> 3;
  int b = int(blockIdx.x);
  return (b & 7) * per + (b >> 3);
}

template <int MODE, int RZ>
__global__ __launch_bounds__(256) void fd_step(StepArgs a) {
  constexpr int BZ = 4 * RZ;
  constexpr int LW = 64 + 4;
  constexpr float w1 = 4.0f / 3.0f, w2 = -1.0f / 12.0f;
  __shared__ float tile[BZ + 4][LW];

  const int t = tile_of_block(a.total_tiles);
  if (t >= a.total_tiles) return;
  const int lp = t / a.tiles_per_pair;
  const int rem = t - lp * a.tiles_per_pair;
  const int tzi = rem / a.tiles_x;
  const int txi = rem - tzi * a.tiles_x;
  const int x0 = txi * 64, z0 = tzi * BZ;
  const int tx = int(threadIdx.x) & 63, ty = int(threadIdx.x) >> 6;
  const int gp = a.pair0 + lp;
  const int particle = gp / a.ns;
  const int shot = gp - particle * a.ns;
  const int NX = a.NX;

  const float *uin = a.u_in + lp * a.in_stride;
  const int x = x0 + tx;
  const int xh = tx < 2 ? x0 - 2 + tx : x0 + 62 + tx;   // halo column for lanes 0..3
  const int ch = tx < 2 ? tx : 64 + tx;                  // its LDS column
  for (int r = ty; r < BZ + 4; r += 4) {
    const int z = z0 - 2 + r;
    const bool zin = z >= 0 && z < a.NZ;
    float v = 0.0f;
    if (!a.zero_in && zin && x < NX) v = uin[z * NX + x];
    tile[r][tx + 2] = v;
    if (tx < 4) {
      float h = 0.0f;
      if (!a.zero_in && zin && xh >= 0 && xh < NX) h = uin[z * NX + xh];
      tile[r][ch] = h;
    }
  }
  __syncthreads();
  if (x >= NX) return;

  const float gxv = a.gx[x];
  const float *cp = a.c + size_t(particle) * size_t(a.N);
  const float *qin = a.q_in + lp * a.in_stride;
  int src = -1;
  float src_amp = 0.0f;
  if (MODE != MODE_ADJ) {
    src = a.src_idx[shot];
    src_amp = a.wavelet[a.n] * a.inv_area;
  }
#pragma unroll
  for (int k = 0; k < RZ; ++k) {
    const int r = ty * RZ + k;
    const int z = z0 + r;
    if (z >= a.NZ) break;
    const int i = z * NX + x;
    const float uc = tile[r + 2][tx + 2];
    const float lx = w1 * ((tile[r + 2][tx + 1] - uc) + (tile[r + 2][tx + 3] - uc)) +
                     w2 * ((tile[r + 2][tx] - uc) + (tile[r + 2][tx + 4] - uc));
    const float lz = w1 * ((tile[r + 1][tx + 2] - uc) + (tile[r + 3][tx + 2] - uc)) +
                     w2 * ((tile[r][tx + 2] - uc) + (tile[r + 4][tx + 2] - uc));
    float lap = a.cx * lx + a.cz * lz;
    int rid = -1;
    if (MODE != MODE_REC) {
      const int rr = a.rrow[z];
      if (rr >= 0) rid = a.rmap[rr * NX + x];
    }
    if (MODE != MODE_ADJ) {
      if (i == src) lap += src_amp;
    } else if (rid >= 0) {
      lap += a.rho[lp * a.rho_stride + (long long)(a.n + 1) * a.nr + rid];
    }
    if (MODE == MODE_REC) a.seg[lp * a.seg_stride + i] = lap;
    const float gv = a.gz[z] * gxv;
    const float qv = a.zero_in ? 0.0f : qin[i];
    const float qn = gv * (qv + cp[i] * lap);
    const float un = gv * uc + qn;
    if (a.u_out) {
      a.u_out[lp * a.out_stride + i] = un;
      a.q_out[lp * a.out_stride + i] = qn;
    }
    if (MODE == MODE_FWD && rid >= 0) {
      float *d = a.data + lp * a.data_stride;
      d[(long long)(a.n + 1) * a.nr + rid] = un;
      if (a.n == 0) d[rid] = 0.0f;   // u^0 = 0
    }
    if (MODE == MODE_ADJ)   // every step's product goes into the FP64 sum (one add per point)
      __hip_atomic_fetch_add(a.acc64 + lp * a.acc64_stride + i,
                             double(un * a.seg[lp * a.seg_stride + i]), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
}

// c = (v_pad dt)^2 for every particle; v_pad replicates the model edges.  The
// product is formed in FP64 and rounded to FP32 once: c scales the whole
// stencil update, and each extra ulp of it shifts the simulated travel times,
// an error that grows linearly along the sweep.
__global__ void coeff_kernel(const float *vel, float *c, int np, int nx, int nz, int nb, int NX,
                             int NZ, double dt, float vmax, uint32_t *status) {
  long long N = (long long)NX * NZ;
  long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * np) return;
  int p = int(idx / N);
  int i = int(idx - (long long)p * N);
  int Z = i / NX, X = i - Z * NX;
  int iz = min(max(Z - nb, 0), nz - 1), ix = min(max(X - nb, 0), nx - 1);
  float v = vel[(long long)p * nx * nz + (long long)iz * nx + ix];
  if (!(v > 0.0f) || !(v <= vmax)) {
    if (!isfinite(v)) atomicOr(status, VIP_FLAG_NONFINITE);
    else atomicOr(status, VIP_FLAG_VMAX);
  }
  const double vd = double(v) * dt;
  c[idx] = float(vd * vd);
}

// Cerjan profile gamma(delta) = exp(-(alpha delta)^2) along one padded axis.
__global__ void sponge_kernel(float *g, int n, int nb, double alpha) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n + 2 * nb) return;
  int delta = max(max(nb - k, k - (nb + n - 1)), 0);
  double ad = alpha * double(delta);
  g[k] = float(exp(-ad * ad));
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Residual rho = w (d - dobs)/sigma^2 in place and J = w/2 sum (d - dobs)^2/sigma^2
// per pair (FP64, fixed reduction order); inv_s2 = w / sigma^2, w the misfit
// scale of a shot subset (1 for the whole survey).
// One block of 1024 threads per pair; 16-byte accesses when the rows allow.
constexpr int RESID_T = 1024;
__global__ __launch_bounds__(RESID_T) void residual_kernel(float *d, long long d_stride,
                                                           const float *dobs, const int *shot_row,
                                                           int pair0, int ns, long long per_pair,
                                                           double inv_s2, double *J,
                                                           uint32_t *status) {
  __shared__ double part[RESID_T / 64];
  const int lp = blockIdx.x;
  const int shot = (pair0 + lp) % ns;
  float *dp = d + lp * d_stride;
  const float *op = dobs + (long long)shot_row[shot] * per_pair;
  double acc = 0.0;
  const bool vec = per_pair % 4 == 0 &&
                   ((reinterpret_cast<uintptr_t>(dp) | reinterpret_cast<uintptr_t>(op)) & 15) == 0;
  if (vec) {
    float4 *d4 = reinterpret_cast<float4 *>(dp);
    const float4 *o4 = reinterpret_cast<const float4 *>(op);
#pragma unroll 4
    for (long long e = threadIdx.x; e < per_pair / 4; e += RESID_T) {
      float4 dv = d4[e];
      const float4 ov = o4[e];
      const double r0 = double(dv.x) - double(ov.x), r1 = double(dv.y) - double(ov.y);
      const double r2 = double(dv.z) - double(ov.z), r3 = double(dv.w) - double(ov.w);
      acc += r0 * r0;
      acc += r1 * r1;
      acc += r2 * r2;
      acc += r3 * r3;
      dv.x = float(r0 * inv_s2);
      dv.y = float(r1 * inv_s2);
      dv.z = float(r2 * inv_s2);
      dv.w = float(r3 * inv_s2);
      d4[e] = dv;
    }
  } else {
    for (long long e = threadIdx.x; e < per_pair; e += RESID_T) {
      const double r = double(dp[e]) - double(op[e]);
      acc += r * r;
      dp[e] = float(r * inv_s2);
    }
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < RESID_T / 64; ++w) t += part[w];
    const double j = 0.5 * t * inv_s2;
    if (!isfinite(j)) atomicOr(status, VIP_FLAG_NONFINITE);
    J[pair0 + lp] = j;
  }
}

// grad[p][iz][ix] = sign * (2 / v) * sum_shots sum_{padded cells copied from (iz, ix)} acc64
__global__ void finalize_grad_kernel(const double *acc64, const float *vel, float *grad, int np,
                                     int ns, int nx, int nz, int nb, int NX, float sign) {
  long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long d = (long long)nx * nz;
  if (idx >= d * np) return;
  int p = int(idx / d);
  int cell = int(idx - (long long)p * d);
  int iz = cell / nx, ix = cell - iz * nx;
  int NZ = nz + 2 * nb;
  int r0 = (iz == 0) ? 0 : nb + iz, r1 = (iz == nz - 1) ? NZ - 1 : nb + iz;
  int c0 = (ix == 0) ? 0 : nb + ix, c1 = (ix == nx - 1) ? NX - 1 : nb + ix;
  long long N = (long long)NX * NZ;
  double s = 0.0;
  if (r0 == r1 && c0 == c1) {
    // an interior cell: one padded cell per shot (loads issued together, sum in shot order)
    const double *a = acc64 + (long long)p * ns * N + (long long)r0 * NX + c0;
#pragma unroll 5
    for (int sh = 0; sh < ns; ++sh) s += a[sh * N];
  } else {
    for (int sh = 0; sh < ns; ++sh) {
      const double *a = acc64 + ((long long)p * ns + sh) * N;
      for (int r = r0; r <= r1; ++r)
        for (int c = c0; c <= c1; ++c) s += a[(long long)r * NX + c];
    }
  }
  grad[idx] = float(double(sign) * 2.0 * s / double(vel[idx]));
}

// logpost[p] = -sum_s J[p][s] + log prior (0 inside a uniform box, -inf outside)
// Prior terms, FP64 per coordinate (section 3, eq:transform).  For the
// transform kind t is theta and s = 1 / (1 + exp(-theta)): m = a + (b - a) s,
// log|dm/dtheta| = log(b - a) + log s + log(1 - s), d/dtheta of it = 1 - 2 s.
__device__ __forceinline__ double softplus(double x) { return fmax(x, 0.0) + log1p(exp(-fabs(x))); }
__device__ __forceinline__ double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

// logpost[p] = -sum_s J[p][s] + log prior; vel holds what the caller passed
// (theta for the transform kind), model the velocities the sweeps used.
__global__ __launch_bounds__(256) void logpost_kernel(const double *J, const float *vel,
                                                      const float *model, int kind,
                                                      const float *lo, const float *hi,
                                                      const float *mean, const float *sd, int ns,
                                                      long long d, double *logpost,
                                                      uint32_t *status) {
  __shared__ double part[4];
  __shared__ int outside_s;
  const int p = blockIdx.x;
  if (threadIdx.x == 0) outside_s = 0;
  __syncthreads();
  double acc = 0.0;
  int out = 0;
  for (long long e = threadIdx.x; e < d; e += 256) {
    const long long i = (long long)p * d + e;
    if (kind == VIP_PRIOR_UNIFORM_CLIP) {
      const float v = model[i];
      out |= !(v >= lo[e] && v <= hi[e]);
    } else if (kind == VIP_PRIOR_UNIFORM_TRANSFORM) {
      const double t = double(vel[i]);
      acc += log(double(hi[e]) - double(lo[e])) - softplus(-t) - softplus(t);
    } else if (kind == VIP_PRIOR_GAUSSIAN) {
      const double z = (double(model[i]) - double(mean[e])) / double(sd[e]);
      acc -= 0.5 * z * z;
    }
  }
  if (out) atomicOr(&outside_s, 1);
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double j = 0.0;
    for (int s = 0; s < ns; ++s) j += J[(long long)p * ns + s];
    double lp = -j + ((part[0] + part[1]) + (part[2] + part[3]));
    if (outside_s) lp = -INFINITY;
    if (!isfinite(j)) atomicOr(status, VIP_FLAG_NONFINITE);
    logpost[p] = lp;
  }
}

// m = a + (b - a) / (1 + exp(-theta)) (direction 0) or theta = log(m - a) -
// log(b - m) (direction 1), elementwise over [n][d].
__global__ void prior_transform_kernel(const float *in, float *out, const float *lo,
                                       const float *hi, long long total, long long d,
                                       int direction) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long long e = i % d;
  const double a = lo[e], b = hi[e], x = in[i];
  out[i] = direction == 0 ? float(a + (b - a) * sigmoid(x)) : float(log(x - a) - log(b - x));
}

// Gradient of the prior terms, in place on grad = d(-J)/dm: the transform
// kind maps it to theta, dlogp/dm dm/dtheta + (1 - 2 s); the Gaussian kind
// adds -(m - mean) / std^2.
__global__ void prior_grad_kernel(float *grad, const float *vel, const float *model, int kind,
                                  const float *lo, const float *hi, const float *mean,
                                  const float *sd, long long total, long long d) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long long e = i % d;
  if (kind == VIP_PRIOR_UNIFORM_TRANSFORM) {
    const double sg = sigmoid(double(vel[i]));
    grad[i] = float(double(grad[i]) * (double(hi[e]) - double(lo[e])) * sg * (1.0 - sg) +
                    (1.0 - 2.0 * sg));
  } else if (kind == VIP_PRIOR_GAUSSIAN) {
    const double sd2 = double(sd[e]) * double(sd[e]);
    grad[i] = float(double(grad[i]) - (double(model[i]) - double(mean[e])) / sd2);
  }
}

// --------------------------------------------------------------------------
// Host side
// --------------------------------------------------------------------------

static vip_status launch_step(vip_ctx *ctx, int mode, int rz, int npairs, StepArgs &a) {
  const int BZ = 4 * rz;
  const int tiles_z = (a.NZ + BZ - 1) / BZ;
  a.tiles_x = (a.NX + 63) / 64;
  a.tiles_per_pair = a.tiles_x * tiles_z;
  long long total = (long long)a.tiles_per_pair * npairs;
  if (total > (1LL << 30)) return VIP_E_UNSUPPORTED;
  a.total_tiles = int(total);
  unsigned blocks = unsigned((total + 7) / 8 * 8);
  dim3 grid(blocks), block(256);
  hipStream_t s = ctx->s();
#define VIP_STEP_CASE(M, R) \
  if (mode == M && rz == R) { fd_step<M, R><<<grid, block, 0, s>>>(a); VIP_LAUNCH_CHECK(); return VIP_OK; }
  VIP_STEP_CASE(MODE_FWD, 2) VIP_STEP_CASE(MODE_FWD, 4) VIP_STEP_CASE(MODE_FWD, 8)
  VIP_STEP_CASE(MODE_REC, 2) VIP_STEP_CASE(MODE_REC, 4) VIP_STEP_CASE(MODE_REC, 8)
  VIP_STEP_CASE(MODE_ADJ, 2) VIP_STEP_CASE(MODE_ADJ, 4) VIP_STEP_CASE(MODE_ADJ, 8)
#undef VIP_STEP_CASE
  return VIP_E_UNSUPPORTED;
}

static StepArgs base_args(const FwiDims &D, const FwiPlan &P, const float *wavelet, int pair0) {
  StepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.NX = D.NX;
  a.NZ = D.NZ;
  a.N = int(D.N);
  a.pair0 = pair0;
  a.ns = D.ns;
  a.nt = D.nt;
  a.nr = D.nr;
  a.cx = D.cx;
  a.cz = D.cz;
  a.inv_area = D.inv_area;
  a.gx = P.gx;
  a.gz = P.gz;
  a.c = P.c;
  a.src_idx = P.src;
  a.rrow = P.rrow;
  a.rmap = P.rmap;
  a.wavelet = wavelet;
  a.status = P.status;
  return a;
}

vip_status upload_tables(vip_ctx *ctx, const FwiDims &D, const vip_grid *grid,
                         const vip_geometry *geom, const FwiPlan &P) {
  hipStream_t s = ctx->s();
  sponge_kernel<<<dim3((D.NX + 255) / 256), dim3(256), 0, s>>>(P.gx, D.nx, D.nb, grid->sponge_alpha);
  VIP_LAUNCH_CHECK();
  sponge_kernel<<<dim3((D.NZ + 255) / 256), dim3(256), 0, s>>>(P.gz, D.nz, D.nb, grid->sponge_alpha);
  VIP_LAUNCH_CHECK();
  std::vector<int32_t> src(D.ns), rrow(D.NZ, -1), rmap(size_t(D.nrows) * D.NX, -1);
  for (int k = 0; k < D.ns; ++k) src[k] = (geom->src_iz[k] + D.nb) * D.NX + geom->src_ix[k] + D.nb;
  int rows = 0;
  for (int r = 0; r < D.nr; ++r) {
    int Z = geom->rec_iz[r] + D.nb;
    if (rrow[Z] < 0) rrow[Z] = rows++;
  }
  for (int r = 0; r < D.nr; ++r) {
    int Z = geom->rec_iz[r] + D.nb, X = geom->rec_ix[r] + D.nb;
    rmap[size_t(rrow[Z]) * D.NX + X] = r;   // nodes are distinct (checked in make_dims)
  }
  VIP_TRY(upload_i32(s, P.src, src.data(), src.size()));
  std::vector<int32_t> shot_row(D.ns);
  for (int k = 0; k < D.ns; ++k) shot_row[k] = geom->shot_index ? geom->shot_index[k] : k;
  VIP_TRY(upload_i32(s, P.shot_row, shot_row.data(), shot_row.size()));
  VIP_TRY(upload_i32(s, P.rrow, rrow.data(), rrow.size()));
  VIP_TRY(upload_i32(s, P.rmap, rmap.data(), rmap.size()));
  return VIP_OK;
}

vip_status launch_coeff(vip_ctx *ctx, const FwiDims &D, const vip_grid *grid, const float *vel,
                        const FwiPlan &P) {
  long long total = D.N * D.np;
  coeff_kernel<<<dim3(unsigned((total + 255) / 256)), dim3(256), 0, ctx->s()>>>(
      vel, P.c, D.np, D.nx, D.nz, D.nb, D.NX, D.NZ, grid->dt, float(grid->vmax), P.status);
  VIP_LAUNCH_CHECK();
  return VIP_OK;
}

// ---- temporally blocked sweeps -----------------------------------------------

struct TileCfg {
  int ex, ez, rz, tmax;
  int pipe;   // 1: persistent pipelined kernel (fd_pipe), one block per compute unit
};
// Instantiated tile shapes (extended width, extended height, rows per thread,
// steps per launch); the interior is (ex - 4 tmax) x (ez - 4 tmax).
static const TileCfg kTiles[] = {
    {112, 112, 14, 8},   // 0: interior 80 x 80, 896 threads
    {80, 80, 10, 4},     // 1: interior 64 x 64, 640 threads
    {96, 96, 12, 4},     // 2: interior 80 x 80, 768 threads
    {64, 64, 8, 4},      // 3: interior 48 x 48, 512 threads
    {128, 64, 8, 4},     // 4: interior 112 x 48, 1024 threads
    {104, 104, 13, 6},   // 5: interior 80 x 80, 832 threads
    {112, 112, 14, 8, 1},   // 6: shape 0, persistent with the next tile's loads in flight
};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);
constexpr int kPipeTile = 6;   // the persistent variant of shape 0

int tile_count() { return kNumTiles; }

// Default shape when no tuned choice exists, from a launch-time model fitted
// to the c2 gradient (240 x 160 padded points, 1280 pairs) timed per shape:
// blocks run in rounds of one per compute unit (two for shapes whose LDS
// allows it, sharing the unit), and a block costs W per extended point-step
// plus a fixed F for loading its tile and writing it back.  The fit gives
// W = 7.0e-5 us and F = 8.1 us (per step, 112^2: 55.8 us measured, 56.7
// modelled; 104^2: 65.0 / 63.2; 96^2 two per unit: 79.5 / 80.1).  The model
// holds while every unit has blocks: a launch with fewer blocks than units is
// bound by one block's latency, which the smaller shapes shorten, so there
// the shape that gives the most blocks (up to two per unit) is taken.
constexpr int kComputeUnits = 256;

static int tile_blocks_per_cu(int c) {
  const TileCfg &t = kTiles[c];
  return 2 * 2 * (t.ez + 4) * (t.ex + 4) * int(sizeof(float)) <= 160 * 1024 ? 2 : 1;
}

static long long tile_blocks(int c, int NX, int NZ, long long pairs) {
  const TileCfg &t = kTiles[c];
  const int ix = t.ex - 4 * t.tmax, iz = t.ez - 4 * t.tmax;
  return (long long)((NX + ix - 1) / ix) * ((NZ + iz - 1) / iz) * std::max(1LL, pairs);
}

// Modelled microseconds per time step of one launch over `pairs` pairs.
static double tile_cost(int c, int NX, int NZ, long long pairs) {
  constexpr double W = 7.0e-5, F = 8.1;
  const TileCfg &t = kTiles[c];
  const long long blocks = tile_blocks(c, NX, NZ, pairs);
  const long long k = tile_blocks_per_cu(c);
  const long long rounds = (blocks + kComputeUnits * k - 1) / (kComputeUnits * k);
  const long long share = std::min(k, (blocks + kComputeUnits - 1) / kComputeUnits);
  return double(rounds * share) * (W * t.ex * t.ez * t.tmax + F) / t.tmax;
}

// Better of two shapes for `pairs` pairs per launch (pairs <= 0: many).
static bool tile_better(int c, int b, int NX, int NZ, long long pairs) {
  if (pairs <= 0) pairs = 1LL << 20;
  const long long nc = tile_blocks(c, NX, NZ, pairs), nb = tile_blocks(b, NX, NZ, pairs);
  const bool fc = nc >= kComputeUnits, fb = nb >= kComputeUnits;
  if (fc != fb) return fc;
  if (!fc) {
    const long long uc = std::min<long long>(nc, kComputeUnits * tile_blocks_per_cu(c));
    const long long ub = std::min<long long>(nb, kComputeUnits * tile_blocks_per_cu(b));
    if (uc != ub) return uc > ub;
  }
  return tile_cost(c, NX, NZ, pairs) < tile_cost(b, NX, NZ, pairs);
}

int default_tile(int NX, int NZ, long long pairs) {
  int best = 0;
  for (int c = 1; c < kNumTiles; ++c)
    if (!kTiles[c].pipe && tile_better(c, best, NX, NZ, pairs)) best = c;
  // The persistent variant of shape 0 steps the same tiles with the next
  // tile's loads in flight; it pays once every unit has several tiles per
  // launch (c2 gradient: adjoint 409 -> 375 us per launch, forward with a^n
  // store unchanged).
  if (best == 0 && tile_blocks(0, NX, NZ, pairs <= 0 ? 1LL << 20 : pairs) >= 4 * kComputeUnits)
    best = kPipeTile;
  return best;
}

// One shape for a batch of problems launched together: the least summed
// modelled time when their blocks fill the units, else the most blocks.
static int default_tile_multi(const std::vector<FwiDims> &Ds) {
  if (Ds.size() == 1) return default_tile(Ds[0].NX, Ds[0].NZ, Ds[0].live);
  int best = 0;
  double best_cost = 1e300;
  long long best_blocks = 0;
  for (int c = 0; c < kNumTiles; ++c) {
    if (kTiles[c].pipe) continue;
    double cost = 0.0;
    long long blocks = 0;
    for (const FwiDims &D : Ds) {
      const long long launches = (D.pairs + D.live - 1) / D.live;
      cost += tile_cost(c, D.NX, D.NZ, D.live) * double(launches) * D.nt;
      blocks += tile_blocks(c, D.NX, D.NZ, D.live);
    }
    blocks = std::min<long long>(blocks, kComputeUnits * tile_blocks_per_cu(c));
    const bool better = blocks >= kComputeUnits && best_blocks >= kComputeUnits
                            ? cost < best_cost
                            : blocks > best_blocks || (blocks == best_blocks && cost < best_cost);
    if (better) best = c, best_cost = cost, best_blocks = blocks;
  }
  return best;
}

static vip_status set_tiles(int cfg, int npairs, BlockArgs &a) {
  const TileCfg &tc = kTiles[cfg];
  // byte offsets into one field (4 N) must stay below 2^31 (see field_rsrc)
  if (a.N >= kMaxBlockedPoints) return VIP_E_UNSUPPORTED;
  const int ix = tc.ex - 4 * tc.tmax, iz = tc.ez - 4 * tc.tmax;
  a.tiles_x = (a.NX + ix - 1) / ix;
  a.tiles_per_pair = a.tiles_x * ((a.NZ + iz - 1) / iz);
  const long long total = (long long)a.tiles_per_pair * npairs;
  if (total > (1LL << 30)) return VIP_E_UNSUPPORTED;
  a.total_tiles = int(total);
  return VIP_OK;
}

static vip_status launch_block(vip_ctx *ctx, int mode, int cfg, int npairs, BlockArgs &a) {
  const TileCfg &tc = kTiles[cfg];
  VIP_TRY(set_tiles(cfg, npairs, a));
  const long long total = a.total_tiles;
  const dim3 block(unsigned(tc.ex * (tc.ez / tc.rz)));
  hipStream_t s = ctx->s();
  if (tc.pipe) {
    // one resident block per compute unit, a multiple of the 8 XCDs
    const dim3 grid(unsigned(std::max(8, ctx->cus / 8 * 8)));
#define VIP_PIPE_MODES(EX, EZ, RZ, TM, ISO)                                                      \
  if (mode == BMODE_FWD) fd_pipe<BMODE_FWD, EX, EZ, RZ, TM, ISO, false><<<grid, block, 0, s>>>(a);      \
  else if (mode == BMODE_REC) fd_pipe<BMODE_REC, EX, EZ, RZ, TM, ISO, false><<<grid, block, 0, s>>>(a); \
  else if (mode == BMODE_FWS) fd_pipe<BMODE_FWS, EX, EZ, RZ, TM, ISO, false><<<grid, block, 0, s>>>(a); \
  else fd_pipe<BMODE_ADJ, EX, EZ, RZ, TM, ISO, false><<<grid, block, 0, s>>>(a);
    if (tc.ex == 112 && tc.ez == 112 && tc.rz == 14 && tc.tmax == 8) {
      if (a.iso) {
        VIP_PIPE_MODES(112, 112, 14, 8, true)
      } else {
        VIP_PIPE_MODES(112, 112, 14, 8, false)
      }
      VIP_LAUNCH_CHECK();
      return VIP_OK;
    }
#undef VIP_PIPE_MODES
    return VIP_E_UNSUPPORTED;
  }
  const dim3 grid(unsigned((total + 7) / 8 * 8));
#define VIP_BLOCK_MODES(EX, EZ, RZ, TM, ISO)                                                   \
  if (mode == BMODE_FWD) fd_block<BMODE_FWD, EX, EZ, RZ, TM, ISO><<<grid, block, 0, s>>>(a);        \
  else if (mode == BMODE_REC) fd_block<BMODE_REC, EX, EZ, RZ, TM, ISO><<<grid, block, 0, s>>>(a);   \
  else if (mode == BMODE_FWS) fd_block<BMODE_FWS, EX, EZ, RZ, TM, ISO><<<grid, block, 0, s>>>(a);   \
  else fd_block<BMODE_ADJ, EX, EZ, RZ, TM, ISO><<<grid, block, 0, s>>>(a);
#define VIP_BLOCK_CASE(C, EX, EZ, RZ, TM)      \
  if (cfg == C) {                              \
    if (a.iso) {                               \
      VIP_BLOCK_MODES(EX, EZ, RZ, TM, true)    \
    } else {                                   \
      VIP_BLOCK_MODES(EX, EZ, RZ, TM, false)   \
    }                                          \
    VIP_LAUNCH_CHECK();                        \
    return VIP_OK;                             \
  }
  VIP_BLOCK_CASE(0, 112, 112, 14, 8)
  VIP_BLOCK_CASE(1, 80, 80, 10, 4)
  VIP_BLOCK_CASE(2, 96, 96, 12, 4)
  VIP_BLOCK_CASE(3, 64, 64, 8, 4)
  VIP_BLOCK_CASE(4, 128, 64, 8, 4)
  VIP_BLOCK_CASE(5, 104, 104, 13, 6)
#undef VIP_BLOCK_CASE
#undef VIP_BLOCK_MODES
  return VIP_E_UNSUPPORTED;
}

static vip_status launch_multi(vip_ctx *ctx, int cfg,
                               const std::vector<const std::pair<int, BlockArgs> *> &items) {
  // a merged launch left with one problem (the others have finished their
  // sweeps) takes that problem's own kernel, which skips the per-tile lookup
  if (items.size() == 1) {
    BlockArgs a = items[0]->second;
    return launch_block(ctx, items[0]->first, cfg, a.total_tiles / a.tiles_per_pair, a);
  }
  MultiArgs m;
  std::memset(&m, 0, sizeof(m));
  m.nprob = int(items.size());
  long long acc = 0;
  for (int p = 0; p < m.nprob; ++p) {
    m.start[p] = int(acc);
    m.mode[p] = items[p]->first;
    m.a[p] = items[p]->second;
    acc += m.a[p].total_tiles;
  }
  if (acc > (1LL << 30)) return VIP_E_UNSUPPORTED;
  m.start[m.nprob] = int(acc);
  const TileCfg &tc = kTiles[cfg];
  const dim3 block(unsigned(tc.ex * (tc.ez / tc.rz)));
  hipStream_t s = ctx->s();
  // The persistent kernel takes the batch when its problems share the sweep
  // mode and the Laplacian form (the kernel is compiled per mode); one block
  // per compute unit then walks the tiles of all of them.
  bool same = tc.pipe != 0;
  for (int p = 1; p < m.nprob && same; ++p)
    same = m.mode[p] == m.mode[0] && m.a[p].iso == m.a[0].iso;
  if (same && tc.ex == 112 && tc.ez == 112 && tc.rz == 14 && tc.tmax == 8) {
    const dim3 grid(unsigned(std::max(8, ctx->cus / 8 * 8)));
    const int mode = m.mode[0];
#define VIP_PIPE_MULTI(ISO)                                                                       \
  if (mode == BMODE_FWD) fd_pipe<BMODE_FWD, 112, 112, 14, 8, ISO, true><<<grid, block, 0, s>>>(m);      \
  else if (mode == BMODE_REC) fd_pipe<BMODE_REC, 112, 112, 14, 8, ISO, true><<<grid, block, 0, s>>>(m); \
  else if (mode == BMODE_FWS) fd_pipe<BMODE_FWS, 112, 112, 14, 8, ISO, true><<<grid, block, 0, s>>>(m); \
  else fd_pipe<BMODE_ADJ, 112, 112, 14, 8, ISO, true><<<grid, block, 0, s>>>(m);
    if (m.a[0].iso) {
      VIP_PIPE_MULTI(true)
    } else {
      VIP_PIPE_MULTI(false)
    }
#undef VIP_PIPE_MULTI
    VIP_LAUNCH_CHECK();
    return VIP_OK;
  }
  const dim3 grid(unsigned((acc + 7) / 8 * 8));
#define VIP_MULTI_CASE(C, EX, EZ, RZ, TM)                            \
  if (cfg == C) {                                                    \
    fd_block_multi<EX, EZ, RZ, TM><<<grid, block, 0, s>>>(m);        \
    VIP_LAUNCH_CHECK();                                              \
    return VIP_OK;                                                   \
  }
  VIP_MULTI_CASE(0, 112, 112, 14, 8)
  VIP_MULTI_CASE(1, 80, 80, 10, 4)
  VIP_MULTI_CASE(2, 96, 96, 12, 4)
  VIP_MULTI_CASE(3, 64, 64, 8, 4)
  VIP_MULTI_CASE(4, 128, 64, 8, 4)
  VIP_MULTI_CASE(5, 104, 104, 13, 6)
  VIP_MULTI_CASE(6, 112, 112, 14, 8)   // shape 6 with mixed sweep modes: one block per tile
#undef VIP_MULTI_CASE
  return VIP_E_UNSUPPORTED;
}

// Launches a blocked step, or records it (mode + arguments with the tile
// geometry filled in) when several problems are merged into one launch.
struct Emitter {
  vip_ctx *ctx;
  int cfg, npairs;
  std::vector<std::pair<int, BlockArgs>> *list;
  vip_status operator()(int mode, BlockArgs &a) const {
    if (list) {
      VIP_TRY(set_tiles(cfg, npairs, a));
      list->emplace_back(mode, a);
      return VIP_OK;
    }
    return launch_block(ctx, mode, cfg, npairs, a);
  }
  int timing_begin_(int kind) const { return list ? -1 : timing_begin(ctx, kind); }
  void timing_end_(int run, int64_t launches, double pts) const {
    if (!list) timing_end(ctx, run, launches, pts);
  }
};

static BlockArgs block_args(const FwiDims &D, const FwiPlan &P, const float *wavelet, int pair0) {
  BlockArgs a;
  std::memset(&a, 0, sizeof(a));
  a.NX = D.NX;
  a.NZ = D.NZ;
  a.N = int(D.N);
  a.pair0 = pair0;
  a.ns = D.ns;
  a.nt = D.nt;
  a.nr = D.nr;
  a.w1x = float(4.0 / 3.0 * D.inv_dx2);
  a.w2x = float(-1.0 / 12.0 * D.inv_dx2);
  a.w1z = float(4.0 / 3.0 * D.inv_dz2);
  a.w2z = float(-1.0 / 12.0 * D.inv_dz2);
  a.iso = a.w1x == a.w1z && a.w2x == a.w2z;
  a.inv_area = D.inv_area;
  a.gx = P.gx;
  a.gz = P.gz;
  a.c = P.c;
  a.src_idx = P.src;
  a.rrow = P.rrow;
  a.rmap = P.rmap;
  a.nb = D.nb;
  a.nrows = D.nrows;
  a.wavelet = wavelet;
  return a;
}

// Forward sweep for pairs [pair0, pair0 + npairs) (blocked kernel): traces
// into data; with ckpt, the state at every segment start but the first into
// ckpt [pair][nseg-1][2][N]; when the dimensions keep a tail segment and the
// segment buffer exists, the tail's steps also store a^n into it.
static vip_status forward_sweep_blocked(const Emitter &emit, const FwiDims &D, const FwiPlan &P,
                                        const float *wavelet, int pair0, int npairs, float *data,
                                        float *ckpt) {
  const long long N = D.N;
  const long long ck_stride = (long long)(D.nseg - 1) * 2 * N;
  const long long seg_stride = (long long)D.seg_slots * N;
  const int tmax = kTiles[D.tile].tmax;
  const float *u_in = P.u[0], *q_in = P.q[0];
  long long in_stride = N;
  int buf = 0;
  for (int s = 0; s < D.nseg; ++s) {
    const int n0 = D.seg_begin(s), n1 = D.seg_end(s);
    const bool store = P.seg && D.stored > 0 && s == D.nseg - 1;
    const int mode = store ? BMODE_FWS : BMODE_FWD;
    const int run = emit.timing_begin_(store ? MODE_FWS : MODE_FWD);
    int launches = 0;
    for (int n = n0; n < n1; n += tmax) {
      const int T = std::min(tmax, n1 - n);
      BlockArgs a = block_args(D, P, wavelet, pair0);
      a.steps = T;
      a.n_start = n;
      a.zero_in = n == 0;
      a.u_in = u_in;
      a.q_in = q_in;
      a.in_stride = in_stride;
      const int m = n + T;
      if (ckpt && m == n1 && s + 1 <= D.nseg - 1) {
        a.u_out = ckpt + (long long)s * 2 * N;   // checkpoint slot s+1 lives at index s
        a.q_out = a.u_out + N;
        a.out_stride = ck_stride;
      } else {
        buf ^= 1;
        a.u_out = P.u[buf];
        a.q_out = P.q[buf];
        a.out_stride = N;
      }
      a.data = data;
      a.data_stride = (long long)D.nt * D.nr;
      if (store) {
        a.seg = P.seg;
        a.seg_stride = seg_stride;
        a.seg_n0 = n0;
      }
      VIP_TRY(emit(mode, a));
      ++launches;
      u_in = a.u_out;
      q_in = a.q_out;
      in_stride = a.out_stride;
    }
    emit.timing_end_(run, launches, double(n1 - n0) * double(N) * npairs);
  }
  return VIP_OK;
}

static vip_status backward_sweep_blocked(const Emitter &emit, const FwiDims &D, const FwiPlan &P,
                                         const float *wavelet, int pair0, int npairs,
                                         const float *rho, const float *ckpt, double *acc64) {
  const long long N = D.N;
  const long long ck_stride = (long long)(D.nseg - 1) * 2 * N;
  const long long seg_stride = (long long)D.seg_slots * N;
  const int tmax = kTiles[D.tile].tmax;
  bool adj_zero = true;
  int abuf = 0;
  for (int s = D.nseg - 1; s >= 0; --s) {
    const int n0 = D.seg_begin(s), n1 = D.seg_end(s);
    const float *u_in = s == 0 ? P.u[0] : ckpt + (long long)(s - 1) * 2 * N;
    const float *q_in = s == 0 ? P.q[0] : u_in + N;
    long long in_stride = s == 0 ? N : ck_stride;
    bool zero = s == 0;
    int buf = 0, launches = 0;
    // the forward sweep already stored the tail segment's a^n
    const bool stored = D.stored > 0 && s == D.nseg - 1;
    const int run_rec = stored ? -1 : emit.timing_begin_(MODE_REC);
    for (int n = n0; n < n1 && !stored; n += tmax) {
      const int T = std::min(tmax, n1 - n);
      BlockArgs a = block_args(D, P, wavelet, pair0);
      a.steps = T;
      a.n_start = n;
      a.seg_n0 = n0;
      a.zero_in = zero;
      a.u_in = u_in;
      a.q_in = q_in;
      a.in_stride = in_stride;
      if (n + T < n1) {
        buf ^= 1;
        a.u_out = P.u[buf];
        a.q_out = P.q[buf];
        a.out_stride = N;
      }
      a.seg = P.seg;
      a.seg_stride = seg_stride;
      VIP_TRY(emit(BMODE_REC, a));
      ++launches;
      u_in = a.u_out;
      q_in = a.q_out;
      in_stride = N;
      zero = false;
    }
    emit.timing_end_(run_rec, launches, double(n1 - n0) * double(N) * npairs);
    launches = 0;
    const int run_adj = emit.timing_begin_(MODE_ADJ);
    for (int n = n1 - 1; n >= n0; n -= tmax) {
      const int T = std::min(tmax, n - n0 + 1);
      BlockArgs a = block_args(D, P, wavelet, pair0);
      a.steps = T;
      a.n_start = n;
      a.seg_n0 = n0;
      a.zero_in = adj_zero;
      a.u_in = P.z[abuf];
      a.q_in = P.Q[abuf];
      a.in_stride = N;
      abuf ^= 1;
      a.u_out = P.z[abuf];
      a.q_out = P.Q[abuf];
      a.out_stride = N;
      a.rho = rho;
      a.rho_stride = (long long)D.nt * D.nr;
      a.seg = P.seg;
      a.seg_stride = seg_stride;
      a.acc64 = acc64;
      a.acc64_stride = N;
      VIP_TRY(emit(BMODE_ADJ, a));
      ++launches;
      adj_zero = false;
    }
    emit.timing_end_(run_adj, launches, double(n1 - n0) * double(N) * npairs);
  }
  return VIP_OK;
}

// Forward sweep for pairs [pair0, pair0 + npairs): traces into data (indexed by
// local pair, stride nt*nr); optional checkpoints (u, q) at every segment
// start but the first into ckpt [pair][nseg-1][2][N].  (This kernel leaves
// the tail segment's a^n to the backward sweep.)
static vip_status forward_sweep_stream(vip_ctx *ctx, const FwiDims &D, const FwiPlan &P,
                                       const float *wavelet, int pair0, int npairs, float *data,
                                       float *ckpt) {
  const long long N = D.N;
  const long long ck_stride = (long long)(D.nseg - 1) * 2 * N;
  const float *u_in = nullptr, *q_in = nullptr;
  long long in_stride = N;
  const int run = timing_begin(ctx, MODE_FWD);
  int next_seg = 1;   // next segment whose start state is checkpointed
  for (int n = 0; n <= D.nt - 2; ++n) {
    StepArgs a = base_args(D, P, wavelet, pair0);
    a.n = n;
    a.zero_in = n == 0;
    a.u_in = n == 0 ? P.u[0] : u_in;
    a.q_in = n == 0 ? P.q[0] : q_in;
    a.in_stride = in_stride;
    const int m = n + 1;
    if (ckpt && next_seg < D.nseg && m == D.seg_begin(next_seg)) {
      a.u_out = ckpt + (long long)(next_seg - 1) * 2 * N;
      ++next_seg;
      a.q_out = a.u_out + N;
      a.out_stride = ck_stride;
    } else {
      a.u_out = P.u[m & 1];
      a.q_out = P.q[m & 1];
      a.out_stride = N;
    }
    a.data = data;
    a.data_stride = (long long)D.nt * D.nr;
    VIP_TRY(launch_step(ctx, MODE_FWD, D.rz, npairs, a));
    u_in = a.u_out;
    q_in = a.q_out;
    in_stride = a.out_stride;
  }
  timing_end(ctx, run, D.nt - 1, double(D.nt - 1) * double(N) * npairs);
  return VIP_OK;
}

// Backward sweep: for each segment from the last, recompute a^n = L u^n + f^n
// from its checkpoint, then run the adjoint over the segment with the imaging
// sum; rho [pair][nt][nr] (local pair), acc64 [pair][N] (local pair, zeroed).
static vip_status backward_sweep_stream(vip_ctx *ctx, const FwiDims &D, const FwiPlan &P,
                                        const float *wavelet, int pair0, int npairs,
                                        const float *rho, const float *ckpt, double *acc64) {
  const long long N = D.N;
  const long long ck_stride = (long long)(D.nseg - 1) * 2 * N;
  const long long seg_stride = (long long)D.seg_slots * N;
  int adj_steps = 0;
  const float *z_in = nullptr, *Q_in = nullptr;
  for (int s = D.nseg - 1; s >= 0; --s) {
    const int n0 = D.seg_begin(s);
    const int n1 = D.seg_end(s);
    const float *u_in = nullptr, *q_in = nullptr;
    long long in_stride = N;
    const int run_rec = timing_begin(ctx, MODE_REC);
    for (int n = n0; n < n1; ++n) {
      StepArgs a = base_args(D, P, wavelet, pair0);
      a.n = n;
      if (n == n0) {
        a.zero_in = s == 0;
        a.u_in = s == 0 ? P.u[0] : ckpt + (long long)(s - 1) * 2 * N;
        a.q_in = s == 0 ? P.q[0] : a.u_in + N;
        a.in_stride = s == 0 ? N : ck_stride;
      } else {
        a.u_in = u_in;
        a.q_in = q_in;
        a.in_stride = in_stride;
      }
      if (n < n1 - 1) {
        a.u_out = P.u[(n + 1) & 1];
        a.q_out = P.q[(n + 1) & 1];
        a.out_stride = N;
      }
      a.seg = P.seg + (long long)(n - n0) * N;
      a.seg_stride = seg_stride;
      VIP_TRY(launch_step(ctx, MODE_REC, D.rz, npairs, a));
      u_in = a.u_out;
      q_in = a.q_out;
      in_stride = N;
    }
    timing_end(ctx, run_rec, n1 - n0, double(n1 - n0) * double(N) * npairs);
    const int run_adj = timing_begin(ctx, MODE_ADJ);
    for (int n = n1 - 1; n >= n0; --n) {
      StepArgs a = base_args(D, P, wavelet, pair0);
      a.n = n;
      a.zero_in = adj_steps == 0;
      a.u_in = adj_steps == 0 ? P.z[0] : z_in;
      a.q_in = adj_steps == 0 ? P.Q[0] : Q_in;
      a.in_stride = N;
      a.u_out = P.z[(adj_steps + 1) & 1];
      a.q_out = P.Q[(adj_steps + 1) & 1];
      a.out_stride = N;
      a.rho = rho;
      a.rho_stride = (long long)D.nt * D.nr;
      a.seg = P.seg + (long long)(n - n0) * N;
      a.seg_stride = seg_stride;
      a.acc64 = acc64;
      a.acc64_stride = N;
      VIP_TRY(launch_step(ctx, MODE_ADJ, D.rz, npairs, a));
      z_in = a.u_out;
      Q_in = a.q_out;
      ++adj_steps;
    }
    timing_end(ctx, run_adj, n1 - n0, double(n1 - n0) * double(N) * npairs);
  }
  return VIP_OK;
}

vip_status forward_sweep(vip_ctx *ctx, const FwiDims &D, const FwiPlan &P, const float *wavelet,
                         int pair0, int npairs, float *data, float *ckpt) {
  if (D.tile < 0) return forward_sweep_stream(ctx, D, P, wavelet, pair0, npairs, data, ckpt);
  const Emitter emit{ctx, D.tile, npairs, nullptr};
  return forward_sweep_blocked(emit, D, P, wavelet, pair0, npairs, data, ckpt);
}

vip_status backward_sweep(vip_ctx *ctx, const FwiDims &D, const FwiPlan &P, const float *wavelet,
                          int pair0, int npairs, const float *rho, const float *ckpt,
                          double *acc64) {
  if (D.tile < 0) return backward_sweep_stream(ctx, D, P, wavelet, pair0, npairs, rho, ckpt, acc64);
  const Emitter emit{ctx, D.tile, npairs, nullptr};
  return backward_sweep_blocked(emit, D, P, wavelet, pair0, npairs, rho, ckpt, acc64);
}

vip_status launch_residual(vip_ctx *ctx, const FwiDims &D, const FwiPlan &P, int pair0,
                           int npairs, const float *dobs, double sigma) {
  long long per_pair = (long long)D.nt * D.nr;
  residual_kernel<<<dim3(npairs), dim3(RESID_T), 0, ctx->s()>>>(
      P.resid, per_pair, dobs, P.shot_row, pair0, D.ns, per_pair, D.misfit_scale / (sigma * sigma), P.J,
      P.status);
  VIP_LAUNCH_CHECK();
  return VIP_OK;
}

vip_status launch_finalize(vip_ctx *ctx, const FwiDims &D, const FwiPlan &P, const float *vel,
                           float *grad, float sign) {
  long long total = (long long)D.nx * D.nz * D.np;
  finalize_grad_kernel<<<dim3(unsigned((total + 255) / 256)), dim3(256), 0, ctx->s()>>>(
      P.acc64, vel, grad, D.np, D.ns, D.nx, D.nz, D.nb, D.NX, sign);
  VIP_LAUNCH_CHECK();
  return VIP_OK;
}

vip_status check_prior(const vip_prior *prior) {
  if (!prior || prior->kind == VIP_PRIOR_NONE) return VIP_OK;
  switch (prior->kind) {
    case VIP_PRIOR_UNIFORM_CLIP:
    case VIP_PRIOR_UNIFORM_TRANSFORM: return (prior->lo && prior->hi) ? VIP_OK : VIP_E_ARG;
    case VIP_PRIOR_GAUSSIAN: return (prior->mean && prior->std) ? VIP_OK : VIP_E_ARG;
    default: return VIP_E_ARG;
  }
}

const float *prior_model(vip_ctx *ctx, const FwiDims &D, const FwiPlan &P, const float *vel,
                         const vip_prior *prior) {
  if (!prior || prior->kind != VIP_PRIOR_UNIFORM_TRANSFORM) return vel;
  const long long d = (long long)D.nx * D.nz, total = d * D.np;
  prior_transform_kernel<<<dim3(unsigned((total + 255) / 256)), dim3(256), 0, ctx->s()>>>(
      vel, P.model, prior->lo, prior->hi, total, d, 0);
  return P.model;
}

vip_status launch_prior_and_logpost(vip_ctx *ctx, const FwiDims &D, const FwiPlan &P,
                                    const float *vel, const float *model, const vip_prior *prior,
                                    float *grad, double *logpost) {
  VIP_LAUNCH_CHECK();
  const int kind = prior ? prior->kind : VIP_PRIOR_NONE;
  const long long d = (long long)D.nx * D.nz, total = d * D.np;
  if (kind == VIP_PRIOR_UNIFORM_TRANSFORM || kind == VIP_PRIOR_GAUSSIAN) {
    prior_grad_kernel<<<dim3(unsigned((total + 255) / 256)), dim3(256), 0, ctx->s()>>>(
        grad, vel, model, kind, prior->lo, prior->hi, prior->mean, prior->std, total, d);
    VIP_LAUNCH_CHECK();
  }
  logpost_kernel<<<dim3(D.np), dim3(256), 0, ctx->s()>>>(
      P.J, vel, model, kind, prior ? prior->lo : nullptr, prior ? prior->hi : nullptr,
      prior ? prior->mean : nullptr, prior ? prior->std : nullptr, D.ns, d, logpost, P.status);
  VIP_LAUNCH_CHECK();
  return VIP_OK;
}


// The rows of d_obs a geometry reads (and with them the misfit scale) are
// baked into a captured graph, so they belong to its cache key.
static void add_shot_rows(KeyBuilder &kb, const vip_geometry &g) {
  kb.add(g.shot_index ? 1 : 0);
  if (g.shot_index) kb.add(g.nobs).add_array(g.shot_index, g.ns);
}

// ---- batches of problems ------------------------------------------------------

static vip_status multi_dims(int32_t nprob, const vip_problem *probs, int32_t k, bool need_wavelet,
                             std::vector<FwiDims> *Ds) {
  if (nprob < 1 || nprob > VIP_MAX_BATCH || !probs) return VIP_E_ARG;
  Ds->resize(size_t(nprob));
  for (int p = 0; p < nprob; ++p)
    VIP_TRY(make_dims(&probs[p].grid, &probs[p].geom, probs[p].np, k, 0, need_wavelet, &(*Ds)[size_t(p)]));
  return VIP_OK;
}

// Sub-workspaces of the problems, one after the other; one status word for all.
static size_t plan_multi(const std::vector<FwiDims> &Ds, char *base, std::vector<FwiPlan> *Ps) {
  size_t off = kStatusBytes;
  Ps->resize(Ds.size());
  for (size_t p = 0; p < Ds.size(); ++p) {
    FwiPlan &P = (*Ps)[p];
    plan_fwi(Ds[p], base ? base + off : nullptr, PLAN_GRAD, &P);
    P.status = reinterpret_cast<uint32_t *>(base);
    off = align_up(off + P.bytes);
  }
  return off;
}

static vip_status launch_merged(vip_ctx *ctx, int cfg,
                                const std::vector<std::vector<std::pair<int, BlockArgs>>> &lists) {
  size_t longest = 0;
  for (auto &l : lists) longest = std::max(longest, l.size());
  for (size_t i = 0; i < longest; ++i) {
    std::vector<const std::pair<int, BlockArgs> *> items;
    for (auto &l : lists)
      if (i < l.size()) items.push_back(&l[i]);
    VIP_TRY(launch_multi(ctx, cfg, items));
  }
  return VIP_OK;
}

}  // namespace vip

using namespace vip;

extern "C" {

int vip_tile_count(void) { return tile_count(); }

vip_status vip_set_tile(vip_ctx *ctx, int tile) {
  if (!ctx || tile < -2 || tile >= tile_count()) return VIP_E_ARG;
  ctx->tile = tile;
  return VIP_OK;
}

vip_status vip_tile_shape(int tile, int32_t shape[4]) {
  if (!shape || tile < 0 || tile >= tile_count()) return VIP_E_ARG;
  shape[0] = kTiles[tile].ex;
  shape[1] = kTiles[tile].ez;
  shape[2] = kTiles[tile].rz;
  shape[3] = kTiles[tile].tmax;
  return VIP_OK;
}

int vip_tile_persistent(int tile) {
  if (tile < 0 || tile >= tile_count()) return VIP_E_ARG;
  return kTiles[tile].pipe;
}

vip_status vip_tile_for_grid(const vip_ctx *ctx, const vip_grid *grid, int64_t pairs, int32_t *tile) {
  if (!ctx || !grid || !tile || grid->nx <= 0 || grid->nz <= 0 || grid->nb < 0) return VIP_E_ARG;
  if (ctx->tile >= -1) {
    *tile = ctx->tile;
  } else {
    const int NX = grid->nx + 2 * grid->nb, NZ = grid->nz + 2 * grid->nb;
    *tile = (long long)NX * NZ < kMaxBlockedPoints ? default_tile(NX, NZ, pairs) : -1;
  }
  return VIP_OK;
}

vip_status vip_forward_workspace(const vip_grid *grid, const vip_geometry *geom, int32_t np,
                                 size_t *bytes) {
  if (!bytes) return VIP_E_ARG;
  FwiDims D;
  VIP_TRY(make_dims(grid, geom, np, grid ? grid->nt : 0, 0, false, &D));
  FwiPlan P;
  plan_fwi(D, nullptr, PLAN_FORWARD, &P);
  *bytes = P.bytes;
  return VIP_OK;
}

vip_status vip_forward(vip_ctx *ctx, const vip_grid *grid, const vip_geometry *geom, int32_t np,
                       const float *vel, float *data, void *ws, size_t ws_bytes) {
  if (!ctx || !vel || !data || !ws) return VIP_E_ARG;
  FwiDims D;
  VIP_TRY(make_dims(grid, geom, np, grid ? grid->nt : 0, 0, true, &D));
  apply_tile_choice(ctx, &D);
  FwiPlan P;
  plan_fwi(D, static_cast<char *>(ws), PLAN_FORWARD, &P);
  if (ws_bytes < P.bytes || !aligned(ws)) return VIP_E_WORKSPACE;
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  KeyBuilder kb;
  kb.add(std::string("fwd")).add(D.tile).add(*grid).add(np).add(vel).add(data).add(ws).add(geom->wavelet)
      .add(geom->ns).add(geom->nr);
  kb.add_array(geom->src_ix, geom->ns).add_array(geom->src_iz, geom->ns)
      .add_array(geom->rec_ix, geom->nr).add_array(geom->rec_iz, geom->nr);
  return run_maybe_graph(ctx, kb.k, [&]() -> vip_status {
    VIP_TRY(upload_tables(ctx, D, grid, geom, P));
    VIP_TRY(launch_coeff(ctx, D, grid, vel, P));
    return forward_sweep(ctx, D, P, geom->wavelet, 0, int(D.pairs), data, nullptr);
  });
}

vip_status vip_grad_logpost_workspace(const vip_grid *grid, const vip_geometry *geom, int32_t np,
                                      int32_t ckpt_every, int32_t stored_steps,
                                      int32_t live_pairs, size_t *bytes) {
  if (!bytes) return VIP_E_ARG;
  FwiDims D;
  VIP_TRY(make_dims(grid, geom, np, ckpt_every, live_pairs, false, &D, stored_steps));
  FwiPlan P;
  plan_fwi(D, nullptr, PLAN_GRAD, &P);
  *bytes = P.bytes;
  return VIP_OK;
}

vip_status vip_grad_logpost(vip_ctx *ctx, const vip_grid *grid, const vip_geometry *geom,
                            const vip_prior *prior, int32_t np, const float *vel,
                            const float *dobs, double sigma, int32_t ckpt_every,
                            int32_t stored_steps, int32_t live_pairs, double *logpost,
                            float *grad, void *ws, size_t ws_bytes) {
  if (!ctx || !vel || !dobs || !logpost || !grad || !ws) return VIP_E_ARG;
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return VIP_E_ARG;
  VIP_TRY(check_prior(prior));
  FwiDims D;
  VIP_TRY(make_dims(grid, geom, np, ckpt_every, live_pairs, true, &D, stored_steps));
  apply_tile_choice(ctx, &D);
  FwiPlan P;
  plan_fwi(D, static_cast<char *>(ws), PLAN_GRAD, &P);
  if (ws_bytes < P.bytes || !aligned(ws)) return VIP_E_WORKSPACE;
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  KeyBuilder kb;
  kb.add(std::string("grad")).add(D.tile).add(*grid).add(np).add(vel).add(dobs).add(sigma).add(ckpt_every)
      .add(stored_steps)
      .add(live_pairs).add(logpost).add(grad).add(ws).add(geom->wavelet).add(geom->ns)
      .add(geom->nr);
  kb.add(prior ? prior->kind : -1).add(prior ? prior->lo : nullptr).add(prior ? prior->hi : nullptr)
      .add(prior ? prior->mean : nullptr).add(prior ? prior->std : nullptr);
  kb.add_array(geom->src_ix, geom->ns).add_array(geom->src_iz, geom->ns)
      .add_array(geom->rec_ix, geom->nr).add_array(geom->rec_iz, geom->nr);
  add_shot_rows(kb, *geom);
  return run_maybe_graph(ctx, kb.k, [&]() -> vip_status {
    VIP_TRY(upload_tables(ctx, D, grid, geom, P));
    const float *model = prior_model(ctx, D, P, vel, prior);
    VIP_TRY(launch_coeff(ctx, D, grid, model, P));
    VIP_TRY(fill_f64(ctx->s(), P.acc64, size_t(D.pairs * D.N), 0.0));
    for (long long p0 = 0; p0 < D.pairs; p0 += D.live) {
      int cnt = int(std::min<long long>(D.live, D.pairs - p0));
      VIP_TRY(forward_sweep(ctx, D, P, geom->wavelet, int(p0), cnt, P.resid, P.ckpt));
      VIP_TRY(launch_residual(ctx, D, P, int(p0), cnt, dobs, sigma));
      VIP_TRY(backward_sweep(ctx, D, P, geom->wavelet, int(p0), cnt, P.resid, P.ckpt,
                             P.acc64 + p0 * D.N));
    }
    VIP_TRY(launch_finalize(ctx, D, P, model, grad, -1.0f));
    return launch_prior_and_logpost(ctx, D, P, vel, model, prior, grad, logpost);
  });
}

vip_status vip_tape_bytes(const vip_grid *grid, const vip_geometry *geom, int32_t np,
                          int32_t ckpt_every, size_t *bytes) {
  if (!bytes) return VIP_E_ARG;
  FwiDims D;
  VIP_TRY(make_dims(grid, geom, np, ckpt_every, 0, false, &D));
  *bytes = size_t(D.pairs) * size_t(D.nseg - 1) * 2 * size_t(D.N) * sizeof(float);
  return VIP_OK;
}

vip_status vip_tape_workspace(const vip_grid *grid, const vip_geometry *geom, int32_t np,
                              int32_t ckpt_every, size_t *bytes) {
  if (!bytes) return VIP_E_ARG;
  FwiDims D;
  VIP_TRY(make_dims(grid, geom, np, ckpt_every, 0, false, &D));
  FwiPlan P;
  plan_fwi(D, nullptr, PLAN_TAPE, &P);
  *bytes = P.bytes;
  return VIP_OK;
}

vip_status vip_forward_tape(vip_ctx *ctx, const vip_grid *grid, const vip_geometry *geom,
                            int32_t np, const float *vel, float *data, int32_t ckpt_every,
                            void *tape, size_t tape_bytes, void *ws, size_t ws_bytes) {
  if (!ctx || !vel || !data || !ws) return VIP_E_ARG;
  FwiDims D;
  VIP_TRY(make_dims(grid, geom, np, ckpt_every, 0, true, &D));
  apply_tile_choice(ctx, &D);
  size_t need = size_t(D.pairs) * size_t(D.nseg - 1) * 2 * size_t(D.N) * sizeof(float);
  if (tape_bytes < need || (need > 0 && !tape)) return VIP_E_WORKSPACE;
  FwiPlan P;
  plan_fwi(D, static_cast<char *>(ws), PLAN_TAPE, &P);
  if (ws_bytes < P.bytes || !aligned(ws)) return VIP_E_WORKSPACE;
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  ctx->active = ctx->user;
  VIP_TRY(upload_tables(ctx, D, grid, geom, P));
  VIP_TRY(launch_coeff(ctx, D, grid, vel, P));
  return forward_sweep(ctx, D, P, geom->wavelet, 0, int(D.pairs), data,
                       static_cast<float *>(tape));
}

vip_status vip_adjoint_tape(vip_ctx *ctx, const vip_grid *grid, const vip_geometry *geom,
                            int32_t np, const float *vel, int32_t ckpt_every, const void *tape,
                            size_t tape_bytes, const float *grad_data, float *grad_vel, void *ws,
                            size_t ws_bytes) {
  if (!ctx || !vel || !grad_data || !grad_vel || !ws) return VIP_E_ARG;
  FwiDims D;
  VIP_TRY(make_dims(grid, geom, np, ckpt_every, 0, true, &D));
  apply_tile_choice(ctx, &D);
  size_t need = size_t(D.pairs) * size_t(D.nseg - 1) * 2 * size_t(D.N) * sizeof(float);
  if (tape_bytes < need || (need > 0 && !tape)) return VIP_E_WORKSPACE;
  FwiPlan P;
  plan_fwi(D, static_cast<char *>(ws), PLAN_TAPE, &P);
  if (ws_bytes < P.bytes || !aligned(ws)) return VIP_E_WORKSPACE;
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  ctx->active = ctx->user;
  VIP_TRY(upload_tables(ctx, D, grid, geom, P));
  VIP_TRY(launch_coeff(ctx, D, grid, vel, P));
  VIP_TRY(fill_f64(ctx->s(), P.acc64, size_t(D.pairs * D.N), 0.0));
  VIP_TRY(backward_sweep(ctx, D, P, geom->wavelet, 0, int(D.pairs), grad_data,
                         static_cast<const float *>(tape), P.acc64));
  return launch_finalize(ctx, D, P, vel, grad_vel, 1.0f);
}

vip_status vip_grad_logpost_multi_workspace(int32_t nprob, const vip_problem *probs,
                                            int32_t ckpt_every, size_t *bytes) {
  if (!bytes) return VIP_E_ARG;
  std::vector<FwiDims> Ds;
  VIP_TRY(multi_dims(nprob, probs, ckpt_every, false, &Ds));
  std::vector<FwiPlan> Ps;
  *bytes = plan_multi(Ds, nullptr, &Ps);
  return VIP_OK;
}

vip_status vip_grad_logpost_multi(vip_ctx *ctx, int32_t nprob, const vip_problem *probs,
                                  int32_t ckpt_every, void *ws, size_t ws_bytes) {
  if (!ctx || !ws) return VIP_E_ARG;
  std::vector<FwiDims> Ds;
  VIP_TRY(multi_dims(nprob, probs, ckpt_every, true, &Ds));
  for (int p = 0; p < nprob; ++p) {
    const vip_problem &q = probs[p];
    if (!q.vel || !q.dobs || !q.logpost || !q.grad) return VIP_E_ARG;
    if (!(q.sigma > 0.0) || !std::isfinite(q.sigma)) return VIP_E_ARG;
    VIP_TRY(check_prior(&q.prior));
  }
  const int cfg = ctx->tile >= 0 ? ctx->tile : default_tile_multi(Ds);
  if (ctx->tile == -1) return VIP_E_UNSUPPORTED;   // batching needs a blocked tile shape
  for (FwiDims &D : Ds) D.tile = cfg;
  std::vector<FwiPlan> Ps;
  const size_t need = plan_multi(Ds, static_cast<char *>(ws), &Ps);
  if (ws_bytes < need || !aligned(ws)) return VIP_E_WORKSPACE;
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  KeyBuilder kb;
  kb.add(std::string("multi")).add(cfg).add(nprob).add(ckpt_every).add(ws);
  for (int p = 0; p < nprob; ++p) {
    const vip_problem &q = probs[p];
    kb.add(q.grid).add(q.np).add(q.vel).add(q.dobs).add(q.sigma).add(q.logpost).add(q.grad)
        .add(q.prior.kind).add(q.prior.lo).add(q.prior.hi).add(q.prior.mean).add(q.prior.std)
        .add(q.geom.wavelet).add(q.geom.ns)
        .add(q.geom.nr);
    kb.add_array(q.geom.src_ix, q.geom.ns).add_array(q.geom.src_iz, q.geom.ns)
        .add_array(q.geom.rec_ix, q.geom.nr).add_array(q.geom.rec_iz, q.geom.nr);
    add_shot_rows(kb, q.geom);
  }
  return run_maybe_graph(ctx, kb.k, [&]() -> vip_status {
    std::vector<std::vector<std::pair<int, BlockArgs>>> fwd(nprob), bwd(nprob);
    std::vector<const float *> models(nprob);
    for (int p = 0; p < nprob; ++p) {
      const FwiDims &D = Ds[p];
      const FwiPlan &P = Ps[p];
      VIP_TRY(upload_tables(ctx, D, &probs[p].grid, &probs[p].geom, P));
      models[p] = prior_model(ctx, D, P, probs[p].vel, &probs[p].prior);
      VIP_TRY(launch_coeff(ctx, D, &probs[p].grid, models[p], P));
      VIP_TRY(fill_f64(ctx->s(), P.acc64, size_t(D.pairs * D.N), 0.0));
      const Emitter ef{ctx, cfg, int(D.pairs), &fwd[p]};
      VIP_TRY(forward_sweep_blocked(ef, D, P, probs[p].geom.wavelet, 0, int(D.pairs), P.resid, P.ckpt));
      const Emitter eb{ctx, cfg, int(D.pairs), &bwd[p]};
      VIP_TRY(backward_sweep_blocked(eb, D, P, probs[p].geom.wavelet, 0, int(D.pairs), P.resid,
                                     P.ckpt, P.acc64));
    }
    VIP_TRY(launch_merged(ctx, cfg, fwd));
    for (int p = 0; p < nprob; ++p)
      VIP_TRY(launch_residual(ctx, Ds[p], Ps[p], 0, int(Ds[p].pairs), probs[p].dobs, probs[p].sigma));
    VIP_TRY(launch_merged(ctx, cfg, bwd));
    for (int p = 0; p < nprob; ++p) {
      VIP_TRY(launch_finalize(ctx, Ds[p], Ps[p], models[p], probs[p].grad, -1.0f));
      VIP_TRY(launch_prior_and_logpost(ctx, Ds[p], Ps[p], probs[p].vel, models[p], &probs[p].prior,
                                       probs[p].grad, probs[p].logpost));
    }
    return VIP_OK;
  });
}

vip_status vip_prior_transform(vip_ctx *ctx, const vip_prior *prior, int32_t n, int64_t d,
                               const float *in, float *out, int32_t direction) {
  if (!ctx || !prior || !in || !out || n < 1 || d < 1 || (direction != 0 && direction != 1))
    return VIP_E_ARG;
  if (prior->kind != VIP_PRIOR_UNIFORM_TRANSFORM || !prior->lo || !prior->hi) return VIP_E_ARG;
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  const long long total = (long long)n * d;
  prior_transform_kernel<<<dim3(unsigned((total + 255) / 256)), dim3(256), 0, ctx->user>>>(
      in, out, prior->lo, prior->hi, total, d, direction);
  VIP_LAUNCH_CHECK();
  return VIP_OK;
}

}  // extern "C"
