// Plain per-pair GPU path for the log-posterior gradient: the baseline the
// batched path is measured against.  Same scheme and the same arithmetic
// forms as fwi.hip, organised the straightforward way:
//   - one (particle, shot) pair at a time;
//   - per time step separate launches for the Laplacian (neighbours read from
//     global memory), the source or residual injection, the update, the
//     receiver gather and the imaging sum;
//   - the whole forward history of L u + f kept for the adjoint (no
//     checkpoints), imaging accumulated directly in FP64.
#include <algorithm>
#include <cmath>

#include "vip_internal.h"
#include "fwi_plan.h"

namespace vip {

__global__ void plain_lap_kernel(const float *u, float *out, int NX, int NZ, float cx, float cz) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NX * NZ) return;
  int z = i / NX, x = i - z * NX;
  const float w1 = 4.0f / 3.0f, w2 = -1.0f / 12.0f;
  float uc = u[i];
  auto at = [&](int zz, int xx) { return (zz >= 0 && zz < NZ && xx >= 0 && xx < NX) ? u[zz * NX + xx] : 0.0f; };
  float lx = w1 * ((at(z, x - 1) - uc) + (at(z, x + 1) - uc)) + w2 * ((at(z, x - 2) - uc) + (at(z, x + 2) - uc));
  float lz = w1 * ((at(z - 1, x) - uc) + (at(z + 1, x) - uc)) + w2 * ((at(z - 2, x) - uc) + (at(z + 2, x) - uc));
  out[i] = cx * lx + cz * lz;
}

__global__ void plain_add_source_kernel(float *a, const int *src, int shot, const float *w, int n,
                                        float inv_area) {
  a[src[shot]] += w[n] * inv_area;
}

__global__ void plain_add_residual_kernel(float *a, const float *rho_n, const int *rec_node, int nr) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nr) a[rec_node[r]] += rho_n[r];
}

__global__ void plain_update_kernel(float *u, float *q, const float *a, const float *c,
                                    const float *gx, const float *gz, int NX, int N) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int z = i / NX, x = i - z * NX;
  float g = gz[z] * gx[x];
  float qn = g * (q[i] + c[i] * a[i]);
  q[i] = qn;
  u[i] = g * u[i] + qn;
}

__global__ void plain_gather_kernel(const float *u, float *d_n, const int *rec_node, int nr) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nr) d_n[r] = u[rec_node[r]];
}

__global__ void plain_image_kernel(double *acc, const float *z, const float *a, int N) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) acc[i] += double(z[i] * a[i]);
}

vip_status launch_residual(vip_ctx *ctx, const FwiDims &D, const FwiPlan &P, int pair0,
                           int npairs, const float *dobs, double sigma);

}  // namespace vip

using namespace vip;

extern "C" {

vip_status vip_grad_logpost_plain_workspace(const vip_grid *grid, const vip_geometry *geom,
                                            int32_t np, size_t *bytes) {
  if (!bytes) return VIP_E_ARG;
  FwiDims D;
  VIP_TRY(make_dims(grid, geom, np, grid ? grid->nt : 1, 1, false, &D));
  FwiPlan P;
  plan_fwi(D, nullptr, PLAN_PLAIN, &P);
  *bytes = align_up(P.bytes + sizeof(int32_t) * size_t(D.nr));
  return VIP_OK;
}

vip_status vip_grad_logpost_plain(vip_ctx *ctx, const vip_grid *grid, const vip_geometry *geom,
                                  const vip_prior *prior, int32_t np, const float *vel,
                                  const float *dobs, double sigma, double *logpost, float *grad,
                                  void *ws, size_t ws_bytes) {
  if (!ctx || !vel || !dobs || !logpost || !grad || !ws) return VIP_E_ARG;
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return VIP_E_ARG;
  VIP_TRY(check_prior(prior));
  FwiDims D;
  VIP_TRY(make_dims(grid, geom, np, grid->nt, 1, true, &D));
  FwiPlan P;
  plan_fwi(D, static_cast<char *>(ws), PLAN_PLAIN, &P);
  int32_t *rec_node = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + P.bytes);
  if (ws_bytes < align_up(P.bytes + sizeof(int32_t) * size_t(D.nr)) || !aligned(ws))
    return VIP_E_WORKSPACE;
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  ctx->active = ctx->user;
  hipStream_t s = ctx->user;
  VIP_TRY(upload_tables(ctx, D, grid, geom, P));
  {
    std::vector<int32_t> nodes(D.nr);
    for (int r = 0; r < D.nr; ++r)
      nodes[r] = (geom->rec_iz[r] + D.nb) * D.NX + geom->rec_ix[r] + D.nb;
    VIP_TRY(upload_i32(s, rec_node, nodes.data(), nodes.size()));
  }
  const float *model = prior_model(ctx, D, P, vel, prior);
  VIP_TRY(launch_coeff(ctx, D, grid, model, P));
  const int N = int(D.N);
  const dim3 gN((N + 255) / 256), b256(256), gR((D.nr + 255) / 256);
  for (long long pair = 0; pair < D.pairs; ++pair) {
    const int particle = int(pair / D.ns), shot = int(pair % D.ns);
    const float *c = P.c + (long long)particle * D.N;
    double *acc = P.acc64 + pair * D.N;
    VIP_TRY(fill_f32(s, P.u[0], size_t(N), 0.0f));
    VIP_TRY(fill_f32(s, P.q[0], size_t(N), 0.0f));
    VIP_TRY(fill_f32(s, P.resid, size_t(D.nr), 0.0f));
    for (int n = 0; n <= D.nt - 2; ++n) {
      float *a = P.hist + (long long)n * N;
      plain_lap_kernel<<<gN, b256, 0, s>>>(P.u[0], a, D.NX, D.NZ, D.cx, D.cz);
      VIP_LAUNCH_CHECK();
      plain_add_source_kernel<<<1, 1, 0, s>>>(a, P.src, shot, geom->wavelet, n, D.inv_area);
      VIP_LAUNCH_CHECK();
      plain_update_kernel<<<gN, b256, 0, s>>>(P.u[0], P.q[0], a, c, P.gx, P.gz, D.NX, N);
      VIP_LAUNCH_CHECK();
      plain_gather_kernel<<<gR, b256, 0, s>>>(P.u[0], P.resid + (long long)(n + 1) * D.nr, rec_node,
                                             D.nr);
      VIP_LAUNCH_CHECK();
    }
    VIP_TRY(launch_residual(ctx, D, P, int(pair), 1, dobs, sigma));
    VIP_TRY(fill_f32(s, P.z[0], size_t(N), 0.0f));
    VIP_TRY(fill_f32(s, P.Q[0], size_t(N), 0.0f));
    VIP_TRY(fill_f64(s, acc, size_t(N), 0.0));
    for (int n = D.nt - 1; n >= 1; --n) {
      plain_lap_kernel<<<gN, b256, 0, s>>>(P.z[0], P.acc32, D.NX, D.NZ, D.cx, D.cz);
      VIP_LAUNCH_CHECK();
      plain_add_residual_kernel<<<gR, b256, 0, s>>>(P.acc32, P.resid + (long long)n * D.nr,
                                                   rec_node, D.nr);
      VIP_LAUNCH_CHECK();
      plain_update_kernel<<<gN, b256, 0, s>>>(P.z[0], P.Q[0], P.acc32, c, P.gx, P.gz, D.NX, N);
      VIP_LAUNCH_CHECK();
      plain_image_kernel<<<gN, b256, 0, s>>>(acc, P.z[0], P.hist + (long long)(n - 1) * N, N);
      VIP_LAUNCH_CHECK();
    }
  }
  VIP_TRY(launch_finalize(ctx, D, P, model, grad, -1.0f));
  return launch_prior_and_logpost(ctx, D, P, vel, model, prior, grad, logpost);
}

}  // extern "C"
