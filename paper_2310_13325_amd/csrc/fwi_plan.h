// Problem dimensions, validation and workspace layout of the FWI calls.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "vip_internal.h"

namespace vip {

struct FwiDims {
  int nx, nz, nb, nt, NX, NZ;
  long long N;          // padded points per field
  int ns, nr, np;
  long long pairs;      // np * ns, pair = particle * ns + shot
  // Rows of d_obs, and the misfit scale nobs / ns of a geometry that lists a
  // subset of them (the unbiased minibatch estimate of section 2.4; 1 without
  // a shot_index).
  int nobs;
  double misfit_scale;
  // Steps n = 0 .. nt-2 (u^n -> u^{n+1}) fall into segments: regular ones of
  // k steps over [0, n_split) and, when stored > 0, one tail segment
  // [n_split, nt-1) of the last `stored` steps.  The state at every segment
  // start but the first is checkpointed; the backward sweep recomputes each
  // segment's a^n from it, except the tail's when the forward stores them.
  int k, nseg;          // checkpoint interval, number of segments
  int stored;           // steps in the tail segment (0: none)
  int n_split;          // first step of the tail segment (nt-1 when stored == 0)
  int nseg_r;           // regular segments
  int seg_slots;        // a^n slots of the segment buffer (the longest segment)
  int seg_begin(int s) const { return s < nseg_r ? s * k : n_split; }
  int seg_end(int s) const { return s + 1 < nseg ? seg_begin(s + 1) : nt - 1; }
  long long live;       // pairs simulated at once
  int nrows;            // distinct receiver rows
  int rz;               // rows per thread in the streaming step kernel (tile height 4*rz)
  int tile;             // temporally blocked tile shape, -1 = one step per launch
  float cx, cz, inv_area;
  double inv_dx2, inv_dz2;   // 1/dx^2, 1/dz^2 before rounding
};

// Stability of the fourth-order / leapfrog scheme: the largest eigenvalue of
// -L is (16/3)(1/dx^2 + 1/dz^2), and leapfrog needs c * lambda_max <= 4.
inline double courant_factor(const vip_grid &g) {
  return g.vmax * g.dt * std::sqrt((4.0 / 3.0) * (1.0 / (g.dx * g.dx) + 1.0 / (g.dz * g.dz)));
}

inline bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Largest padded grid (points) the temporally blocked kernel accepts.
constexpr long long kMaxBlockedPoints = 1LL << 29;
int default_tile(int NX, int NZ, long long pairs);   // fwi.hip; pairs <= 0: many
int tile_count();

inline int default_rz(int NZ) { return NZ >= 96 ? 8 : (NZ >= 40 ? 4 : 2); }

inline vip_status make_dims(const vip_grid *grid, const vip_geometry *geom, int32_t np,
                            int32_t ckpt_every, int32_t live, bool need_wavelet, FwiDims *D,
                            int32_t stored_steps = 0) {
  if (!grid || !geom || !D) return VIP_E_ARG;
  const vip_grid &g = *grid;
  if (g.nx < 1 || g.nz < 1 || g.nb < 0 || g.nt < 2) return VIP_E_ARG;
  if (!finite_pos(g.dx) || !finite_pos(g.dz) || !finite_pos(g.dt) || !finite_pos(g.vmax))
    return VIP_E_ARG;
  if (!std::isfinite(g.sponge_alpha) || g.sponge_alpha < 0.0) return VIP_E_ARG;
  if (np < 1 || geom->ns < 1 || geom->nr < 1) return VIP_E_ARG;
  if (!geom->src_ix || !geom->src_iz || !geom->rec_ix || !geom->rec_iz) return VIP_E_ARG;
  if (need_wavelet && !geom->wavelet) return VIP_E_ARG;
  for (int s = 0; s < geom->ns; ++s)
    if (geom->src_ix[s] < 0 || geom->src_ix[s] >= g.nx || geom->src_iz[s] < 0 ||
        geom->src_iz[s] >= g.nz)
      return VIP_E_ARG;
  for (int r = 0; r < geom->nr; ++r)
    if (geom->rec_ix[r] < 0 || geom->rec_ix[r] >= g.nx || geom->rec_iz[r] < 0 ||
        geom->rec_iz[r] >= g.nz)
      return VIP_E_ARG;
  if (geom->shot_index) {
    if (geom->nobs < 1) return VIP_E_ARG;
    for (int s = 0; s < geom->ns; ++s)
      if (geom->shot_index[s] < 0 || geom->shot_index[s] >= geom->nobs) return VIP_E_ARG;
  }
  {
    // receivers must sit on distinct nodes (each node maps to one trace)
    std::vector<long long> nodes(geom->nr);
    for (int r = 0; r < geom->nr; ++r) nodes[r] = (long long)geom->rec_iz[r] * g.nx + geom->rec_ix[r];
    std::sort(nodes.begin(), nodes.end());
    if (std::adjacent_find(nodes.begin(), nodes.end()) != nodes.end()) return VIP_E_ARG;
  }
  if (courant_factor(g) > 1.0) return VIP_E_CFL;
  if (ckpt_every < 1 || live < 0) return VIP_E_ARG;
  if (stored_steps < 0 || stored_steps > g.nt - 1) return VIP_E_ARG;
  FwiDims d;
  d.nx = g.nx;
  d.nz = g.nz;
  d.nb = g.nb;
  d.nt = g.nt;
  d.NX = g.nx + 2 * g.nb;
  d.NZ = g.nz + 2 * g.nb;
  d.N = (long long)d.NX * d.NZ;
  if (d.N >= (1LL << 31)) return VIP_E_UNSUPPORTED;
  d.ns = geom->ns;
  d.nr = geom->nr;
  d.nobs = geom->shot_index ? geom->nobs : geom->ns;
  d.misfit_scale = double(d.nobs) / double(d.ns);
  d.np = np;
  d.pairs = (long long)np * geom->ns;
  if (d.pairs >= (1LL << 31)) return VIP_E_UNSUPPORTED;
  d.k = std::min(ckpt_every, g.nt - 1);
  d.stored = stored_steps;
  d.n_split = g.nt - 1 - stored_steps;
  d.nseg_r = (d.n_split + d.k - 1) / d.k;
  d.nseg = d.nseg_r + (stored_steps > 0 ? 1 : 0);
  d.seg_slots = std::max(d.nseg_r > 0 ? std::min(d.k, d.n_split) : 0, stored_steps);
  d.live = live == 0 ? d.pairs : std::min<long long>(live, d.pairs);
  {
    std::vector<int> rows(geom->rec_iz, geom->rec_iz + geom->nr);
    std::sort(rows.begin(), rows.end());
    d.nrows = int(std::unique(rows.begin(), rows.end()) - rows.begin());
  }
  d.rz = default_rz(d.NZ);
  d.tile = d.N < kMaxBlockedPoints ? default_tile(d.NX, d.NZ, d.live) : -1;
  d.inv_dx2 = 1.0 / (double(g.dx) * g.dx);
  d.inv_dz2 = 1.0 / (double(g.dz) * g.dz);
  d.cx = float(1.0 / (g.dx * g.dx));
  d.cz = float(1.0 / (g.dz * g.dz));
  d.inv_area = float(1.0 / (g.dx * g.dz));
  *D = d;
  return VIP_OK;
}

enum PlanKind { PLAN_FORWARD = 0, PLAN_GRAD = 1, PLAN_TAPE = 2, PLAN_PLAIN = 3 };

struct FwiPlan {
  uint32_t *status = nullptr;
  float *gx = nullptr, *gz = nullptr;
  int32_t *src = nullptr, *rrow = nullptr, *rmap = nullptr;
  int32_t *shot_row = nullptr;   // row of d_obs holding each shot
  float *c = nullptr;
  float *u[2] = {nullptr, nullptr}, *q[2] = {nullptr, nullptr};
  float *z[2] = {nullptr, nullptr}, *Q[2] = {nullptr, nullptr};
  float *ckpt = nullptr, *seg = nullptr;
  float *acc32 = nullptr;   // plain path: Laplacian scratch of one field
  double *acc64 = nullptr;
  float *resid = nullptr;
  double *J = nullptr;
  float *model = nullptr;   // velocities from theta (transform prior) [np][nz][nx]
  float *hist = nullptr;    // plain path: full a-history of one pair
  size_t bytes = 0;
};

inline void plan_fwi(const FwiDims &D, char *base, int kind, FwiPlan *P) {
  Arena A;
  A.base = base;
  P->status = reinterpret_cast<uint32_t *>(base);
  P->gx = A.take<float>(D.NX);
  P->gz = A.take<float>(D.NZ);
  P->src = A.take<int32_t>(D.ns);
  P->shot_row = A.take<int32_t>(D.ns);
  P->rrow = A.take<int32_t>(D.NZ);
  P->rmap = A.take<int32_t>(size_t(D.nrows) * D.NX);
  P->c = A.take<float>(size_t(D.np) * D.N);
  const long long live = (kind == PLAN_GRAD) ? D.live : (kind == PLAN_PLAIN ? 1 : D.pairs);
  const size_t field = size_t(live) * size_t(D.N);
  for (int b = 0; b < 2; ++b) {
    P->u[b] = A.take<float>(field);
    P->q[b] = A.take<float>(field);
  }
  if (kind != PLAN_FORWARD) {
    for (int b = 0; b < 2; ++b) {
      P->z[b] = A.take<float>(field);
      P->Q[b] = A.take<float>(field);
    }
    P->acc64 = A.take<double>(size_t(D.pairs) * D.N);
  }
  if (kind == PLAN_GRAD) {
    P->ckpt = A.take<float>(size_t(live) * size_t(D.nseg - 1) * 2 * D.N);
    P->seg = A.take<float>(size_t(live) * size_t(D.seg_slots) * D.N);
    P->resid = A.take<float>(size_t(live) * D.nt * D.nr);
    P->J = A.take<double>(D.pairs);
    P->model = A.take<float>(size_t(D.np) * D.nx * D.nz);
  } else if (kind == PLAN_TAPE) {
    P->seg = A.take<float>(size_t(live) * size_t(D.seg_slots) * D.N);
  } else if (kind == PLAN_PLAIN) {
    P->hist = A.take<float>(size_t(D.nt - 1) * D.N);
    P->resid = A.take<float>(size_t(D.nt) * D.nr);
    P->J = A.take<double>(D.pairs);
    P->acc32 = A.take<float>(D.N);
    P->model = A.take<float>(size_t(D.np) * D.nx * D.nz);
  }
  P->bytes = A.bytes();
}

// The context may force a tile shape (-1 = one step per launch).
inline void apply_tile_choice(const vip_ctx *ctx, FwiDims *D) {
  if (ctx && ctx->tile >= -1) D->tile = ctx->tile;
}

// Implemented in fwi.hip, shared with the plain path.
vip_status upload_tables(vip_ctx *ctx, const FwiDims &D, const vip_grid *grid,
                         const vip_geometry *geom, const FwiPlan &P);
vip_status launch_coeff(vip_ctx *ctx, const FwiDims &D, const vip_grid *grid, const float *vel,
                        const FwiPlan &P);
vip_status launch_finalize(vip_ctx *ctx, const FwiDims &D, const FwiPlan &P, const float *vel,
                           float *grad, float sign);
vip_status check_prior(const vip_prior *prior);
// theta -> m into the plan's model buffer for the transform prior (returns the
// velocities the sweeps use: vel itself for the other kinds)
const float *prior_model(vip_ctx *ctx, const FwiDims &D, const FwiPlan &P, const float *vel,
                         const vip_prior *prior);
// prior terms of the gradient (in place, after the misfit gradient) and logpost
vip_status launch_prior_and_logpost(vip_ctx *ctx, const FwiDims &D, const FwiPlan &P,
                                    const float *vel, const float *model, const vip_prior *prior,
                                    float *grad, double *logpost);

}  // namespace vip
