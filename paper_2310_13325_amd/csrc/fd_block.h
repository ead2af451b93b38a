// Temporally blocked time stepping: one launch advances every live pair by up
// to TMAX steps.
//
// A block owns an interior tile IX x IZ of one pair's padded grid and loads the
// extended tile EX x EZ = (IX + 4 TMAX) x (IZ + 4 TMAX) of u, q and c once.  Each
// step invalidates two more cells at the edges of the extended tile (the
// stencil reaches two cells out), so after T <= TMAX steps the interior is still
// exact; it is written back once.  Halo cells are recomputed by the
// neighbouring blocks instead of being exchanged, trading VALU work for HBM
// traffic: per point and step the kernel moves (12 e + 8) / T bytes
// (e = EX EZ / (IX IZ)) instead of 20.
//
// Thread layout: thread t owns column t % EX of the extended tile and the RZ
// consecutive rows of strip t / EX, keeping u, q, c and the damping of those
// points in registers.  Per step the current u of every point is published in
// a double-buffered LDS tile (two zero cells of padding on each side); a
// thread reads its x-neighbours and the two rows beyond each end of its strip
// from LDS and the rows inside its strip from registers.  One barrier per
// step.
//
// Points outside the padded grid have g = c = 0, so they stay exactly 0 (the
// zero ghost layers of the scheme).  The source (forward, recompute) and the
// residual (adjoint) are injected at every point of the extended tile that
// carries one, so halo points evolve exactly like the owner's; receiver
// traces, the aⁿ segment stores and loads, and the imaging sum are handled for
// owned points only.
#pragma once

#include "fwi_plan.h"

namespace vip {

enum { BMODE_FWD = 0, BMODE_REC = 1, BMODE_ADJ = 2 };

struct BlockArgs {
  int NX, NZ, N;
  int tiles_x, tiles_per_pair, total_tiles;
  int pair0, ns, nt, nr;
  int steps;              // T <= TMAX
  int n_start;            // FWD/REC: first input time index; ADJ: first n (produces z^{n+1}), descending
  int seg_n0;             // REC/ADJ: time index of segment slot 0
  float cx, cz, inv_area;
  const float *gx, *gz, *c;
  const int *src_idx, *rrow, *rmap;
  const float *wavelet;
  int zero_in;
  const float *u_in, *q_in;
  long long in_stride;
  float *u_out, *q_out;   // null: the final state is not needed
  long long out_stride;
  float *data;            // FWD: traces [pair][nt][nr]
  long long data_stride;
  float *seg;             // REC: a^n written at slot n - seg_n0; ADJ: read
  long long seg_stride;
  const float *rho;       // ADJ: residual [pair][nt][nr]
  long long rho_stride;
  double *acc64;          // ADJ: imaging sum [pair][N] (+= per launch)
  long long acc64_stride;
};

template <int MODE, int EX, int EZ, int RZ, int TMAX>
__global__ __launch_bounds__(EX *(EZ / RZ)) void fd_block(BlockArgs a) {
  constexpr int NTHREADS = EX * (EZ / RZ);
  constexpr int H = 2 * TMAX;                 // halo width
  constexpr int IX = EX - 2 * H, IZ = EZ - 2 * H;
  constexpr int LW = EX + 4;                  // LDS row with 2 zero cells each side
  constexpr float w1 = 4.0f / 3.0f, w2 = -1.0f / 12.0f;
  // The adjoint keeps one u buffer (two barriers per step) and c and the
  // imaging sum in LDS, which leaves registers for prefetching the next
  // step's aⁿ; forward and recompute double-buffer u and keep c in registers.
  constexpr bool ADJ = MODE == BMODE_ADJ;
  constexpr int NBUF = ADJ ? 1 : 2;
  static_assert(IX > 0 && IZ > 0 && EZ % RZ == 0 && RZ >= 2 && RZ <= 32, "tile shape");
  __shared__ float lds[NBUF][EZ + 4][LW];
  __shared__ float gzs[EZ];     // z damping of each extended-tile row (0 outside the grid)
  __shared__ int rrs[EZ];       // receiver-row index of each extended-tile row (-1: none)
  __shared__ float injs[TMAX];  // forward / recompute: source term w(t_n)/(dx dz) of each step
  __shared__ float cs[ADJ ? EZ : 1][ADJ ? EX : 1];     // adjoint: c of each point
  __shared__ float accs[ADJ ? EZ : 1][ADJ ? EX : 1];   // adjoint: FP32 imaging sum of this launch

  // tile index, contiguous ranges per XCD (blocks are dealt round-robin to 8 XCDs)
  const int per = int(gridDim.x) >> 3;
  const int b = int(blockIdx.x);
  const int t = (b & 7) * per + (b >> 3);
  if (t >= a.total_tiles) return;
  const int lp = t / a.tiles_per_pair;
  const int rem = t - lp * a.tiles_per_pair;
  const int tzi = rem / a.tiles_x, txi = rem - (rem / a.tiles_x) * a.tiles_x;
  const int X0 = txi * IX - H, Z0 = tzi * IZ - H;   // extended-tile origin in the padded grid
  const int gp = a.pair0 + lp;
  const int particle = gp / a.ns, shot = gp - (gp / a.ns) * a.ns;
  const int NX = a.NX, NZ = a.NZ;

  // zero the u buffers (padding cells must read 0); per-row tables; wavelet samples
  for (int e = threadIdx.x; e < NBUF * (EZ + 4) * LW; e += NTHREADS) (&lds[0][0][0])[e] = 0.0f;
  for (int e = threadIdx.x; e < EZ; e += NTHREADS) {
    const int Z = Z0 + e;
    const bool zin = Z >= 0 && Z < NZ;
    gzs[e] = zin ? a.gz[Z] : 0.0f;
    rrs[e] = (zin && MODE != BMODE_REC) ? a.rrow[Z] : -1;
  }
  if (!ADJ && int(threadIdx.x) < a.steps)
    injs[threadIdx.x] = a.wavelet[a.n_start + int(threadIdx.x)] * a.inv_area;

  const int col = int(threadIdx.x) % EX;
  const int strip = int(threadIdx.x) / EX;
  const int zl0 = strip * RZ;              // first extended-tile row of my strip
  const int X = X0 + col;
  const bool xin = X >= 0 && X < NX;
  const bool xown = col >= H && col < H + IX && X < NX;
  const float gxv = xin ? a.gx[X] : 0.0f;
  const int idx0 = (Z0 + zl0) * NX + X;    // grid index of my first row (rows follow at +NX)

  float u[RZ], q[RZ], cc[ADJ ? 1 : RZ];
  uint32_t own = 0;
  const float *uin = a.u_in + lp * a.in_stride;
  const float *qin = a.q_in + lp * a.in_stride;
  const float *cp = a.c + (long long)particle * a.N;
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const int Z = Z0 + zl0 + r;
    const bool in = xin && Z >= 0 && Z < NZ;
    const int i = in ? idx0 + r * NX : 0;
    u[r] = (in && !a.zero_in) ? uin[i] : 0.0f;
    q[r] = (in && !a.zero_in) ? qin[i] : 0.0f;
    const float cv = in ? cp[i] : 0.0f;
    if (ADJ) {
      cs[zl0 + r][col] = cv;
      accs[zl0 + r][col] = 0.0f;
    } else {
      cc[r] = cv;
    }
    const int zl = zl0 + r;
    if (in && xown && zl >= H && zl < H + IZ) own |= 1u << r;
  }
  // row of my strip that holds the shot's source (forward / recompute), or -1
  int src_r = -1;
  if (!ADJ) {
    const int sidx = a.src_idx[shot];
    const int sz = sidx / NX, sx = sidx - (sidx / NX) * NX;
    if (sx == X && sz >= Z0 + zl0 && sz < Z0 + zl0 + RZ) src_r = sz - (Z0 + zl0);
  }
  __syncthreads();   // buffers zeroed, row tables ready

  // Receivers in my strip: the first one is kept in registers (the common case
  // of receivers along rows); any further ones take a table lookup per step.
  int rec_r0 = -1, rec_id0 = 0;
  uint32_t rec_rest = 0;
  if (MODE != BMODE_REC && xin) {
#pragma unroll
    for (int r = 0; r < RZ; ++r) {
      const int rr = rrs[zl0 + r];
      if (rr >= 0) {
        const int rid = a.rmap[rr * NX + X];
        if (rid >= 0) {
          if (rec_r0 < 0) {
            rec_r0 = r;
            rec_id0 = rid;
          } else {
            rec_rest |= 1u << r;
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RZ; ++r) lds[0][zl0 + r + 2][col + 2] = u[r];

  // adjoint prefetch of step 0: aⁿ of owned rows (others read a harmless
  // in-bounds slot) and the residual at my first receiver
  const long long seg_pair = lp * a.seg_stride;
  float av[ADJ ? RZ : 1], rv = 0.0f;
  if (ADJ) {
    const float *segp = a.seg + seg_pair + (long long)(a.n_start - a.seg_n0) * a.N;
#pragma unroll
    for (int r = 0; r < RZ; ++r) av[r] = segp[((own >> r) & 1u) ? idx0 + r * NX : 0];
    if (rec_r0 >= 0) rv = a.rho[lp * a.rho_stride + (long long)(a.n_start + 1) * a.nr + rec_id0];
  }

  for (int s = 0; s < a.steps; ++s) {
    const int cur = ADJ ? 0 : (s & 1), nxt = ADJ ? 0 : (cur ^ 1);
    const int n = ADJ ? a.n_start - s : a.n_start + s;
    float avn[ADJ ? RZ : 1], rvn = 0.0f;
    if (ADJ && s + 1 < a.steps) {
      const float *segp = a.seg + seg_pair + (long long)(n - 1 - a.seg_n0) * a.N;
#pragma unroll
      for (int r = 0; r < RZ; ++r) avn[r] = segp[((own >> r) & 1u) ? idx0 + r * NX : 0];
      if (rec_r0 >= 0) rvn = a.rho[lp * a.rho_stride + (long long)n * a.nr + rec_id0];
    }
    __syncthreads();
    const float inj = ADJ ? rv : injs[s];
    float prev1 = lds[cur][zl0 + 1][col + 2];   // u at row zl0 - 1
    float prev2 = lds[cur][zl0][col + 2];       // u at row zl0 - 2
    const float nextA = lds[cur][zl0 + RZ + 2][col + 2];   // row zl0 + RZ
    const float nextB = lds[cur][zl0 + RZ + 3][col + 2];   // row zl0 + RZ + 1
#pragma unroll
    for (int r = 0; r < RZ; ++r) {
      const int zl = zl0 + r;
      const float uc = u[r];
      const float dn1 = (r + 1 < RZ) ? u[r + 1] : nextA;
      const float dn2 = (r + 2 < RZ) ? u[r + 2] : (r + 2 == RZ ? nextA : nextB);
      const float xm1 = lds[cur][zl + 2][col + 1], xp1 = lds[cur][zl + 2][col + 3];
      const float xm2 = lds[cur][zl + 2][col], xp2 = lds[cur][zl + 2][col + 4];
      const float lx = w1 * ((xm1 - uc) + (xp1 - uc)) + w2 * ((xm2 - uc) + (xp2 - uc));
      const float lz = w1 * ((prev1 - uc) + (dn1 - uc)) + w2 * ((prev2 - uc) + (dn2 - uc));
      float lap = a.cx * lx + a.cz * lz;
      const bool owned = (own >> r) & 1u;
      if (!ADJ) {
        if (r == src_r) lap += inj;
      } else {
        if (r == rec_r0) lap += inj;
        if ((rec_rest >> r) & 1u) {
          const int rid = a.rmap[rrs[zl] * NX + X];
          lap += a.rho[lp * a.rho_stride + (long long)(n + 1) * a.nr + rid];
        }
      }
      if (MODE == BMODE_REC && owned)
        a.seg[seg_pair + (long long)(n - a.seg_n0) * a.N + idx0 + r * NX] = lap;
      const float g = gzs[zl] * gxv;
      const float cv = ADJ ? cs[zl][col] : cc[r];
      const float qn = g * (q[r] + cv * lap);
      const float un = g * uc + qn;
      prev2 = prev1;
      prev1 = uc;
      u[r] = un;
      q[r] = qn;
      if (!ADJ) lds[nxt][zl + 2][col + 2] = un;
      if (MODE == BMODE_FWD && owned) {
        int rid = -1;
        if (r == rec_r0) rid = rec_id0;
        else if ((rec_rest >> r) & 1u) rid = a.rmap[rrs[zl] * NX + X];
        if (rid >= 0) {
          float *d = a.data + lp * a.data_stride;
          d[(long long)(n + 1) * a.nr + rid] = un;
          if (n == 0) d[rid] = 0.0f;   // u^0 = 0
        }
      }
      if (ADJ && owned) accs[zl][col] += un * av[r];
    }
    if (ADJ) {
      __syncthreads();   // every read of the old u is done
#pragma unroll
      for (int r = 0; r < RZ; ++r) {
        lds[0][zl0 + r + 2][col + 2] = u[r];
        av[r] = avn[r];
      }
      rv = rvn;
    }
  }
  // write back the owned interior
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    if (!((own >> r) & 1u)) continue;
    const int i = idx0 + r * NX;
    if (a.u_out) {
      a.u_out[lp * a.out_stride + i] = u[r];
      a.q_out[lp * a.out_stride + i] = q[r];
    }
    if (ADJ) a.acc64[lp * a.acc64_stride + i] += double(accs[zl0 + r][col]);
  }
}

}  // namespace vip
