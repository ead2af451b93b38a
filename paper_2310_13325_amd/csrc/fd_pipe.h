// Persistent, software-pipelined variant of the temporally blocked step kernel.
//
// The arithmetic of a tile is that of fd_block (the same operations in the same
// order, so the results are bitwise the same); what changes is how a compute
// unit moves from one tile to the next.  fd_block runs one block per tile, and
// with one 112 x 112 block per compute unit its start (loading u, q and c of
// the extended tile) and its end (writing the interior back, adding the
// imaging partial) leave the unit idle: about 40 % of a block's time on the
// 240 x 160 grid.  Here one block per compute unit stays resident and walks a
// run of tiles; while it steps tile i the loads of tile i+1 are in flight:
//
//  * u of tile i+1 goes straight from memory into an LDS staging area
//    (buffer loads with the LDS flag: no registers are held while they fly),
//    laid out thread-major so that every thread later reads back only the
//    words its own wave wrote;
//  * q of tile i+1 goes into registers where the mode leaves room (forward,
//    forward-with-store, recompute); the adjoint, whose imaging sum and a^n
//    prefetch fill its registers, loads it once tile i is written back;
//  * c of tile i+1 is reloaded only when the particle or the position
//    changes;
//  * what the set-up of a tile needs besides the fields (the sponge factors,
//    which receivers lie in a thread's rows) comes from small per-problem LDS
//    tables filled once per block and problem, so that a tile starts without a
//    barrier or a dependent memory round trip of its own.
//
// Each XCD takes a contiguous range of tiles; its blocks step through that
// range J tiles apart (J blocks per XCD), so that the blocks of an XCD work on
// neighbouring tiles at the same time and share their halos in its L2.  The
// grid is one block per compute unit (the LDS of one block exceeds half a
// unit's), so every block is resident from the start.
#pragma once

#include <type_traits>

#include "fd_block.h"

namespace vip {

// Per-problem LDS tables of the persistent kernel: the sponge profile g(d) at
// depth d = 0 .. nb into the sponge (gx and gz are the same profile), the grid
// row of each receiver row and the receiver id of each (receiver row, column).
// A problem whose sponge or receiver rows exceed them takes the sponge factors
// and receiver ids from global memory instead.
constexpr int kPipeProf = 64;     // sponge widths nb < 64
constexpr int kPipeRows = 8;      // receiver rows
constexpr int kPipeRmap = 1400;   // receiver rows x NX

// LDS of one persistent block.
template <int EX, int EZ, int RZ, int TMAX>
constexpr int pipe_lds_bytes() {
  return 2 * (EZ + 4) * (EX + 4) * 4 + RZ * EX * (EZ / RZ) * 4 + 4 * TMAX +
         4 * (kPipeProf + kPipeRows + kPipeRmap);
}

// MULTI: the launch carries several problems (MultiArgs: tile ranges
// [start[p], start[p + 1]) of one shape and one sweep mode) and a block's run
// of tiles may cross from one problem to the next; otherwise one problem
// (BlockArgs).
template <bool MULTI>
using PipeParams = typename std::conditional<MULTI, MultiArgs, BlockArgs>::type;

template <int MODE, int EX, int EZ, int RZ, int TMAX, bool ISO, bool MULTI>
__global__ __launch_bounds__(EX *(EZ / RZ)) void fd_pipe(PipeParams<MULTI> args) {
  // The arguments are read through the kernel-argument segment pointer and,
  // inside the tile loop, through a copy of it that the compiler cannot see
  // through: it then reloads them (scalar loads) on each tile instead of
  // holding them all in scalar registers across the loop, which would spill.
  (void)args;
  typedef const __attribute__((address_space(4))) BlockArgs KArgs;
  typedef const __attribute__((address_space(4))) PipeParams<MULTI> KParams;
  KParams *const kp0 = (KParams *)__builtin_amdgcn_kernarg_segment_ptr();
  // tiles of the launch, the problem of tile tt and its first tile, its arguments
  auto total_of = [](KParams *kp) -> int {
    if constexpr (MULTI) return kp->start[kp->nprob];
    else return kp->total_tiles;
  };
  // (tiles only move forward, so the search starts at a known problem p0 <= the answer)
  auto prob_of = [](KParams *kp, int tt, int p0) -> int {
    if constexpr (MULTI) {
      int p = p0;
      while (p + 1 < kp->nprob && tt >= kp->start[p + 1]) ++p;
      return p;
    } else {
      return 0;
    }
  };
  auto first_of = [](KParams *kp, int p) -> int {
    if constexpr (MULTI) return kp->start[p];
    else return 0;
  };
  auto args_of = [](KParams *kp, int p) -> KArgs & {
    if constexpr (MULTI) return kp->a[p];
    else return *kp;
  };
  constexpr int NTHREADS = EX * (EZ / RZ);
  constexpr int H = 2 * TMAX;                 // halo width
  constexpr int IX = EX - 2 * H, IZ = EZ - 2 * H;
  constexpr int LW = EX + 4;                  // LDS row with 2 zero cells each side
  constexpr bool ADJ = MODE == BMODE_ADJ;
  constexpr bool TRACES = MODE == BMODE_FWD || MODE == BMODE_FWS;   // record receiver traces
  constexpr bool STORE = MODE == BMODE_REC || MODE == BMODE_FWS;    // store a^n
  constexpr bool PREQ = !ADJ;                 // q of the next tile prefetched into registers
  static_assert(IX > 0 && IZ > 0 && EZ % RZ == 0 && RZ >= 2 && RZ <= 32, "tile shape");
  static_assert(NTHREADS % 64 == 0, "whole waves");
  static_assert(pipe_lds_bytes<EX, EZ, RZ, TMAX>() <= kLdsBytes, "LDS");
  __shared__ float lds[2][EZ + 4][LW];
  __shared__ float stage[RZ][NTHREADS];   // u of the next tile: row r of thread t at [r][t]
  __shared__ float injs[TMAX];  // source term w(t_n)/(dx dz) of each step of the launch
  __shared__ float prof[kPipeProf];   // sponge factor at depth d into the sponge
  __shared__ int rowz[kPipeRows];     // grid row of receiver row k
  __shared__ int rmapl[kPipeRmap];    // receiver id at (receiver row k, column X), -1: none

  // This block's run of tiles: XCD x = blockIdx % 8 owns [x per, (x + 1) per),
  // its j-th block the tiles j, j + J, j + 2 J, ... of that range.  Local tile
  // lt of a problem stands for position lt % tiles_per_pair of its local pair
  // lt / tiles_per_pair.
  const int J = int(gridDim.x) >> 3;
  const int total = total_of(kp0);
  const int per = (total + 7) >> 3;
  const int xbeg = (int(blockIdx.x) & 7) * per;
  const int tend = min(total, xbeg + per);
  int t = xbeg + (int(blockIdx.x) >> 3);
  if (t >= tend) return;

  int col = int(threadIdx.x) % EX;
  int zl0 = (int(threadIdx.x) / EX) * RZ;  // first extended-tile row of my strip

  // once per block: zero the padding cells of both u buffers (every other cell
  // is written before it is read)
  {
    constexpr int PR = 4 * LW, PC = 4 * EZ;   // padding rows, padding columns
    for (int e = threadIdx.x; e < 2 * (PR + PC); e += NTHREADS) {
      const int b = e / (PR + PC), k = e - (e / (PR + PC)) * (PR + PC);
      int row, colp;
      if (k < PR) {
        const int rr = k / LW;
        row = rr < 2 ? rr : EZ + rr;        // rows 0, 1, EZ + 2, EZ + 3
        colp = k - rr * LW;
      } else {
        const int cc = (k - PR) / EZ;
        row = 2 + (k - PR) - cc * EZ;
        colp = cc < 2 ? cc : LW - 4 + cc;   // columns 0, 1, LW - 2, LW - 1
      }
      lds[b][row][colp] = 0.0f;
    }
  }

  // Local tile lt of problem a: local pair, position, my column's byte offset
  // in a field (see fd_block for the wrap-around that the range check turns
  // into zeros above, below and beside the grid).
  auto tile_lp = [](KArgs &a, int lt) { return lt / a.tiles_per_pair; };
  auto tile_pos = [](KArgs &a, int lt) { return lt - (lt / a.tiles_per_pair) * a.tiles_per_pair; };
  auto tile_particle = [&](KArgs &a, int lt) { return (a.pair0 + tile_lp(a, lt)) / a.ns; };
  auto tile_off = [&](KArgs &a, int lt) -> uint32_t {
    const int pos = tile_pos(a, lt);
    const int tzi = pos / a.tiles_x, txi = pos - (pos / a.tiles_x) * a.tiles_x;
    const int X = txi * IX - H + col;
    return (X >= 0 && X < a.NX) ? uint32_t((tzi * IZ - H + zl0) * a.NX + X) * 4u : 0x80000000u;
  };
  // u of a tile straight into the staging area: wave w's lanes write
  // stage[r][64 w .. 64 w + 63], i.e. thread t's row r lands at stage[r][t].
  auto stage_u = [&](KArgs &a, int lt) {
    if (a.zero_in) return;
    const uint32_t offn = tile_off(a, lt);
    const uint32_t rb = uint32_t(a.NX) * 4u;
    const BufRsrc ru = field_rsrc_uniform(a.u_in + tile_lp(a, lt) * a.in_stride, a.N);
    // the wave's first thread, as a scalar, so the LDS addresses (M0) are too
    const int wave0 = __builtin_amdgcn_readfirstlane(int(threadIdx.x) & ~63);
    float *srow = &stage[0][wave0];
#pragma unroll
    for (int r = 0; r < RZ; ++r)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ru, srow + r * NTHREADS, 4,
                                               int(offn + uint32_t(r) * rb), 0, 0, 0);
  };
  auto load_q = [&](KArgs &a, int lt, float (&qq)[RZ]) {
    const uint32_t offn = tile_off(a, lt);
    const uint32_t rb = uint32_t(a.NX) * 4u;
    // zero initial state: a buffer of no records reads 0
    const BufRsrc rq =
        field_rsrc_uniform(a.q_in + tile_lp(a, lt) * a.in_stride, a.zero_in ? 0 : a.N);
#pragma unroll
    for (int r = 0; r < RZ; ++r) qq[r] = field_load(rq, offn + uint32_t(r) * rb);
  };
  auto load_c = [&](KArgs &a, int lt, float (&cv)[RZ]) {
    const uint32_t offn = tile_off(a, lt);
    const uint32_t rb = uint32_t(a.NX) * 4u;
    const BufRsrc rc = field_rsrc_uniform(a.c + (long long)tile_particle(a, lt) * a.N, a.N);
#pragma unroll
    for (int r = 0; r < RZ; ++r) cv[r] = field_load(rc, offn + uint32_t(r) * rb);
  };

  float u[RZ], q[RZ], cc[RZ], acc[ADJ ? RZ : 1];
  // q of the next tile: prefetched into qn (not the adjoint), or (adjoint)
  // loaded into av once the last step's imaging term has used it
  float qn[PREQ ? RZ : 1];
  float av[ADJ ? RZ : 1];
  int pb = 0;   // the LDS u buffer the next tile's u is published into
  {
    const int p0 = prob_of(kp0, t, 0);
    KArgs &a0 = args_of(kp0, p0);
    const int lt0 = t - first_of(kp0, p0);
    stage_u(a0, lt0);
    load_q(a0, lt0, q);
    load_c(a0, lt0, cc);
  }
  bool first = true;
  // What depends on the problem and tile position only, kept from tile to
  // tile (the 32 blocks of an XCD step neighbouring tiles, so a block's next
  // tile is often at the same position of another pair).
  int cur_p = -1, cur_pos = -1;
  int Z0 = 0, X = 0;
  bool xin = false;
  uint32_t off0 = 0, own = 0;
  float gr[RZ];   // sponge factor g = gz gx of my rows
  int rec_r0 = -1, rec_id0 = 0;   // receivers in my strip: the first one in registers
  uint32_t rec_rest = 0;          // (the common case of receivers along rows), any
                                  // further ones take a table lookup per step
  for (;;) {
    KParams *kp = kp0;
    asm volatile("" : "+s"(kp));
    int tid = int(threadIdx.x);
    if constexpr (MULTI) asm volatile("" : "+v"(col), "+v"(zl0), "+v"(tid));
    const int prob = prob_of(kp, t, cur_p < 0 ? 0 : cur_p);
    KArgs &a = args_of(kp, prob);
    const int lt = t - first_of(kp, prob);
    const int NX = a.NX, NZ = a.NZ;
    const uint32_t row_bytes = uint32_t(NX) * 4u;
    const int lp = tile_lp(a, lt);
    const int pos = tile_pos(a, lt);
    const int gp = a.pair0 + lp;
    const int particle = gp / a.ns, shot = gp - (gp / a.ns) * a.ns;
    const int sidx = a.src_idx[shot];
    const bool newprob = prob != cur_p;
    const bool newpos = newprob || pos != cur_pos;
    if (newpos) {
      const int tzi = pos / a.tiles_x, txi = pos - (pos / a.tiles_x) * a.tiles_x;
      const int X0 = txi * IX - H;
      Z0 = tzi * IZ - H;
      X = X0 + col;
      xin = X >= 0 && X < NX;
      const bool xown = col >= H && col < H + IX && X < NX;
      off0 = tile_off(a, lt);
      own = 0;
#pragma unroll
      for (int r = 0; r < RZ; ++r) {
        const int Z = Z0 + zl0 + r;
        const int zl = zl0 + r;
        if (xown && Z < NZ && zl >= H && zl < H + IZ) own |= 1u << r;
      }
    }

    // All loads of tile t have landed (vmcnt 0): u in the staging area, q and
    // c in registers.
    __builtin_amdgcn_s_waitcnt(0x0F70);
    if (!first) {
#pragma unroll
      for (int r = 0; r < RZ; ++r) q[r] = PREQ ? qn[r] : av[r];
    }
#pragma unroll
    for (int r = 0; r < RZ; ++r) u[r] = a.zero_in ? 0.0f : stage[r][tid];
    if (ADJ) {
#pragma unroll
      for (int r = 0; r < RZ; ++r) acc[r] = 0.0f;
    }
    // row of my strip that holds the shot's source, or -1
    int src_r = -1;
    {
      const int sz = sidx / NX, sx = sidx - (sidx / NX) * NX;
      if (sx == X && sz >= Z0 + zl0 && sz < Z0 + zl0 + RZ) src_r = sz - (Z0 + zl0);
    }
    if (newprob) {
      // this problem's tables (every thread is done with the last problem's;
      // on the first tile the padding of the u buffers is being zeroed)
      if (!first) __syncthreads();
      const int nrows = a.nrows;
      for (int d = tid; d <= a.nb && d < kPipeProf; d += NTHREADS) prof[d] = a.gz[a.nb - d];
      for (int Z = tid; Z < NZ; Z += NTHREADS) {
        const int rr = a.rrow[Z];
        if (rr >= 0 && rr < kPipeRows) rowz[rr] = Z;
      }
      if (nrows <= kPipeRows && nrows * NX <= kPipeRmap)
        for (int e = tid; e < nrows * NX; e += NTHREADS) rmapl[e] = a.rmap[e];
      // wavelet samples of this launch's steps (the adjoint's for its imaging
      // term: a load of its own there would wait for the step's a^n loads)
      if (tid < a.steps) injs[tid] = a.wavelet[ADJ ? a.n_start - tid : a.n_start + tid] * a.inv_area;
      __syncthreads();
    }
    if (newpos) {
      cur_p = prob;
      cur_pos = pos;
      // sponge factors g = gz gx of my rows: depth into the sponge, as the
      // profile is tabulated (0 off the grid)
      const int nb = a.nb;
      const bool tab = nb < kPipeProf;
      const int dx = max(max(nb - X, X - (NX - 1 - nb)), 0);
      const float gxv = xin ? (tab ? prof[dx] : a.gx[X]) : 0.0f;
#pragma unroll
      for (int r = 0; r < RZ; ++r) {
        const int Z = Z0 + zl0 + r;
        const int dz = max(max(nb - Z, Z - (NZ - 1 - nb)), 0);
        const float gzv = (Z >= 0 && Z < NZ) ? (tab ? prof[dz] : a.gz[Z]) : 0.0f;
        gr[r] = gzv * gxv;
      }
      // receivers in my rows and column: the first in registers, any further
      // ones as a row mask (their ids are looked up per step)
      rec_r0 = -1;
      rec_id0 = 0;
      rec_rest = 0;
      if (MODE != BMODE_REC && xin) {
        uint32_t mask = 0;
        int best = RZ, best_id = 0;
        const int nrows = a.nrows;
        if (nrows <= kPipeRows && nrows * NX <= kPipeRmap) {
          for (int k = 0; k < nrows; ++k) {
            const int r = rowz[k] - (Z0 + zl0);
            if (r >= 0 && r < RZ) {
              const int rid = rmapl[k * NX + X];
              if (rid >= 0) {
                mask |= 1u << r;
                if (r < best) {
                  best = r;
                  best_id = rid;
                }
              }
            }
          }
        } else {
#pragma unroll
          for (int r = 0; r < RZ; ++r) {
            const int Z = Z0 + zl0 + r;
            const int rr = (Z >= 0 && Z < NZ) ? a.rrow[Z] : -1;
            if (rr >= 0) {
              const int rid = a.rmap[rr * NX + X];
              if (rid >= 0) {
                mask |= 1u << r;
                if (r < best) {
                  best = r;
                  best_id = rid;
                }
              }
            }
          }
        }
        if (mask) {
          rec_r0 = best;
          rec_id0 = best_id;
          rec_rest = mask & ~(1u << best);
        }
      }
    }
    first = false;
    // Publish u into the buffer the previous tile's last step did not read:
    // no thread reads it until the barrier that opens step 0, and every
    // thread writes only its own cells, which only it wrote before.
#pragma unroll
    for (int r = 0; r < RZ; ++r) lds[pb][zl0 + r + 2][col + 2] = u[r];
    const int tnext = t + J;
    const bool more = tnext < tend;
    // the next tile's loads fly while this tile steps (my staging words are
    // free: their values are in u)
    if (more) {
      const int pn = prob_of(kp, tnext, prob);
      KArgs &an = args_of(kp, pn);
      const int ltn = tnext - first_of(kp, pn);
      stage_u(an, ltn);
      if constexpr (PREQ) load_q(an, ltn, qn);
    }

    // Adjoint imaging, one step late, as in fd_block.
    const long long seg_pair = lp * a.seg_stride;
    const uint32_t off_av = own ? off0 : 0x80000000u;
    float rv = 0.0f, rvn = 0.0f;
    if (ADJ) {
#pragma unroll
      for (int r = 0; r < RZ; ++r) av[r] = 0.0f;
      if (rec_r0 >= 0) rv = a.rho[lp * a.rho_stride + (long long)(a.n_start + 1) * a.nr + rec_id0];
    }

    for (int s = 0; s < a.steps; ++s) {
      const int cur = (s + pb) & 1, nxt = cur ^ 1;
      const int n = ADJ ? a.n_start - s : a.n_start + s;
      if (ADJ && s + 1 < a.steps && rec_r0 >= 0)
        rvn = a.rho[lp * a.rho_stride + (long long)n * a.nr + rec_id0];
      // lds[cur] holds the current u; lds[nxt] is no longer read.  A plain
      // barrier after the LDS writes: __syncthreads() would also wait for
      // every vector memory operation in flight, the next tile's staging
      // loads among them, since those write LDS.
      asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
      if (!ADJ) {
        if (src_r >= 0) {
          const float f = injs[s];
#pragma unroll
          for (int r = 0; r < RZ; ++r)
            if (r == src_r) q[r] = fmaf(cc[r], f, q[r]);
        }
      } else {
        if (rec_r0 >= 0) {
#pragma unroll
          for (int r = 0; r < RZ; ++r)
            if (r == rec_r0) q[r] = fmaf(cc[r], rv, q[r]);
        }
        if (rec_rest) {
#pragma unroll
          for (int r = 0; r < RZ; ++r) {
            if ((rec_rest >> r) & 1u) {
              const int rid = a.rmap[a.rrow[Z0 + zl0 + r] * NX + X];
              const float rho = a.rho[lp * a.rho_stride + (long long)(n + 1) * a.nr + rid];
              q[r] = fmaf(cc[r], rho, q[r]);
            }
          }
        }
      }
      uint32_t off_s = ADJ ? off_av : off0;
      if (STORE || ADJ) asm volatile("" : "+v"(off_s));
      BufRsrc rseg;
      if (STORE || ADJ)
        rseg = field_rsrc_uniform(a.seg + seg_pair + (long long)(n - a.seg_n0) * a.N, a.N);
      float prev1 = lds[cur][zl0 + 1][col + 2];   // u at row zl0 - 1
      float prev2 = lds[cur][zl0][col + 2];       // u at row zl0 - 2
      const float nextA = lds[cur][zl0 + RZ + 2][col + 2];   // row zl0 + RZ
      const float nextB = lds[cur][zl0 + RZ + 3][col + 2];   // row zl0 + RZ + 1
#pragma unroll
      for (int r = 0; r < RZ; ++r) {
        const int zl = zl0 + r;
        const float uc = u[r];
        if (ADJ) {
          acc[r] = fmaf(uc, av[r], acc[r]);
          av[r] = field_load(rseg, off_s + uint32_t(r) * row_bytes);
        }
        const float dn1 = (r + 1 < RZ) ? u[r + 1] : nextA;
        const float dn2 = (r + 2 < RZ) ? u[r + 2] : (r + 2 == RZ ? nextA : nextB);
        const float xm1 = lds[cur][zl + 2][col + 1], xp1 = lds[cur][zl + 2][col + 3];
        const float xm2 = lds[cur][zl + 2][col], xp2 = lds[cur][zl + 2][col + 4];
        float lap;
        if (ISO) {
          const float s1 = (xm1 + xp1) + (prev1 + dn1), s2 = (xm2 + xp2) + (prev2 + dn2);
          lap = fmaf(a.w1x, fmaf(-4.0f, uc, s1), a.w2x * fmaf(-4.0f, uc, s2));
        } else {
          const float d1x = fmaf(-2.0f, uc, xm1 + xp1), d2x = fmaf(-2.0f, uc, xm2 + xp2);
          const float d1z = fmaf(-2.0f, uc, prev1 + dn1), d2z = fmaf(-2.0f, uc, prev2 + dn2);
          lap = fmaf(a.w1x, d1x, fmaf(a.w2x, d2x, fmaf(a.w1z, d1z, a.w2z * d2z)));
        }
        if (STORE && ((own >> r) & 1u))
          field_store(rseg, off_s + uint32_t(r) * row_bytes, lap);
        const float qn1 = gr[r] * fmaf(cc[r], lap, q[r]);
        const float un = fmaf(gr[r], uc, qn1);
        prev2 = prev1;
        prev1 = uc;
        u[r] = un;
        q[r] = qn1;
        lds[nxt][zl + 2][col + 2] = un;
      }
      if (TRACES) {
        if (rec_r0 >= 0 && ((own >> rec_r0) & 1u)) {
          const float val = lds[nxt][zl0 + rec_r0 + 2][col + 2];
          float *d = a.data + lp * a.data_stride;
          d[(long long)(n + 1) * a.nr + rec_id0] = val;
          if (n == 0) d[rec_id0] = 0.0f;   // u^0 = 0
        }
        if (rec_rest & own) {
          float *d = a.data + lp * a.data_stride;
#pragma unroll
          for (int r = 0; r < RZ; ++r) {
            if (((rec_rest & own) >> r) & 1u) {
              const int rid = a.rmap[a.rrow[Z0 + zl0 + r] * NX + X];
              d[(long long)(n + 1) * a.nr + rid] = u[r];
              if (n == 0) d[rid] = 0.0f;
            }
          }
        }
      }
      if (ADJ) {
        if (src_r >= 0 && ((own >> src_r) & 1u)) {
          const float f = injs[s];
#pragma unroll
          for (int r = 0; r < RZ; ++r)
            if (r == src_r) acc[r] = fmaf(u[r], f, acc[r]);
        }
        rv = rvn;
      }
    }
    pb = (pb + a.steps) & 1;   // the buffer the last step wrote, not read
    if (ADJ) {
#pragma unroll
      for (int r = 0; r < RZ; ++r) acc[r] = fmaf(u[r], av[r], acc[r]);   // the last step's term
    }
    // The next tile's c (when it differs) and the adjoint's q go out before
    // the write-back, into registers this tile no longer needs.
    if (more) {
      // (the next tile's problem is looked up again rather than kept live
      // across the steps)
      KParams *kq = kp;
      const int pn = prob_of(kq, tnext, prob);
      KArgs &an = args_of(kq, pn);
      const int ltn = tnext - first_of(kq, pn);
      if (pn != prob || tile_particle(an, ltn) != particle || tile_pos(an, ltn) != pos)
        load_c(an, ltn, cc);
      if constexpr (!PREQ) load_q(an, ltn, av);
    }
    // write back the owned interior: u, q and (adjoint) the launch's imaging
    // partial into the FP64 sum (one add per point and launch, so the
    // no-return atomic adds what a read, add and store would)
    // (the bases of my pair's fields are formed once, as values the compiler
    // cannot recompute from the arguments: otherwise it reloads the arguments
    // and redoes the 64-bit arithmetic for every row)
    // grid index of my first row: an owned point is on the grid, so off0 is 4
    // times that index taken modulo 2^32; the row may lie above the grid (a
    // negative index), hence the signed division
    const int i0 = int(off0) / 4;
    if (a.u_out) {
      typedef __attribute__((address_space(1))) float GFloat;
      GFloat *uo = (GFloat *)(a.u_out + lp * a.out_stride);
      GFloat *qo = (GFloat *)(a.q_out + lp * a.out_stride);
      asm volatile("" : "+s"(uo), "+s"(qo));
#pragma unroll
      for (int r = 0; r < RZ; ++r) {
        if (!((own >> r) & 1u)) continue;
        uo[i0 + r * NX] = u[r];
        qo[i0 + r * NX] = q[r];
      }
    }
    if (ADJ) {
      typedef __attribute__((address_space(1))) double GDouble;
      GDouble *ao = (GDouble *)(a.acc64 + lp * a.acc64_stride);
      asm volatile("" : "+s"(ao));
#pragma unroll
      for (int r = 0; r < RZ; ++r)
        if ((own >> r) & 1u)
          __hip_atomic_fetch_add(ao + i0 + r * NX, double(acc[r]), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!more) break;
    t = tnext;
  }
}

}  // namespace vip
