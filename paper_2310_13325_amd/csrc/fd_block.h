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
// consecutive rows of strip t / EX, keeping u, q and (forward, recompute) c of
// those points in registers.  Per step the current u of every point is
// published in a double-buffered LDS tile (two zero cells of padding on each
// side); a thread reads its x-neighbours and the two rows beyond each end of
// its strip from LDS and the rows inside its strip from registers.  One
// barrier per step.  The adjoint keeps its imaging sum over the launch's steps
// in FP32 registers and adds it into the FP64 accumulator once per launch.
//
// Points outside the padded grid have g = c = 0, so they stay exactly 0 (the
// zero ghost layers of the scheme).  The source (forward, recompute) and the
// residual (adjoint) are added to q at every point of the extended tile that
// carries one, so halo points evolve exactly like the owner's; receiver
// traces, the aⁿ segment stores and loads, and the imaging sum are handled for
// owned points only.
//
// Field loads go through buffer descriptors whose range check returns 0 for
// rows above or below the grid, so a strip needs no per-row bounds test.
#pragma once

#include "fwi_plan.h"

namespace vip {

// Sweep modes: forward (traces), recompute (stores a^n), adjoint (reads a^n,
// images), and forward that also stores a^n (the tail segment kept by the
// forward sweep).
enum { BMODE_FWD = 0, BMODE_REC = 1, BMODE_ADJ = 2, BMODE_FWS = 3 };

// Raw buffer descriptor over one [N] float field (stride 0, N * 4 bytes, the
// gfx9-family data-format word).  Offsets are bytes in the VGPR offset, which
// the hardware checks against the size: loads out of range return 0 and
// stores out of range are dropped.
using BufRsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ BufRsrc field_rsrc(const float *base, int n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), (short)0, n * 4, 0x00020000);
}
// The same over a base address that is the same for the whole wave, taken as
// such: the compiler then keeps the descriptor in scalar registers even when
// register pressure would otherwise move it to vector registers (and make
// every access loop over the distinct descriptors of the wave).
__device__ __forceinline__ BufRsrc field_rsrc_uniform(const float *base, int n) {
  const uint64_t p = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(p));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(p >> 32));
  return field_rsrc(reinterpret_cast<const float *>((uint64_t(hi) << 32) | lo),
                    __builtin_amdgcn_readfirstlane(n));
}
// (The b32 builtins move raw 32-bit words, hence the bit casts.)
__device__ __forceinline__ float field_load(BufRsrc r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(off), 0, 0));
}
__device__ __forceinline__ void field_store(BufRsrc r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, int(off), 0, 0);
}

struct BlockArgs {
  int NX, NZ, N;
  int tiles_x, tiles_per_pair, total_tiles;
  int pair0, ns, nt, nr;
  int steps;              // T <= TMAX
  int n_start;            // FWD/REC: first input time index; ADJ: first n (produces z^{n+1}), descending
  int seg_n0;             // REC/FWS/ADJ: time index of segment slot 0
  float w1x, w2x, w1z, w2z;   // Laplacian weights 4/3, -1/12 times 1/dx^2 (x) or 1/dz^2 (z)
  int iso;                    // w1x == w1z and w2x == w2z (dx == dz): the fused Laplacian applies
  float inv_area;
  const float *gx, *gz, *c;
  const int *src_idx, *rrow, *rmap;
  int nb;                 // sponge width (gx, gz: one profile of depth into the sponge)
  int nrows;              // distinct receiver rows (rows of rmap)
  const float *wavelet;
  int zero_in;
  const float *u_in, *q_in;
  long long in_stride;
  float *u_out, *q_out;   // null: the final state is not needed
  long long out_stride;
  float *data;            // FWD/FWS: traces [pair][nt][nr]
  long long data_stride;
  float *seg;             // REC/FWS: a^n written at slot n - seg_n0; ADJ: read
  long long seg_stride;
  const float *rho;       // ADJ: residual [pair][nt][nr]
  long long rho_stride;
  double *acc64;          // ADJ: FP64 imaging sum [pair][N]; each launch adds its FP32 partial
  long long acc64_stride;
};

constexpr int kLdsBytes = 160 * 1024;
// The adjoint keeps c of each point in LDS when that still lets two blocks
// share a CU (registers are then tight), and in registers otherwise (one
// block per CU leaves registers to spare, and the LDS reads go).
template <int EX, int EZ>
constexpr bool adj_c_in_lds() {
  constexpr int U = (EZ + 4) * (EX + 4) * 4, C = EZ * EX * 4, T = 8 * EZ + 64;
  return 2 * (U + C + T) <= kLdsBytes;
}

// LDS of one block, per mode: double-buffered u; the adjoint may also keep c.
template <int MODE, int EX, int EZ, int TMAX>
struct BlockLds {
  static constexpr bool ADJ = MODE == BMODE_ADJ;
  static constexpr bool CLDS = ADJ && adj_c_in_lds<EX, EZ>();
  static constexpr int LW = EX + 4;           // 2 zero cells each side
  float u[2][EZ + 4][LW];
  float gz[EZ];                               // z damping per tile row (0 off the grid)
  int rr[EZ];                                 // receiver-row index per tile row (-1: none)
  float inj[TMAX];                            // forward / recompute: w(t_n)/(dx dz) per step
  float c[CLDS ? EZ : 1][CLDS ? EX : 1];      // adjoint: c per point
};

template <int EX, int EZ, int TMAX>
union BlockLdsAny {
  BlockLds<BMODE_FWD, EX, EZ, TMAX> fwd;
  BlockLds<BMODE_REC, EX, EZ, TMAX> rec;
  BlockLds<BMODE_ADJ, EX, EZ, TMAX> adj;
};

// Tile index of this block, contiguous ranges per XCD (blocks are dealt
// round-robin to the 8 XCDs, so neighbouring tiles share an L2).
__device__ __forceinline__ int xcd_tile() {
  const int per = int(gridDim.x) >> 3;
  const int b = int(blockIdx.x);
  return (b & 7) * per + (b >> 3);
}

// LDS bytes of one single-problem block with nbuf u buffers.
template <int MODE, int EX, int EZ>
constexpr int block_lds_bytes(int nbuf) {
  return nbuf * (EZ + 4) * (EX + 4) * 4 +
         (MODE == BMODE_ADJ && adj_c_in_lds<EX, EZ>() ? EZ * EX * 4 : 0) + 8 * EZ + 64;
}
// u buffers: two when two blocks fit in one CU's LDS that way; else one if
// that lets two blocks share a CU (one block's loads and stores then overlap
// the other's steps, at the price of a second barrier per step); else two.
// The modes that store a^n, and the adjoint with c in registers, keep two:
// with one they need more registers than two blocks leave.
template <int MODE, int EX, int EZ>
constexpr int block_nbuf() {
  return 2 * block_lds_bytes<MODE, EX, EZ>(2) <= kLdsBytes ? 2
         : MODE != BMODE_REC && MODE != BMODE_FWS &&
                   !(MODE == BMODE_ADJ && !adj_c_in_lds<EX, EZ>()) &&
                   2 * block_lds_bytes<MODE, EX, EZ>(1) <= kLdsBytes
             ? 1
             : 2;
}
// Waves per SIMD that let two blocks share a CU (1: no constraint).
template <int MODE, int EX, int EZ, int RZ>
constexpr int block_waves_per_eu() {
  return 2 * block_lds_bytes<MODE, EX, EZ>(block_nbuf<MODE, EX, EZ>()) <= kLdsBytes
             ? (2 * (EX * (EZ / RZ) / 64) + 3) / 4
             : 1;
}

template <int MODE, int EX, int EZ, int RZ, int TMAX, bool ISO>
__global__ __launch_bounds__(EX *(EZ / RZ))
__attribute__((amdgpu_waves_per_eu(block_waves_per_eu<MODE, EX, EZ, RZ>()))) void fd_block(BlockArgs a) {
  constexpr int NTHREADS = EX * (EZ / RZ);
  constexpr int H = 2 * TMAX;                 // halo width
  constexpr int IX = EX - 2 * H, IZ = EZ - 2 * H;
  constexpr int LW = EX + 4;                  // LDS row with 2 zero cells each side
  constexpr bool ADJ = MODE == BMODE_ADJ;
  constexpr int NBUF = block_nbuf<MODE, EX, EZ>();
  constexpr bool CLDS = ADJ && adj_c_in_lds<EX, EZ>();
  // one block per CU leaves registers for g of each row
  constexpr bool GREG = block_waves_per_eu<MODE, EX, EZ, RZ>() == 1;
  static_assert(IX > 0 && IZ > 0 && EZ % RZ == 0 && RZ >= 2 && RZ <= 32, "tile shape");
  __shared__ float lds[NBUF][EZ + 4][LW];
  __shared__ float gzs[EZ];     // z damping of each extended-tile row (0 outside the grid)
  __shared__ int rrs[EZ];       // receiver-row index of each extended-tile row (-1: none)
  __shared__ float injs[TMAX];  // forward / recompute: source term w(t_n)/(dx dz) of each step
  __shared__ float cs[CLDS ? EZ : 1][CLDS ? EX : 1];   // adjoint: c of each point (or registers)
  const int t = xcd_tile();
  if (t >= a.total_tiles) return;
#include "fd_block_body.inc"
}

template <int MODE, int EX, int EZ, int RZ, int TMAX, bool ISO>
__device__ __forceinline__ void fd_block_multi_body(const BlockArgs &a, const int t,
                                                    BlockLds<MODE, EX, EZ, TMAX> &sh) {
  constexpr int NTHREADS = EX * (EZ / RZ);
  constexpr int H = 2 * TMAX;                 // halo width
  constexpr int IX = EX - 2 * H, IZ = EZ - 2 * H;
  constexpr int LW = EX + 4;                  // LDS row with 2 zero cells each side
  constexpr bool ADJ = MODE == BMODE_ADJ;
  constexpr int NBUF = 2;
  constexpr bool CLDS = BlockLds<MODE, EX, EZ, TMAX>::CLDS;
  constexpr bool GREG = false;
  static_assert(IX > 0 && IZ > 0 && EZ % RZ == 0 && RZ >= 2 && RZ <= 32, "tile shape");
  auto &lds = sh.u;
  auto &gzs = sh.gz;
  auto &rrs = sh.rr;
  auto &injs = sh.inj;
  auto &cs = sh.c;
#include "fd_block_body.inc"
}

// Several independent problems (different grids, shot counts, time ranges and
// even different sweep modes) in one launch: block t belongs to the problem
// whose tile range [start[p], start[p+1]) contains it.
constexpr int kMaxMulti = 4;
struct MultiArgs {
  int nprob;
  int start[kMaxMulti + 1];
  int mode[kMaxMulti];
  BlockArgs a[kMaxMulti];
};

template <int EX, int EZ, int RZ, int TMAX>
__global__ __launch_bounds__(EX *(EZ / RZ)) void fd_block_multi(MultiArgs m) {
  __shared__ BlockLdsAny<EX, EZ, TMAX> sh;
  const int t = xcd_tile();
  if (t >= m.start[m.nprob]) return;
  int p = 0;
  while (p + 1 < m.nprob && t >= m.start[p + 1]) ++p;
  const int local = t - m.start[p];
  // the same Laplacian form as the single-problem kernel, so a problem's
  // result does not depend on the company it is launched in
  const bool iso = m.a[p].iso;
  switch (m.mode[p]) {
    case BMODE_FWD:
      if (iso) fd_block_multi_body<BMODE_FWD, EX, EZ, RZ, TMAX, true>(m.a[p], local, sh.fwd);
      else fd_block_multi_body<BMODE_FWD, EX, EZ, RZ, TMAX, false>(m.a[p], local, sh.fwd);
      break;
    case BMODE_REC:
      if (iso) fd_block_multi_body<BMODE_REC, EX, EZ, RZ, TMAX, true>(m.a[p], local, sh.rec);
      else fd_block_multi_body<BMODE_REC, EX, EZ, RZ, TMAX, false>(m.a[p], local, sh.rec);
      break;
    default:
      if (iso) fd_block_multi_body<BMODE_ADJ, EX, EZ, RZ, TMAX, true>(m.a[p], local, sh.adj);
      else fd_block_multi_body<BMODE_ADJ, EX, EZ, RZ, TMAX, false>(m.a[p], local, sh.adj);
      break;
  }
}

}  // namespace vip
