// Batched ensembles: many independent lattices ("channels", each with its
// own size, walls, tau, forces and droplets) advanced together.
//
// A step is two batched launches over a flat list of tile items, first every
// channel's phase tiles, then every channel's collision tiles (each a TX x TY
// column over a block of z-planes).  Workgroup b processes item b; the item
// names the channel and the tile.  The launch boundary between the two
// passes orders them and makes every channel's phase field visible, exactly
// as in the single-lattice step, so a workgroup runs the same tile code as
// the single-lattice kernels and never waits on another one.  Channel-table
// values are made wave-uniform explicitly so that buffer descriptors stay in
// scalar registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "step_kernels.hpp"

namespace lbm {

struct ChannelDev {
  StepArgs a;        // per-channel constants; tiles_x/tiles_y/z_per_block of the ensemble tiling
  void* f[2];        // population copies (ping-pong)
  float* sc[2];      // recolouring scalars (total layout)
  void* phi;
  FieldPtrs fo;
  uint32_t ntiles;   // phase tiles (= collision tiles) of this channel
  uint32_t pad;
  // read-once step: phase field buffers (phis[p] is read by the collision
  // pass of a step of parity p, phis[1 - p] written by its combine pass), the
  // partial densities and the halo blocks
  void* phis[2];
  void* part;
  void* halo;
};

// item encoding: bit 31 = collision tile, bits 20..30 = channel, bits 0..19 = tile
constexpr uint32_t ITEM_COLLIDE = 1u << 31;
constexpr int ITEM_CH_SHIFT = 20;
constexpr uint32_t ITEM_TILE_MASK = (1u << ITEM_CH_SHIFT) - 1;
constexpr uint32_t ITEM_CH_MASK = 0x7FFu;

template <class P>
__device__ __forceinline__ P* uniform_ptr(P* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (P*)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ StepArgs uniform_args(const StepArgs& in) {
  // copy word by word through readfirstlane: every field is the same for the
  // whole workgroup
  StepArgs out;
  static_assert(sizeof(StepArgs) % 4 == 0, "StepArgs must be a whole number of words");
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&in);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(StepArgs) / 4); ++k) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
  return out;
}

// one tile item per workgroup; `items` holds only phase items or only
// collision items
// LDS of an ensemble workgroup: a collision tile or a total-layout phase tile
template <class L, class S, class T, bool TOT>
union EnsembleSmem {
  CollideSmem<L, S, T, TOT> c;
  PhaseTotalSmem<Tile<T::TX, T::TY, 1, L::D>> p;
};

// phase items only: the phase pass's registers and LDS, not those of the
// collision tile it shares k_ensemble with
template <class L, class S, class TS, bool TOT>
__global__ void __launch_bounds__(TS::NT) k_ensemble_phase(const ChannelDev* __restrict__ chans,
                                                           const uint32_t* __restrict__ items, int parity) {
  using R = typename Storage<S>::real;
  const uint32_t e = __builtin_amdgcn_readfirstlane(items[xcd_range_index(blockIdx.x, gridDim.x)]);
  const uint32_t c = (e >> ITEM_CH_SHIFT) & ITEM_CH_MASK;
  const ChannelDev* C = chans + c;
  const StepArgs a = uniform_args(C->a);
  const TileCoord tc = tile_coord(e & ITEM_TILE_MASK, a, TS::TX, TS::TY);
  const S* fin = uniform_ptr((const S*)C->f[parity]);
  void* phi = uniform_ptr(C->phi);
  if constexpr (TOT) {
    __shared__ PhaseTotalSmem<TS> sm;
    const float* scin = uniform_ptr((const float*)C->sc[parity]);
    phase_total_tile<L, S, TS>(fin, scin, (float*)phi, a, tc, sm);
  } else {
    phase_tile<L, S>(fin, (R*)phi, a, tc, TS::TX);
  }
}

template <class L, class S, class T, bool NC, bool FIELDS, bool TOT>
__global__ void __launch_bounds__(T::NT) k_ensemble(const ChannelDev* __restrict__ chans,
                                                     const uint32_t* __restrict__ items, int parity) {
  using R = typename Storage<S>::real;
  using TS = Tile<T::TX, T::TY, 1, L::D>;
  __shared__ EnsembleSmem<L, S, T, TOT> sm;
  // consecutive items (x-neighbour tiles of one channel) go to one XCD
  const uint32_t e = __builtin_amdgcn_readfirstlane(items[xcd_range_index(blockIdx.x, gridDim.x)]);
  const uint32_t c = (e >> ITEM_CH_SHIFT) & ITEM_CH_MASK;
  const ChannelDev* C = chans + c;
  const StepArgs a = uniform_args(C->a);
  const TileCoord tc = tile_coord(e & ITEM_TILE_MASK, a, T::TX, T::TY);
  const S* fin = uniform_ptr((const S*)C->f[parity]);
  S* fout = uniform_ptr((S*)C->f[1 - parity]);
  const float* scin = uniform_ptr((const float*)C->sc[parity]);
  float* scout = uniform_ptr(C->sc[1 - parity]);
  void* phi = uniform_ptr(C->phi);
  if (!(e & ITEM_COLLIDE)) {
    if constexpr (TOT) {
      phase_total_tile<L, S, TS>(fin, scin, (float*)phi, a, tc, sm.p);
    } else {
      phase_tile<L, S>(fin, (R*)phi, a, tc, T::TX);
    }
  } else {
    FieldPtrs fo;
    fo.rho_a = uniform_ptr(C->fo.rho_a);
    fo.rho_b = uniform_ptr(C->fo.rho_b);
    fo.u = uniform_ptr(C->fo.u);
    fo.fnc = uniform_ptr(C->fo.fnc);
    fo.flags = uniform_ptr(C->fo.flags);
    collide_tile<L, S, T, NC, FIELDS, TOT>(fin, fout, (const R*)phi, scout, fo, a, tc, sm.c);
  }
}

// Read-once ensemble step, first launch: every channel's collision tiles with
// the read-once scatter (one tile-march per workgroup; the item names the
// channel and the tile-march, as for the two-pass collision).
template <class L, class S, class T, bool NC, bool FIELDS, bool TOT, int SCP = CPOL_NT>
__global__ void __launch_bounds__(T::NT, (collide_min_waves<S, TOT, true>()))
    k_ensemble_ro(const ChannelDev* __restrict__ chans, const uint32_t* __restrict__ items, int parity) {
  using R = typename Storage<S>::real;
  __shared__ CollideSmem<L, S, T, TOT, false, true> sm;
  const uint32_t e = __builtin_amdgcn_readfirstlane(items[xcd_range_index(blockIdx.x, gridDim.x)]);
  const uint32_t c = (e >> ITEM_CH_SHIFT) & ITEM_CH_MASK;
  const ChannelDev* C = chans + c;
  const StepArgs a = uniform_args(C->a);
  const TileCoord tc = tile_coord(e & ITEM_TILE_MASK, a, T::TX, T::TY);
  const S* fin = uniform_ptr((const S*)C->f[parity]);
  S* fout = uniform_ptr((S*)C->f[1 - parity]);
  float* scout = uniform_ptr(C->sc[1 - parity]);
  const R* phi = uniform_ptr((const R*)C->phis[parity]);
  FieldPtrs fo;
  fo.rho_a = uniform_ptr(C->fo.rho_a);
  fo.rho_b = uniform_ptr(C->fo.rho_b);
  fo.u = uniform_ptr(C->fo.u);
  fo.fnc = uniform_ptr(C->fo.fnc);
  fo.flags = uniform_ptr(C->fo.flags);
  const ScatterOut so{uniform_ptr(C->part), uniform_ptr(C->halo)};
  collide_tile<L, S, T, NC, FIELDS, TOT, false, STREAM_AB, false, true, false, SCP>(fin, fout, phi, scout, fo, a, tc,
                                                                                    sm, nullptr, so);
}

// Read-once ensemble step, second launch: every channel's combine blocks.
// Item index: ((tm G + j) tiles_y + ty) tiles_x + tx with G = ceil(march
// depth / COMBINE_PLANES), the channel's own tiling.
template <class L, class R, int TX, int TY, bool SHIFTED>
__global__ void __launch_bounds__(TX * TY)
    k_ensemble_combine(const ChannelDev* __restrict__ chans, const uint32_t* __restrict__ items, int parity) {
  const uint32_t e = __builtin_amdgcn_readfirstlane(items[xcd_range_index(blockIdx.x, gridDim.x)]);
  const uint32_t c = (e >> ITEM_CH_SHIFT) & ITEM_CH_MASK;
  const ChannelDev* C = chans + c;
  const StepArgs a = uniform_args(C->a);
  const uint32_t idx = e & ITEM_TILE_MASK;
  const int G = (a.z_per_block + COMBINE_PLANES - 1) / COMBINE_PLANES;
  const uint32_t txy = (uint32_t)a.tiles_x * a.tiles_y;
  const int zg = idx / txy;
  const uint32_t r = idx - (uint32_t)zg * txy;
  const int ty = r / a.tiles_x, tx = r - ty * a.tiles_x;
  const int tm = zg / G, j = zg - tm * G;
  combine_block<L, R, TX, TY, SHIFTED>(uniform_ptr((const R*)C->part), uniform_ptr((const RPair<R>*)C->halo),
                                               uniform_ptr((R*)C->phis[1 - parity]), a, tx, ty, tm, j);
}

}  // namespace lbm
