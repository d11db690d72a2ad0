// Host-side launchers of the moment-based (regularised) step for one velocity
// set; included by lattice_*_llb.hip.
#pragma once

#include "engine.hpp"
#include "llb_kernels.hpp"

namespace lbm {

template <class L>
struct LlbLaunch {
  template <class S>
  static hipError_t init_t(void* M, void* phi, const FieldPtrs& fo, const double* drops, const InitArgs& a,
                           hipStream_t s) {
    dim3 block(256), grid((a.N + 255) / 256);
    k_llb_init<L, S><<<grid, block, 0, s>>>((S*)M, (S*)phi, fo, drops, a);
    return hipGetLastError();
  }
  static hipError_t init(int st, void* M, void* phi, const FieldPtrs& fo, const double* drops, const InitArgs& a,
                         hipStream_t s) {
    if (st == ST_F64) return init_t<double>(M, phi, fo, drops, a, s);
    if (st == ST_F32) return init_t<float>(M, phi, fo, drops, a, s);
    return hipErrorInvalidValue;
  }

  template <class S>
  static hipError_t pull_t(const void* M, void* W, void* phi, const StepArgs& a, hipStream_t s) {
    // one block spans up to 256 consecutive x-sites of a row (as the phase pass)
    const int bx = a.nx >= 192 ? 256 : (a.nx >= 96 ? 128 : 64);
    dim3 block(bx, 256 / bx, 1);
    StepArgs b = a;
    b.tiles_x = (a.nx + bx - 1) / bx;
    b.tiles_y = (a.ny + block.y - 1) / block.y;
    dim3 grid((unsigned)b.tiles_x * b.tiles_y * a.nz);
    k_llb_pull<L, S><<<grid, block, 0, s>>>((const S*)M, (S*)W, (S*)phi, b);
    return hipGetLastError();
  }
  // FP32: the moments of a tile plus halo staged in an LDS ring (15 channels,
  // about 95 KB for a 3D 64 x 4 tile); FP64 would not fit and reads memory
  static hipError_t pull_ring(const void* M, void* W, void* phi, const StepArgs& a, hipStream_t s) {
    using TS = Tile<TILE_X, TILE_Y, 1, L::D>;
    dim3 block(TS::TX, TS::TY, 1);
    const int zb = a.z_per_block;
    StepArgs b = a;
    b.tiles_x = (a.nx + TS::TX - 1) / TS::TX;
    b.tiles_y = (a.ny + TS::TY - 1) / TS::TY;
    dim3 grid((unsigned)b.tiles_x * b.tiles_y * ((a.nz + zb - 1) / zb));
    k_llb_pull_ring<L, TS><<<grid, block, 0, s>>>((const float*)M, (float*)W, (float*)phi, b);
    return hipGetLastError();
  }
  static hipError_t pull(int st, const void* M, void* W, void* phi, const StepArgs& a, hipStream_t s) {
    if (st == ST_F64) return pull_t<double>(M, W, phi, a, s);
    if (st == ST_F32) return pull_ring(M, W, phi, a, s);
    return hipErrorInvalidValue;
  }

  template <class S, int RAD, bool NC, bool FIELDS>
  static hipError_t collide_t(const void* W, void* M, const void* phi, const FieldPtrs& fo, const StepArgs& a,
                              hipStream_t s) {
    using T = Tile<TILE_X, TILE_Y, RAD, L::D>;
    dim3 block(T::TX, T::TY, 1);
    const int zb = a.z_per_block;
    StepArgs b = a;
    b.tiles_x = (a.nx + T::TX - 1) / T::TX;
    b.tiles_y = (a.ny + T::TY - 1) / T::TY;
    dim3 grid((unsigned)b.tiles_x * b.tiles_y * ((a.nz + zb - 1) / zb));
    k_llb_collide<L, S, T, NC, FIELDS><<<grid, block, 0, s>>>((const S*)W, (S*)M, (const S*)phi, fo, b);
    return hipGetLastError();
  }
  template <class S>
  static hipError_t collide_s(bool nc, bool fields, const void* W, void* M, const void* phi, const FieldPtrs& fo,
                              const StepArgs& a, hipStream_t s) {
    if (nc)
      return fields ? collide_t<S, 4, true, true>(W, M, phi, fo, a, s) : collide_t<S, 4, true, false>(W, M, phi, fo, a, s);
    return fields ? collide_t<S, 1, false, true>(W, M, phi, fo, a, s) : collide_t<S, 1, false, false>(W, M, phi, fo, a, s);
  }
  static hipError_t collide(int st, bool nc, bool fields, const void* W, void* M, const void* phi,
                            const FieldPtrs& fo, const StepArgs& a, hipStream_t s) {
    if (st == ST_F64) return collide_s<double>(nc, fields, W, M, phi, fo, a, s);
    if (st == ST_F32) return collide_s<float>(nc, fields, W, M, phi, fo, a, s);
    return hipErrorInvalidValue;
  }

  static LlbOps ops() { return LlbOps{&init, &pull, &collide}; }
};

}  // namespace lbm
