// Host-side launchers of the step kernels for one velocity set; included once
// per lattice by lattice_d2q9.hip / lattice_d3q19.hip / lattice_d3q27.hip so
// that the heavy instantiations compile in parallel.
#pragma once

#include "engine.hpp"

namespace lbm {

template <class L>
struct Launch {
  // OWN / STREAM: read mode of the phase pass and streaming mode of the
  // collision pass (step_kernels.hpp); the in-place launchers
  // (lattice_inplace.hpp) instantiate the other modes
  template <class S, bool OWN = false>
  static hipError_t phase_t(const void* fin, void* phi, const StepArgs& a, hipStream_t s) {
    using R = typename Storage<S>::real;
    // one block spans up to 256 consecutive x-sites of a row, so the cache
    // lines the +-1 pulls share between neighbouring waves stay in one CU
    const int bx = a.nx >= 192 ? 256 : (a.nx >= 96 ? 128 : 64);
    dim3 block(bx, 256 / bx, 1);
    StepArgs b = a;
    b.tiles_x = (a.nx + bx - 1) / bx;
    b.tiles_y = (a.ny + block.y - 1) / block.y;
    dim3 grid((unsigned)b.tiles_x * b.tiles_y * a.nz);
    k_phase<L, S, OWN><<<grid, block, 0, s>>>((const S*)fin, (R*)phi, b);
    return hipGetLastError();
  }

  template <class S, bool OWN = false>
  static hipError_t phase_total_t(const void* fin, const float* scin, void* phi, const StepArgs& a,
                                  hipStream_t s) {
    using TS = Tile<TILE_X, TILE_Y, 1, L::D>;
    dim3 block(TS::TX, TS::TY, 1);
    const int zb = a.z_per_block;
    StepArgs b = a;
    b.tiles_x = (a.nx + TS::TX - 1) / TS::TX;
    b.tiles_y = (a.ny + TS::TY - 1) / TS::TY;
    dim3 grid((unsigned)b.tiles_x * b.tiles_y * ((a.nz + zb - 1) / zb));
    k_phase_total<L, S, TS, OWN><<<grid, block, 0, s>>>((const S*)fin, scin, (float*)phi, b);
    return hipGetLastError();
  }

  static hipError_t phase(int st, const void* fin, const float* scin, void* phi, const StepArgs& a,
                          hipStream_t s) {
    switch (st) {
      case ST_F64: return phase_t<double>(fin, phi, a, s);
      case ST_F32: return phase_t<float>(fin, phi, a, s);
      case ST_F16: return phase_t<_Float16>(fin, phi, a, s);
      case ST_BF16: return phase_t<__bf16>(fin, phi, a, s);
      case ST_F32S: return phase_t<F32S>(fin, phi, a, s);
      case ST_F32T: return phase_total_t<float>(fin, scin, phi, a, s);
      case ST_F16T: return phase_total_t<_Float16>(fin, scin, phi, a, s);
      case ST_BF16T: return phase_total_t<__bf16>(fin, scin, phi, a, s);
      case ST_F16CT: return phase_total_t<F16C>(fin, scin, phi, a, s);
    }
    return hipErrorInvalidValue;
  }

  template <class S, int RAD, bool NC, bool FIELDS, bool TOT, int STREAM = STREAM_AB, bool SR = false>
  static hipError_t collide_t(const void* fin, void* fout, float* scout, const void* phi,
                              const FieldPtrs& fo, const StepArgs& a, hipStream_t s) {
    using R = typename Storage<S>::real;
    using T = Tile<TILE_X, TILE_Y, RAD, L::D>;
    dim3 block(T::TX, T::TY, 1);
    StepArgs b = a;
    b.tiles_x = (a.nx + T::TX - 1) / T::TX;
    b.tiles_y = (a.ny + T::TY - 1) / T::TY;
    int zb = a.z_per_block;
    // two-copy 4-byte per-colour layouts: when the grid is small (at most
    // 1024 workgroups), marches twice as long halve it so that it runs in a
    // single round instead of a full round and a partial one.  Measured on
    // the 256 x 128 x 128 channel: 399 -> 384 us for the FP32 pass; on grids
    // of several thousand workgroups longer marches were 1-2% slower, and
    // the in-place, FP64 and total-layout passes did not gain
    if constexpr (!TOT && sizeof(S) == 4 && STREAM == STREAM_AB) {
      const long g = (long)b.tiles_x * b.tiles_y * ((a.nz + zb - 1) / zb);
      if (g <= 1024 && 2 * zb <= a.nz) zb *= 2;
    }
    b.z_per_block = zb;
    dim3 grid((unsigned)b.tiles_x * b.tiles_y * ((a.nz + zb - 1) / zb));
    k_collide<L, S, T, NC, FIELDS, TOT, STREAM, SR><<<grid, block, 0, s>>>((const S*)fin, (S*)fout, (const R*)phi, scout, fo, b);
    return hipGetLastError();
  }

  template <class S, bool TOT, int STREAM = STREAM_AB, bool SR = false>
  static hipError_t collide_n(bool nc, bool fields, const void* fin, void* fout, float* scout,
                              const void* phi, const FieldPtrs& fo, const StepArgs& a, hipStream_t s) {
    if (nc) {
      return fields ? collide_t<S, 4, true, true, TOT, STREAM, SR>(fin, fout, scout, phi, fo, a, s)
                    : collide_t<S, 4, true, false, TOT, STREAM, SR>(fin, fout, scout, phi, fo, a, s);
    }
    return fields ? collide_t<S, 1, false, true, TOT, STREAM, SR>(fin, fout, scout, phi, fo, a, s)
                  : collide_t<S, 1, false, false, TOT, STREAM, SR>(fin, fout, scout, phi, fo, a, s);
  }
  // the stochastic-rounding kernels exist for the FP16 and BF16 totals only
  template <class S, bool TOT, int STREAM = STREAM_AB>
  static hipError_t collide_s(bool nc, bool fields, const void* fin, void* fout, float* scout,
                              const void* phi, const FieldPtrs& fo, const StepArgs& a, hipStream_t s) {
    if constexpr (TOT && sizeof(S) == 2 && !std::is_same_v<S, F16C>) {
      if (a.sround) return collide_n<S, TOT, STREAM, true>(nc, fields, fin, fout, scout, phi, fo, a, s);
    }
    return collide_n<S, TOT, STREAM, false>(nc, fields, fin, fout, scout, phi, fo, a, s);
  }

  static hipError_t collide(int st, bool nc, bool fields, const void* fin, void* fout, float* scout, const void* phi,
                            const FieldPtrs& fo, const StepArgs& a, hipStream_t s) {
    switch (st) {
      case ST_F64: return collide_s<double, false>(nc, fields, fin, fout, scout, phi, fo, a, s);
      case ST_F32: return collide_s<float, false>(nc, fields, fin, fout, scout, phi, fo, a, s);
      case ST_F16: return collide_s<_Float16, false>(nc, fields, fin, fout, scout, phi, fo, a, s);
      case ST_BF16: return collide_s<__bf16, false>(nc, fields, fin, fout, scout, phi, fo, a, s);
      case ST_F32S: return collide_s<F32S, false>(nc, fields, fin, fout, scout, phi, fo, a, s);
      case ST_F32T: return collide_s<float, true>(nc, fields, fin, fout, scout, phi, fo, a, s);
      case ST_F16T: return collide_s<_Float16, true>(nc, fields, fin, fout, scout, phi, fo, a, s);
      case ST_BF16T: return collide_s<__bf16, true>(nc, fields, fin, fout, scout, phi, fo, a, s);
      case ST_F16CT: return collide_s<F16C, true>(nc, fields, fin, fout, scout, phi, fo, a, s);
    }
    return hipErrorInvalidValue;
  }

  // collision pass with the learned near-contact closure (3D lattices)
  template <class S, bool FIELDS, bool TOT, int STREAM = STREAM_AB>
  static hipError_t collide_mlp_t(const void* fin, void* fout, float* scout, const void* phi,
                                  const FieldPtrs& fo, const StepArgs& a, const MlpPacked* net, hipStream_t s) {
    using R = typename Storage<S>::real;
    // radius-1 phase ring: the network needs the 3x3x3 neighbourhood; the
    // explicit scan for sites outside its range reads the phase field from memory
    using T = Tile<TILE_X, TILE_Y, 1, L::D>;
    dim3 block(T::TX, T::TY, 1);
    // half the planes per workgroup of the other passes: this pass holds the
    // network and its row queues in LDS and runs three workgroups per CU,
    // and measured faster with twice as many, shorter marches
    const int zb = a.z_per_block > 1 ? a.z_per_block / 2 : 1;
    StepArgs b = a;
    b.z_per_block = zb;
    b.tiles_x = (a.nx + T::TX - 1) / T::TX;
    b.tiles_y = (a.ny + T::TY - 1) / T::TY;
    dim3 grid((unsigned)b.tiles_x * b.tiles_y * ((a.nz + zb - 1) / zb));
    k_collide_mlp<L, S, T, FIELDS, TOT, STREAM><<<grid, block, 0, s>>>((const S*)fin, (S*)fout, (const R*)phi, scout, fo, b,
                                                               net);
    return hipGetLastError();
  }

  static hipError_t collide_mlp(int st, bool fields, const void* fin, void* fout, float* scout, const void* phi,
                                const FieldPtrs& fo, const StepArgs& a, const MlpPacked* net, hipStream_t s) {
    if constexpr (L::D == 3) {
#define LB_MLP_CASE(ST, TYPE, TOT)                                                          \
  case ST:                                                                                  \
    return fields ? collide_mlp_t<TYPE, true, TOT>(fin, fout, scout, phi, fo, a, net, s) \
                  : collide_mlp_t<TYPE, false, TOT>(fin, fout, scout, phi, fo, a, net, s);
      switch (st) {
        LB_MLP_CASE(ST_F64, double, false)
        LB_MLP_CASE(ST_F32, float, false)
        LB_MLP_CASE(ST_F32T, float, true)
        LB_MLP_CASE(ST_F16T, _Float16, true)
        LB_MLP_CASE(ST_BF16T, __bf16, true)
        LB_MLP_CASE(ST_F16CT, F16C, true)
      }
#undef LB_MLP_CASE
    }
    return hipErrorInvalidValue;
  }

  template <class S>
  static hipError_t init_t(void* f, void* phi, const FieldPtrs& fo, const double* drops, const InitArgs& a,
                           hipStream_t s) {
    using R = typename Storage<S>::real;
    dim3 block(256);
    dim3 grid((a.N + 255) / 256);
    k_init<L, S><<<grid, block, 0, s>>>((S*)f, (R*)phi, fo, drops, a);
    return hipGetLastError();
  }

  template <class S>
  static hipError_t init_total_t(void* f, float* sc, void* phi, const FieldPtrs& fo, const double* drops,
                                 const InitArgs& a, hipStream_t s) {
    dim3 block(256);
    dim3 grid((a.N + 255) / 256);
    k_init_total<L, S><<<grid, block, 0, s>>>((S*)f, sc, (float*)phi, fo, drops, a);
    return hipGetLastError();
  }

  static hipError_t init(int st, void* f, float* sc, void* phi, const FieldPtrs& fo, const double* drops,
                         const InitArgs& a, hipStream_t s) {
    switch (st) {
      case ST_F64: return init_t<double>(f, phi, fo, drops, a, s);
      case ST_F32: return init_t<float>(f, phi, fo, drops, a, s);
      case ST_F16: return init_t<_Float16>(f, phi, fo, drops, a, s);
      case ST_BF16: return init_t<__bf16>(f, phi, fo, drops, a, s);
      case ST_F32S: return init_t<F32S>(f, phi, fo, drops, a, s);
      case ST_F32T: return init_total_t<float>(f, sc, phi, fo, drops, a, s);
      case ST_F16T: return init_total_t<_Float16>(f, sc, phi, fo, drops, a, s);
      case ST_BF16T: return init_total_t<__bf16>(f, sc, phi, fo, drops, a, s);
      case ST_F16CT: return init_total_t<F16C>(f, sc, phi, fo, drops, a, s);
    }
    return hipErrorInvalidValue;
  }

  template <class S, bool NC, bool FIELDS, bool TOT>
  static auto ens_kernel() {
    using T = Tile<TILE_X, TILE_Y, NC ? 4 : 1, L::D>;
    return &k_ensemble<L, S, T, NC, FIELDS, TOT>;
  }

  template <class S, bool TOT>
  static hipError_t ensemble_s(bool nc, bool fields, bool phase_only, const ChannelDev* chans, const uint32_t* items,
                               uint32_t nitems, int parity, hipStream_t s) {
    dim3 block(TILE_X, TILE_Y, 1), grid(nitems);
    if (phase_only) {
      using TS = Tile<TILE_X, TILE_Y, 1, L::D>;
      k_ensemble_phase<L, S, TS, TOT><<<grid, block, 0, s>>>(chans, items, parity);
      return hipGetLastError();
    }
    if (nc) {
      if (fields) ens_kernel<S, true, true, TOT>()<<<grid, block, 0, s>>>(chans, items, parity);
      else ens_kernel<S, true, false, TOT>()<<<grid, block, 0, s>>>(chans, items, parity);
    } else {
      if (fields) ens_kernel<S, false, true, TOT>()<<<grid, block, 0, s>>>(chans, items, parity);
      else ens_kernel<S, false, false, TOT>()<<<grid, block, 0, s>>>(chans, items, parity);
    }
    return hipGetLastError();
  }

  static hipError_t ensemble(int st, bool nc, bool fields, bool phase_only, const ChannelDev* chans,
                             const uint32_t* items, uint32_t nitems, int parity, hipStream_t s) {
    if (nitems == 0) return hipSuccess;
    switch (st) {
      case ST_F64: return ensemble_s<double, false>(nc, fields, phase_only, chans, items, nitems, parity, s);
      case ST_F32: return ensemble_s<float, false>(nc, fields, phase_only, chans, items, nitems, parity, s);
      case ST_F32T: return ensemble_s<float, true>(nc, fields, phase_only, chans, items, nitems, parity, s);
      case ST_F16T: return ensemble_s<_Float16, true>(nc, fields, phase_only, chans, items, nitems, parity, s);
      case ST_BF16T: return ensemble_s<__bf16, true>(nc, fields, phase_only, chans, items, nitems, parity, s);
      case ST_F16CT: return ensemble_s<F16C, true>(nc, fields, phase_only, chans, items, nitems, parity, s);
    }
    return hipErrorInvalidValue;
  }

  static LatticeOps ops() {
    return LatticeOps{L::Q, L::D, &phase, &collide, &init, &ensemble, L::D == 3 ? &collide_mlp : nullptr};
  }
};

}  // namespace lbm
