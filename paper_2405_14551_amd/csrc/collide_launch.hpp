// Host-side launchers of the collision pass for one velocity set, streaming
// mode and read-once setting.  Each lattice_*_collide_*.hip file includes
// this header and instantiates collide_impl / collide_mlp_impl for one
// (lattice, streaming, read-once) combination, so that the heavy kernel
// instantiations compile in parallel.
#pragma once

#include "lattice_ops.hpp"

namespace lbm {

template <class L, int STREAM, bool RO>
struct CollideLaunch {
  template <class S, int RAD, bool NC, bool FIELDS, bool TOT, bool SR>
  static hipError_t collide_t(const void* fin, void* fout, float* scout, const void* phi,
                              const FieldPtrs& fo, const StepArgs& a, const ScatterOut* ro, hipStream_t s) {
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
    // the in-place, FP64 and total-layout passes did not gain.  (The
    // read-once launch takes the depth its caller chose.)
    if constexpr (!RO && !TOT && sizeof(S) == 4 && STREAM == STREAM_AB) {
      const long g = (long)b.tiles_x * b.tiles_y * ((a.nz + zb - 1) / zb);
      if (g <= 1024 && 2 * zb <= a.nz) zb *= 2;
    }
    b.z_per_block = zb;
    dim3 grid((unsigned)b.tiles_x * b.tiles_y * ((a.nz + zb - 1) / zb));
    if constexpr (RO) {
      if (!ro) return hipErrorInvalidValue;
      k_collide<L, S, T, NC, FIELDS, TOT, STREAM, SR, true><<<grid, block, 0, s>>>((const S*)fin, (S*)fout,
                                                                                 (const R*)phi, scout, fo, b, *ro);
    } else {
      k_collide<L, S, T, NC, FIELDS, TOT, STREAM, SR, false><<<grid, block, 0, s>>>(
          (const S*)fin, (S*)fout, (const R*)phi, scout, fo, b, ScatterOut{nullptr, nullptr});
    }
    return hipGetLastError();
  }

  template <class S, bool TOT, bool SR>
  static hipError_t collide_n(bool nc, bool fields, const void* fin, void* fout, float* scout, const void* phi,
                              const FieldPtrs& fo, const StepArgs& a, const ScatterOut* ro, hipStream_t s) {
    if (nc) {
      return fields ? collide_t<S, 4, true, true, TOT, SR>(fin, fout, scout, phi, fo, a, ro, s)
                    : collide_t<S, 4, true, false, TOT, SR>(fin, fout, scout, phi, fo, a, ro, s);
    }
    return fields ? collide_t<S, 1, false, true, TOT, SR>(fin, fout, scout, phi, fo, a, ro, s)
                  : collide_t<S, 1, false, false, TOT, SR>(fin, fout, scout, phi, fo, a, ro, s);
  }

  // the stochastic-rounding kernels exist for the FP16 and BF16 totals only
  template <class S, bool TOT>
  static hipError_t collide_s(bool nc, bool fields, const void* fin, void* fout, float* scout, const void* phi,
                              const FieldPtrs& fo, const StepArgs& a, const ScatterOut* ro, hipStream_t s) {
    if constexpr (TOT && sizeof(S) == 2 && !std::is_same_v<S, F16C>) {
      if (a.sround) return collide_n<S, TOT, true>(nc, fields, fin, fout, scout, phi, fo, a, ro, s);
    }
    return collide_n<S, TOT, false>(nc, fields, fin, fout, scout, phi, fo, a, ro, s);
  }

  static hipError_t collide(int st, bool nc, bool fields, const void* fin, void* fout, float* scout, const void* phi,
                            const FieldPtrs& fo, const StepArgs& a, const ScatterOut* ro, hipStream_t s) {
    switch (st) {
      case ST_F64: return collide_s<double, false>(nc, fields, fin, fout, scout, phi, fo, a, ro, s);
      case ST_F32: return collide_s<float, false>(nc, fields, fin, fout, scout, phi, fo, a, ro, s);
      case ST_F16: return collide_s<_Float16, false>(nc, fields, fin, fout, scout, phi, fo, a, ro, s);
      case ST_BF16: return collide_s<__bf16, false>(nc, fields, fin, fout, scout, phi, fo, a, ro, s);
      case ST_F32S: return collide_s<F32S, false>(nc, fields, fin, fout, scout, phi, fo, a, ro, s);
      case ST_F32T: return collide_s<float, true>(nc, fields, fin, fout, scout, phi, fo, a, ro, s);
      case ST_F16T: return collide_s<_Float16, true>(nc, fields, fin, fout, scout, phi, fo, a, ro, s);
      case ST_BF16T: return collide_s<__bf16, true>(nc, fields, fin, fout, scout, phi, fo, a, ro, s);
      case ST_F16CT: return collide_s<F16C, true>(nc, fields, fin, fout, scout, phi, fo, a, ro, s);
    }
    return hipErrorInvalidValue;
  }

  // collision pass with the learned near-contact closure (3D lattices).
  // Without ro it marches half the planes of the other passes: it holds the
  // network and its row queues in LDS and measured faster with twice as
  // many, shorter marches.  With ro it takes the caller's depth (the one the
  // halo blocks are sized for).
  template <class S, bool FIELDS, bool TOT>
  static hipError_t collide_mlp_t(const void* fin, void* fout, float* scout, const void* phi, const FieldPtrs& fo,
                                  const StepArgs& a, const MlpPacked* net, const ScatterOut* ro, hipStream_t s) {
    using R = typename Storage<S>::real;
    // radius-1 phase ring: the network needs the 3x3x3 neighbourhood; the
    // explicit scan for sites outside its range reads the phase field from memory
    using T = Tile<TILE_X, TILE_Y, 1, L::D>;
    dim3 block(T::TX, T::TY, 1);
    const int zb = RO ? a.z_per_block : (a.z_per_block > 1 ? a.z_per_block / 2 : 1);
    StepArgs b = a;
    b.z_per_block = zb;
    b.tiles_x = (a.nx + T::TX - 1) / T::TX;
    b.tiles_y = (a.ny + T::TY - 1) / T::TY;
    dim3 grid((unsigned)b.tiles_x * b.tiles_y * ((a.nz + zb - 1) / zb));
    if constexpr (RO) {
      if (!ro) return hipErrorInvalidValue;
      k_collide_mlp<L, S, T, FIELDS, TOT, STREAM, true><<<grid, block, 0, s>>>((const S*)fin, (S*)fout, (const R*)phi,
                                                                              scout, fo, b, net, *ro);
    } else {
      k_collide_mlp<L, S, T, FIELDS, TOT, STREAM, false><<<grid, block, 0, s>>>(
          (const S*)fin, (S*)fout, (const R*)phi, scout, fo, b, net, ScatterOut{nullptr, nullptr});
    }
    return hipGetLastError();
  }

  static hipError_t collide_mlp(int st, bool fields, const void* fin, void* fout, float* scout, const void* phi,
                                const FieldPtrs& fo, const StepArgs& a, const MlpPacked* net, const ScatterOut* ro,
                                hipStream_t s) {
    if constexpr (L::D == 3) {
#define LB_MLP_CASE(ST, TYPE, TOT)                                                            \
  case ST:                                                                                    \
    return fields ? collide_mlp_t<TYPE, true, TOT>(fin, fout, scout, phi, fo, a, net, ro, s) \
                  : collide_mlp_t<TYPE, false, TOT>(fin, fout, scout, phi, fo, a, net, ro, s);
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
};

// read-once batched ensemble launches (two-copy streaming)
template <class L>
struct EnsembleRoLaunch {
  template <class S, bool TOT, int SCP = CPOL_NT>
  static hipError_t run_s(bool nc, bool fields, bool combine, const ChannelDev* chans, const uint32_t* items,
                          uint32_t nitems, int parity, hipStream_t s) {
    using R = typename Storage<S>::real;
    dim3 block(TILE_X, TILE_Y, 1), grid(nitems);
    if (combine) {
      // per-colour FP64 / FP32 scatter the stored populations themselves
      constexpr bool SHIFTED = !(std::is_same_v<S, double> || (std::is_same_v<S, float> && !TOT));
      k_ensemble_combine<L, R, TILE_X, TILE_Y, SHIFTED><<<grid, block, 0, s>>>(chans, items, parity);
      return hipGetLastError();
    }
    if (nc) {
      using T = Tile<TILE_X, TILE_Y, 4, L::D>;
      if (fields) k_ensemble_ro<L, S, T, true, true, TOT, SCP><<<grid, block, 0, s>>>(chans, items, parity);
      else k_ensemble_ro<L, S, T, true, false, TOT, SCP><<<grid, block, 0, s>>>(chans, items, parity);
    } else {
      using T = Tile<TILE_X, TILE_Y, 1, L::D>;
      if (fields) k_ensemble_ro<L, S, T, false, true, TOT, SCP><<<grid, block, 0, s>>>(chans, items, parity);
      else k_ensemble_ro<L, S, T, false, false, TOT, SCP><<<grid, block, 0, s>>>(chans, items, parity);
    }
    return hipGetLastError();
  }
  static hipError_t run(int st, bool nc, bool fields, bool combine, bool cached, const ChannelDev* chans,
                        const uint32_t* items, uint32_t nitems, int parity, hipStream_t s) {
    // cached stores for the 4- and 8-byte storages (16-bit ensembles take the
    // two-pass step unless asked otherwise)
    if (cached && !combine) {
      switch (st) {
        case ST_F64: return run_s<double, false, 0>(nc, fields, combine, chans, items, nitems, parity, s);
        case ST_F32: return run_s<float, false, 0>(nc, fields, combine, chans, items, nitems, parity, s);
        case ST_F32T: return run_s<float, true, 0>(nc, fields, combine, chans, items, nitems, parity, s);
      }
    }
    switch (st) {
      case ST_F64: return run_s<double, false>(nc, fields, combine, chans, items, nitems, parity, s);
      case ST_F32: return run_s<float, false>(nc, fields, combine, chans, items, nitems, parity, s);
      case ST_F32T: return run_s<float, true>(nc, fields, combine, chans, items, nitems, parity, s);
      case ST_F16T: return run_s<_Float16, true>(nc, fields, combine, chans, items, nitems, parity, s);
      case ST_BF16T: return run_s<__bf16, true>(nc, fields, combine, chans, items, nitems, parity, s);
      case ST_F16CT: return run_s<F16C, true>(nc, fields, combine, chans, items, nitems, parity, s);
    }
    return hipErrorInvalidValue;
  }
};

template <class L>
hipError_t ensemble_ro_impl(int st, bool nc, bool fields, bool combine, bool cached, const ChannelDev* chans,
                            const uint32_t* items, uint32_t nitems, int parity, hipStream_t s) {
  return EnsembleRoLaunch<L>::run(st, nc, fields, combine, cached, chans, items, nitems, parity, s);
}

template <class L, int STREAM, bool RO>
hipError_t collide_impl(int st, bool nc, bool fields, const void* fin, void* fout, float* scout, const void* phi,
                        const FieldPtrs& fo, const StepArgs& a, const ScatterOut* ro, hipStream_t s) {
  return CollideLaunch<L, STREAM, RO>::collide(st, nc, fields, fin, fout, scout, phi, fo, a, ro, s);
}

template <class L, int STREAM, bool RO>
hipError_t collide_mlp_impl(int st, bool fields, const void* fin, void* fout, float* scout, const void* phi,
                            const FieldPtrs& fo, const StepArgs& a, const MlpPacked* net, const ScatterOut* ro,
                            hipStream_t s) {
  return CollideLaunch<L, STREAM, RO>::collide_mlp(st, fields, fin, fout, scout, phi, fo, a, net, ro, s);
}

}  // namespace lbm

// explicit instantiation of one (lattice, streaming, read-once) combination
#define LB_INSTANTIATE_COLLIDE(LAT, STREAM, RO)                                                                 \
  namespace lbm {                                                                                               \
  template hipError_t collide_impl<LAT, STREAM, RO>(int, bool, bool, const void*, void*, float*, const void*,  \
                                                    const FieldPtrs&, const StepArgs&, const ScatterOut*,       \
                                                    hipStream_t);                                               \
  template hipError_t collide_mlp_impl<LAT, STREAM, RO>(int, bool, const void*, void*, float*, const void*,     \
                                                        const FieldPtrs&, const StepArgs&, const MlpPacked*,    \
                                                        const ScatterOut*, hipStream_t);                        \
  }

// the read-once ensemble launches of one lattice (in its two-copy read-once unit)
#define LB_INSTANTIATE_ENSEMBLE_RO(LAT)                                                                      \
  namespace lbm {                                                                                          \
  template hipError_t ensemble_ro_impl<LAT>(int, bool, bool, bool, bool, const ChannelDev*, const uint32_t*,\
                                            uint32_t, int, hipStream_t);                                   \
  }
