// Host-side launchers of the step kernels for one velocity set; included once
// per lattice by lattice_d2q9.hip / lattice_d3q19.hip / lattice_d3q27.hip so
// that the heavy instantiations compile in parallel.
#pragma once

#include "engine.hpp"

namespace lbm {

// collision passes of one streaming mode and read-once setting, defined in
// collide_launch.hpp and instantiated per lattice in their own translation
// units (lattice_*_collide*.hip) so that the builds run in parallel.  ro: the
// read-once scatter's outputs (NULL without); with ro, a.z_per_block is the
// march depth the caller sized the halo blocks for and is used as given.
template <class L, int STREAM, bool RO>
hipError_t collide_impl(int st, bool nc, bool fields, const void* fin, void* fout, float* scout, const void* phi,
                        const FieldPtrs& fo, const StepArgs& a, const ScatterOut* ro, hipStream_t s);
// the same with the learned near-contact closure (3D lattices)
template <class L, int STREAM, bool RO>
hipError_t collide_mlp_impl(int st, bool fields, const void* fin, void* fout, float* scout, const void* phi,
                            const FieldPtrs& fo, const StepArgs& a, const MlpPacked* net, const ScatterOut* ro,
                            hipStream_t s);
template <class L>
hipError_t ensemble_ro_impl(int st, bool nc, bool fields, bool combine, bool cached, const ChannelDev* chans,
                            const uint32_t* items, uint32_t nitems, int parity, hipStream_t s);

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

  // collision pass (two-copy streaming): the kernels of each read-once
  // setting are instantiated in their own translation unit (collide_launch.hpp)
  static hipError_t collide(int st, bool nc, bool fields, const void* fin, void* fout, float* scout, const void* phi,
                            const FieldPtrs& fo, const StepArgs& a, const ScatterOut* ro, hipStream_t s) {
    return ro ? collide_impl<L, STREAM_AB, true>(st, nc, fields, fin, fout, scout, phi, fo, a, ro, s)
              : collide_impl<L, STREAM_AB, false>(st, nc, fields, fin, fout, scout, phi, fo, a, ro, s);
  }

  // read-once step after an initialisation or a restore: scatter the stored
  // state (canonical layout) as the collision pass would have; a: with the
  // read-once march depth
  template <class S, bool TOT>
  static hipError_t boot_t(const void* f, const float* sc, const ScatterOut& ro, const StepArgs& a, hipStream_t s) {
    using T = Tile<TILE_X, TILE_Y, 1, L::D>;
    dim3 block(T::TX, T::TY, 1);
    StepArgs b = a;
    b.tiles_x = (a.nx + T::TX - 1) / T::TX;
    b.tiles_y = (a.ny + T::TY - 1) / T::TY;
    dim3 grid((unsigned)b.tiles_x * b.tiles_y * ((a.nz + a.z_per_block - 1) / a.z_per_block));
    k_boot_scatter<L, S, T, TOT><<<grid, block, 0, s>>>((const S*)f, sc, b, ro);
    return hipGetLastError();
  }
  static hipError_t boot(int st, const void* f, const float* sc, const ScatterOut& ro, const StepArgs& a,
                         hipStream_t s) {
    switch (st) {
      case ST_F64: return boot_t<double, false>(f, sc, ro, a, s);
      case ST_F32: return boot_t<float, false>(f, sc, ro, a, s);
      case ST_F16: return boot_t<_Float16, false>(f, sc, ro, a, s);
      case ST_BF16: return boot_t<__bf16, false>(f, sc, ro, a, s);
      case ST_F32S: return boot_t<F32S, false>(f, sc, ro, a, s);
      case ST_F32T: return boot_t<float, true>(f, sc, ro, a, s);
      case ST_F16T: return boot_t<_Float16, true>(f, sc, ro, a, s);
      case ST_BF16T: return boot_t<__bf16, true>(f, sc, ro, a, s);
      case ST_F16CT: return boot_t<F16C, true>(f, sc, ro, a, s);
    }
    return hipErrorInvalidValue;
  }

  // read-once step, second launch: the phase field of the next step from the
  // scatter's outputs; a: the arguments the collision launch used
  static hipError_t combine(int st, const ScatterOut& ro, void* phi, const StepArgs& a, hipStream_t s) {
    StepArgs b = a;
    b.tiles_x = (a.nx + TILE_X - 1) / TILE_X;
    b.tiles_y = (a.ny + TILE_Y - 1) / TILE_Y;
    dim3 block(TILE_X, TILE_Y, 1);
    const unsigned marches = (unsigned)((a.nz + a.z_per_block - 1) / a.z_per_block);
    const unsigned groups = (unsigned)((a.z_per_block + COMBINE_PLANES - 1) / COMBINE_PLANES);
    dim3 grid((unsigned)b.tiles_x, (unsigned)b.tiles_y, marches * groups);
    // per-colour FP64 / FP32 storage scatter the stored populations
    // themselves; every other layout scatters shifted values
    if (st == ST_F64)
      k_combine<L, double, TILE_X, TILE_Y, false><<<grid, block, 0, s>>>((const double*)ro.part,
                                                                         (const RPair<double>*)ro.halo, (double*)phi, b);
    else if (st == ST_F32)
      k_combine<L, float, TILE_X, TILE_Y, false><<<grid, block, 0, s>>>((const float*)ro.part,
                                                                        (const RPair<float>*)ro.halo, (float*)phi, b);
    else
      k_combine<L, float, TILE_X, TILE_Y, true><<<grid, block, 0, s>>>((const float*)ro.part,
                                                                       (const RPair<float>*)ro.halo, (float*)phi, b);
    return hipGetLastError();
  }

  static hipError_t collide_mlp(int st, bool fields, const void* fin, void* fout, float* scout, const void* phi,
                                const FieldPtrs& fo, const StepArgs& a, const MlpPacked* net, const ScatterOut* ro,
                                hipStream_t s) {
    if constexpr (L::D == 3) {
      return ro ? collide_mlp_impl<L, STREAM_AB, true>(st, fields, fin, fout, scout, phi, fo, a, net, ro, s)
                : collide_mlp_impl<L, STREAM_AB, false>(st, fields, fin, fout, scout, phi, fo, a, net, ro, s);
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
    return LatticeOps{L::Q, L::D, &phase, &collide, &init, &ensemble, L::D == 3 ? &collide_mlp : nullptr, &combine,
                      &boot, &ensemble_ro_impl<L>};
  }
};

}  // namespace lbm
