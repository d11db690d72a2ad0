// Host-side launchers of the one-copy (in-place) streaming modes for one
// velocity set.  Included by lattice_*_inplace.hip, so that these
// instantiations compile in parallel with the two-copy ones.
#pragma once

#include "lattice_ops.hpp"

namespace lbm {

template <class L>
struct InPlaceLaunch {
  using B = Launch<L>;

  // phase pass of an odd step: the pulled populations are in the site's own
  // reversed slots (an even step reads as two-copy streaming does)
  static hipError_t phase_odd(int st, const void* f, const float* scin, void* phi, const StepArgs& a,
                              hipStream_t s) {
    switch (st) {
      case ST_F64: return B::template phase_t<double, true>(f, phi, a, s);
      case ST_F32: return B::template phase_t<float, true>(f, phi, a, s);
      case ST_F16: return B::template phase_t<_Float16, true>(f, phi, a, s);
      case ST_BF16: return B::template phase_t<__bf16, true>(f, phi, a, s);
      case ST_F32S: return B::template phase_t<F32S, true>(f, phi, a, s);
      case ST_F32T: return B::template phase_total_t<float, true>(f, scin, phi, a, s);
      case ST_F16T: return B::template phase_total_t<_Float16, true>(f, scin, phi, a, s);
      case ST_BF16T: return B::template phase_total_t<__bf16, true>(f, scin, phi, a, s);
      case ST_F16CT: return B::template phase_total_t<F16C, true>(f, scin, phi, a, s);
    }
    return hipErrorInvalidValue;
  }

  // collision pass of either kind (collide_launch.hpp, instantiated in the
  // lattice_*_collide_*.hip files); one copy: fin == fout
  static hipError_t collide(int st, int odd, bool nc, bool fields, void* f, float* scout, const void* phi,
                            const FieldPtrs& fo, const StepArgs& a, const ScatterOut* ro, hipStream_t s) {
    if (ro)
      return odd ? collide_impl<L, STREAM_ODD, true>(st, nc, fields, f, f, scout, phi, fo, a, ro, s)
                 : collide_impl<L, STREAM_EVEN, true>(st, nc, fields, f, f, scout, phi, fo, a, ro, s);
    return odd ? collide_impl<L, STREAM_ODD, false>(st, nc, fields, f, f, scout, phi, fo, a, ro, s)
               : collide_impl<L, STREAM_EVEN, false>(st, nc, fields, f, f, scout, phi, fo, a, ro, s);
  }

  static hipError_t collide_mlp(int st, int odd, bool fields, void* f, float* scout, const void* phi,
                                const FieldPtrs& fo, const StepArgs& a, const MlpPacked* net, const ScatterOut* ro,
                                hipStream_t s) {
    if constexpr (L::D == 3) {
      if (ro)
        return odd ? collide_mlp_impl<L, STREAM_ODD, true>(st, fields, f, f, scout, phi, fo, a, net, ro, s)
                   : collide_mlp_impl<L, STREAM_EVEN, true>(st, fields, f, f, scout, phi, fo, a, net, ro, s);
      return odd ? collide_mlp_impl<L, STREAM_ODD, false>(st, fields, f, f, scout, phi, fo, a, net, ro, s)
                 : collide_mlp_impl<L, STREAM_EVEN, false>(st, fields, f, f, scout, phi, fo, a, net, ro, s);
    }
    return hipErrorInvalidValue;
  }

  static hipError_t canonical(int st, const void* f, void* out, int i0, int i1, const StepArgs& a, hipStream_t s) {
    if (i0 < 0 || i1 > L::Q || i0 >= i1) return hipErrorInvalidValue;
    dim3 block(256), grid((a.N + 255) / 256);
    switch (st) {
      case ST_F64:
        k_canonical<L, uint64_t><<<grid, block, 0, s>>>((const uint64_t*)f, (uint64_t*)out, i0, i1, a);
        break;
      case ST_F32:
      case ST_F32T:
      case ST_F32S:
        k_canonical<L, uint32_t><<<grid, block, 0, s>>>((const uint32_t*)f, (uint32_t*)out, i0, i1, a);
        break;
      case ST_F16:
      case ST_BF16:
      case ST_F16T:
      case ST_BF16T:
      case ST_F16CT:
        k_canonical<L, uint16_t><<<grid, block, 0, s>>>((const uint16_t*)f, (uint16_t*)out, i0, i1, a);
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }

  static InPlaceOps ops() {
    return InPlaceOps{&phase_odd, &collide, L::D == 3 ? &collide_mlp : nullptr, &canonical};
  }
};

}  // namespace lbm
