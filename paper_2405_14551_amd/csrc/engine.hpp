// Internal launch interface between the C ABI (api.hip) and the per-lattice
// kernel instantiations (lattice_*.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aux_kernels.hpp"

namespace lbm {

enum StorageKind { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3 };

// pass-2 tile: 64 x-sites (one wave per row) by 4 rows
constexpr int TILE_X = 64;
constexpr int TILE_Y = 4;

struct LatticeOps {
  int q, d;
  hipError_t (*phase)(int storage, const void* fin, void* phi, const StepArgs& a, hipStream_t s);
  hipError_t (*collide)(int storage, bool nc, bool fields, const void* fin, void* fout, const void* phi,
                        const FieldPtrs& fo, const StepArgs& a, hipStream_t s);
  hipError_t (*init)(int storage, void* f, void* phi, const FieldPtrs& fo, const double* drops,
                     const InitArgs& a, hipStream_t s);
};

const LatticeOps* ops_d2q9();
const LatticeOps* ops_d3q19();
const LatticeOps* ops_d3q27();

}  // namespace lbm
