// Internal launch interface between the C ABI (api.hip) and the per-lattice
// kernel instantiations (lattice_*.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aux_kernels.hpp"
#include "ensemble.hpp"

namespace lbm {

// per-colour layouts, then the total layout (total population + recolouring scalars)
enum StorageKind {
  ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3, ST_F32T = 4, ST_F16T = 5, ST_BF16T = 6, ST_F16CT = 7,
  ST_F32S = 8  // per-colour, shifted populations in FP32
};
inline bool is_total(int st) { return st >= ST_F32T && st <= ST_F16CT; }

// pass-2 tile: 64 x-sites (one wave per row) by 4 rows unless overridden at build time
#ifndef LB_TILE_X
#define LB_TILE_X 64
#endif
#ifndef LB_TILE_Y
#define LB_TILE_Y 4
#endif
// collision tile: TILE_X x TILE_Y columns of sites, one thread each
constexpr int TILE_X = LB_TILE_X;
constexpr int TILE_Y = LB_TILE_Y;
static_assert(TILE_X * TILE_Y == 256 && TILE_X % 64 == 0, "a collision tile is 256 threads, whole waves per row");

struct LatticeOps {
  int q, d;
  // scin / scout: recolouring scalars of the total layout (unused otherwise);
  // the collision pass writes them but never reads them
  hipError_t (*phase)(int storage, const void* fin, const float* scin, void* phi, const StepArgs& a, hipStream_t s);
  // ro: read-once step (NULL: two-pass step), see step_kernels.hpp
  hipError_t (*collide)(int storage, bool nc, bool fields, const void* fin, void* fout, float* scout,
                        const void* phi, const FieldPtrs& fo, const StepArgs& a, const ScatterOut* ro,
                        hipStream_t s);
  hipError_t (*init)(int storage, void* f, float* sc, void* phi, const FieldPtrs& fo, const double* drops,
                     const InitArgs& a, hipStream_t s);
  // batched ensemble launch: one workgroup per entry of `items` (storages
  // ST_F64, ST_F32 and the total layouts); phase_only: every item is a
  // phase tile, launched with the phase pass's own (smaller) kernel
  hipError_t (*ensemble)(int storage, bool nc, bool fields, bool phase_only, const ChannelDev* chans,
                         const uint32_t* items, uint32_t nitems, int parity, hipStream_t s);
  // collision pass with the learned near-contact closure (3D; storages
  // ST_F64, ST_F32 and the total layouts); NULL for 2D
  hipError_t (*collide_mlp)(int storage, bool fields, const void* fin, void* fout, float* scout, const void* phi,
                            const FieldPtrs& fo, const StepArgs& a, const MlpPacked* net, const ScatterOut* ro,
                            hipStream_t s);
  // read-once step: the next phase field from the scatter's outputs; a: the
  // collision launch's arguments
  hipError_t (*combine)(int storage, const ScatterOut& ro, void* phi, const StepArgs& a, hipStream_t s);
  // read-once step after an initialisation or a restore: the scatter of the
  // stored state (canonical layout; sc: the total layout's scalars) that the
  // collision pass storing it would have made
  hipError_t (*boot)(int storage, const void* f, const float* sc, const ScatterOut& ro, const StepArgs& a,
                     hipStream_t s);
  // read-once batched ensemble launch (storages as for `ensemble`): combine
  // false: every item is a collision tile-march (collision with the
  // scatter); combine true: every item is a combine block.  cached: the
  // populations are stored through L2 instead of non-temporally (for rows
  // that do not start on 64-byte boundaries, whose line ends two tiles write)
  hipError_t (*ensemble_ro)(int storage, bool nc, bool fields, bool combine, bool cached, const ChannelDev* chans,
                            const uint32_t* items, uint32_t nitems, int parity, hipStream_t s);
};

// One-copy (in-place) streaming: even and odd steps alternate, the even kind
// starting from the canonical layout (step_kernels.hpp, STREAM_EVEN /
// STREAM_ODD).  An even step's phase pass is LatticeOps::phase.
struct InPlaceOps {
  hipError_t (*phase_odd)(int storage, const void* f, const float* scin, void* phi, const StepArgs& a,
                          hipStream_t s);
  hipError_t (*collide)(int storage, int odd, bool nc, bool fields, void* f, float* scout, const void* phi,
                        const FieldPtrs& fo, const StepArgs& a, const ScatterOut* ro, hipStream_t s);
  // NULL for 2D; storages as LatticeOps::collide_mlp
  hipError_t (*collide_mlp)(int storage, int odd, bool fields, void* f, float* scout, const void* phi,
                            const FieldPtrs& fo, const StepArgs& a, const MlpPacked* net, const ScatterOut* ro,
                            hipStream_t s);
  // planes i0 .. i1-1 of the colour block at f, in the canonical layout, from
  // the layout an even step leaves; out holds (i1 - i0) N elements
  hipError_t (*canonical)(int storage, const void* f, void* out, int i0, int i1, const StepArgs& a, hipStream_t s);
};

// Moment-based (regularised) step: the state is 15 moments per site
// (llb_kernels.hpp); storages ST_F64 and ST_F32.  W holds the 11 pre-collision
// moments pass 1 writes and pass 2 reads.
struct LlbOps {
  hipError_t (*init)(int storage, void* M, void* phi, const FieldPtrs& fo, const double* drops, const InitArgs& a,
                     hipStream_t s);
  hipError_t (*pull)(int storage, const void* M, void* W, void* phi, const StepArgs& a, hipStream_t s);
  hipError_t (*collide)(int storage, bool nc, bool fields, const void* W, void* M, const void* phi,
                        const FieldPtrs& fo, const StepArgs& a, hipStream_t s);
};

// storages the learned closure is built for
inline bool mlp_storage(int st) { return st == ST_F64 || st == ST_F32 || is_total(st); }

// storages the ensemble kernel is built for
inline bool ensemble_storage(int st) { return st == ST_F64 || st == ST_F32 || is_total(st); }

const LatticeOps* ops_d2q9();
const LatticeOps* ops_d3q19();
const LatticeOps* ops_d3q27();
const InPlaceOps* inplace_d2q9();
const InPlaceOps* inplace_d3q19();
const InPlaceOps* inplace_d3q27();
const LlbOps* llb_d2q9();
const LlbOps* llb_d3q19();
const LlbOps* llb_d3q27();

}  // namespace lbm
