// Moment-based (regularised) step for the D3Q19 velocity set.
#include "lattice_llb.hpp"

namespace lbm {
const LlbOps* llb_d3q19() {
  static const LlbOps o = LlbLaunch<D3Q19>::ops();
  return &o;
}
}  // namespace lbm
