// Moment-based (regularised) step for the D3Q27 velocity set.
#include "lattice_llb.hpp"

namespace lbm {
const LlbOps* llb_d3q27() {
  static const LlbOps o = LlbLaunch<D3Q27>::ops();
  return &o;
}
}  // namespace lbm
