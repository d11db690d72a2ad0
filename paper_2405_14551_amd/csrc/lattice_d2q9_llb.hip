// Moment-based (regularised) step for the D2Q9 velocity set.
#include "lattice_llb.hpp"

namespace lbm {
const LlbOps* llb_d2q9() {
  static const LlbOps o = LlbLaunch<D2Q9>::ops();
  return &o;
}
}  // namespace lbm
