// Kernel instantiations for the D2Q9 velocity set.
#include "lattice_ops.hpp"

namespace lbm {
const LatticeOps* ops_d2q9() {
  static const LatticeOps o = Launch<D2Q9>::ops();
  return &o;
}
}  // namespace lbm
