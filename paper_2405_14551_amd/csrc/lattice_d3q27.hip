// Kernel instantiations for the D3Q27 velocity set.
#include "lattice_ops.hpp"

namespace lbm {
const LatticeOps* ops_d3q27() {
  static const LatticeOps o = Launch<D3Q27>::ops();
  return &o;
}
}  // namespace lbm
