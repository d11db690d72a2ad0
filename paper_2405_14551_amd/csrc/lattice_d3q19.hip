// Kernel instantiations for the D3Q19 velocity set.
#include "lattice_ops.hpp"

namespace lbm {
const LatticeOps* ops_d3q19() {
  static const LatticeOps o = Launch<D3Q19>::ops();
  return &o;
}
}  // namespace lbm
