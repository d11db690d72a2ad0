// In-place streaming instantiations for the D3Q27 velocity set.
#include "lattice_inplace.hpp"

namespace lbm {
const InPlaceOps* inplace_d3q27() {
  static const InPlaceOps o = InPlaceLaunch<D3Q27>::ops();
  return &o;
}
}  // namespace lbm
