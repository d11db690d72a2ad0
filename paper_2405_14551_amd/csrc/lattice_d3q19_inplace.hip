// In-place streaming instantiations for the D3Q19 velocity set.
#include "lattice_inplace.hpp"

namespace lbm {
const InPlaceOps* inplace_d3q19() {
  static const InPlaceOps o = InPlaceLaunch<D3Q19>::ops();
  return &o;
}
}  // namespace lbm
