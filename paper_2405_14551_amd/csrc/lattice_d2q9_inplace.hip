// In-place streaming instantiations for the D2Q9 velocity set.
#include "lattice_inplace.hpp"

namespace lbm {
const InPlaceOps* inplace_d2q9() {
  static const InPlaceOps o = InPlaceLaunch<D2Q9>::ops();
  return &o;
}
}  // namespace lbm
