// Kernel instantiations for the F16O population storage format.
#include "chromo_launch.hpp"

namespace chromo {
const Ops& ops_f16o() {
  static const Ops o = launch::make_ops<F16O>();
  return o;
}
}  // namespace chromo
