// Kernel instantiations for the F64 population storage format.
#include "chromo_launch.hpp"

namespace chromo {
const Ops& ops_f64() {
  static const Ops o = launch::make_ops<F64>();
  return o;
}
}  // namespace chromo
