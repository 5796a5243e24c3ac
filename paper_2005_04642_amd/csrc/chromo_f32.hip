// Kernel instantiations for the F32 population storage format.
#include "chromo_launch.hpp"

namespace chromo {
const Ops& ops_f32() {
  static const Ops o = launch::make_ops<F32>();
  return o;
}
}  // namespace chromo
