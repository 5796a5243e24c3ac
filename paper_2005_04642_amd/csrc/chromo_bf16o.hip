// Kernel instantiations for the BF16O population storage format.
#include "chromo_launch.hpp"

namespace chromo {
const Ops& ops_bf16o() {
  static const Ops o = launch::make_ops<BF16O>();
  return o;
}
}  // namespace chromo
