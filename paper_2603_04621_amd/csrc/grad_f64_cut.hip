// Fused gradient kernel instantiated for double storage of a and c, variant with capped-simplex blocks.
#include "grad_impl.hpp"

namespace dl {
DL_INSTANTIATE_GRAD(double, true, false)
}  // namespace dl
