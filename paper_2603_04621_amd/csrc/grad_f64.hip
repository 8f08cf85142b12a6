// Fused gradient kernel instantiated for double storage of a and c.
#include "grad_impl.hpp"

namespace dl {
DL_INSTANTIATE_GRAD(double, false, false)
}  // namespace dl
