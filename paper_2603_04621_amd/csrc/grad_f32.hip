// Fused gradient kernel instantiated for float storage of a and c.
#include "grad_impl.hpp"

namespace dl {
DL_INSTANTIATE_GRAD(float, false, false)
}  // namespace dl
