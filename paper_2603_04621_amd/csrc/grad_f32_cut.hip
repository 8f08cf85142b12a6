// Fused gradient kernel instantiated for float storage of a and c, variant with capped-simplex blocks.
#include "grad_impl.hpp"

namespace dl {
DL_INSTANTIATE_GRAD(float, true, false)
}  // namespace dl
