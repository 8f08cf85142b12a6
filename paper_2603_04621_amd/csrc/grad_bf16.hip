// Fused gradient kernel instantiated for uint16_t storage of a and c.
#include "grad_impl.hpp"

namespace dl {
DL_INSTANTIATE_GRAD(uint16_t, false, false)
}  // namespace dl
