// Fused gradient kernel instantiated for uint16_t storage of a and c, deterministic variant (integer per-destination sums; all block types).
#include "grad_impl.hpp"

namespace dl {
DL_INSTANTIATE_GRAD(uint16_t, true, true)
}  // namespace dl
