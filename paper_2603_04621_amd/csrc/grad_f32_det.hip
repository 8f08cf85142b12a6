// Fused gradient kernel instantiated for float storage of a and c, deterministic variant (integer per-destination sums; all block types).
#include "grad_impl.hpp"

namespace dl {
DL_INSTANTIATE_GRAD(float, true, true)
}  // namespace dl
