// Fused gradient kernel instantiated for double storage of a and c, deterministic variant (integer per-destination sums; all block types).
#include "grad_impl.hpp"

namespace dl {
DL_INSTANTIATE_GRAD(double, true, true)
}  // namespace dl
