// Multi-entry-column gradient kernel (several families, dense rows)
// instantiated for float storage of the coefficients and costs.
#include "grad_mf.hpp"

namespace dl {
DL_INSTANTIATE_GRAD_MF(float)
}  // namespace dl
