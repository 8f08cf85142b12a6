// Multi-entry-column gradient kernel (several families, dense rows)
// instantiated for double storage of the coefficients and costs.
#include "grad_mf.hpp"

namespace dl {
DL_INSTANTIATE_GRAD_MF(double)
}  // namespace dl
