// Implicit adjoint of the converged field solve (kernels added with the backward pass).
#include "dgp_internal.h"

namespace dgp {}  // namespace dgp
