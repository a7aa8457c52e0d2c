// Discrete-adjoint instantiations: Wilson-Cowan pair (register tape of 8 states).
#include "ff_adjoint.h"

namespace ff {

hipError_t launch_adj_wc(const AdjLaunch& A) { return dispatch_adj<WilsonCowan, 8>(A); }

}  // namespace ff
