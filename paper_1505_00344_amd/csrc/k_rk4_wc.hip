// Fused RK4 instantiations: Wilson-Cowan pair.
#include "ff_rk4.h"

namespace ff {

hipError_t launch_rk4_wc(const RK4Launch& L) { return dispatch_rk4<WilsonCowan, 4>(L); }

}  // namespace ff
