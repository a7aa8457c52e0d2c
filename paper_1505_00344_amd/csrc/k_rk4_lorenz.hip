// Fused RK4 instantiations: Lorenz and the linear test systems.
#include "ff_rk4.h"

namespace ff {

template <typename R> using Lin1 = Linear<R, 1>;
template <typename R> using Lin2 = Linear<R, 2>;
template <typename R> using Lin3 = Linear<R, 3>;
template <typename R> using Lin4 = Linear<R, 4>;

hipError_t launch_rk4_lorenz(const RK4Launch& L) { return dispatch_rk4<Lorenz, 4>(L); }

hipError_t launch_rk4_linear(int dim, const RK4Launch& L) {
    switch (dim) {
        case 1: return dispatch_rk4<Lin1, 4>(L);
        case 2: return dispatch_rk4<Lin2, 4>(L);
        case 3: return dispatch_rk4<Lin3, 4>(L);
        case 4: return dispatch_rk4<Lin4, 4>(L);
    }
    return hipErrorInvalidValue;
}

}  // namespace ff
