// Discrete-adjoint instantiations: Lorenz and the linear test systems
// (register tape of 8 states).
#include "ff_adjoint.h"

namespace ff {

template <typename R> using Lin1 = Linear<R, 1>;
template <typename R> using Lin2 = Linear<R, 2>;
template <typename R> using Lin3 = Linear<R, 3>;
template <typename R> using Lin4 = Linear<R, 4>;

hipError_t launch_adj_lorenz(const AdjLaunch& A) { return dispatch_adj<Lorenz, 8>(A); }

hipError_t launch_adj_linear(int dim, const AdjLaunch& A) {
    switch (dim) {
        case 1: return dispatch_adj<Lin1, 8>(A);
        case 2: return dispatch_adj<Lin2, 8>(A);
        case 3: return dispatch_adj<Lin3, 8>(A);
        case 4: return dispatch_adj<Lin4, 8>(A);
    }
    return hipErrorInvalidValue;
}

}  // namespace ff
