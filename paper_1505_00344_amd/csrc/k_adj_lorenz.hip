// Discrete-adjoint instantiations: Lorenz and the linear test systems
// (register tape of 8 states, 4 for Lorenz in double precision).
#include "ff_adjoint.h"

namespace ff {

template <typename R> using Lin1 = Linear<R, 1>;
template <typename R> using Lin2 = Linear<R, 2>;
template <typename R> using Lin3 = Linear<R, 3>;
template <typename R> using Lin4 = Linear<R, 4>;

// Lorenz keeps the stage points of its tape states (CAPTURE): single
// precision with the 8-state tape (138 VGPRs), double precision with a
// 4-state tape (162 VGPRs; with 8 states it would take 258, one wave per
// SIMD).  Measured on the 8M-particle, 200-step adjoint: FP64 12.0 -> 11.6 ms,
// FP32-Kahan 7.33 -> 7.15 ms, FP32 6.61 -> 6.40 ms, results bitwise unchanged.
hipError_t launch_adj_lorenz(const AdjLaunch& A) { return dispatch_adj<Lorenz, 8, false, true, 4, true>(A); }

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
