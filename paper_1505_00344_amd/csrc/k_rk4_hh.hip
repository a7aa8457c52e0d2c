// Fused RK4 instantiations: Hodgkin-Huxley rings of 1 and 3 neurons (at most
// two particles per thread: one 15-dimensional FP64 particle already holds
// ~100 live VGPRs across a stage).
#include "ff_rk4.h"

namespace ff {

template <typename R> using HH1 = HHRing<R, 1>;
template <typename R> using HH3 = HHRing<R, 3>;

hipError_t launch_rk4_hh(int neurons, const RK4Launch& L) {
    switch (neurons) {
        case 1: return dispatch_rk4<HH1, 2>(L);
        case 3: return dispatch_rk4<HH3, 2>(L);
    }
    return hipErrorInvalidValue;
}

}  // namespace ff
