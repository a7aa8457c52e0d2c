// Discrete-adjoint instantiations: Hodgkin-Huxley rings.  No register tape
// (every state of a segment is a sub-checkpoint in HBM: 15 doubles per step
// next to ~4 RK4 steps of exp-heavy arithmetic) and stage points recomputed
// on demand, so that the 15-dimensional reverse step fits in registers.
#include "ff_adjoint.h"

namespace ff {

template <typename R> using HH1 = HHRing<R, 1>;
template <typename R> using HH3 = HHRing<R, 3>;

// The compensated single-precision three-neuron step takes 268 VGPRs, one
// wave per SIMD; capped at 256 (two waves, 12 registers spilled) its reverse
// sweep of 1M particles x 2000 steps took 313 instead of 360 ms.  Double
// precision would spill 184 registers (1198 instead of 960 ms): no cap.
template <int N> struct AdjMinBlocks<HHRing<float, N>> {
    static constexpr int value = 2;
};

hipError_t launch_adj_hh(int neurons, const AdjLaunch& A) {
    switch (neurons) {
        case 1: return dispatch_adj<HH1, 1, true>(A);
        case 3: return dispatch_adj<HH3, 1, true>(A);
    }
    return hipErrorInvalidValue;
}

}  // namespace ff
