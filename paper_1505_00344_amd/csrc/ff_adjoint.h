// ff_adjoint.h — host-side launch of the discrete adjoint kernel
// (ff_adjoint_kernel.h) for the built-in right-hand sides.
#pragma once
#include "ff_adjoint_kernel.h"
#include "ff_rk4.h"

namespace ff {

inline AdjArgs make_adj_args(const AdjLaunch& A) {
    AdjArgs a;
    a.pp = A.f.pp;
    a.n = A.f.n;
    a.ld = A.f.ld;
    a.n_pp = A.f.n_pp;
    for (int k = 0; k < kMaxPP; ++k) a.slot[k] = A.f.slot[k];
    a.p = A.f.p;
    a.h = A.f.h;
    a.h2 = A.f.h2;
    a.h6 = A.f.h6;
    a.h3 = A.h3;
    a.ckpt = A.ckpt;
    a.ckpt_c = A.ckpt_c;
    a.sub = A.sub;
    a.sub_c = A.sub_c;
    a.lam = A.lam;
    a.mu = A.mu;
    a.mu_part = A.mu_part;
    a.carry = A.carry;
    a.seg_len = A.seg_len;
    a.first = A.first;
    a.last = A.last;
    return a;
}

// T: register-tape length; CAPTURE: keep the stage points too (single
// precision with T32, double with T64 and CAPTURE64, where registers allow).
template <template <typename> class SysT, int T, bool LOWREG = false, bool CAPTURE = false, int T64 = T,
          bool CAPTURE64 = CAPTURE>
hipError_t dispatch_adj(const AdjLaunch& A) {
    const int64_t grid = (A.f.n + kAdjBlock - 1) / kAdjBlock;
    if (grid <= 0) return hipSuccess;
    const AdjArgs a = make_adj_args(A);
    switch (A.f.prec) {
        case FF_FP64:
            hipLaunchKernelGGL((k_adj<SysT<double>, double, false, T64, LOWREG, CAPTURE64>), dim3((unsigned)grid),
                               dim3(kAdjBlock), 0, A.f.stream, a);
            break;
        case FF_FP32:
            hipLaunchKernelGGL((k_adj<SysT<float>, float, false, T, LOWREG, CAPTURE>), dim3((unsigned)grid),
                               dim3(kAdjBlock), 0, A.f.stream, a);
            break;
        case FF_FP32_KAHAN:
            hipLaunchKernelGGL((k_adj<SysT<float>, float, true, T, LOWREG, CAPTURE>), dim3((unsigned)grid),
                               dim3(kAdjBlock), 0, A.f.stream, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ff
