// ff_rk4.h — host-side launch of the fused RK4 kernel (ff_kernel.h) for the
// built-in right-hand sides: argument packing and the dispatch over
// precision and particles per thread.
#pragma once
#include "ff_internal.h"
#include "ff_kernel.h"
#include "ff_rhs.h"

namespace ff {

inline RK4Args make_args(const RK4Launch& L) {
    RK4Args a;
    a.state = L.state;
    a.comp = L.comp;
    a.pp = L.pp;
    a.n = L.n;
    a.ld = L.ld;
    a.n_pp = L.n_pp;
    for (int k = 0; k < kMaxPP; ++k) a.slot[k] = L.slot[k];
    a.p = L.p;
    a.h = L.h;
    a.h2 = L.h2;
    a.h6 = L.h6;
    a.steps = L.steps;
    a.ckpt = L.ckpt;
    a.ckpt_c = L.ckpt_c;
    a.ckpt_ld = L.ckpt_ld;
    return a;
}

template <class S, typename R, bool KAHAN, int PPT>
hipError_t launch_rk4_t(const RK4Launch& L) {
    const int64_t per_block = (int64_t)L.block * PPT;
    const int64_t grid = (L.n + per_block - 1) / per_block;
    if (grid <= 0) return hipSuccess;
    if (L.record) {
        if constexpr (PPT <= 2) {
            const ResetArgs none{};
            if (L.reset)
                hipLaunchKernelGGL((k_rk4_record<S, R, KAHAN, PPT, true>), dim3((unsigned)grid), dim3(L.block), 0,
                                   L.stream, make_args(L), *L.reset, *L.record);
            else
                hipLaunchKernelGGL((k_rk4_record<S, R, KAHAN, PPT, false>), dim3((unsigned)grid), dim3(L.block), 0,
                                   L.stream, make_args(L), none, *L.record);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;  // the launcher clamps PPT to 2 for recording
    }
    if (L.reset) {
        if constexpr (PPT <= 2) {
            hipLaunchKernelGGL((k_rk4_reset<S, R, KAHAN, PPT>), dim3((unsigned)grid), dim3(L.block), 0, L.stream,
                               make_args(L), *L.reset);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;  // the launcher clamps PPT to 2 for resets
    }
    hipLaunchKernelGGL((k_rk4<S, R, KAHAN, PPT>), dim3((unsigned)grid), dim3(L.block), 0, L.stream,
                       make_args(L));
    return hipGetLastError();
}

// Dispatch over precision and particles per thread (PPT above MAXPPT is
// clamped to MAXPPT).
template <template <typename> class SysT, int MAXPPT>
hipError_t dispatch_rk4(const RK4Launch& L) {
    int ppt = L.ppt > MAXPPT ? MAXPPT : L.ppt;
    if ((L.reset || L.record) && ppt > 2) ppt = 2;
    switch (L.prec) {
        case FF_FP64:
            if (ppt >= 4 && MAXPPT >= 4) return launch_rk4_t<SysT<double>, double, false, (MAXPPT >= 4 ? 4 : 1)>(L);
            if (ppt >= 2 && MAXPPT >= 2) return launch_rk4_t<SysT<double>, double, false, (MAXPPT >= 2 ? 2 : 1)>(L);
            return launch_rk4_t<SysT<double>, double, false, 1>(L);
        case FF_FP32:
            if (ppt >= 4 && MAXPPT >= 4) return launch_rk4_t<SysT<float>, float, false, (MAXPPT >= 4 ? 4 : 1)>(L);
            if (ppt >= 2 && MAXPPT >= 2) return launch_rk4_t<SysT<float>, float, false, (MAXPPT >= 2 ? 2 : 1)>(L);
            return launch_rk4_t<SysT<float>, float, false, 1>(L);
        case FF_FP32_KAHAN:
            if (ppt >= 4 && MAXPPT >= 4) return launch_rk4_t<SysT<float>, float, true, (MAXPPT >= 4 ? 4 : 1)>(L);
            if (ppt >= 2 && MAXPPT >= 2) return launch_rk4_t<SysT<float>, float, true, (MAXPPT >= 2 ? 2 : 1)>(L);
            return launch_rk4_t<SysT<float>, float, true, 1>(L);
    }
    return hipErrorInvalidValue;
}

}  // namespace ff
