// ff_internal.h — host-side declarations shared by the library's translation
// units (launch descriptors, per-system launchers, error reporting).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/fireflies.h"
#include "ff_kernel.h"

namespace ff {

static_assert(kMaxPP == FF_MAX_PP, "kernel and ABI disagree on per-particle parameters");

// Everything one fused-RK4 launch needs (kernel arguments are built from it).
struct RK4Launch {
    int prec;            // ff_prec
    void* state;
    void* comp;          // FF_FP32_KAHAN only
    const void* pp;      // per-particle parameters, SoA [n_pp][ld], dtype of prec
    int64_t n, ld;
    int n_pp;
    int slot[kMaxPP];
    ParamBlock p;
    double h, h2, h6;    // step, half step, step/6 (already rounded to prec)
    int64_t steps;       // steps in this launch
    int ppt;             // particles per thread: 1, 2, 4
    int block;           // threads per block: 64..256 (multiple of 64)
    hipStream_t stream;
    void* ckpt;          // if set: the launch first stores its starting state here
    void* ckpt_c;        //   (and the compensation here), SoA [dim][ckpt_ld]
    int64_t ckpt_ld;
    const ResetArgs* reset;  // if set: apply the reset rule after every step
    RecordArgs* record;      // if set: store every stride-th particle every `every` steps
};

// Adjoint launch: one reverse segment of a checkpointed run.
struct AdjLaunch {
    RK4Launch f;         // forward description (pp, n, ld, params, steps; f.h3 below)
    double h3;           // step/3 rounded to the precision
    const void* ckpt;    // segment start state, SoA [dim][n]
    const void* ckpt_c;  // matching Kahan compensation, or null
    void* sub;           // sub-checkpoint scratch [nsub][dim][n] (+ compensation after it)
    void* sub_c;
    void* lam;           // adjoint of the state, SoA [dim][ld], in/out
    void* mu;            // per-particle parameter adjoints, SoA [n_pp][ld]
    double* mu_part;     // per-block FP64 partial sums of all parameter adjoints [nblk][kMaxParams]
    void* carry;         // per-particle parameter adjoints between segments [NP][n]
    int64_t seg_len;     // steps in this segment
    int first;           // 1 for the first segment processed (last in time)
    int last;            // 1 for the last segment processed (first in time)
};

// Steps held in registers by the adjoint's innermost recompute (per system).
int adj_tape_len(const ff_system_s* sys, int prec);

// Per-system fused RK4 launchers (one translation unit each).
hipError_t launch_rk4_linear(int dim, const RK4Launch& L);
hipError_t launch_rk4_lorenz(const RK4Launch& L);
hipError_t launch_rk4_wc(const RK4Launch& L);
hipError_t launch_rk4_hh(int neurons, const RK4Launch& L);

hipError_t launch_adj_linear(int dim, const AdjLaunch& A);
hipError_t launch_adj_lorenz(const AdjLaunch& A);
hipError_t launch_adj_wc(const AdjLaunch& A);
hipError_t launch_adj_hh(int neurons, const AdjLaunch& A);

// Right-hand sides compiled at run time from expressions (ff_expr.hip).
struct ExprProgram;
constexpr int kExprKernels = 8;  // {step, reset, record, record+reset} x {1, 2} particles per thread

// Thread-local last-error text.
void set_error(const std::string& msg);
ff_status fail(ff_status code, const std::string& msg);
ff_status device_fail(hipError_t e, const char* where);

// Library-owned device scratch, one buffer per device and use, allocated on
// first need and grown (after a sync of `stream`) when a call needs more;
// refused under stream capture when it would have to grow.
constexpr int kScratchHistogram = 0, kScratchRender = 1, kScratchUses = 2;
ff_status library_scratch(int use, size_t need, hipStream_t stream, void** out);

}  // namespace ff

// The opaque system handle.
struct ff_system_s {
    int32_t rhs;
    int32_t dim;
    int32_t n_params;
    double params[ff::kMaxParams];
    ff::ExprProgram* expr = nullptr;  // FF_RHS_EXPR only
};

namespace ff {

// Host-side validation shared by the entry points (no device access).
ff_status check_system(const ff_system_s* sys);
ff_status check_batch(const ff_system_s* sys, const ff_batch* b, bool need_state);
ff_status check_tuning(const ff_system_s* sys, const ff_tuning* t);
size_t prec_size(int prec);

// Fill a launch descriptor (step rounding, parameters, per-particle slots).
RK4Launch make_launch(const ff_system_s* sys, const ff_batch* b, double dt, const ff_tuning* t,
                      hipStream_t stream);
// Launch the fused RK4 kernel of the system for L.steps steps.
hipError_t launch_rk4(const ff_system_s* sys, const RK4Launch& L);
// Expression systems: compile and load the kernels of `prec` (the fused RK4
// kernels, or the adjoint kernel) for the current device unless that was done
// before (thread-safe).
constexpr int kExprForward = 0, kExprAdjoint = 1;
ff_status expr_prepare(const ff_system_s* sys, int prec, int kind);
hipError_t launch_rk4_expr(const ff_system_s* sys, const RK4Launch& L);
hipError_t launch_adj_expr(const ff_system_s* sys, const AdjLaunch& A);
void expr_destroy(ExprProgram* p);
// Default particles per thread / block for a system and precision.
ff_tuning default_tuning(const ff_system_s* sys, int prec, int64_t nsteps);

}  // namespace ff
