// ff_api.hip — C ABI: system handles, validation, errors, and ff_integrate.
#include <cfloat>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "ff_internal.h"
#include "ff_rk4.h"

namespace ff {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }

ff_status fail(ff_status code, const std::string& msg) {
    g_error = msg;
    return code;
}

ff_status device_fail(hipError_t e, const char* where) {
    // the error is reported here: clear the runtime's sticky last error so
    // that the caller's next, unrelated HIP call does not report it again
    (void)hipGetLastError();
    return fail(FF_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

size_t prec_size(int prec) { return prec == FF_FP64 ? sizeof(double) : sizeof(float); }

static int expected_params(int rhs, int dim) {
    switch (rhs) {
        case FF_RHS_LINEAR: return (dim >= 1 && dim <= 4) ? dim * dim : -1;
        case FF_RHS_LORENZ: return dim == 3 ? 3 : -1;
        case FF_RHS_WILSON_COWAN: return dim == 2 ? 10 : -1;
        case FF_RHS_HH_RING: return (dim == 5 || dim == 15) ? 14 : -1;
    }
    return -1;
}

ff_status check_system(const ff_system_s* sys) {
    if (!sys) return fail(FF_E_INVALID, "system handle is NULL");
    return FF_OK;
}

ff_status check_batch(const ff_system_s* sys, const ff_batch* b, bool need_state) {
    if (!b) return fail(FF_E_INVALID, "batch is NULL");
    if (b->prec != FF_FP32 && b->prec != FF_FP32_KAHAN && b->prec != FF_FP64)
        return fail(FF_E_INVALID, "batch.prec must be FF_FP32, FF_FP32_KAHAN or FF_FP64");
    if (b->n < 0) return fail(FF_E_INVALID, "batch.n < 0");
    if (b->ld < b->n) return fail(FF_E_INVALID, "batch.ld < batch.n");
    if (b->ld > 0 && (int64_t)sys->dim > INT64_MAX / b->ld)
        return fail(FF_E_INVALID, "dim * ld overflows");
    if (b->n_pp < 0 || b->n_pp > FF_MAX_PP)
        return fail(FF_E_INVALID, "batch.n_pp must be in [0, FF_MAX_PP]");
    for (int k = 0; k < b->n_pp; ++k)
        if (b->pp_slot[k] < 0 || b->pp_slot[k] >= sys->n_params)
            return fail(FF_E_INVALID, "batch.pp_slot[" + std::to_string(k) + "] = " +
                                          std::to_string(b->pp_slot[k]) + " is not a parameter index");
    for (int k = 0; k < b->n_pp; ++k)
        for (int l = 0; l < k; ++l)
            if (b->pp_slot[k] == b->pp_slot[l])
                return fail(FF_E_INVALID, "batch.pp_slot repeats parameter " + std::to_string(b->pp_slot[k]));
    if (b->n > 0) {
        if (need_state && !b->state) return fail(FF_E_INVALID, "batch.state is NULL");
        if (b->n_pp > 0 && !b->pparams) return fail(FF_E_INVALID, "batch.pparams is NULL but n_pp > 0");
        if (need_state && b->prec == FF_FP32_KAHAN && !b->comp)
            return fail(FF_E_INVALID, "FF_FP32_KAHAN needs batch.comp");
    }
    return FF_OK;
}

ff_status check_tuning(const ff_system_s* sys, const ff_tuning* t) {
    if (!t) return FF_OK;
    if (t->steps_per_launch < 1) return fail(FF_E_INVALID, "tuning.steps_per_launch < 1");
    if (t->particles_per_thread != 1 && t->particles_per_thread != 2 && t->particles_per_thread != 4)
        return fail(FF_E_INVALID, "tuning.particles_per_thread must be 1, 2 or 4");
    if (t->block < 64 || t->block > 256 || t->block % 64 != 0)
        return fail(FF_E_INVALID, "tuning.block must be 64, 128, 192 or 256");
    (void)sys;
    return FF_OK;
}

ff_tuning default_tuning(const ff_system_s* sys, int prec, int64_t nsteps) {
    ff_tuning t;
    t.steps_per_launch = (int32_t)(nsteps < 4096 ? (nsteps > 0 ? nsteps : 1) : 4096);
    t.block = 256;
    t.particles_per_thread = 1;
    if (sys->rhs == FF_RHS_HH_RING) t.block = 128;
    // Two particles per thread where a sweep of particles per thread x block
    // on gfx950 found it faster: Wilson-Cowan with the compensated update
    // (3.6%) and Lorenz in FP32 (0.7%).  Plain FP32 Wilson-Cowan is 5% slower
    // with two; FP64 and the Hodgkin-Huxley ring gain nothing.
    if ((sys->rhs == FF_RHS_WILSON_COWAN && prec == FF_FP32_KAHAN) ||
        (sys->rhs == FF_RHS_LORENZ && prec != FF_FP64))
        t.particles_per_thread = 2;
    return t;
}

RK4Launch make_launch(const ff_system_s* sys, const ff_batch* b, double dt, const ff_tuning* t,
                      hipStream_t stream) {
    RK4Launch L;
    std::memset(&L, 0, sizeof L);
    L.prec = b->prec;
    L.state = b->state;
    L.comp = b->comp;
    L.pp = b->pparams;
    L.n = b->n;
    L.ld = b->ld;
    L.n_pp = b->n_pp;
    for (int k = 0; k < kMaxPP; ++k) L.slot[k] = k < b->n_pp ? b->pp_slot[k] : -1;
    for (int q = 0; q < kMaxParams; ++q) L.p.v[q] = q < sys->n_params ? sys->params[q] : 0.0;
    if (b->prec == FF_FP64) {
        L.h = dt;
        L.h2 = dt * 0.5;
        L.h6 = dt / 6.0;
    } else {
        const float h = (float)dt;
        const float h2 = h * 0.5f;
        const float h6 = h / 6.0f;
        L.h = h;
        L.h2 = h2;
        L.h6 = h6;
    }
    L.ppt = t->particles_per_thread;
    L.block = t->block;
    L.stream = stream;
    return L;
}

hipError_t launch_rk4(const ff_system_s* sys, const RK4Launch& L) {
    switch (sys->rhs) {
        case FF_RHS_LINEAR: return launch_rk4_linear(sys->dim, L);
        case FF_RHS_LORENZ: return launch_rk4_lorenz(L);
        case FF_RHS_WILSON_COWAN: return launch_rk4_wc(L);
        case FF_RHS_HH_RING: return launch_rk4_hh(sys->dim / 5, L);
        case FF_RHS_EXPR: return launch_rk4_expr(sys, L);
    }
    return hipErrorInvalidValue;
}

}  // namespace ff

using namespace ff;

extern "C" {

int32_t ff_abi_version(void) { return FF_ABI_VERSION; }

const char* ff_last_error(void) { return g_error.c_str(); }

ff_status ff_system_create(int32_t rhs, int32_t dim, int32_t n_params, const double* params,
                           ff_system_t* out) {
    g_error.clear();
    if (!out) return fail(FF_E_INVALID, "out is NULL");
    *out = nullptr;
    const int want = expected_params(rhs, dim);
    if (want < 0) {
        if (rhs == FF_RHS_EXPR) return fail(FF_E_INVALID, "expression systems are made by ff_system_create_expr");
        if (rhs < 0 || rhs > FF_RHS_HH_RING) return fail(FF_E_INVALID, "unknown right-hand side");
        if (rhs == FF_RHS_HH_RING && dim > 0 && dim % 5 == 0)
            return fail(FF_E_UNSUPPORTED, "Hodgkin-Huxley ring: this build has 1 or 3 neurons (dim 5 or 15)");
        return fail(FF_E_INVALID, "dimension " + std::to_string(dim) + " does not fit the right-hand side");
    }
    if (n_params != want)
        return fail(FF_E_INVALID, "right-hand side expects " + std::to_string(want) + " parameters, got " +
                                      std::to_string(n_params));
    if (!params) return fail(FF_E_INVALID, "params is NULL");
    ff_system_s* s = new (std::nothrow) ff_system_s;
    if (!s) return fail(FF_E_NOMEM, "out of host memory");
    s->rhs = rhs;
    s->dim = dim;
    s->n_params = n_params;
    for (int q = 0; q < kMaxParams; ++q) s->params[q] = q < n_params ? params[q] : 0.0;
    *out = s;
    return FF_OK;
}

ff_status ff_system_destroy(ff_system_t sys) {
    g_error.clear();
    if (sys) expr_destroy(sys->expr);
    delete sys;
    return FF_OK;
}

ff_status ff_system_set_params(ff_system_t sys, const double* params, int32_t n_params) {
    g_error.clear();
    if (ff_status s = check_system(sys)) return s;
    if (!params) return fail(FF_E_INVALID, "params is NULL");
    if (n_params != sys->n_params) return fail(FF_E_INVALID, "wrong parameter count");
    for (int q = 0; q < n_params; ++q) sys->params[q] = params[q];
    return FF_OK;
}

ff_status ff_system_get_params(ff_system_t sys, double* params, int32_t n_params) {
    g_error.clear();
    if (ff_status s = check_system(sys)) return s;
    if (!params) return fail(FF_E_INVALID, "params is NULL");
    if (n_params != sys->n_params) return fail(FF_E_INVALID, "wrong parameter count");
    for (int q = 0; q < n_params; ++q) params[q] = sys->params[q];
    return FF_OK;
}

ff_status ff_system_info(ff_system_t sys, int32_t* rhs, int32_t* dim, int32_t* n_params) {
    g_error.clear();
    if (ff_status s = check_system(sys)) return s;
    if (rhs) *rhs = sys->rhs;
    if (dim) *dim = sys->dim;
    if (n_params) *n_params = sys->n_params;
    return FF_OK;
}

ff_status ff_integrate(ff_system_t sys, const ff_batch* b, double dt_signed, int64_t nsteps,
                       const ff_tuning* tuning, void* stream) {
    g_error.clear();
    if (ff_status s = check_system(sys)) return s;
    if (ff_status s = check_batch(sys, b, true)) return s;
    if (ff_status s = check_tuning(sys, tuning)) return s;
    if (nsteps < 0) return fail(FF_E_INVALID, "nsteps < 0");
    if (!std::isfinite(dt_signed)) return fail(FF_E_INVALID, "dt_signed is not finite");
    if (b->n == 0 || nsteps == 0 || dt_signed == 0.0) return FF_OK;
    if (sys->expr) {
        if (ff_status s = expr_prepare(sys, b->prec, kExprForward)) return s;
    }
    const ff_tuning t = tuning ? *tuning : default_tuning(sys, b->prec, nsteps);
    RK4Launch L = make_launch(sys, b, dt_signed, &t, (hipStream_t)stream);
    for (int64_t done = 0; done < nsteps;) {
        L.steps = nsteps - done < t.steps_per_launch ? nsteps - done : t.steps_per_launch;
        const hipError_t e = launch_rk4(sys, L);
        if (e != hipSuccess) return device_fail(e, "ff_integrate launch");
        done += L.steps;
    }
    return FF_OK;
}

}  // extern "C"

namespace ff {
namespace {
// The smallest float >= b and the largest float <= b (b not NaN): a float
// state compared with them decides exactly as the double comparison would.
float float_at_or_above(double b) {
    if (b > FLT_MAX) return INFINITY;
    if (b < -FLT_MAX) return std::isinf(b) ? -INFINITY : -FLT_MAX;
    const float f = (float)b;  // nearest; in range here
    return (double)f < b ? std::nextafter(f, INFINITY) : f;
}
float float_at_or_below(double b) {
    if (b < -FLT_MAX) return -INFINITY;
    if (b > FLT_MAX) return std::isinf(b) ? INFINITY : FLT_MAX;
    const float f = (float)b;
    return (double)f > b ? std::nextafter(f, -INFINITY) : f;
}

ff_status fill_reset(const ff_system_s* sys, const ff_batch* b, const ff_reset* reset, ResetArgs* r) {
    if (!reset->bound_lo || !reset->bound_hi || !reset->box_lo || !reset->box_hi)
        return fail(FF_E_INVALID, "reset bounds and box must be given");
    if (sys->dim > kMaxDim) return fail(FF_E_UNSUPPORTED, "reset supports up to 15 state variables");
    for (int d = 0; d < sys->dim; ++d) {
        const double bl = reset->bound_lo[d], bh = reset->bound_hi[d], xl = reset->box_lo[d], xh = reset->box_hi[d];
        if (std::isnan(bl) || std::isnan(bh) || !(bl <= bh)) return fail(FF_E_INVALID, "reset bounds need lo <= hi");
        if (!std::isfinite(xl) || !std::isfinite(xh) || !(xl < xh))
            return fail(FF_E_INVALID, "reset box must be finite with lo < hi");
    }
    if (b->n > 0 && (!reset->age || !reset->n_resets)) return fail(FF_E_INVALID, "reset age / n_resets are NULL");
    std::memset(r, 0, sizeof *r);
    for (int d = 0; d < sys->dim; ++d) {
        r->blo[d] = reset->bound_lo[d];
        r->bhi[d] = reset->bound_hi[d];
        r->blf[d] = float_at_or_above(r->blo[d]);
        r->bhf[d] = float_at_or_below(r->bhi[d]);
        r->wd[d] = reset->box_hi[d] - reset->box_lo[d];
        r->lod[d] = reset->box_lo[d];
        r->wf[d] = (float)r->wd[d];
        r->lof[d] = (float)reset->box_lo[d];
    }
    r->max_age = reset->max_age;
    r->seed = reset->seed;
    r->id_offset = reset->id_offset;
    r->age = reset->age;
    r->nres = reset->n_resets;
    return FF_OK;
}

ff_status run_steps(const ff_system_s* sys, RK4Launch& L, int64_t nsteps, int64_t per_launch, const char* what) {
    for (int64_t done = 0; done < nsteps;) {
        L.steps = nsteps - done < per_launch ? nsteps - done : per_launch;
        if (L.record) L.record->step0 = done;
        const hipError_t e = launch_rk4(sys, L);
        if (e != hipSuccess) return device_fail(e, what);
        done += L.steps;
    }
    return FF_OK;
}
}  // namespace
}  // namespace ff

extern "C" ff_status ff_integrate_reset(ff_system_t sys, const ff_batch* b, double dt_signed, int64_t nsteps,
                                        const ff_reset* reset, const ff_tuning* tuning, void* stream) {
    g_error.clear();
    if (ff_status s = check_system(sys)) return s;
    if (ff_status s = check_batch(sys, b, true)) return s;
    if (ff_status s = check_tuning(sys, tuning)) return s;
    if (nsteps < 0) return fail(FF_E_INVALID, "nsteps < 0");
    if (!std::isfinite(dt_signed)) return fail(FF_E_INVALID, "dt_signed is not finite");
    if (!reset) return fail(FF_E_INVALID, "reset is NULL");
    ResetArgs r;
    if (ff_status s = fill_reset(sys, b, reset, &r)) return s;
    if (b->n == 0 || nsteps == 0 || dt_signed == 0.0) return FF_OK;
    if (sys->expr) {
        if (ff_status s = expr_prepare(sys, b->prec, kExprForward)) return s;
    }
    const ff_tuning t = tuning ? *tuning : default_tuning(sys, b->prec, nsteps);
    RK4Launch L = make_launch(sys, b, dt_signed, &t, (hipStream_t)stream);
    L.reset = &r;
    return run_steps(sys, L, nsteps, t.steps_per_launch, "ff_integrate_reset launch");
}

extern "C" ff_status ff_integrate_record(ff_system_t sys, const ff_batch* b, double dt_signed, int64_t nsteps,
                                         int64_t every, int64_t stride, void* out, const ff_reset* reset,
                                         const ff_tuning* tuning, void* stream) {
    g_error.clear();
    if (ff_status s = check_system(sys)) return s;
    if (ff_status s = check_batch(sys, b, true)) return s;
    if (ff_status s = check_tuning(sys, tuning)) return s;
    if (nsteps < 0) return fail(FF_E_INVALID, "nsteps < 0");
    if (!std::isfinite(dt_signed)) return fail(FF_E_INVALID, "dt_signed is not finite");
    if (every < 1 || stride < 1) return fail(FF_E_INVALID, "every and stride must be >= 1");
    if (b->n > 0 && nsteps >= every && !out) return fail(FF_E_INVALID, "out is NULL");
    ResetArgs r;
    if (reset) {
        if (ff_status s = fill_reset(sys, b, reset, &r)) return s;
    }
    if (b->n == 0 || nsteps == 0 || dt_signed == 0.0) return FF_OK;
    if (sys->expr) {
        if (ff_status s = expr_prepare(sys, b->prec, kExprForward)) return s;
    }
    const ff_tuning t = tuning ? *tuning : default_tuning(sys, b->prec, nsteps);
    RK4Launch L = make_launch(sys, b, dt_signed, &t, (hipStream_t)stream);
    RecordArgs rc;
    rc.out = out;
    rc.every = every;
    rc.stride = stride;
    rc.m = (b->n + stride - 1) / stride;
    rc.step0 = 0;
    L.reset = reset ? &r : nullptr;
    L.record = &rc;
    return run_steps(sys, L, nsteps, t.steps_per_launch, "ff_integrate_record launch");
}
