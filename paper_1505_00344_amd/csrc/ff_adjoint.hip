// ff_adjoint.hip — C ABI of the checkpointed forward pass and the discrete
// adjoint (see ff_adjoint.h for the kernel).
//
// Workspace layout (each region 256-byte aligned; n = batch.n, D = dim):
//   ckpt   [nseg][D][n]  state at the start of every K-step segment
//   ckpt_c [nseg][D][n]  its Kahan compensation (FF_FP32_KAHAN only)
//   sub    [nsub][D][n]  sub-checkpoints inside one segment (T steps apart)
//   sub_c  [nsub][D][n]  their compensation (FF_FP32_KAHAN only)
//   carry  [NP][n]       per-particle adjoints of every parameter, carried
//                        from one segment to the next (so the result does
//                        not depend on K)
//   mu_part [nblk][16]   FP64 per-block sums of the parameter adjoints
// with nseg = ceil(nsteps / K), nsub = ceil(min(K, nsteps) / T) and
// nblk = ceil(n / 256).
#include <cmath>
#include <cstring>
#include <string>

#include "ff_internal.h"

namespace ff {

// The 15-variable ring (and expression systems of more than four variables)
// keep one step on the tape and recompute stage points (LOWREG); the small
// systems keep eight, Lorenz in double precision four (it also keeps every
// tape state's stage points; the launcher in k_adj_lorenz.hip must agree).
int adj_tape_len(const ff_system_s* sys, int prec) {
    if (sys->rhs == FF_RHS_HH_RING) return 1;
    if (sys->rhs == FF_RHS_EXPR) return sys->dim <= 4 ? 8 : 1;
    if (sys->rhs == FF_RHS_LORENZ && prec == FF_FP64) return 4;
    return 8;
}

namespace {

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct AdjLayout {
    size_t ckpt, ckpt_c, sub, sub_c, carry, mu_part, total;
    int64_t nseg, nsub, nblk;
};

AdjLayout adj_layout(const ff_system_s* sys, const ff_batch* b, int64_t nsteps, int32_t K) {
    AdjLayout L{};
    const size_t esz = prec_size(b->prec);
    const bool kahan = b->prec == FF_FP32_KAHAN;
    const int64_t T = adj_tape_len(sys, b->prec);
    L.nseg = nsteps > 0 ? (nsteps + K - 1) / K : 0;
    const int64_t seg = nsteps < K ? nsteps : K;
    L.nsub = seg > 0 ? (seg + T - 1) / T : 0;
    L.nblk = (b->n + kAdjBlock - 1) / kAdjBlock;
    const size_t st = (size_t)sys->dim * (size_t)b->n * esz;
    size_t off = 0;
    L.ckpt = off;
    off += al((size_t)L.nseg * st);
    L.ckpt_c = off;
    if (kahan) off += al((size_t)L.nseg * st);
    L.sub = off;
    off += al((size_t)L.nsub * st);
    L.sub_c = off;
    if (kahan) off += al((size_t)L.nsub * st);
    L.carry = off;
    off += al((size_t)sys->n_params * (size_t)b->n * esz);
    L.mu_part = off;
    off += al((size_t)L.nblk * kMaxParams * sizeof(double));
    L.total = off;
    return L;
}

__global__ void k_zero(void* p, int64_t bytes) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < bytes) static_cast<unsigned char*>(p)[i] = 0;
}

// mu_global[q] = sum over blocks of mu_part[b][q]: strided partial sums then
// a fixed-shape tree, so the result does not depend on scheduling.
__global__ void __launch_bounds__(256) k_reduce_mu(const double* mu_part, int64_t nblk, double* out) {
    __shared__ double s[256];
    const int q = blockIdx.x;
    double v = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += 256) v += mu_part[b * kMaxParams + q];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = s[0];
}

hipError_t zero_async(void* p, int64_t bytes, hipStream_t st) {
    if (!p || bytes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((bytes + 255) / 256)), dim3(256), 0, st, p, bytes);
    return hipGetLastError();
}

ff_status check_adj_args(const ff_system_s* sys, const ff_batch* b, double dt, int64_t nsteps, int32_t K) {
    if (ff_status s = check_system(sys)) return s;
    if (ff_status s = check_batch(sys, b, false)) return s;
    if (nsteps < 0) return fail(FF_E_INVALID, "nsteps < 0");
    if (K < 1) return fail(FF_E_INVALID, "K must be >= 1");
    if (!std::isfinite(dt)) return fail(FF_E_INVALID, "dt_signed is not finite");
    return FF_OK;
}

}  // namespace

}  // namespace ff

using namespace ff;

extern "C" {

ff_status ff_adjoint_workspace_size(ff_system_t sys, const ff_batch* b, int64_t nsteps, int32_t K,
                                    size_t* bytes) {
    set_error("");
    if (ff_status s = check_adj_args(sys, b, 0.0, nsteps, K)) return s;
    if (!bytes) return fail(FF_E_INVALID, "bytes is NULL");
    *bytes = adj_layout(sys, b, nsteps, K).total;
    return FF_OK;
}

ff_status ff_integrate_checkpointed(ff_system_t sys, const ff_batch* b, double dt_signed, int64_t nsteps,
                                    int32_t K, void* workspace, size_t workspace_bytes, void* stream) {
    set_error("");
    if (ff_status s = check_adj_args(sys, b, dt_signed, nsteps, K)) return s;
    if (ff_status s = check_batch(sys, b, true)) return s;
    if (b->n == 0 || nsteps == 0 || dt_signed == 0.0) return FF_OK;
    const AdjLayout W = adj_layout(sys, b, nsteps, K);
    if (!workspace || workspace_bytes < W.total)
        return fail(FF_E_NOMEM, "adjoint workspace too small: need " + std::to_string(W.total) + " bytes");
    if (sys->expr) {
        if (ff_status s = expr_prepare(sys, b->prec, kExprForward)) return s;
    }
    const ff_tuning t = default_tuning(sys, b->prec, K);
    RK4Launch L = make_launch(sys, b, dt_signed, &t, (hipStream_t)stream);
    const size_t st = (size_t)sys->dim * (size_t)b->n * prec_size(b->prec);
    char* ws = (char*)workspace;
    L.ckpt_ld = b->n;
    for (int64_t s = 0; s < W.nseg; ++s) {
        L.ckpt = ws + W.ckpt + (size_t)s * st;
        L.ckpt_c = b->prec == FF_FP32_KAHAN ? ws + W.ckpt_c + (size_t)s * st : nullptr;
        L.steps = (nsteps - s * K) < K ? (nsteps - s * K) : K;
        const hipError_t e = launch_rk4(sys, L);
        if (e != hipSuccess) return device_fail(e, "ff_integrate_checkpointed launch");
    }
    return FF_OK;
}

ff_status ff_adjoint(ff_system_t sys, const ff_batch* b, double dt_signed, int64_t nsteps, int32_t K,
                     void* workspace, size_t workspace_bytes, void* lambda, void* mu, double* mu_global,
                     void* stream) {
    set_error("");
    if (ff_status s = check_adj_args(sys, b, dt_signed, nsteps, K)) return s;
    if (b->n > 0 && !lambda) return fail(FF_E_INVALID, "lambda is NULL");
    if (b->n > 0 && b->n_pp > 0 && !mu) return fail(FF_E_INVALID, "mu is NULL but the batch has per-particle parameters");
    hipStream_t st = (hipStream_t)stream;
    const size_t esz = prec_size(b->prec);
    if (b->n == 0 || nsteps == 0 || dt_signed == 0.0) {
        // identity map: dL/dx(0) = dL/dx(T), parameter gradients vanish
        hipError_t e = hipSuccess;
        if (b->n_pp > 0 && b->n > 0)
            for (int k = 0; k < b->n_pp && e == hipSuccess; ++k)
                e = zero_async((char*)mu + (size_t)k * b->ld * esz, b->n * (int64_t)esz, st);
        if (e == hipSuccess && mu_global) e = zero_async(mu_global, sys->n_params * (int64_t)sizeof(double), st);
        return e == hipSuccess ? FF_OK : device_fail(e, "ff_adjoint");
    }
    const AdjLayout W = adj_layout(sys, b, nsteps, K);
    if (!workspace || workspace_bytes < W.total)
        return fail(FF_E_NOMEM, "adjoint workspace too small: need " + std::to_string(W.total) + " bytes");
    if (sys->expr) {
        if (ff_status s = expr_prepare(sys, b->prec, kExprAdjoint)) return s;
    }
    const ff_tuning t = default_tuning(sys, b->prec, K);
    AdjLaunch A;
    std::memset(&A, 0, sizeof A);
    A.f = make_launch(sys, b, dt_signed, &t, st);
    if (b->prec == FF_FP64) {
        A.h3 = dt_signed / 3.0;
    } else {
        const float h = (float)dt_signed;
        A.h3 = h / 3.0f;
    }
    char* ws = (char*)workspace;
    const size_t stb = (size_t)sys->dim * (size_t)b->n * esz;
    A.sub = ws + W.sub;
    A.sub_c = b->prec == FF_FP32_KAHAN ? ws + W.sub_c : nullptr;
    A.lam = lambda;
    A.mu = mu;
    A.mu_part = (double*)(ws + W.mu_part);
    A.carry = ws + W.carry;
    for (int64_t s = W.nseg - 1; s >= 0; --s) {
        A.ckpt = ws + W.ckpt + (size_t)s * stb;
        A.ckpt_c = b->prec == FF_FP32_KAHAN ? ws + W.ckpt_c + (size_t)s * stb : nullptr;
        A.seg_len = (nsteps - s * K) < K ? (nsteps - s * K) : K;
        A.first = s == W.nseg - 1;
        A.last = s == 0;
        hipError_t e;
        switch (sys->rhs) {
            case FF_RHS_LINEAR: e = launch_adj_linear(sys->dim, A); break;
            case FF_RHS_LORENZ: e = launch_adj_lorenz(A); break;
            case FF_RHS_WILSON_COWAN: e = launch_adj_wc(A); break;
            case FF_RHS_HH_RING: e = launch_adj_hh(sys->dim / 5, A); break;
            case FF_RHS_EXPR: e = launch_adj_expr(sys, A); break;
            default: e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return device_fail(e, "ff_adjoint launch");
    }
    if (mu_global) {
        hipLaunchKernelGGL(k_reduce_mu, dim3(sys->n_params), dim3(256), 0, st, A.mu_part, W.nblk, mu_global);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return device_fail(e, "ff_adjoint reduction");
    }
    return FF_OK;
}

}  // extern "C"
