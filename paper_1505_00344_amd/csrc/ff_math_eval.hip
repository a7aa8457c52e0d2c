// ff_math_eval.hip — the double-precision elementary kernels of the built-in
// right-hand sides (M<double> in ff_math.h, the clamped logistics and psi of
// ff_rhs.h) evaluated elementwise, so that their accuracy can be measured on
// the device against an independent reference.
#include "ff_internal.h"
#include "ff_rhs.h"

namespace ff {
namespace {

constexpr int kMathBlock = 256;

__global__ void __launch_bounds__(kMathBlock)
k_math_eval(int fn, const double* __restrict__ x, double* __restrict__ y, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v = x[i];
        double r;
        switch (fn) {
            case FF_MATH_EXP: r = M<double>::exp_k(v); break;
            case FF_MATH_EXP2: r = M<double>::exp2_k(v); break;
            case FF_MATH_EXPM1: r = M<double>::expm1_k(v); break;
            case FF_MATH_RCP: r = M<double>::rcp_k(v); break;
            case FF_MATH_LOGISTIC: r = logistic_k<true>(v); break;
            case FF_MATH_LOGISTIC2: r = logistic2_k<true>(v); break;
            default: r = hh_psi<double>(v); break;
        }
        y[i] = r;
    }
}

}  // namespace
}  // namespace ff

using namespace ff;

extern "C" ff_status ff_math_eval(int32_t fn, const double* x, double* y, int64_t n, void* stream) {
    set_error("");
    if (fn < FF_MATH_EXP || fn > FF_MATH_PSI) return fail(FF_E_INVALID, "unknown ff_math function");
    if (n < 0) return fail(FF_E_INVALID, "n < 0");
    if (n == 0) return FF_OK;
    if (!x || !y) return fail(FF_E_INVALID, "x or y is NULL");
    const int64_t blocks = (n + kMathBlock - 1) / kMathBlock;
    const unsigned grid = (unsigned)(blocks < 8192 ? blocks : 8192);
    hipLaunchKernelGGL(k_math_eval, dim3(grid), dim3(kMathBlock), 0, (hipStream_t)stream, (int)fn, x, y, n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FF_OK : device_fail(e, "ff_math_eval");
}
