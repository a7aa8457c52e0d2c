// ff_math.h — working-precision arithmetic used by the device code: fused
// multiply-add and the exponential / reciprocal policy of each precision.
// Compiles both in the library and in the kernels the library builds at run
// time from user expressions (there the HIP headers are implicit).
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

namespace ff {

template <typename R> struct M;
template <> struct M<double> {
    static constexpr bool kFast = false;
    static __device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
    static __device__ __forceinline__ double exp_(double x) { return exp(x); }
    // exp(x * c) for a compile-time constant c: the product is rounded, then exp
    static __device__ __forceinline__ double expc(double x, double c) { return exp(x * c); }
    static __device__ __forceinline__ double expm1_(double x) { return expm1(x); }
    // 1/x: the hardware estimate (v_rcp_f64) refined by two Newton steps,
    // within 1 ulp (not always the correctly rounded quotient, which costs
    // about twice the instructions).  Where the estimate is +-0 or +-inf
    // (x infinite or zero, or |x| < 2^-1024 so that 1/x overflows) it is
    // IEEE's 1/x and is returned as it is, since a Newton step would turn it
    // into NaN; every other x, subnormal ones included, takes the refined
    // value.
    static constexpr int kZeroInf = (1 << 2) | (1 << 5) | (1 << 6) | (1 << 9);
    static __device__ __forceinline__ double rcp_(double x) {
        const double r0 = __builtin_amdgcn_rcp(x);
        double r = __builtin_fma(__builtin_fma(-x, r0, 1.0), r0, r0);
        r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
        return __builtin_amdgcn_class(r0, kZeroInf) ? r0 : r;
    }
    // a/b: a times that reciprocal with one residual correction (within
    // 1 ulp).  Where the estimate is +-0 or +-inf the result is a times it:
    // IEEE's a/b for b zero or infinite, and for |b| < 2^-1024 unless |a|
    // is small enough for a/b to be finite (then +-inf or NaN instead).
    static __device__ __forceinline__ double div_(double a, double b) {
        const double r0 = __builtin_amdgcn_rcp(b);
        double r = __builtin_fma(__builtin_fma(-b, r0, 1.0), r0, r0);
        r = __builtin_fma(__builtin_fma(-b, r, 1.0), r, r);
        const double q = a * r;
        const double qc = __builtin_fma(__builtin_fma(-b, q, a), r, q);
        return __builtin_amdgcn_class(r0, kZeroInf) ? a * r0 : qc;
    }
};
// Single precision.  By default (FF_FAST_F32 = 1) the exponential is the
// hardware 2^x (v_exp_f32) with log2(e) folded into the argument's scale, and
// reciprocals/divisions use v_rcp_f32 (each about 1 ulp); expm1 stays the
// library function because psi(u) near u = 0 needs it.  FF_FAST_F32 = 0 uses
// the library expf and correctly rounded division instead.  Double precision
// uses the library exp/expm1 and a Newton-refined reciprocal (below).
#ifndef FF_FAST_F32
#define FF_FAST_F32 1
#endif
constexpr double kLog2e = 1.4426950408889634074;
template <> struct M<float> {
    static constexpr bool kFast = FF_FAST_F32 != 0;
    static __device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
#if FF_FAST_F32
    static __device__ __forceinline__ float exp_(float x) { return __builtin_amdgcn_exp2f(x * (float)kLog2e); }
    static __device__ __forceinline__ float exp2_(float x) { return __builtin_amdgcn_exp2f(x); }
    static __device__ __forceinline__ float expc(float x, double c) { return __builtin_amdgcn_exp2f(x * (float)(c * kLog2e)); }
    static __device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float div_(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
#else
    static __device__ __forceinline__ float exp_(float x) { return expf(x); }
    static __device__ __forceinline__ float exp2_(float x) { return exp2f(x); }
    static __device__ __forceinline__ float expc(float x, double c) { return expf(x * (float)c); }
    static __device__ __forceinline__ float rcp_(float x) { return 1.0f / x; }
    static __device__ __forceinline__ float div_(float a, float b) { return a / b; }
#endif
    static __device__ __forceinline__ float expm1_(float x) { return expm1f(x); }
};

}  // namespace ff
