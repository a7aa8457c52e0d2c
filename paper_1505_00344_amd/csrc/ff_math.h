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
    static __device__ __forceinline__ double expm1_(double x) { return expm1(x); }

    // Kernels of exp and expm1 for arguments a caller has checked (they leave
    // out the library functions' handling of extreme arguments): Cody and
    // Waite's argument reduction x = n ln2 + r, n = rint(x log2 e),
    // |r| <= ln2/2 (ln 2 split into a double and its remainder), a polynomial
    // in r, and 2^n by ldexp.  The polynomials are Chebyshev interpolants on
    // [-0.3466, 0.3466] computed in 60-digit arithmetic and rounded to
    // double: degree 11 for e^r (Horner), degree 10 for
    // g(r) = (e^r - 1 - r)/r^2, so that e^r - 1 = r + r^2 g(r) has no
    // cancellation near 0.  expm1 adds 2^n - 1 and 2^n r_hi
    // (r_hi = x - n ln2_hi, exact for |n| = 1) as a Fast2Sum, then the small
    // terms, so that n = +-1 does not amplify the rounding of r.  Valid (IEEE
    // results, gradual underflow included) for |x| <= 708; measured against
    // long-double references on 4M points each of [-700, 700], [-1, 1] and
    // [-1e-3, 1e-3]: exp_k within 0.94 ulp (mean 0.26), expm1_k within 1.10
    // ulp (mean 0.13-0.25).
    static constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;   // ln 2 rounded
    static constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;  // ln 2 - kLn2Hi
    static constexpr double kLog2E = 1.4426950408889634074;
    static __device__ __forceinline__ double exp_k(double x) {
        const double n = __builtin_rint(x * kLog2E);
        const double r = __builtin_fma(-n, kLn2Lo, __builtin_fma(-n, kLn2Hi, x));
        double p = 0x1.af6326f3df789p-26;
        p = __builtin_fma(p, r, 0x1.28b40d95cf927p-22);
        p = __builtin_fma(p, r, 0x1.71ddf56f3c074p-19);
        p = __builtin_fma(p, r, 0x1.a01991a3c8c2ep-16);
        p = __builtin_fma(p, r, 0x1.a01a01b1457b9p-13);
        p = __builtin_fma(p, r, 0x1.6c16c187ff24ap-10);
        p = __builtin_fma(p, r, 0x1.111111110f220p-7);
        p = __builtin_fma(p, r, 0x1.555555554f0bfp-5);
        p = __builtin_fma(p, r, 0x1.555555555555ap-3);
        p = __builtin_fma(p, r, 0x1.0000000000011p-1);
        p = __builtin_fma(p, r, 1.0);
        p = __builtin_fma(p, r, 1.0);
        return __builtin_ldexp(p, (int)n);
    }
    static __device__ __forceinline__ double expm1_k(double x) {
        const double n = __builtin_rint(x * kLog2E);
        const double rh = __builtin_fma(-n, kLn2Hi, x);
        const double rl = -n * kLn2Lo;
        const double r = rh + rl;
        double g = 0x1.1f7301a8efa5cp-29;
        g = __builtin_fma(g, r, 0x1.af4de6a36d4fcp-26);
        g = __builtin_fma(g, r, 0x1.27e4db653346ep-22);
        g = __builtin_fma(g, r, 0x1.71de0232f4775p-19);
        g = __builtin_fma(g, r, 0x1.a01a01a6d84aap-16);
        g = __builtin_fma(g, r, 0x1.a01a01abe78f9p-13);
        g = __builtin_fma(g, r, 0x1.6c16c16c162d5p-10);
        g = __builtin_fma(g, r, 0x1.11111111100dcp-7);
        g = __builtin_fma(g, r, 0x1.5555555555556p-5);
        g = __builtin_fma(g, r, 0x1.5555555555557p-3);
        g = __builtin_fma(g, r, 0.5);
        const double s = __builtin_ldexp(1.0, (int)n), sm1 = s - 1.0;
        const double a = __builtin_fma(s, rh, sm1);             // (2^n - 1) + 2^n r_hi, rounded
        const double e = __builtin_fma(s, rh, -(a - sm1));      // its rounding error, exactly
        return a + __builtin_fma(s, __builtin_fma(r * r, g, rl), e);
    }
    // 2^t by the same method in base 2: t = n + f with n = rint(t) and
    // |f| <= 1/2, a reduction that is exact (no split constant), then the
    // degree-11 Chebyshev interpolant of 2^f on [-1/2, 1/2] (computed in
    // 60-digit arithmetic, rounded to double) and ldexp.  For |t| <= 2^31
    // (callers clamp their arguments far inside that); measured against
    // long-double references on 4M points each of [-1000, 1000], [-30, 30],
    // [-1, 1] and [-1e-3, 1e-3]: within 0.89 ulp (mean 0.26).
    static __device__ __forceinline__ double exp2_k(double t) {
        const double n = __builtin_rint(t);
        const double f = t - n;
        double p = 0x1.e9ec1fcb69a7fp-32;
        p = __builtin_fma(p, f, 0x1.e6228acd1c6e5p-28);
        p = __builtin_fma(p, f, 0x1.b524ebd13a55fp-24);
        p = __builtin_fma(p, f, 0x1.62bfc2c86d700p-20);
        p = __builtin_fma(p, f, 0x1.ffcbfc6da6ed1p-17);
        p = __builtin_fma(p, f, 0x1.430913112c61bp-13);
        p = __builtin_fma(p, f, 0x1.5d87fe78a3f9cp-10);
        p = __builtin_fma(p, f, 0x1.3b2ab6fb9f1a5p-7);
        p = __builtin_fma(p, f, 0x1.c6b08d704a0c6p-5);
        p = __builtin_fma(p, f, 0x1.ebfbdff82c5aep-3);
        p = __builtin_fma(p, f, 0x1.62e42fefa39efp-1);
        p = __builtin_fma(p, f, 1.0);
        return __builtin_ldexp(p, (int)n);
    }
    // 1/x: the hardware estimate r0 = v_rcp_f64(x) refined by one
    // third-order step: with e = 1 - x r0 (one fma, exact up to its
    // rounding), 1/x = r0/(1 - e) = r0 (1 + e + e^2 + ...), taken as
    // r0 + r0 (e + e^2); the estimate's |e| is below about 2^-25, so the
    // truncated e^3 term is below 2^-75 and the result is within 1 ulp
    // (measured on the device: correctly rounded on 1M points over the
    // exponent range).  Three fmas, where two Newton steps take four.
    static __device__ __forceinline__ double refine_(double x, double r0) {
        const double e = __builtin_fma(-x, r0, 1.0);
        return __builtin_fma(r0, __builtin_fma(e, e, e), r0);
    }
    // Where the estimate is +-0 or +-inf (x infinite or zero, or
    // |x| < 2^-1024 so that 1/x overflows) it is IEEE's 1/x and is returned as
    // it is, since the refinement would turn it into NaN; every other x,
    // subnormal ones included, takes the refined value.
    static constexpr int kZeroInf = (1 << 2) | (1 << 5) | (1 << 6) | (1 << 9);
    static __device__ __forceinline__ double rcp_(double x) {
        const double r0 = __builtin_amdgcn_rcp(x);
        const double r = refine_(x, r0);
        return __builtin_amdgcn_class(r0, kZeroInf) ? r0 : r;
    }
    // a/b: a times that reciprocal with one residual correction (within
    // 1 ulp).  Where the estimate is +-0 or +-inf the result is a times it:
    // IEEE's a/b for b zero or infinite, and for |b| < 2^-1024 unless |a|
    // is small enough for a/b to be finite (then +-inf or NaN instead).
    static __device__ __forceinline__ double div_(double a, double b) {
        const double r0 = __builtin_amdgcn_rcp(b);
        const double r = refine_(b, r0);
        const double q = a * r;
        const double qc = __builtin_fma(__builtin_fma(-b, q, a), r, q);
        return __builtin_amdgcn_class(r0, kZeroInf) ? a * r0 : qc;
    }
    // rcp_ and div_ without the fallback, for divisors whose estimate is
    // finite and nonzero (|x| between about 2^-1022 and 2^1022): the same
    // values bit for bit
    static __device__ __forceinline__ double rcp_k(double x) { return refine_(x, __builtin_amdgcn_rcp(x)); }
    static __device__ __forceinline__ double div_k(double a, double b) {
        const double r = rcp_k(b);
        const double q = a * r;
        return __builtin_fma(__builtin_fma(-b, q, a), r, q);
    }
};
// Single precision.  By default (FF_FAST_F32 = 1) the exponential is the
// hardware 2^x (v_exp_f32) with log2(e) folded into the argument's scale, and
// reciprocals/divisions use v_rcp_f32 (each about 1 ulp); expm1 stays the
// library function because psi(u) near u = 0 needs it.  FF_FAST_F32 = 0 uses
// the library expf and correctly rounded division instead.  In double
// precision the built-in right-hand sides use the kernels above on clamped
// arguments, and the refined reciprocal with its fallback where the divisor
// is a parameter (1/C).
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
    static __device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float div_(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
#else
    static __device__ __forceinline__ float exp_(float x) { return expf(x); }
    static __device__ __forceinline__ float exp2_(float x) { return exp2f(x); }
    static __device__ __forceinline__ float rcp_(float x) { return 1.0f / x; }
    static __device__ __forceinline__ float div_(float a, float b) { return a / b; }
#endif
    static __device__ __forceinline__ float expm1_(float x) { return expm1f(x); }
};

}  // namespace ff
