// ff_rhs.h — device right-hand sides of the particle systems, and their
// vector-Jacobian products, for the gfx950 kernels.
//
// Each system is a struct template over the working precision R with
//   D   number of state components,  NP  number of parameters,
//   UNROLL  RK4 steps per trip of the fused kernel's step loop,
//   FUSED_INC  nonzero: the compensated update forms inc - c as one fma
//           (systems evaluated with the fast single-precision functions,
//           which leave the canonical order anyway),
//   NQ  number of constants derived from the parameters once per particle,
//   derive(p, q)                 fill q from p,
//   f(p, q, x, out)              the right-hand side (autonomous: no t),
//   vjp(p, q, x, a, gx, gp)      gx += J(x)^T a, gp += (df/dp)^T a.
// Parameters live in a per-particle register array p[NP] (global values with
// per-particle overrides already applied).
//
// Evaluation order is fixed (explicit fma(), compiled with
// -ffp-contract=off).  The canonical orders below are the ones a CPU
// evaluation of the formulas follows; Lorenz and linear FP64 runs reproduce
// it operation for operation, HH FP64 keeps its order with the exp/expm1
// kernels of M<double>, and the Wilson-Cowan sigmoids fold their gain in
// double and fast single precision (WilsonCowan below):
//   Lorenz:  fx = s*(y - x); fy = fma(x, r - z, -y); fz = fma(x, y, -(b*z))
//   WC:      u = fma(c1, E, fma(-c2, I, P)); S = 1/(1 + exp(-(a*(u - th))))
//   HH:      rates with multiplications by the doubles nearest -1/10, -1/18,
//            -1/20, -1/80; membrane sum ((((IL + INa) + IK) + Isyn) + Iext)*(1/C)
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ff_math.h"

namespace ff {

// Double precision evaluates the exponentials and reciprocals of the built-in
// right-hand sides with the kernels of M<double> (no branches, so no result
// depends on the other particles of a wave).  Their arguments are clamped
// where the function is flat anyway, so that the kernels never see an
// argument outside their range on any trajectory, however far it escapes.

// 1/(1 + e^z) from the exp and reciprocal kernels.  z is clamped to
// [-700, 700] first: beyond it the logistic is 0 or 1 to within 1e-304
// (e^-700 = 9.9e-305), and inside it 1 + e^z is finite and its reciprocal
// normal, so the kernels need no fallback.  The clamp (IEEE max and min)
// turns a NaN argument into a bound; with KEEP_NAN the result is
// fma(0, z, S), which is S for every finite z and NaN when z is NaN or
// infinite, so that a NaN argument reaches the result (an infinite z, from an
// infinite state or one within a factor ~16 of overflow, then gives NaN
// instead of 0 or 1); without it a NaN z gives a finite result, for callers
// whose NaN z implies a NaN state component anyway.
template <bool KEEP_NAN>
__device__ __forceinline__ double logistic_k(double z) {
    const double zc = __builtin_fmin(__builtin_fmax(z, -700.0), 700.0);
    const double s = M<double>::rcp_k(1.0 + M<double>::exp_k(zc));
    return KEEP_NAN ? __builtin_fma(0.0, z, s) : s;
}

// 1/(1 + 2^t), the same in base 2 for arguments that already carry the
// factor log2(e): t clamped to [-1000, 1000] (2^-1000 = 9.3e-302).
template <bool KEEP_NAN>
__device__ __forceinline__ double logistic2_k(double t) {
    const double tc = __builtin_fmin(__builtin_fmax(t, -1000.0), 1000.0);
    const double s = M<double>::rcp_k(1.0 + M<double>::exp2_k(tc));
    return KEEP_NAN ? __builtin_fma(0.0, t, s) : s;
}

template <typename R> constexpr bool kHasKernels = std::is_same<R, double>::value;

// ---------------------------------------------------------------- linear
// x' = A x with A row-major in p (Dm <= 4); the acc starts with column 0.
template <typename R, int Dm> struct Linear {
    static constexpr int D = Dm, NP = Dm * Dm, NQ = 1, UNROLL = 2, FUSED_INC = 0;
    static __device__ __forceinline__ void derive(const R (&)[NP], R (&q)[NQ]) { q[0] = R(0); }
    static __device__ __forceinline__ void f(const R (&p)[NP], const R (&)[NQ], const R (&x)[D], R (&o)[D]) {
#pragma unroll
        for (int r = 0; r < D; ++r) {
            R acc = p[r * D] * x[0];
#pragma unroll
            for (int c = 1; c < D; ++c) acc = M<R>::fma_(p[r * D + c], x[c], acc);
            o[r] = acc;
        }
    }
    static __device__ __forceinline__ void vjp(const R (&p)[NP], const R (&)[NQ], const R (&x)[D],
                                               const R (&a)[D], R (&gx)[D], R (&gp)[NP]) {
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) {
                gx[c] += p[r * D + c] * a[r];
                gp[r * D + c] += x[c] * a[r];
            }
    }
};

// ---------------------------------------------------------------- Lorenz
// Section 2.2: x' = s (y - x), y' = x (r - z) - y, z' = x y - b z; p = [s, r, b].
template <typename R> struct Lorenz {
    static constexpr int D = 3, NP = 3, NQ = 1, UNROLL = 2, FUSED_INC = 0;
    static __device__ __forceinline__ void derive(const R (&)[NP], R (&q)[NQ]) { q[0] = R(0); }
    static __device__ __forceinline__ void f(const R (&p)[NP], const R (&)[NQ], const R (&x)[D], R (&o)[D]) {
        o[0] = p[0] * (x[1] - x[0]);
        o[1] = M<R>::fma_(x[0], p[1] - x[2], -x[1]);
        o[2] = M<R>::fma_(x[0], x[1], -(p[2] * x[2]));
    }
    // J = [[-s, s, 0], [r - z, -1, -x], [y, x, -b]];  df/dp = diag-like
    // (y - x, x, -z) on (s, r, b).
    static __device__ __forceinline__ void vjp(const R (&p)[NP], const R (&)[NQ], const R (&x)[D],
                                               const R (&a)[D], R (&gx)[D], R (&gp)[NP]) {
        gx[0] += -p[0] * a[0] + (p[1] - x[2]) * a[1] + x[1] * a[2];
        gx[1] += p[0] * a[0] - a[1] + x[0] * a[2];
        gx[2] += -x[0] * a[1] - p[2] * a[2];
        gp[0] += (x[1] - x[0]) * a[0];
        gp[1] += x[0] * a[1];
        gp[2] += -x[2] * a[2];
    }
};

// ---------------------------------------------------------------- Wilson-Cowan
// E' = -E + S_E(c1 E - c2 I + P), I' = -I + S_I(c3 E - c4 I + Q),
// S(u) = 1/(1 + exp(-a (u - th)));  p = [c1, c2, c3, c4, aE, thE, aI, thI, P, Q].
template <typename R> struct WilsonCowan {
    // Fast single precision and double precision fold the gain into the
    // sigmoid's argument: with g = -a*log2(e),
    // (u - th)*g = fma(c1*g, E, fma(-c2*g, I, (P - th)*g)), three constants
    // per population derived once per particle, so each S = 1/(1 + 2^t)
    // costs two fma, exp2, add and rcp (in double precision the kernels of
    // logistic2_k, which also clamp t and keep a NaN).  The folded constants
    // round the same number of times as the canonical order, with errors of
    // the same size.  Single precision with the library functions keeps the
    // canonical order below.
    static constexpr bool kFold = M<R>::kFast || kHasKernels<R>;
    static constexpr int D = 2, NP = 10, NQ = kFold ? 6 : 1, UNROLL = 1, FUSED_INC = M<R>::kFast;
    static __device__ __forceinline__ void derive(const R (&p)[NP], R (&q)[NQ]) {
        if constexpr (kFold) {
            const R gE = -p[4] * R(kLog2e), gI = -p[6] * R(kLog2e);
            q[0] = p[0] * gE;
            q[1] = -p[1] * gE;
            q[2] = (p[8] - p[5]) * gE;
            q[3] = p[2] * gI;
            q[4] = -p[3] * gI;
            q[5] = (p[9] - p[7]) * gI;
        } else {
            q[0] = R(0);
        }
    }
    static __device__ __forceinline__ void sigmoids(const R (&p)[NP], const R (&q)[NQ], const R (&x)[D], R& sE, R& sI) {
        if constexpr (kHasKernels<R>) {
            // a NaN per-particle P must reach the state through S_E
            sE = logistic2_k<true>(M<R>::fma_(q[0], x[0], M<R>::fma_(q[1], x[1], q[2])));
            sI = logistic2_k<true>(M<R>::fma_(q[3], x[0], M<R>::fma_(q[4], x[1], q[5])));
        } else if constexpr (kFold) {
            sE = M<R>::rcp_(R(1) + M<R>::exp2_(M<R>::fma_(q[0], x[0], M<R>::fma_(q[1], x[1], q[2]))));
            sI = M<R>::rcp_(R(1) + M<R>::exp2_(M<R>::fma_(q[3], x[0], M<R>::fma_(q[4], x[1], q[5]))));
        } else {
            const R uE = M<R>::fma_(p[0], x[0], M<R>::fma_(-p[1], x[1], p[8]));
            const R uI = M<R>::fma_(p[2], x[0], M<R>::fma_(-p[3], x[1], p[9]));
            sE = M<R>::rcp_(R(1) + M<R>::exp_(-(p[4] * (uE - p[5]))));
            sI = M<R>::rcp_(R(1) + M<R>::exp_(-(p[6] * (uI - p[7]))));
        }
    }
    static __device__ __forceinline__ void f(const R (&p)[NP], const R (&q)[NQ], const R (&x)[D], R (&o)[D]) {
        R sE, sI;
        sigmoids(p, q, x, sE, sI);
        o[0] = sE - x[0];
        o[1] = sI - x[1];
    }
    static __device__ __forceinline__ void vjp(const R (&p)[NP], const R (&q)[NQ], const R (&x)[D],
                                               const R (&a)[D], R (&gx)[D], R (&gp)[NP]) {
        const R uE = M<R>::fma_(p[0], x[0], M<R>::fma_(-p[1], x[1], p[8]));
        const R uI = M<R>::fma_(p[2], x[0], M<R>::fma_(-p[3], x[1], p[9]));
        R sE, sI;
        sigmoids(p, q, x, sE, sI);
        const R qE = sE * (R(1) - sE), qI = sI * (R(1) - sI);
        const R dE = p[4] * qE * a[0];   // dS_E/du_E * a_E
        const R dI = p[6] * qI * a[1];
        gx[0] += p[0] * dE - a[0] + p[2] * dI;
        gx[1] += -p[1] * dE - p[3] * dI - a[1];
        gp[0] += dE * x[0];
        gp[1] += -dE * x[1];
        gp[2] += dI * x[0];
        gp[3] += -dI * x[1];
        gp[4] += (uE - p[5]) * qE * a[0];
        gp[5] += -dE;
        gp[6] += (uI - p[7]) * qI * a[1];
        gp[7] += -dI;
        gp[8] += dE;
        gp[9] += dI;
    }
};

// ---------------------------------------------------------------- HH ring
// N Hodgkin-Huxley neurons (Section 3) with first-order synapses; neuron j is
// [V, m, h, n, s] at 5j and receives the synapse of neuron (j + N - 1) % N.
// p = [gNa, gK, gL, ENa, EK, EL, C, Iext, gsyn, Esyn, r_rise, r_decay,
//      th_syn, sg_syn].  Rates (modern convention, rest near -65 mV):
//   am = psi(-(V+40)/10), bm = 4 e^{-(V+65)/18}, ah = 0.07 e^{-(V+65)/20},
//   bh = 1/(1 + e^{-(V+35)/10}), an = 0.1 psi(-(V+55)/10),
//   bn = 0.125 e^{-(V+65)/80},  T = 1/(1 + e^{-sg (V - th)}),
//   psi(u) = u / (e^u - 1) with psi(0) = 1 taken by a select (fast single
//   precision: a Bernoulli series near 0 and the hardware exp2 elsewhere).
template <typename R> struct HHRate {
    R am, bm, ah, bh, an, bn, tv;
};

// k psi(u) with the fast single-precision functions, given den = (e^u - 1)/k
// from the caller: for |u| < 1/2 the Bernoulli series of u/(e^u - 1),
// 1 - u/2 + u^2/12 - u^4/720 + u^6/30240 (the next term, u^8/1209600, is below
// 3.3e-9), with its coefficients scaled by k; otherwise u * rcp(den)
// (cancellation in e^u - 1 costs at most a factor 2.6 there).  Both are
// computed and one is selected.
template <typename R>
__device__ __forceinline__ R hh_psi_fast(R u, R den, double k) {
    const R w = u * u;
    const R series = M<R>::fma_(w, M<R>::fma_(w, M<R>::fma_(w, R(k / 30240.0), R(-k / 720.0)), R(k / 12.0)),
                                M<R>::fma_(R(-0.5 * k), u, R(k)));
    const R direct = u * M<R>::rcp_(den);
    return __builtin_fabsf(u) < R(0.5) ? series : direct;
}

template <typename R>
__device__ __forceinline__ R hh_psi(R u) {
    if constexpr (kHasKernels<R>) {
        // u > 700 (V < -7040 mV): psi is below 1e-301 and e^u would overflow
        // (a NaN u gives a NaN quotient through the numerator)
        const R q = M<double>::div_k(u, M<double>::expm1_k(__builtin_fmin(u, 700.0)));
        return (u == R(0)) ? R(1) : q;
    } else {
        const R q = M<R>::div_(u, M<R>::expm1_(u));
        return (u == R(0)) ? R(1) : q;
    }
}

// Rates of one neuron.  sgl = -sg * log2(e) (derived once per particle) is
// used by the fast single-precision path only.
template <typename R>
__device__ __forceinline__ HHRate<R> hh_rates(R V, R th, R sg, R sgl) {
    const R c10 = R(-1.0 / 10.0);
    const R v65 = V + R(65.0);
    HHRate<R> q;
    if constexpr (M<R>::kFast) {
        // One exponential serves three rates: with E = e^{-(V+40)/10},
        // e^{-(V+35)/10} = E e^{1/2} and e^{-(V+55)/10} = E e^{-3/2}.  The
        // constants are split into two floats (hi + lo, added by two fmas) so
        // that their rounding does not bias the rates; the 1/10 of an scales
        // psi's series and denominator, and the factors 4 and 1/8 of bm and bn
        // are added to the base-2 exponent exactly.
        constexpr double kE05 = 1.6487212707001281468, kE15x10 = 2.2313016014842982893;
        const R um = (V + R(40.0)) * c10, un = (V + R(55.0)) * c10;
        const R E = M<R>::exp2_(um * R(kLog2e));
        q.am = hh_psi_fast<R>(um, E - R(1), 1.0);
        q.an = hh_psi_fast<R>(
            un, M<R>::fma_(E, R(kE15x10 - double(R(kE15x10))), M<R>::fma_(E, R(kE15x10), R(-10))), 0.1);
        q.bh = M<R>::rcp_(M<R>::fma_(E, R(kE05 - double(R(kE05))), M<R>::fma_(E, R(kE05), R(1))));
        q.bm = M<R>::exp2_(M<R>::fma_(v65, R(-kLog2e / 18.0), R(2)));
        q.ah = R(0.07) * M<R>::exp2_(v65 * R(-kLog2e / 20.0));
        q.bn = M<R>::exp2_(M<R>::fma_(v65, R(-kLog2e / 80.0), R(-3)));
        q.tv = M<R>::rcp_(R(1) + M<R>::exp2_((V - th) * sgl));
    } else {
        q.am = hh_psi<R>((V + R(40.0)) * c10);
        q.an = R(0.1) * hh_psi<R>((V + R(55.0)) * c10);
        if constexpr (kHasKernels<R>) {
            // the exp kernel overflows to inf and underflows to 0 like the
            // library function for |x| <= 1e15 (|V| <= 1.8e16 mV)
            q.bm = R(4.0) * M<double>::exp_k(v65 * R(-1.0 / 18.0));
            q.ah = R(0.07) * M<double>::exp_k(v65 * R(-1.0 / 20.0));
            // a NaN V makes V' NaN by itself; the synapse's argument also
            // carries the parameters th and sg, whose NaN must propagate
            q.bh = logistic_k<false>((V + R(35.0)) * R(-1.0 / 10.0));
            q.bn = R(0.125) * M<double>::exp_k(v65 * R(-1.0 / 80.0));
            q.tv = logistic_k<true>((V - th) * (-sg));
        } else {
            q.bm = R(4.0) * M<R>::exp_(v65 * R(-1.0 / 18.0));
            q.ah = R(0.07) * M<R>::exp_(v65 * R(-1.0 / 20.0));
            q.bh = M<R>::rcp_(R(1) + M<R>::exp_((V + R(35.0)) * R(-1.0 / 10.0)));
            q.bn = R(0.125) * M<R>::exp_(v65 * R(-1.0 / 80.0));
            q.tv = M<R>::rcp_(R(1) + M<R>::exp_((V - th) * (-sg)));
        }
    }
    return q;
}

// dx/dt = a (1 - x) - b x of a gate; the fast path evaluates a - (a + b) x.
template <typename R>
__device__ __forceinline__ R hh_gate(R a, R b, R x) {
    if constexpr (M<R>::kFast) return M<R>::fma_(-(a + b), x, a);
    else return M<R>::fma_(a, R(1) - x, -(b * x));
}

template <typename R, int N> struct HHRing {
    static constexpr int D = 5 * N, NP = 14, NQ = 1, UNROLL = 1, FUSED_INC = M<R>::kFast;
    static __device__ __forceinline__ void derive(const R (&p)[NP], R (&q)[NQ]) {
        q[0] = M<R>::kFast ? -p[13] * R(kLog2e) : R(0);
    }
    static __device__ __forceinline__ void f(const R (&p)[NP], const R (&qd)[NQ], const R (&x)[D], R (&o)[D]) {
        const R invC = M<R>::rcp_(p[6]);
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const R V = x[5 * j], m = x[5 * j + 1], h = x[5 * j + 2], n = x[5 * j + 3], s = x[5 * j + 4];
            const R spre = x[5 * ((j + N - 1) % N) + 4];
            const HHRate<R> q = hh_rates<R>(V, p[12], p[13], qd[0]);
            const R gNa = (p[0] * ((m * m) * m)) * h;
            const R n2 = n * n;
            const R gK = p[1] * (n2 * n2);
            const R gS = p[8] * spre;
            if constexpr (M<R>::kFast) {
                // the membrane currents accumulated by fma, Iext first
                R I = M<R>::fma_(p[2], p[5] - V, p[7]);
                I = M<R>::fma_(gNa, p[3] - V, I);
                I = M<R>::fma_(gK, p[4] - V, I);
                I = M<R>::fma_(gS, p[9] - V, I);
                o[5 * j] = I * invC;
            } else {
                const R IL = p[2] * (p[5] - V);
                o[5 * j] = ((((IL + gNa * (p[3] - V)) + gK * (p[4] - V)) + gS * (p[9] - V)) + p[7]) * invC;
            }
            o[5 * j + 1] = hh_gate(q.am, q.bm, m);
            o[5 * j + 2] = hh_gate(q.ah, q.bh, h);
            o[5 * j + 3] = hh_gate(q.an, q.bn, n);
            o[5 * j + 4] = hh_gate(p[10] * q.tv, p[11], s);
        }
    }
    // psi'(u) = (expm1(u) - u e^u) / expm1(u)^2, psi'(0) = -1/2.  The
    // numerator is a difference of two terms of size |u| that cancel to
    // -u^2/2, so in fast single precision |u| < 1/2 takes the derivative of
    // the Bernoulli series instead, -1/2 + u/6 - u^3/180 + u^5/5040 -
    // u^7/151200 (the next term, u^9/4790016, is below 4.1e-10 there), and
    // the rest the hardware exponential (cancellation there costs a few
    // ulp).  Both are computed and one is selected.
    static __device__ __forceinline__ R dpsi(R u) {
        if constexpr (M<R>::kFast) {
            const R w = u * u;
            const R series = M<R>::fma_(
                u, M<R>::fma_(w, M<R>::fma_(w, M<R>::fma_(w, R(-1.0 / 151200.0), R(1.0 / 5040.0)), R(-1.0 / 180.0)),
                              R(1.0 / 6.0)),
                R(-0.5));
            const R e = M<R>::exp2_(u * R(kLog2e));
            const R em1 = e - R(1);
            const R direct = (em1 - u * e) * M<R>::rcp_(em1 * em1);
            return __builtin_fabsf(u) < R(0.5) ? series : direct;
        } else if constexpr (kHasKernels<R>) {
            // u > 350 (V < -3540 mV): psi' is below 1e-149 and expm1(u)^2 would
            // overflow (a NaN u: the state's V is NaN already)
            const R uc = __builtin_fmin(u, 350.0);
            const R em1 = M<double>::expm1_k(uc);
            const R d = M<double>::div_k(em1 - uc * (em1 + R(1)), em1 * em1);
            return (u == R(0)) ? R(-0.5) : d;
        } else {
            const R em1 = M<R>::expm1_(u);
            const R d = M<R>::div_(em1 - u * (em1 + R(1)), em1 * em1);
            return (u == R(0)) ? R(-0.5) : d;
        }
    }
    static __device__ __forceinline__ void vjp(const R (&p)[NP], const R (&qd)[NQ], const R (&x)[D],
                                               const R (&a)[D], R (&gx)[D], R (&gp)[NP]) {
        const R invC = M<R>::rcp_(p[6]);
        const R th = p[12], sg = p[13];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const int o = 5 * j, q5 = 5 * ((j + N - 1) % N);
            const R V = x[o], m = x[o + 1], h = x[o + 2], n = x[o + 3], s = x[o + 4];
            const R spre = x[q5 + 4];
            const HHRate<R> q = hh_rates<R>(V, th, sg, qd[0]);
            const R um = (V + R(40.0)) * R(-1.0 / 10.0), un = (V + R(55.0)) * R(-1.0 / 10.0);
            const R dam = dpsi(um) * R(-0.1);
            const R dbm = q.bm * R(-1.0 / 18.0);
            const R dah = q.ah * R(-1.0 / 20.0);
            const R dbh = R(0.1) * q.bh * (R(1) - q.bh);
            const R dan = R(0.1) * dpsi(un) * R(-0.1);
            const R dbn = q.bn * R(-1.0 / 80.0);
            const R dT = sg * q.tv * (R(1) - q.tv);
            const R m2 = m * m, m3 = m2 * m, n2 = n * n, n3 = n2 * n, n4 = n2 * n2;
            const R eNa = p[3] - V, eK = p[4] - V, eL = p[5] - V, eS = p[9] - V;
            const R aV = a[o] * invC;      // membrane adjoint scaled by 1/C
            const R am_ = a[o + 1], ah_ = a[o + 2], an_ = a[o + 3], as_ = a[o + 4];
            // d/dV
            gx[o] += aV * (-p[2] - p[0] * m3 * h - p[1] * n4 - p[8] * spre)
                   + am_ * (dam * (R(1) - m) - dbm * m)
                   + ah_ * (dah * (R(1) - h) - dbh * h)
                   + an_ * (dan * (R(1) - n) - dbn * n)
                   + as_ * (p[10] * dT * (R(1) - s));
            gx[o + 1] += aV * (R(3) * p[0] * m2 * h * eNa) - am_ * (q.am + q.bm);
            gx[o + 2] += aV * (p[0] * m3 * eNa) - ah_ * (q.ah + q.bh);
            gx[o + 3] += aV * (R(4) * p[1] * n3 * eK) - an_ * (q.an + q.bn);
            gx[o + 4] += -as_ * (p[10] * q.tv + p[11]);
            gx[q5 + 4] += aV * (p[8] * eS);
            // parameters
            const R dV = (p[2] * eL + p[0] * m3 * h * eNa + p[1] * n4 * eK + p[8] * spre * eS + p[7]) * invC;
            gp[0] += aV * m3 * h * eNa;
            gp[1] += aV * n4 * eK;
            gp[2] += aV * eL;
            gp[3] += aV * p[0] * m3 * h;
            gp[4] += aV * p[1] * n4;
            gp[5] += aV * p[2];
            gp[6] += -aV * dV;
            gp[7] += aV;
            gp[8] += aV * spre * eS;
            gp[9] += aV * p[8] * spre;
            const R tq = q.tv * (R(1) - q.tv);
            gp[10] += as_ * q.tv * (R(1) - s);
            gp[11] += -as_ * s;
            gp[12] += as_ * p[10] * (R(1) - s) * (-sg * tq);
            gp[13] += as_ * p[10] * (R(1) - s) * ((V - th) * tq);
        }
    }
};

}  // namespace ff
