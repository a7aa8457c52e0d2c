// ffo.cpp — CPU oracle for the Fireflies particle-RK4 hot path.
//
// TEST INFRASTRUCTURE ONLY (see ffo.h).  Plain loops, one particle at a time,
// no blocking or fusion.  Build: g++ -std=c++17 -O2 -fopenmp -ffp-contract=off
// -fno-fast-math -fPIC -shared.  fp-contract is off so that every fused
// multiply-add below is one written out with std::fma and nothing else is
// contracted.
//
// Evaluation order.  Floating-point results depend on the order of operations,
// and the Lorenz system is chaotic, so the order is fixed here once and for all
// (it is one admissible way to write the formulas of the paper; any other order
// is equally correct mathematically):
//   RK4 step with h2 = h*0.5 and h6 = h/6 (working precision):
//     k1 = f(x); y = fma(h2, k1, x); k2 = f(y); y = fma(h2, k2, x); k3 = f(y);
//     y = fma(h, k3, x); k4 = f(y);
//     s = k2 + k3; s = fma(2, s, k1); s = s + k4; x = fma(h6, s, x)
//   compensated (Kahan) update, single precision only:
//     inc = h6*s; yk = inc - c; t = x + yk; c = (t - x) - yk; x = t
#include "ffo.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include <omp.h>

namespace {

using cplx = std::complex<double>;
constexpr int kMaxDim = 20;
constexpr int kMaxParams = 16;
constexpr int kMaxPP = 8;

// ---------------------------------------------------------------- arithmetic
// fma / exp / expm1 for the three scalar types the oracle is instantiated on.
inline double fma_(double a, double b, double c) { return std::fma(a, b, c); }
inline float fma_(float a, float b, float c) { return std::fma(a, b, c); }
// Complex-step only needs an analytic extension, so a*b + c is exact enough.
inline cplx fma_(cplx a, cplx b, cplx c) { return a * b + c; }

inline double exp_(double x) { return std::exp(x); }
inline float exp_(float x) { return std::exp(x); }
inline cplx exp_(cplx z) { return std::exp(z); }

inline double expm1_(double x) { return std::expm1(x); }
inline float expm1_(float x) { return std::expm1(x); }
// expm1(a + ib) = e^a cos b - 1 + i e^a sin b, with the real part written as
// expm1(a) cos b - 2 sin^2(b/2) so that it does not cancel for small a, b.
inline cplx expm1_(cplx z) {
    const double a = z.real(), b = z.imag();
    const double sb2 = std::sin(0.5 * b);
    return cplx(std::expm1(a) * std::cos(b) - 2.0 * sb2 * sb2, std::exp(a) * std::sin(b));
}

// psi(u) = u / (e^u - 1), continued by psi(0) = 1.  It is the common factor of
// the Hodgkin-Huxley alpha_m and alpha_n rates.
template <class T> inline T psi(T u) {
    return (u == T(0)) ? T(1) : u / expm1_(u);
}
// psi'(u) = (e^u - 1 - u e^u) / (e^u - 1)^2, continued by psi'(0) = -1/2.
inline double dpsi(double u) {
    if (u == 0.0) return -0.5;
    const double em1 = std::expm1(u);
    return (em1 - u * (em1 + 1.0)) / (em1 * em1);
}

// ---------------------------------------------------------------- systems
// Every right-hand side takes the parameter vector p (global values already
// replaced by the particle's own values where it has them), a point x and
// writes f(x).  The systems are autonomous: no time argument.

// x' = A x, A row-major in p (dim <= 4).
template <class T> void rhs_linear(int dim, const T* p, const T* x, T* f) {
    for (int r = 0; r < dim; ++r) {
        T acc = p[r * dim + 0] * x[0];
        for (int c = 1; c < dim; ++c) acc = fma_(p[r * dim + c], x[c], acc);
        f[r] = acc;
    }
}

// Lorenz (Section 2.2, Eqs. lorenz_x, lorenz_y, lorenz_z): p = [sigma, r, beta].
//   x' = sigma (y - x),  y' = x (r - z) - y,  z' = x y - beta z
template <class T> void rhs_lorenz(const T* p, const T* x, T* f) {
    const T sigma = p[0], r = p[1], beta = p[2];
    f[0] = sigma * (x[1] - x[0]);
    f[1] = fma_(x[0], r - x[2], -x[1]);
    f[2] = fma_(x[0], x[1], -(beta * x[2]));
}

// Wilson-Cowan excitatory/inhibitory pair, the same sigmoid-coupled structure
// as Eqs. stn_gpe/eqnGPe with unit time constants:
//   E' = -E + S_E(c1 E - c2 I + P),  I' = -I + S_I(c3 E - c4 I + Q),
//   S(u) = 1 / (1 + exp(-a (u - theta))).
// p = [c1, c2, c3, c4, aE, thetaE, aI, thetaI, P, Q].
template <class T> void rhs_wilson_cowan(const T* p, const T* x, T* f) {
    const T E = x[0], I = x[1];
    const T uE = fma_(p[0], E, fma_(-p[1], I, p[8]));
    const T sE = T(1) / (T(1) + exp_(-(p[4] * (uE - p[5]))));
    const T uI = fma_(p[2], E, fma_(-p[3], I, p[9]));
    const T sI = T(1) / (T(1) + exp_(-(p[6] * (uI - p[7]))));
    f[0] = sE - E;
    f[1] = sI - I;
}

// Hodgkin-Huxley ring of N neurons (Section 3, Eqs. hh_v, hh_h, hh_m, hh_n with
// the synaptic current hh_isyn and the synapse variable hh_s).  State of
// neuron j: [V, m, h, n, s] at offset 5j.  Neuron j receives the synapse of
// neuron (j + N - 1) mod N (0-based reading of the ring index).
// p = [gNa, gK, gL, ENa, EK, EL, C, Iext, gsyn, Esyn, r_rise, r_decay,
//      theta_syn, sigma_syn].  Rate functions: the Hodgkin-Huxley squid-axon
// forms in the modern sign convention (rest near -65 mV):
//   alpha_m = psi(-(V+40)/10)           beta_m = 4 exp(-(V+65)/18)
//   alpha_h = 0.07 exp(-(V+65)/20)      beta_h = 1 / (1 + exp(-(V+35)/10))
//   alpha_n = 0.1 psi(-(V+55)/10)       beta_n = 0.125 exp(-(V+65)/80)
//   synapse: s' = r_rise T(V) (1 - s) - r_decay s,
//            T(V) = 1 / (1 + exp(-sigma_syn (V - theta_syn)))
// Divisions by the constants 10, 18, 20, 80 are written as multiplications by
// the nearest double of -1/10, -1/18, -1/20, -1/80; the membrane equation is
// multiplied by 1/C.
template <class T> struct HHRates { T am, bm, ah, bh, an, bn, tv; };

template <class T> HHRates<T> hh_rates(const T* p, T V) {
    const T km10 = T(-1.0 / 10.0), km18 = T(-1.0 / 18.0), km20 = T(-1.0 / 20.0),
            km80 = T(-1.0 / 80.0);
    HHRates<T> r;
    const T v65 = V + T(65.0);
    r.am = psi((V + T(40.0)) * km10);
    r.bm = T(4.0) * exp_(v65 * km18);
    r.ah = T(0.07) * exp_(v65 * km20);
    r.bh = T(1) / (T(1) + exp_((V + T(35.0)) * km10));
    r.an = T(0.1) * psi((V + T(55.0)) * km10);
    r.bn = T(0.125) * exp_(v65 * km80);
    r.tv = T(1) / (T(1) + exp_((V - p[12]) * (-p[13])));
    return r;
}

template <class T> void rhs_hh_ring(int N, const T* p, const T* x, T* f) {
    const T gNa = p[0], gK = p[1], gL = p[2], ENa = p[3], EK = p[4], EL = p[5];
    const T invC = T(1) / p[6];
    const T Iext = p[7], gsyn = p[8], Esyn = p[9], rr = p[10], rd = p[11];
    for (int j = 0; j < N; ++j) {
        const T V = x[5 * j + 0], m = x[5 * j + 1], h = x[5 * j + 2], n = x[5 * j + 3],
                s = x[5 * j + 4];
        const T s_pre = x[5 * ((j + N - 1) % N) + 4];
        const HHRates<T> r = hh_rates(p, V);
        const T IL = gL * (EL - V);
        const T INa = ((gNa * ((m * m) * m)) * h) * (ENa - V);
        const T n2 = n * n;
        const T IK = (gK * (n2 * n2)) * (EK - V);
        const T Isyn = (gsyn * s_pre) * (Esyn - V);
        f[5 * j + 0] = ((((IL + INa) + IK) + Isyn) + Iext) * invC;
        f[5 * j + 1] = fma_(r.am, T(1) - m, -(r.bm * m));
        f[5 * j + 2] = fma_(r.ah, T(1) - h, -(r.bh * h));
        f[5 * j + 3] = fma_(r.an, T(1) - n, -(r.bn * n));
        f[5 * j + 4] = fma_(rr * r.tv, T(1) - s, -(rd * s));
    }
}

// y' = y^2 (oracle only; exact solution y0 / (1 - y0 t)).
template <class T> void rhs_riccati(const T* x, T* f) { f[0] = x[0] * x[0]; }

template <class T> void rhs(int sys, int dim, const T* p, const T* x, T* f) {
    switch (sys) {
        case FFO_LINEAR: rhs_linear(dim, p, x, f); break;
        case FFO_LORENZ: rhs_lorenz(p, x, f); break;
        case FFO_WILSON_COWAN: rhs_wilson_cowan(p, x, f); break;
        case FFO_HH_RING: rhs_hh_ring(dim / 5, p, x, f); break;
        case FFO_RICCATI: rhs_riccati(x, f); break;
    }
}

int n_params_of(int sys, int dim) {
    switch (sys) {
        case FFO_LINEAR: return (dim >= 1 && dim <= 4) ? dim * dim : -1;
        case FFO_LORENZ: return dim == 3 ? 3 : -1;
        case FFO_WILSON_COWAN: return dim == 2 ? 10 : -1;
        case FFO_HH_RING: return (dim >= 5 && dim <= 20 && dim % 5 == 0) ? 14 : -1;
        case FFO_RICCATI: return dim == 1 ? 0 : -1;
    }
    return -1;
}

// ---------------------------------------------------------------- Jacobians
// J[r*dim + c] = d f_r / d x_c;  Fp[r*np + k] = d f_r / d p_k.  Written out
// from the formulas above by hand; the complex-step derivative of the RK4 map
// checks them.
void jac_linear(int dim, const double* p, const double* x, double* J, double* Fp) {
    const int np = dim * dim;
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c) {
            J[r * dim + c] = p[r * dim + c];
            Fp[r * np + r * dim + c] = x[c];
        }
}

void jac_lorenz(const double* p, const double* x, double* J, double* Fp) {
    const double sigma = p[0], r = p[1], beta = p[2];
    const double X = x[0], Y = x[1], Z = x[2];
    const double Jl[9] = {-sigma, sigma, 0.0, r - Z, -1.0, -X, Y, X, -beta};
    std::memcpy(J, Jl, sizeof Jl);
    Fp[0 * 3 + 0] = Y - X;   // d f_x / d sigma
    Fp[1 * 3 + 1] = X;       // d f_y / d r
    Fp[2 * 3 + 2] = -Z;      // d f_z / d beta
}

void jac_wilson_cowan(const double* p, const double* x, double* J, double* Fp) {
    const double E = x[0], I = x[1];
    const double c1 = p[0], c2 = p[1], c3 = p[2], c4 = p[3];
    const double aE = p[4], thE = p[5], aI = p[6], thI = p[7];
    const double uE = c1 * E - c2 * I + p[8];
    const double uI = c3 * E - c4 * I + p[9];
    const double sE = 1.0 / (1.0 + std::exp(-aE * (uE - thE)));
    const double sI = 1.0 / (1.0 + std::exp(-aI * (uI - thI)));
    const double gE = sE * (1.0 - sE), gI = sI * (1.0 - sI);  // S/(a) slopes
    const double dE = aE * gE, dI = aI * gI;                    // dS/du
    J[0] = c1 * dE - 1.0;  J[1] = -c2 * dE;
    J[2] = c3 * dI;        J[3] = -c4 * dI - 1.0;
    const int np = 10;
    Fp[0 * np + 0] = dE * E;             // c1
    Fp[0 * np + 1] = -dE * I;            // c2
    Fp[1 * np + 2] = dI * E;             // c3
    Fp[1 * np + 3] = -dI * I;            // c4
    Fp[0 * np + 4] = (uE - thE) * gE;    // aE
    Fp[0 * np + 5] = -dE;                // thetaE
    Fp[1 * np + 6] = (uI - thI) * gI;    // aI
    Fp[1 * np + 7] = -dI;                // thetaI
    Fp[0 * np + 8] = dE;                 // P
    Fp[1 * np + 9] = dI;                 // Q
}

void jac_hh_ring(int N, const double* p, const double* x, double* J, double* Fp) {
    const int dim = 5 * N, np = 14;
    const double gNa = p[0], gK = p[1], gL = p[2], ENa = p[3], EK = p[4], EL = p[5];
    const double C = p[6], Iext = p[7], gsyn = p[8], Esyn = p[9], rr = p[10], rd = p[11];
    const double th = p[12], sg = p[13];
    for (int j = 0; j < N; ++j) {
        const int o = 5 * j, q = 5 * ((j + N - 1) % N);
        const double V = x[o], m = x[o + 1], h = x[o + 2], n = x[o + 3], s = x[o + 4];
        const double sp = x[q + 4];
        // rates and their V-derivatives
        const double um = -(V + 40.0) / 10.0, un = -(V + 55.0) / 10.0;
        const double am = psi(um), dam = dpsi(um) * (-0.1);
        const double bm = 4.0 * std::exp(-(V + 65.0) / 18.0), dbm = bm * (-1.0 / 18.0);
        const double ah = 0.07 * std::exp(-(V + 65.0) / 20.0), dah = ah * (-1.0 / 20.0);
        const double bh = 1.0 / (1.0 + std::exp(-(V + 35.0) / 10.0)), dbh = 0.1 * bh * (1.0 - bh);
        const double an = 0.1 * psi(un), dan = 0.1 * dpsi(un) * (-0.1);
        const double bn = 0.125 * std::exp(-(V + 65.0) / 80.0), dbn = bn * (-1.0 / 80.0);
        const double T = 1.0 / (1.0 + std::exp(-sg * (V - th))), dT = sg * T * (1.0 - T);
        const double m3h = m * m * m * h, n4 = n * n * n * n;
        const double dV = (gL * (EL - V) + gNa * m3h * (ENa - V) + gK * n4 * (EK - V) +
                           gsyn * sp * (Esyn - V) + Iext) / C;
        // membrane row
        double* JV = J + (o + 0) * dim;
        JV[o + 0] += (-gL - gNa * m3h - gK * n4 - gsyn * sp) / C;
        JV[o + 1] += 3.0 * gNa * m * m * h * (ENa - V) / C;
        JV[o + 2] += gNa * m * m * m * (ENa - V) / C;
        JV[o + 3] += 4.0 * gK * n * n * n * (EK - V) / C;
        JV[q + 4] += gsyn * (Esyn - V) / C;
        // gate rows
        J[(o + 1) * dim + o] = dam * (1.0 - m) - dbm * m;
        J[(o + 1) * dim + o + 1] = -am - bm;
        J[(o + 2) * dim + o] = dah * (1.0 - h) - dbh * h;
        J[(o + 2) * dim + o + 2] = -ah - bh;
        J[(o + 3) * dim + o] = dan * (1.0 - n) - dbn * n;
        J[(o + 3) * dim + o + 3] = -an - bn;
        // synapse row
        J[(o + 4) * dim + o] = rr * dT * (1.0 - s);
        J[(o + 4) * dim + o + 4] = -rr * T - rd;
        // parameter Jacobian
        double* FV = Fp + (o + 0) * np;
        FV[0] = m3h * (ENa - V) / C;
        FV[1] = n4 * (EK - V) / C;
        FV[2] = (EL - V) / C;
        FV[3] = gNa * m3h / C;
        FV[4] = gK * n4 / C;
        FV[5] = gL / C;
        FV[6] = -dV / C;
        FV[7] = 1.0 / C;
        FV[8] = sp * (Esyn - V) / C;
        FV[9] = gsyn * sp / C;
        double* FS = Fp + (o + 4) * np;
        FS[10] = T * (1.0 - s);
        FS[11] = -s;
        FS[12] = rr * (1.0 - s) * (-sg * T * (1.0 - T));
        FS[13] = rr * (1.0 - s) * ((V - th) * T * (1.0 - T));
    }
}

void jacobians(int sys, int dim, int np, const double* p, const double* x, double* J,
               double* Fp) {
    std::fill(J, J + dim * dim, 0.0);
    std::fill(Fp, Fp + dim * np, 0.0);
    switch (sys) {
        case FFO_LINEAR: jac_linear(dim, p, x, J, Fp); break;
        case FFO_LORENZ: jac_lorenz(p, x, J, Fp); break;
        case FFO_WILSON_COWAN: jac_wilson_cowan(p, x, J, Fp); break;
        case FFO_HH_RING: jac_hh_ring(dim / 5, p, x, J, Fp); break;
        case FFO_RICCATI: J[0] = 2.0 * x[0]; break;
    }
}

// ---------------------------------------------------------------- RK4
template <class T> void rk4_step(int sys, int dim, const T* p, T* x, T h, T h2, T h6) {
    T k1[kMaxDim], k2[kMaxDim], k3[kMaxDim], k4[kMaxDim], y[kMaxDim];
    rhs(sys, dim, p, x, k1);
    for (int d = 0; d < dim; ++d) y[d] = fma_(h2, k1[d], x[d]);
    rhs(sys, dim, p, y, k2);
    for (int d = 0; d < dim; ++d) y[d] = fma_(h2, k2[d], x[d]);
    rhs(sys, dim, p, y, k3);
    for (int d = 0; d < dim; ++d) y[d] = fma_(h, k3[d], x[d]);
    rhs(sys, dim, p, y, k4);
    for (int d = 0; d < dim; ++d) {
        T s = k2[d] + k3[d];
        s = fma_(T(2), s, k1[d]);
        s = s + k4[d];
        x[d] = fma_(h6, s, x[d]);
    }
}

// Same stages; the increment h6*s is added with Kahan's compensated summation.
void rk4_step_kahan(int sys, int dim, const float* p, float* x, float* c, float h, float h2,
                    float h6) {
    float k1[kMaxDim], k2[kMaxDim], k3[kMaxDim], k4[kMaxDim], y[kMaxDim];
    rhs(sys, dim, p, x, k1);
    for (int d = 0; d < dim; ++d) y[d] = fma_(h2, k1[d], x[d]);
    rhs(sys, dim, p, y, k2);
    for (int d = 0; d < dim; ++d) y[d] = fma_(h2, k2[d], x[d]);
    rhs(sys, dim, p, y, k3);
    for (int d = 0; d < dim; ++d) y[d] = fma_(h, k3[d], x[d]);
    rhs(sys, dim, p, y, k4);
    for (int d = 0; d < dim; ++d) {
        float s = k2[d] + k3[d];
        s = fma_(2.0f, s, k1[d]);
        s = s + k4[d];
        const float inc = h6 * s;
        const float yk = inc - c[d];
        const float t = x[d] + yk;
        c[d] = (t - x[d]) - yk;
        x[d] = t;
    }
}

bool valid_common(int sys, int dim, int n_params, const int32_t* pp_slot, int n_pp, int64_t n,
                  int64_t ld) {
    if (n_params_of(sys, dim) != n_params) return false;
    if (n < 0 || ld < n || n_pp < 0 || n_pp > kMaxPP) return false;
    if (n_pp > 0 && pp_slot == nullptr) return false;
    for (int k = 0; k < n_pp; ++k)
        if (pp_slot[k] < 0 || pp_slot[k] >= n_params) return false;
    return true;
}

template <class T, class S>
void particle_params(const double* params, int n_params, const int32_t* pp_slot, int n_pp,
                     const S* pparams, int64_t ld, int64_t i, T* p) {
    for (int j = 0; j < n_params; ++j) p[j] = T(params[j]);
    for (int k = 0; k < n_pp; ++k) p[pp_slot[k]] = T(pparams[k * ld + i]);
}

int threads_or_default(int nthreads) { return nthreads > 0 ? nthreads : omp_get_max_threads(); }

// ---------------------------------------------------------------- Philox
// Philox4x32-10 as defined by Salmon et al. (SC'11): ten rounds of
//   (c0, c1, c2, c3) -> (hi(B*c2) ^ c1 ^ k0, lo(B*c2), hi(A*c0) ^ c3 ^ k1, lo(A*c0))
// with A = 0xD2511F53, B = 0xCD9E8D57, the key bumped by the Weyl constants
// (0x9E3779B9, 0xBB67AE85) after every round but the last.
void philox(const uint32_t in[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {in[0], in[1], in[2], in[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
        c[0] = n0;
        c[1] = n1;
        c[2] = n2;
        c[3] = n3;
        if (round < 9) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
    }
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

// Word w of the random stream of (particle g, draw r).
uint32_t stream_word(uint64_t seed, uint64_t g, uint32_t r, int w) {
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const uint32_t ctr[4] = {(uint32_t)g, (uint32_t)(g >> 32), r, (uint32_t)(w / 4)};
    uint32_t out[4];
    philox(ctr, key, out);
    return out[w % 4];
}

void redraw(int dim, const double* lo, const double* hi, uint64_t seed, uint64_t g, uint32_t r, double* x) {
    for (int d = 0; d < dim; ++d) {
        const uint32_t a = stream_word(seed, g, r, 2 * d), b = stream_word(seed, g, r, 2 * d + 1);
        const double u = ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
        x[d] = std::fma(hi[d] - lo[d], u, lo[d]);
    }
}

void redraw(int dim, const double* lo, const double* hi, uint64_t seed, uint64_t g, uint32_t r, float* x) {
    for (int d = 0; d < dim; ++d) {
        const uint32_t a = stream_word(seed, g, r, d);
        const float u = (float)(a >> 8) * (1.0f / 16777216.0f);
        x[d] = std::fma((float)(hi[d] - lo[d]), u, (float)lo[d]);
    }
}

template <class T> bool escaped(int dim, const T* x, const double* blo, const double* bhi) {
    for (int d = 0; d < dim; ++d) {
        const double v = (double)x[d];
        if (!(v >= blo[d] && v <= bhi[d])) return true;
    }
    return false;
}

}  // namespace

extern "C" {

int ffo_n_params(int sys, int dim) { return n_params_of(sys, dim); }

int ffo_rhs(int sys, int dim, const double* params, int n_params, const double* x, double* f,
            int64_t m) {
    if (n_params_of(sys, dim) != n_params || m < 0) return -1;
    for (int64_t i = 0; i < m; ++i) rhs(sys, dim, params, x + i * dim, f + i * dim);
    return 0;
}

int ffo_jacobians(int sys, int dim, const double* params, int n_params, const double* x,
                  double* J, double* Fp, int64_t m) {
    if (n_params_of(sys, dim) != n_params || m < 0) return -1;
    for (int64_t i = 0; i < m; ++i)
        jacobians(sys, dim, n_params, params, x + i * dim, J + i * dim * dim,
                  Fp + i * dim * n_params);
    return 0;
}

int ffo_rk4(int sys, int dim, const double* params, int n_params, const int32_t* pp_slot,
            int n_pp, const double* pparams, double* state, int64_t n, int64_t ld, double h,
            int64_t nsteps, int nthreads) {
    if (!valid_common(sys, dim, n_params, pp_slot, n_pp, n, ld) || nsteps < 0) return -1;
    const double h2 = h * 0.5, h6 = h / 6.0;
#pragma omp parallel for schedule(static) num_threads(threads_or_default(nthreads))
    for (int64_t i = 0; i < n; ++i) {
        double p[kMaxParams], x[kMaxDim];
        particle_params(params, n_params, pp_slot, n_pp, pparams, ld, i, p);
        for (int d = 0; d < dim; ++d) x[d] = state[d * ld + i];
        for (int64_t s = 0; s < nsteps; ++s) rk4_step(sys, dim, p, x, h, h2, h6);
        for (int d = 0; d < dim; ++d) state[d * ld + i] = x[d];
    }
    return 0;
}

int ffo_rk4_f32(int sys, int dim, const double* params, int n_params, const int32_t* pp_slot,
                int n_pp, const float* pparams, float* state, float* comp, int kahan,
                int64_t n, int64_t ld, float h, int64_t nsteps, int nthreads) {
    if (!valid_common(sys, dim, n_params, pp_slot, n_pp, n, ld) || nsteps < 0) return -1;
    if (kahan && comp == nullptr) return -1;
    const float h2 = h * 0.5f, h6 = h / 6.0f;
#pragma omp parallel for schedule(static) num_threads(threads_or_default(nthreads))
    for (int64_t i = 0; i < n; ++i) {
        float p[kMaxParams], x[kMaxDim], c[kMaxDim];
        particle_params(params, n_params, pp_slot, n_pp, pparams, ld, i, p);
        for (int d = 0; d < dim; ++d) {
            x[d] = state[d * ld + i];
            c[d] = kahan ? comp[d * ld + i] : 0.0f;
        }
        for (int64_t s = 0; s < nsteps; ++s) {
            if (kahan) rk4_step_kahan(sys, dim, p, x, c, h, h2, h6);
            else rk4_step(sys, dim, p, x, h, h2, h6);
        }
        for (int d = 0; d < dim; ++d) {
            state[d * ld + i] = x[d];
            if (kahan) comp[d * ld + i] = c[d];
        }
    }
    return 0;
}

int ffo_rk4_cstep(int sys, int dim, const double* params, int n_params, const int32_t* pp_slot,
                  int n_pp, const double* pparams, const double* x0, const double* dx0,
                  const double* dparams, const double* dpp, double eps, double* xT,
                  double* dxT, int64_t n, int64_t ld, double h, int64_t nsteps, int nthreads) {
    if (!valid_common(sys, dim, n_params, pp_slot, n_pp, n, ld) || nsteps < 0 || eps == 0.0)
        return -1;
    const cplx hc(h, 0.0), h2(h * 0.5, 0.0), h6(h / 6.0, 0.0);
#pragma omp parallel for schedule(static) num_threads(threads_or_default(nthreads))
    for (int64_t i = 0; i < n; ++i) {
        cplx p[kMaxParams], x[kMaxDim];
        for (int j = 0; j < n_params; ++j)
            p[j] = cplx(params[j], dparams ? eps * dparams[j] : 0.0);
        for (int k = 0; k < n_pp; ++k)
            p[pp_slot[k]] = cplx(pparams[k * ld + i], dpp ? eps * dpp[k * ld + i] : 0.0);
        for (int d = 0; d < dim; ++d)
            x[d] = cplx(x0[d * ld + i], dx0 ? eps * dx0[d * ld + i] : 0.0);
        for (int64_t s = 0; s < nsteps; ++s) rk4_step(sys, dim, p, x, hc, h2, h6);
        for (int d = 0; d < dim; ++d) {
            xT[d * ld + i] = x[d].real();
            dxT[d * ld + i] = x[d].imag() / eps;
        }
    }
    return 0;
}

// Reverse mode through x_{k+1} = x_k + (h/6)(k1 + 2 k2 + 2 k3 + k4), treated
// as exact arithmetic.  With lam' = dL/dx_{k+1} the adjoints of the stage
// slopes are abar4 = (h/6) lam', abar3 = (h/3) lam' + h b4,
// abar2 = (h/3) lam' + (h/2) b3, abar1 = (h/6) lam' + (h/2) b2, where
// b_i = J(stage point i)^T abar_i; then dL/dx_k = lam' + b1 + b2 + b3 + b4
// and dL/dp gains sum_i Fp(stage point i)^T abar_i.  The whole trajectory of
// each particle is stored (no checkpointing: it is the plain definition).
int ffo_adjoint(int sys, int dim, const double* params, int n_params, const int32_t* pp_slot,
                int n_pp, const double* pparams, const double* x0, double* lam, double* mu_pp,
                double* mu_global, int64_t n, int64_t ld, double h, int64_t nsteps,
                int nthreads) {
    if (!valid_common(sys, dim, n_params, pp_slot, n_pp, n, ld) || nsteps < 0) return -1;
    if (n_pp > 0 && mu_pp == nullptr) return -1;
    const double h2 = h * 0.5, h6 = h / 6.0, h3 = h / 3.0;
    std::vector<double> mu_all(static_cast<size_t>(n) * (n_params > 0 ? n_params : 1), 0.0);
#pragma omp parallel for schedule(static) num_threads(threads_or_default(nthreads))
    for (int64_t i = 0; i < n; ++i) {
        double p[kMaxParams];
        particle_params(params, n_params, pp_slot, n_pp, pparams, ld, i, p);
        std::vector<double> tape(static_cast<size_t>(nsteps + 1) * dim);
        for (int d = 0; d < dim; ++d) tape[d] = x0[d * ld + i];
        for (int64_t s = 0; s < nsteps; ++s) {
            double* x = &tape[(s + 1) * dim];
            for (int d = 0; d < dim; ++d) x[d] = tape[s * dim + d];
            rk4_step(sys, dim, p, x, h, h2, h6);
        }
        double l[kMaxDim], mu[kMaxParams] = {0};
        for (int d = 0; d < dim; ++d) l[d] = lam[d * ld + i];
        std::vector<double> J(dim * dim), Fp(dim * (n_params > 0 ? n_params : 1));
        for (int64_t s = nsteps - 1; s >= 0; --s) {
            const double* x = &tape[s * dim];
            double k[kMaxDim], pts[4][kMaxDim];
            for (int d = 0; d < dim; ++d) pts[0][d] = x[d];
            rhs(sys, dim, p, x, k);
            for (int d = 0; d < dim; ++d) pts[1][d] = std::fma(h2, k[d], x[d]);
            rhs(sys, dim, p, pts[1], k);
            for (int d = 0; d < dim; ++d) pts[2][d] = std::fma(h2, k[d], x[d]);
            rhs(sys, dim, p, pts[2], k);
            for (int d = 0; d < dim; ++d) pts[3][d] = std::fma(h, k[d], x[d]);
            // stage adjoints, last stage first
            const double wlam[4] = {h6, h3, h3, h6};
            const double wprev[4] = {h2, h2, h, 0.0};  // how stage i+1's point uses k_i
            double b[4][kMaxDim];
            for (int st = 3; st >= 0; --st) {
                double abar[kMaxDim];
                for (int d = 0; d < dim; ++d)
                    abar[d] = wlam[st] * l[d] + (st < 3 ? wprev[st] * b[st + 1][d] : 0.0);
                jacobians(sys, dim, n_params, p, pts[st], J.data(), Fp.data());
                for (int c = 0; c < dim; ++c) {
                    double acc = 0.0;
                    for (int r = 0; r < dim; ++r) acc += J[r * dim + c] * abar[r];
                    b[st][c] = acc;
                }
                for (int q = 0; q < n_params; ++q) {
                    double acc = 0.0;
                    for (int r = 0; r < dim; ++r) acc += Fp[r * n_params + q] * abar[r];
                    mu[q] += acc;
                }
            }
            for (int d = 0; d < dim; ++d) l[d] = l[d] + b[0][d] + b[1][d] + b[2][d] + b[3][d];
        }
        for (int d = 0; d < dim; ++d) lam[d * ld + i] = l[d];
        for (int k = 0; k < n_pp; ++k) mu_pp[k * ld + i] = mu[pp_slot[k]];
        for (int q = 0; q < n_params; ++q) mu_all[static_cast<size_t>(i) * n_params + q] = mu[q];
    }
    if (mu_global) {
        for (int q = 0; q < n_params; ++q) {
            double acc = 0.0;
            for (int64_t i = 0; i < n; ++i) acc += mu_all[static_cast<size_t>(i) * n_params + q];
            mu_global[q] = acc;
        }
    }
    return 0;
}

int ffo_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    philox(ctr, key, out);
    return 0;
}

int ffo_rk4_reset(int sys, int dim, const double* params, int n_params, const int32_t* pp_slot,
                  int n_pp, const double* pparams, double* state, int64_t n, int64_t ld, double h,
                  int64_t nsteps, const double* bound_lo, const double* bound_hi,
                  const double* box_lo, const double* box_hi, int64_t max_age, uint64_t seed,
                  uint64_t id_offset, int32_t* age, uint32_t* n_resets, int nthreads) {
    if (!valid_common(sys, dim, n_params, pp_slot, n_pp, n, ld) || nsteps < 0) return -1;
    if (!bound_lo || !bound_hi || !box_lo || !box_hi || !age || !n_resets) return -1;
    const double h2 = h * 0.5, h6 = h / 6.0;
#pragma omp parallel for schedule(static) num_threads(threads_or_default(nthreads))
    for (int64_t i = 0; i < n; ++i) {
        double p[kMaxParams], x[kMaxDim];
        particle_params(params, n_params, pp_slot, n_pp, pparams, ld, i, p);
        for (int d = 0; d < dim; ++d) x[d] = state[d * ld + i];
        int32_t a = age[i];
        uint32_t r = n_resets[i];
        for (int64_t s = 0; s < nsteps; ++s) {
            rk4_step(sys, dim, p, x, h, h2, h6);
            a += 1;
            if (escaped(dim, x, bound_lo, bound_hi) || (max_age >= 0 && a > max_age)) {
                redraw(dim, box_lo, box_hi, seed, id_offset + (uint64_t)i, r, x);
                a = 0;
                r += 1;
            }
        }
        for (int d = 0; d < dim; ++d) state[d * ld + i] = x[d];
        age[i] = a;
        n_resets[i] = r;
    }
    return 0;
}

int ffo_rk4_reset_f32(int sys, int dim, const double* params, int n_params, const int32_t* pp_slot,
                      int n_pp, const float* pparams, float* state, float* comp, int kahan,
                      int64_t n, int64_t ld, float h, int64_t nsteps, const double* bound_lo,
                      const double* bound_hi, const double* box_lo, const double* box_hi,
                      int64_t max_age, uint64_t seed, uint64_t id_offset, int32_t* age,
                      uint32_t* n_resets, int nthreads) {
    if (!valid_common(sys, dim, n_params, pp_slot, n_pp, n, ld) || nsteps < 0) return -1;
    if (!bound_lo || !bound_hi || !box_lo || !box_hi || !age || !n_resets) return -1;
    if (kahan && comp == nullptr) return -1;
    const float h2 = h * 0.5f, h6 = h / 6.0f;
#pragma omp parallel for schedule(static) num_threads(threads_or_default(nthreads))
    for (int64_t i = 0; i < n; ++i) {
        float p[kMaxParams], x[kMaxDim], c[kMaxDim];
        particle_params(params, n_params, pp_slot, n_pp, pparams, ld, i, p);
        for (int d = 0; d < dim; ++d) {
            x[d] = state[d * ld + i];
            c[d] = kahan ? comp[d * ld + i] : 0.0f;
        }
        int32_t a = age[i];
        uint32_t r = n_resets[i];
        for (int64_t s = 0; s < nsteps; ++s) {
            if (kahan) rk4_step_kahan(sys, dim, p, x, c, h, h2, h6);
            else rk4_step(sys, dim, p, x, h, h2, h6);
            a += 1;
            if (escaped(dim, x, bound_lo, bound_hi) || (max_age >= 0 && a > max_age)) {
                redraw(dim, box_lo, box_hi, seed, id_offset + (uint64_t)i, r, x);
                for (int d = 0; d < dim; ++d) c[d] = 0.0f;
                a = 0;
                r += 1;
            }
        }
        for (int d = 0; d < dim; ++d) {
            state[d * ld + i] = x[d];
            if (kahan) comp[d * ld + i] = c[d];
        }
        age[i] = a;
        n_resets[i] = r;
    }
    return 0;
}

int ffo_histogram(int dim, const double* state, int n_pp, const double* pparams, int64_t n,
                  int64_t ld, int axis_x, int axis_y, double x_lo, double x_hi, double y_lo,
                  double y_hi, int nx, int ny, uint32_t* hist, uint64_t* n_dropped,
                  int accumulate) {
    auto axis_ok = [&](int a) { return (a >= 0 && a < dim) || (a < 0 && -1 - a < n_pp); };
    if (!axis_ok(axis_x) || !axis_ok(axis_y) || nx <= 0 || ny <= 0 || n < 0 || ld < n)
        return -1;
    if (!(x_hi > x_lo) || !(y_hi > y_lo)) return -1;
    if (!accumulate) {
        std::fill(hist, hist + static_cast<int64_t>(nx) * ny, 0u);
        *n_dropped = 0;
    }
    const double sx = nx / (x_hi - x_lo), sy = ny / (y_hi - y_lo);
    auto coord = [&](int a, int64_t i) {
        return a >= 0 ? state[a * ld + i] : pparams[(-1 - a) * ld + i];
    };
    for (int64_t i = 0; i < n; ++i) {
        const double vx = (coord(axis_x, i) - x_lo) * sx;
        const double vy = (coord(axis_y, i) - y_lo) * sy;
        if (vx >= 0.0 && vx < nx && vy >= 0.0 && vy < ny) {
            const int64_t ix = static_cast<int64_t>(vx), iy = static_cast<int64_t>(vy);
            hist[iy * nx + ix] += 1u;
        } else {
            *n_dropped += 1;
        }
    }
    return 0;
}

}  // extern "C"

extern "C" int ffo_render(int dim, const double* state, int n_pp, const double* pparams, int64_t n,
                          int64_t ld, const ffo_render_t* r, uint32_t* img, uint64_t* n_culled,
                          int accumulate) {
    auto axis_ok = [&](int a) { return (a >= 0 && a < dim) || (a < 0 && -1 - a < n_pp); };
    if (!r || !img || !n_culled || n < 0 || ld < n || r->width <= 0 || r->height <= 0 ||
        r->radius < 0)
        return -1;
    for (int i = 0; i < 3; ++i)
        if (!axis_ok(r->axis[i])) return -1;
    const int64_t W = r->width, H = r->height;
    if (!accumulate) {
        std::fill(img, img + W * H * 3, 0u);
        *n_culled = 0;
    }
    auto coord = [&](int a, int64_t i) {
        return a >= 0 ? state[a * ld + i] : pparams[(-1 - a) * ld + i];
    };
    const double reach = r->radius + 1.0;
    for (int64_t i = 0; i < n; ++i) {
        const double a[3] = {coord(r->axis[0], i), coord(r->axis[1], i), coord(r->axis[2], i)};
        double c[4];
        for (int row = 0; row < 4; ++row) {
            const double* m = r->mvp + 4 * row;
            c[row] = m[0] * a[0] + m[1] * a[1] + m[2] * a[2] + m[3];
        }
        bool keep = c[3] > 0.0;
        double ndc[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < 3 && keep; ++k) {
            ndc[k] = c[k] / c[3];
            keep = ndc[k] >= -1.0 && ndc[k] <= 1.0;
        }
        if (!keep) {
            *n_culled += 1;
            continue;
        }
        const double px = (ndc[0] + 1.0) * (double)W / 2.0;
        const double py = (1.0 - ndc[1]) * (double)H / 2.0;
        double rgb[3];
        for (int k = 0; k < 3; ++k) {
            double v = r->base[k];
            for (int j = 0; j < 3; ++j) v += r->grad[3 * k + j] * (a[j] - r->origin[j]);
            rgb[k] = std::min(std::max(v, 0.0), 1.0);
        }
        // radius 0: the pixel containing (px, py); radius R: every pixel whose
        // centre lies closer than R + 1 to (px, py)
        int64_t x0 = (int64_t)std::floor(px), x1 = x0, y0 = (int64_t)std::floor(py), y1 = y0;
        if (r->radius > 0) {
            x0 = (int64_t)std::floor(px - reach);
            x1 = (int64_t)std::floor(px + reach);
            y0 = (int64_t)std::floor(py - reach);
            y1 = (int64_t)std::floor(py + reach);
        }
        for (int64_t iy = y0; iy <= y1; ++iy) {
            for (int64_t ix = x0; ix <= x1; ++ix) {
                if (ix < 0 || ix >= W || iy < 0 || iy >= H) continue;
                double wgt = r->weight;
                if (r->radius > 0) {
                    const double dx = ((double)ix + 0.5) - px, dy = ((double)iy + 0.5) - py;
                    const double d = std::sqrt(dx * dx + dy * dy);
                    if (!(d < reach)) continue;
                    const double f = 1.0 - d / reach;
                    wgt = r->weight * (f * f);
                }
                for (int k = 0; k < 3; ++k)
                    img[(iy * W + ix) * 3 + k] += (uint32_t)std::nearbyint(256.0 * (wgt * rgb[k]));
            }
        }
    }
    return 0;
}
