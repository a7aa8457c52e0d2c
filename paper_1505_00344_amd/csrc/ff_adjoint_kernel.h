// ff_adjoint_kernel.h — discrete adjoint of the fused RK4 map (exact reverse-mode
// gradient of the classical RK4 step of Section 2.1 / Appendix A.1 with
// respect to the state and the parameters).
//
// For one step x' = x + (h/6)(k1 + 2k2 + 2k3 + k4) with stage points
// y1 = x, y2 = x + (h/2)k1, y3 = x + (h/2)k2, y4 = x + h k3 and an incoming
// adjoint lam' = dL/dx':
//   abar4 = (h/6) lam'            g4 = J(y4)^T abar4
//   abar3 = (h/3) lam' + h g4     g3 = J(y3)^T abar3
//   abar2 = (h/3) lam' + h/2 g3   g2 = J(y2)^T abar2
//   abar1 = (h/6) lam' + h/2 g2   g1 = J(y1)^T abar1
//   lam = lam' + (((g4 + g3) + g2) + g1),  mu += sum_i (df/dp)(y_i)^T abar_i.
// The compensated (Kahan) update is differentiated as exact addition.
//
// Memory: one kernel launch per checkpoint segment (the forward pass stored
// the state every K steps).  Inside a segment each thread
//   A. replays the segment from its checkpoint, storing its state every T
//      steps into a sub-checkpoint buffer in HBM (its own slots only), then
//   B. walks the sub-blocks backwards: re-runs T steps from the
//      sub-checkpoint into a register tape of T states (compile-time indices,
//      so no scratch), then applies T reverse steps.
// The replays run the same rk4_step code as the forward kernel, so every
// recomputed state is bitwise the forward state.  Cost per step: two forward
// steps (A and B), three right-hand sides for the stage points and four VJPs;
// with CAPTURE, B keeps the stage points it computes anyway (and computes
// those of its last state), so the reverse steps evaluate no right-hand side.
//
// Device code only: the library instantiates it for its built-in systems and
// hands the same text to hipRTC for systems given as expressions.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>

#include <cstdint>
#endif
#include "ff_kernel.h"

namespace ff {

struct AdjArgs {
    const void* pp;
    int64_t n, ld;
    int n_pp;
    int slot[kMaxPP];
    ParamBlock p;
    double h, h2, h6, h3;
    const void* ckpt;
    const void* ckpt_c;
    void* sub;
    void* sub_c;
    void* lam;
    void* mu;
    double* mu_part;
    void* carry;  // [NP][n] per-particle parameter adjoints carried between segments
    int64_t seg_len;
    int first;    // first segment processed (the last in time): start from zero
    int last;     // last segment processed (the first in time): write mu, mu_part
};

// One reverse step.  LOWREG keeps the stage points y2, y3, y4 out of
// registers, where the large systems would spill: they are computed once and
// parked in LDS, in this thread's own column of `lds` (3 * D rows of
// kAdjBlock entries, no sharing between threads, so no barrier), and each is
// loaded back when its vector-Jacobian product needs it.
// With HAVE_YS the stage points come in `given` (kept by the replay that
// produced x) instead of being recomputed.
template <class S, typename R, bool LOWREG, bool HAVE_YS = false>
__device__ __forceinline__ void vjp_step(const R (&p)[S::NP], const R (&q)[S::NQ], const R (&x)[S::D],
                                         R (&lam)[S::D], R (&gp)[S::NP], R h, R h2, R h6, R h3,
                                         R* lds = nullptr, const R (*given)[S::D] = nullptr) {
    constexpr int D = S::D;
    R ys[3][D];  // y2, y3, y4 when !LOWREG
    if constexpr (HAVE_YS) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int d = 0; d < D; ++d) ys[j][d] = given[j][d];
    } else if constexpr (LOWREG) {
        R y[D], k[D];
#pragma unroll
        for (int d = 0; d < D; ++d) y[d] = x[d];
#pragma unroll 1
        for (int j = 0; j < 3; ++j) {
            S::f(p, q, y, k);
            const R w = (j == 2) ? h : h2;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                y[d] = M<R>::fma_(w, k[d], x[d]);
                lds[(j * D + d) * kAdjBlock] = y[d];
            }
        }
    } else {
        R k[D];
        S::f(p, q, x, k);
#pragma unroll
        for (int d = 0; d < D; ++d) ys[0][d] = M<R>::fma_(h2, k[d], x[d]);
        S::f(p, q, ys[0], k);
#pragma unroll
        for (int d = 0; d < D; ++d) ys[1][d] = M<R>::fma_(h2, k[d], x[d]);
        S::f(p, q, ys[1], k);
#pragma unroll
        for (int d = 0; d < D; ++d) ys[2][d] = M<R>::fma_(h, k[d], x[d]);
    }
    R a[D], g[D], gs[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        a[d] = h6 * lam[d];
        gs[d] = R(0);
    }
    // stages 4, 3, 2, 1: the weight that carries g_s into abar_{s-1} is
    // h (stage 4 -> 3) or h/2; the lam' weight of abar_{s-1} is h/3, h/3, h/6
    auto stage = [&](int s) {
#pragma unroll
        for (int d = 0; d < D; ++d) g[d] = R(0);
        if (s == 1) {
            S::vjp(p, q, x, a, g, gp);
        } else if constexpr (LOWREG) {
            R y[D];
#pragma unroll
            for (int d = 0; d < D; ++d) y[d] = lds[((s - 2) * D + d) * kAdjBlock];
            S::vjp(p, q, y, a, g, gp);
        } else {
            S::vjp(p, q, ys[s - 2], a, g, gp);
        }
        const R wg = (s == 4) ? h : h2;
        const R wl = (s == 2) ? h6 : h3;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            gs[d] = gs[d] + g[d];
            if (s > 1) a[d] = M<R>::fma_(wg, g[d], wl * lam[d]);
        }
    };
    if constexpr (LOWREG) {
        // kept as a loop so the scheduler cannot hoist the loads of later
        // stage points above earlier VJPs (that would defeat LOWREG)
#pragma unroll 1
        for (int s = 4; s >= 1; --s) stage(s);
    } else {
        stage(4);
        stage(3);
        stage(2);
        stage(1);
    }
#pragma unroll
    for (int d = 0; d < D; ++d) lam[d] = lam[d] + gs[d];
}

// Blocks of kAdjBlock threads that the adjoint kernel of system S must fit
// on one CU, i.e. a register cap (1: none); specialised where measured.
template <class S> struct AdjMinBlocks {
    static constexpr int value = 1;
};

// CAPTURE (register tape only): the replay of a sub-block also keeps the
// stage points of every tape state, so that the reverse steps need no right-hand
// side evaluations of their own (3 * T more values in registers).
template <class S, typename R, bool KAHAN, int T, bool LOWREG, bool CAPTURE = false>
__global__ void __launch_bounds__(kAdjBlock, AdjMinBlocks<S>::value) k_adj(AdjArgs a) {
    constexpr int D = S::D, NP = S::NP;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i0 < a.n;
    const int64_t i = act ? i0 : a.n - 1;
    const int64_t n = a.n;

    R p[NP];
    {
        const R* pp = static_cast<const R*>(a.pp);
        R v[kMaxPP];
#pragma unroll
        for (int k = 0; k < kMaxPP; ++k) v[k] = (k < a.n_pp) ? pp[k * a.ld + i] : R(0);
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            R val = R(a.p.v[q]);
#pragma unroll
            for (int k = 0; k < kMaxPP; ++k)
                if (k < a.n_pp && a.slot[k] == q) val = v[k];
            p[q] = val;
        }
    }
    R qd[S::NQ];
    S::derive(p, qd);
    const R h = R(a.h), h2 = R(a.h2), h6 = R(a.h6), h3 = R(a.h3);

    const R* ck = static_cast<const R*>(a.ckpt);
    const R* ckc = static_cast<const R*>(a.ckpt_c);
    R* sub = static_cast<R*>(a.sub);
    R* subc = static_cast<R*>(a.sub_c);

    // A. replay the segment, keeping the state every T steps
    R x[D], c[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        x[d] = ck[d * n + i];
        c[d] = KAHAN ? ckc[d * n + i] : R(0);
    }
    const int64_t L = a.seg_len;
    const int64_t nsub = (L + T - 1) / T;
    for (int64_t b = 0; b < nsub; ++b) {
        R* sb = sub + b * D * n;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            sb[d * n + i] = x[d];
            // the compensation is only needed to replay steps inside a
            // sub-block, and a sub-block of one step replays none
            if (KAHAN && T > 1) subc[b * D * n + d * n + i] = c[d];
        }
        if (b + 1 < nsub)
            for (int t = 0; t < T; ++t) rk4_step<S, R, KAHAN>(p, qd, x, c, h, h2, h6);
    }

    // B. reverse sweep
    R* stage_lds = nullptr;  // this thread's column of the stage-point store
    if constexpr (LOWREG) {
        __shared__ R stage_store[3 * D * kAdjBlock];
        stage_lds = stage_store + threadIdx.x;
    }
    R lam[D], gp[NP];
    R* lm = static_cast<R*>(a.lam);
#pragma unroll
    for (int d = 0; d < D; ++d) lam[d] = lm[d * a.ld + i];
    R* carry = static_cast<R*>(a.carry);
#pragma unroll
    for (int q = 0; q < NP; ++q) gp[q] = a.first ? R(0) : carry[q * n + i];
    for (int64_t b = nsub - 1; b >= 0; --b) {
        const int64_t len = (L - b * T) < T ? (L - b * T) : T;
        R tape[T][D];
        R stages[CAPTURE ? T : 1][3][D];  // y2, y3, y4 of every tape state (CAPTURE)
        R xs[D], cs[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            xs[d] = sub[b * D * n + d * n + i];
            cs[d] = (KAHAN && T > 1) ? subc[b * D * n + d * n + i] : R(0);
            tape[0][d] = xs[d];
        }
        if constexpr (CAPTURE) {
#pragma unroll
            for (int t = 0; t < T; ++t) {
                if (t + 1 < len) {
                    rk4_step<S, R, KAHAN, true>(p, qd, xs, cs, h, h2, h6, stages[t]);
#pragma unroll
                    for (int d = 0; d < D; ++d) tape[t + 1][d] = xs[d];
                } else if (t + 1 == len) {  // the last state: its stage points only
                    rk4_step<S, R, KAHAN, true, false>(p, qd, xs, cs, h, h2, h6, stages[t]);
                }
            }
        } else {
#pragma unroll
            for (int t = 1; t < T; ++t) {
                if (t < len) {
                    rk4_step<S, R, KAHAN>(p, qd, xs, cs, h, h2, h6);
#pragma unroll
                    for (int d = 0; d < D; ++d) tape[t][d] = xs[d];
                }
            }
        }
#pragma unroll
        for (int t = T - 1; t >= 0; --t) {
            if (t < len) {
                if constexpr (CAPTURE)
                    vjp_step<S, R, false, true>(p, qd, tape[t], lam, gp, h, h2, h6, h3, nullptr, stages[t]);
                else
                    vjp_step<S, R, LOWREG>(p, qd, tape[t], lam, gp, h, h2, h6, h3, stage_lds);
            }
        }
    }
    if (act) {
#pragma unroll
        for (int d = 0; d < D; ++d) lm[d * a.ld + i] = lam[d];
        if (!a.last) {
#pragma unroll
            for (int q = 0; q < NP; ++q) carry[q * n + i] = gp[q];
        } else {
            R* mu = static_cast<R*>(a.mu);
#pragma unroll
            for (int k = 0; k < kMaxPP; ++k) {
                if (k < a.n_pp) {
                    R g = R(0);
#pragma unroll
                    for (int q = 0; q < NP; ++q)
                        if (a.slot[k] == q) g = gp[q];
                    mu[k * a.ld + i] = g;
                }
            }
        }
    }
    // per-block FP64 sums of every parameter adjoint, in a fixed order
    if (a.last && a.mu_part) {
        __shared__ double red[kAdjBlock / 64][kMaxParams];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            double v = act ? (double)gp[q] : 0.0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) red[wv][q] = v;
        }
        __syncthreads();
        if (threadIdx.x < NP) {
            double s = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w][threadIdx.x];
            a.mu_part[(int64_t)blockIdx.x * kMaxParams + threadIdx.x] = s;
        }
    }
}

}  // namespace ff
