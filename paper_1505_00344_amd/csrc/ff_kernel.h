// ff_kernel.h — the fused classical-RK4 particle kernel for gfx950 (device
// code only).  The library instantiates it for its built-in right-hand sides,
// and the kernels it compiles at run time from user expressions include this
// same text, so both kinds of system share one kernel skeleton.
//
// One thread owns PPT particles.  Particle i of block b, slot j, is
//   i = b * (blockDim * PPT) + j * blockDim + threadIdx.x,
// so every load and store of a component row state[d*ld + i] is a coalesced,
// contiguous 64-lane access.  The state (and the Kahan compensation) is read
// once, advanced `steps` RK4 steps entirely in VGPRs, and written once: the
// HBM traffic of a launch is 2*D*sizeof(R) bytes per particle (+ parameters,
// + compensation) whatever the number of fused steps, so for steps >= ~8 the
// kernel is bound by the vector ALU, not by HBM.
//
// Step (Section 2.1 / Appendix A.1: classical fourth-order Runge-Kutta with a
// constant, signed step h), written to keep few registers live while
// preserving the order of operations
//   s = k2 + k3; s = fma(2, s, k1); s = s + k4; x = fma(h6, s, x):
//   k1 = f(x); y = fma(h2,k1,x); k = f(y) [k2]; y = fma(h2,k,x); acc = k;
//   k = f(y) [k3]; y = fma(h,k,x); acc = acc + k; acc = fma(2,acc,k1);
//   k = f(y) [k4]; acc = acc + k; update.
// Kahan-compensated update (single precision): inc = h6*acc; y = inc - c;
// t = x + y; c = (t - x) - y; x = t.  Systems with FUSED_INC (those evaluated
// with the fast single-precision functions) form y = fma(h6, acc, -c) instead:
// one instruction fewer per component, and the product's rounding, which the
// compensation would otherwise not see, is left out.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>

#include <cstdint>
#endif
#include "ff_math.h"
#include "ff_rng.h"

namespace ff {

constexpr int kMaxParams = 16;
constexpr int kMaxPP = 4;  // per-particle parameter overrides (FF_MAX_PP)
constexpr int kMaxDim = 15;
constexpr int kAdjBlock = 256;  // threads per block of the adjoint kernel

struct ParamBlock {
    double v[kMaxParams];
};

// With STAGES the stage points y2, y3, y4 of the step are also written to
// ys[0..2] (the adjoint's replay keeps them for the reverse step); with
// UPDATE false only they are computed and x, c are left unchanged.
template <class S, typename R, bool KAHAN, bool STAGES = false, bool UPDATE = true>
__device__ __forceinline__ void rk4_step(const R (&p)[S::NP], const R (&q)[S::NQ], R (&x)[S::D], R (&c)[S::D],
                                         R h, R h2, R h6, R (*ys)[S::D] = nullptr) {
    constexpr int D = S::D;
    R k1[D], k[D], y[D], acc[D];
    S::f(p, q, x, k1);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        y[d] = M<R>::fma_(h2, k1[d], x[d]);
        if constexpr (STAGES) ys[0][d] = y[d];
    }
    S::f(p, q, y, k);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        y[d] = M<R>::fma_(h2, k[d], x[d]);
        if constexpr (STAGES) ys[1][d] = y[d];
        acc[d] = k[d];
    }
    S::f(p, q, y, k);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        y[d] = M<R>::fma_(h, k[d], x[d]);
        if constexpr (STAGES) ys[2][d] = y[d];
        acc[d] = acc[d] + k[d];
        acc[d] = M<R>::fma_(R(2), acc[d], k1[d]);
    }
    if constexpr (!UPDATE) return;
    S::f(p, q, y, k);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        acc[d] = acc[d] + k[d];
        if constexpr (KAHAN) {
            const R yk = S::FUSED_INC ? M<R>::fma_(h6, acc[d], -c[d]) : h6 * acc[d] - c[d];
            const R t = x[d] + yk;
            c[d] = (t - x[d]) - yk;
            x[d] = t;
        } else {
            x[d] = M<R>::fma_(h6, acc[d], x[d]);
        }
    }
}

struct RK4Args {
    void* state;
    void* comp;
    const void* pp;
    int64_t n, ld;
    int n_pp;
    int slot[kMaxPP];
    ParamBlock p;
    double h, h2, h6;
    int64_t steps;
    void* ckpt;
    void* ckpt_c;
    int64_t ckpt_ld;
};

// The reset rule (Section 2.1): after every step a particle that left the
// bounds (NaN counts as outside) or whose age exceeds max_age is redrawn
// uniformly in its group's box from Philox4x32-10 (draw number = its reset
// count, identity = id_offset + index), its compensation and age are zeroed.
// FP64: u = ((a >> 5) * 2^26 + (b >> 6)) * 2^-53 from words 2d, 2d+1;
// FP32: u = (a >> 8) * 2^-24 from word d; x = fma(width, u, lo).
struct ResetArgs {
    double blo[kMaxDim], bhi[kMaxDim];  // bounds, compared in double
    float blf[kMaxDim], bhf[kMaxDim];   // smallest float >= blo, largest float <= bhi
    double wd[kMaxDim], lod[kMaxDim];   // box width and low end (double)
    float wf[kMaxDim], lof[kMaxDim];    // the same rounded to float
    int64_t max_age;
    uint64_t seed, id_offset;
    int32_t* age;
    uint32_t* nres;
};

// Trajectory recording: after global step g (1-based) with g % every == 0,
// particle i with i % stride == 0 stores its state in
// out[(g / every - 1)][d][i / stride] (m = recorded particles per record).
struct RecordArgs {
    void* out;
    int64_t every, stride, m, step0;  // step0: global index of this launch's first step
};

// Lanes of a wave that must need a redraw before the wave draws for them.
constexpr int kRefillLanes = 8;

// For a float v, v >= blo exactly when v >= blf (and likewise above), so
// single-precision states are tested against the float thresholds without a
// conversion to double.
template <typename R, int D>
__device__ __forceinline__ bool escaped(const R (&x)[D], const ResetArgs& r) {
    bool out = false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if constexpr (sizeof(R) == sizeof(float)) out = out || !(x[d] >= r.blf[d] && x[d] <= r.bhf[d]);
        else out = out || !(x[d] >= r.blo[d] && x[d] <= r.bhi[d]);
    }
    return out;
}

template <int D>
__device__ __forceinline__ void redraw(double (&x)[D], const ResetArgs& r, uint64_t g, uint32_t k) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const uint32_t a = draw_word(r.seed, g, k, 2 * d), b = draw_word(r.seed, g, k, 2 * d + 1);
        const double u = ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
        x[d] = __builtin_fma(r.wd[d], u, r.lod[d]);
    }
}

template <int D>
__device__ __forceinline__ void redraw(float (&x)[D], const ResetArgs& r, uint64_t g, uint32_t k) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const float u = (float)(draw_word(r.seed, g, k, d) >> 8) * (1.0f / 16777216.0f);
        x[d] = __builtin_fmaf(r.wf[d], u, r.lof[d]);
    }
}

// Apply per-particle overrides with compile-time indices only, so the
// parameter array stays in registers (no scratch).
template <class S, typename R>
__device__ __forceinline__ void load_params(const RK4Args& a, int64_t i, R (&p)[S::NP]) {
    const R* pp = static_cast<const R*>(a.pp);
    R v[kMaxPP];
#pragma unroll
    for (int k = 0; k < kMaxPP; ++k) v[k] = (k < a.n_pp) ? pp[k * a.ld + i] : R(0);
#pragma unroll
    for (int q = 0; q < S::NP; ++q) {
        R val = R(a.p.v[q]);
#pragma unroll
        for (int k = 0; k < kMaxPP; ++k)
            if (k < a.n_pp && a.slot[k] == q) val = v[k];
        p[q] = val;
    }
}

// Advance the tile of blockDim*PPT particles starting at particle `first`.
// Shared by the one-group launch (k_rk4) and the persistent ragged-batch
// launch, so both produce the same bits.
template <class S, typename R, bool KAHAN, int PPT, bool RESET = false, bool RECORD = false>
__device__ __forceinline__ void rk4_tile(const RK4Args& a, int64_t first, const ResetArgs* rs = nullptr,
                                         const RecordArgs* rc = nullptr) {
    constexpr int D = S::D;
    R* st = static_cast<R*>(a.state);
    R* cp = static_cast<R*>(a.comp);
    const int64_t base = first + threadIdx.x;
    R x[PPT][D], c[PPT][D], p[PPT][S::NP], q[PPT][S::NQ];
    int64_t idx[PPT];
    bool act[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int64_t i = base + (int64_t)j * blockDim.x;
        act[j] = i < a.n;
        idx[j] = act[j] ? i : a.n - 1;  // n >= 1: inactive lanes shadow a valid particle
        load_params<S, R>(a, idx[j], p[j]);
        S::derive(p[j], q[j]);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            x[j][d] = st[d * a.ld + idx[j]];
            c[j][d] = KAHAN ? cp[d * a.ld + idx[j]] : R(0);
        }
    }
    if (a.ckpt) {  // checkpointed forward: keep the starting state of this launch
        R* ck = static_cast<R*>(a.ckpt);
        R* ckc = static_cast<R*>(a.ckpt_c);
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (!act[j]) continue;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                ck[d * a.ckpt_ld + idx[j]] = x[j][d];
                if (KAHAN) ckc[d * a.ckpt_ld + idx[j]] = c[j][d];
            }
        }
    }
    const R h = R(a.h), h2 = R(a.h2), h6 = R(a.h6);
    int32_t age[PPT];
    uint32_t nres[PPT];
    // A redraw depends only on (particle, reset count), so each particle's
    // next one is drawn ahead: nxt[j] holds draw number nres[j] while
    // fresh[j].  Drawing inside the reset branch would run Philox's ten
    // multiply rounds for most waves at most steps (a few lanes of a wave
    // reset in most steps); instead a reset takes nxt[j] and a wave refills
    // its consumed draws together once kRefillLanes lanes need one.  The
    // values are the same draws, so results do not change.
    R nxt[PPT][RESET ? D : 1];
    bool fresh[PPT];
    if constexpr (RESET) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            age[j] = rs->age[idx[j]];
            nres[j] = rs->nres[idx[j]];
            redraw<D>(nxt[j], *rs, rs->id_offset + (uint64_t)idx[j], nres[j]);
            fresh[j] = true;
        }
    }
    // steps per loop trip: each system's own measured choice (two lets the
    // loop-carried state of Lorenz avoid register copies); one with the reset
    // rule, whose wave-wide refill vote cannot be unrolled
    constexpr int kStepsPerTrip = RESET ? 1 : S::UNROLL;
#pragma unroll kStepsPerTrip
    for (int64_t s = 0; s < a.steps; ++s) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            rk4_step<S, R, KAHAN>(p[j], q[j], x[j], c[j], h, h2, h6);
            if constexpr (RESET) {
                age[j] += 1;
                if (escaped<R, D>(x[j], *rs) || (rs->max_age >= 0 && age[j] > rs->max_age)) {
                    // a second reset before the refill draws here
                    if (!fresh[j]) redraw<D>(nxt[j], *rs, rs->id_offset + (uint64_t)idx[j], nres[j]);
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        x[j][d] = nxt[j][d];
                        c[j][d] = R(0);
                    }
                    age[j] = 0;
                    nres[j] += 1;
                    fresh[j] = false;
                }
            }
        }
        if constexpr (RESET) {
            bool need = false;
#pragma unroll
            for (int j = 0; j < PPT; ++j) need = need || !fresh[j];
            if (__popcll(__ballot(need)) >= kRefillLanes) {  // uniform over the wave
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    if (!fresh[j]) {
                        redraw<D>(nxt[j], *rs, rs->id_offset + (uint64_t)idx[j], nres[j]);
                        fresh[j] = true;
                    }
                }
            }
        }
        if constexpr (RECORD) {
            const int64_t g = rc->step0 + s + 1;
            if (g % rc->every == 0) {
                R* out = static_cast<R*>(rc->out) + (g / rc->every - 1) * D * rc->m;
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    if (act[j] && idx[j] % rc->stride == 0) {
                        const int64_t slot = idx[j] / rc->stride;
#pragma unroll
                        for (int d = 0; d < D; ++d) out[d * rc->m + slot] = x[j][d];
                    }
                }
            }
        }
    }
    if constexpr (RESET) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (!act[j]) continue;
            rs->age[idx[j]] = age[j];
            rs->nres[idx[j]] = nres[j];
        }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        if (!act[j]) continue;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            st[d * a.ld + idx[j]] = x[j][d];
            if (KAHAN) cp[d * a.ld + idx[j]] = c[j][d];
        }
    }
}

template <class S, typename R, bool KAHAN, int PPT>
__global__ void __launch_bounds__(256) k_rk4(RK4Args a) {
    rk4_tile<S, R, KAHAN, PPT>(a, (int64_t)blockIdx.x * ((int64_t)blockDim.x * PPT));
}

template <class S, typename R, bool KAHAN, int PPT>
__global__ void __launch_bounds__(256) k_rk4_reset(RK4Args a, ResetArgs r) {
    rk4_tile<S, R, KAHAN, PPT, true>(a, (int64_t)blockIdx.x * ((int64_t)blockDim.x * PPT), &r);
}

template <class S, typename R, bool KAHAN, int PPT, bool RESET>
__global__ void __launch_bounds__(256) k_rk4_record(RK4Args a, ResetArgs r, RecordArgs rc) {
    rk4_tile<S, R, KAHAN, PPT, RESET, true>(a, (int64_t)blockIdx.x * ((int64_t)blockDim.x * PPT),
                                            RESET ? &r : nullptr, &rc);
}

}  // namespace ff
