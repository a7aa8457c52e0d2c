/*
 * ffo.h — the CPU oracle for the Fireflies particle-RK4 hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, constant or helper with the HIP library; both sides are written
 * independently from the paper (Merrison-Hort, "Fireflies", arXiv:1505.00344).
 *
 * What it computes (plain, slow, obviously correct; FP64 unless stated):
 *   - classical fourth-order Runge-Kutta with a constant, signed step for every
 *     particle independently (Section 2.1: one solver, RK4 with constant step;
 *     Appendix A.1: read position, RK4 update, write back; Appendix A.2: the
 *     step may be positive or negative);
 *   - the right-hand sides of the paper's systems: Lorenz (Section 2.2,
 *     Eqs. lorenz_x/y/z), a Wilson-Cowan E/I pair standing in for the
 *     STN-GPe model (Section 2.1, Eqs. stn_gpe/eqnGPe, whose constants the
 *     paper does not print), the Hodgkin-Huxley ring with first-order
 *     synapses (Section 3, Eqs. hh_v/hh_h/hh_m/hh_n/hh_isyn/hh_s), linear
 *     test systems x' = A x, and (oracle only, for pinning the tableau) the
 *     scalar Riccati equation y' = y^2;
 *   - per-particle parameter values, the paper's "parameter as a state with
 *     zero derivative" bifurcation trick (Section 2.1 and Section 2.2);
 *   - the 2D density projection as integer counts (Appendix A.1, additive
 *     blending of unit-weight points = counting);
 *   - the exact gradient of the discrete RK4 map (reverse mode), with the
 *     full Jacobian and parameter Jacobian formed explicitly;
 *   - the same RK4 map in complex arithmetic (complex-step derivative,
 *     Squire & Trapp 1998), used to pin the adjoint;
 *   - the same RK4 map in single precision, plain and with a Kahan-compensated
 *     update, for bit-level checks of single-precision kernels on systems
 *     without transcendental functions.
 *
 * Layout: structure of arrays.  state[d*ld + i] is component d of particle i;
 * pparams[k*ld + i] is per-particle parameter k of particle i, which replaces
 * global parameter pp_slot[k].  All pointers are host memory owned by the
 * caller.  Every function returns 0 on success and a negative code on invalid
 * arguments (nothing is written then).
 */
#ifndef FFO_H
#define FFO_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { FFO_LINEAR = 0, FFO_LORENZ = 1, FFO_WILSON_COWAN = 2, FFO_HH_RING = 3, FFO_RICCATI = 100 };

/* Number of global parameters a system expects for a given dimension, or -1. */
int ffo_n_params(int sys, int dim);

/* f(x) for m points x[m][dim] (row-major, one point per row) -> f[m][dim]. */
int ffo_rhs(int sys, int dim, const double* params, int n_params,
            const double* x, double* f, int64_t m);

/* Jacobian J[m][dim][dim] (J[r][c] = d f_r / d x_c) and parameter Jacobian
 * Fp[m][dim][n_params] at m points, both formed explicitly. */
int ffo_jacobians(int sys, int dim, const double* params, int n_params,
                  const double* x, double* J, double* Fp, int64_t m);

/* nsteps classical RK4 steps of size h on every particle (FP64). */
int ffo_rk4(int sys, int dim, const double* params, int n_params,
            const int32_t* pp_slot, int n_pp, const double* pparams,
            double* state, int64_t n, int64_t ld, double h, int64_t nsteps,
            int nthreads);

/* The same map in single precision: state/pparams are float; params are
 * rounded to float once.  kahan != 0 uses the compensated update with the
 * compensation array comp (same layout as state, carried in and out). */
int ffo_rk4_f32(int sys, int dim, const double* params, int n_params,
                const int32_t* pp_slot, int n_pp, const float* pparams,
                float* state, float* comp, int kahan, int64_t n, int64_t ld,
                float h, int64_t nsteps, int nthreads);

/* Complex-step directional derivative of the FP64 map.  Inputs are perturbed
 * by i*eps times the directions dx0 (SoA like state), dparams (n_params) and
 * dpp (SoA like pparams); any direction pointer may be NULL (= zero).
 * Outputs: xT (real part, SoA) and dxT (imaginary part / eps, SoA). */
int ffo_rk4_cstep(int sys, int dim, const double* params, int n_params,
                  const int32_t* pp_slot, int n_pp, const double* pparams,
                  const double* x0, const double* dx0, const double* dparams,
                  const double* dpp, double eps, double* xT, double* dxT,
                  int64_t n, int64_t ld, double h, int64_t nsteps, int nthreads);

/* Exact reverse-mode gradient of the FP64 map.  On entry lam[dim][ld] holds
 * dL/dx_T; on exit dL/dx_0.  x0 is the initial state (not modified).
 * mu_pp[n_pp][ld] receives dL/d(per-particle parameter k) (may be NULL when
 * n_pp == 0); mu_global[n_params] receives the sum over particles of
 * dL/d(parameter j) (may be NULL). */
int ffo_adjoint(int sys, int dim, const double* params, int n_params,
                const int32_t* pp_slot, int n_pp, const double* pparams,
                const double* x0, double* lam, double* mu_pp, double* mu_global,
                int64_t n, int64_t ld, double h, int64_t nsteps, int nthreads);

/* 2D density projection.  axis >= 0 selects state component axis, axis < 0
 * selects per-particle parameter (-1 - axis).  Half-open ranges
 * [x_lo, x_hi) x [y_lo, y_hi) with nx x ny bins; hist[iy*nx + ix] += 1;
 * particles outside or with NaN coordinates increment *n_dropped.
 * accumulate == 0 clears hist and *n_dropped first. */
int ffo_histogram(int dim, const double* state, int n_pp, const double* pparams,
                  int64_t n, int64_t ld, int axis_x, int axis_y,
                  double x_lo, double x_hi, double y_lo, double y_hi,
                  int nx, int ny, uint32_t* hist, uint64_t* n_dropped,
                  int accumulate);

/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11): out = the 10-round
 * bijection of counter ctr[4] under key key[2]. */
int ffo_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out);

/* RK4 with the paper's reset rule (Section 2.1: a trajectory that leaves the
 * region, or that has not been reset for more than T_max, restarts from new
 * random initial conditions; Appendix A: state-variable bounds and the
 * group's initial-condition box).  After every step: age += 1; if a component
 * is outside [bound_lo, bound_hi] (NaN counts as outside) or age > max_age
 * (max_age < 0: never), the particle is redrawn uniformly in
 * [box_lo, box_hi), age = 0 and n_resets += 1.  Draw number r (= n_resets
 * before the reset) of particle g = id_offset + i uses Philox4x32-10 with key
 * (seed low, seed high) and counter (g low, g high, r, j) for block j.
 * FP64: component d takes words 2d, 2d+1 of the stream (a, b) and
 * u = ((a >> 5) * 2^26 + (b >> 6)) * 2^-53; x = fma(box_hi - box_lo, u, box_lo).
 * FP32: component d takes word d, u = (a >> 8) * 2^-24,
 * x = fmaf((float)(box_hi - box_lo), u, (float)box_lo); a reset also zeroes
 * the Kahan compensation.  age (int32) and n_resets (uint32) are [ld] arrays,
 * carried in and out. */
int ffo_rk4_reset(int sys, int dim, const double* params, int n_params, const int32_t* pp_slot,
                  int n_pp, const double* pparams, double* state, int64_t n, int64_t ld, double h,
                  int64_t nsteps, const double* bound_lo, const double* bound_hi,
                  const double* box_lo, const double* box_hi, int64_t max_age, uint64_t seed,
                  uint64_t id_offset, int32_t* age, uint32_t* n_resets, int nthreads);
int ffo_rk4_reset_f32(int sys, int dim, const double* params, int n_params, const int32_t* pp_slot,
                      int n_pp, const float* pparams, float* state, float* comp, int kahan,
                      int64_t n, int64_t ld, float h, int64_t nsteps, const double* bound_lo,
                      const double* bound_hi, const double* box_lo, const double* box_hi,
                      int64_t max_age, uint64_t seed, uint64_t id_offset, int32_t* age,
                      uint32_t* n_resets, int nthreads);

/* Particle image (Appendix A "Render Technique"; Appendix A.1 vertex,
 * geometry and fragment shaders with additive blending).  For each particle:
 * the axis values a = (a0, a1, a2) (state component or per-particle parameter
 * -1-k) form p = (a0, a1, a2, 1); c = M p with M the row-major 4x4
 * projection * view * model matrix; the particle is culled if c3 <= 0 or a
 * normalised coordinate c_i / c3 (i = 0, 1, 2) lies outside [-1, 1] or is
 * NaN; otherwise its pixel position is px = (c0/c3 + 1) * W / 2,
 * py = (1 - c1/c3) * H / 2.  Colour: rgb_k = min(max(base_k + sum_i
 * grad[k][i] (a_i - origin_i), 0), 1).  Sprite: radius 0 gives
 * w = weight to the pixel (floor(px), floor(py)); radius R > 0 gives every
 * pixel (ix, iy) with floor(px - R - 1) <= ix <= floor(px + R + 1) (likewise
 * iy) whose centre (ix + 0.5, iy + 0.5) lies at distance d < R + 1 from
 * (px, py) the weight w = weight * (1 - d / (R + 1))^2.  Each such pixel receives w * rgb, added
 * into img[(iy*W + ix)*3 + k] as the fixed-point integer
 * nearbyint(256 * (w * rgb_k)) (pixels outside the image are skipped).  Everything is evaluated in double
 * precision in the order written here; n_culled counts culled particles. */
typedef struct {
    int axis[3];
    double mvp[16];
    int width, height;
    double base[3], grad[9], origin[3];
    double weight;
    int radius;
} ffo_render_t;
int ffo_render(int dim, const double* state, int n_pp, const double* pparams, int64_t n,
               int64_t ld, const ffo_render_t* r, uint32_t* img, uint64_t* n_culled,
               int accumulate);

/* User right-hand sides given as expressions (Appendix A: one expression per
 * state variable; Appendix A.1: turned into the step kernel).  exprs[d] is the
 * expression of x_d' over x0..x{dim-1} and p0..p{n_params-1} (grammar in
 * ffo_expr.cpp), evaluated as written, left to right, every operation
 * rounded to the working precision (double, or float for the _f32 form,
 * where comp != NULL selects the Kahan-compensated update).  dim <= 16,
 * n_params <= 32, n_pp <= 4.  Returns -1 for bad sizes, -2 with
 * ffo_expr_error() set when an expression does not parse. */
int ffo_expr_rk4(int dim, const char* const* exprs, const double* params, int n_params,
                 const int32_t* pp_slot, int n_pp, const double* pparams, double* state,
                 int64_t n, int64_t ld, double h, int64_t nsteps);
int ffo_expr_rk4_f32(int dim, const char* const* exprs, const double* params, int n_params,
                     const int32_t* pp_slot, int n_pp, const float* pparams, float* state,
                     float* comp, int64_t n, int64_t ld, float h, int64_t nsteps);
const char* ffo_expr_error(void);
/* The FP64 expression map with its directional derivative (forward-mode
 * differentiation of every operation): inputs perturbed along dx0 (SoA like
 * the state), dparams (n_params) and dpp (SoA like pparams), any of them NULL
 * for zero.  xT equals ffo_expr_rk4's result; dxT is d xT along the direction.
 * fabs has slope +1 at 0; fmin/fmax follow the returned argument (the first on
 * a tie); pow's log term is dropped when the exponent's direction is zero. */
int ffo_expr_rk4_dual(int dim, const char* const* exprs, const double* params, int n_params,
                      const int32_t* pp_slot, int n_pp, const double* pparams, const double* x0,
                      const double* dx0, const double* dparams, const double* dpp, double* xT,
                      double* dxT, int64_t n, int64_t ld, double h, int64_t nsteps);

#ifdef __cplusplus
}
#endif
#endif
