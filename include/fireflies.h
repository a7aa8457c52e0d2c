/*
 * fireflies.h — C ABI of libfireflies.so, the MI355X (gfx950) hot path of
 * "Fireflies: New software for interactively exploring dynamical systems
 * using GPU computing" (R. Merrison-Hort, arXiv:1505.00344).
 *
 * The method (Section 2.1; Appendix A, Appendix A.1, Appendix A.2): many
 * independent trajectories ("particles") of an autonomous N-dimensional ODE
 * are advanced with the classical fourth-order Runge-Kutta method at a
 * constant, signed step (forward groups h > 0, backward groups h < 0); a
 * parameter may take a separate value per particle (the paper's trick of a
 * parameter turned into a state variable with zero derivative, Section 2.1
 * and Section 2.2); the current positions are projected onto two chosen axes
 * and accumulated additively on a pixel grid (Appendix A "Render Technique",
 * Appendix A.1 fragment shader with additive blending).  This library
 * computes that: the RK4 advance in single precision (optionally with a
 * compensated update) or double precision, the projection as an exact count
 * histogram and as the paper's sprite image, the paper's reset rule, trajectory
 * recording, right-hand sides given as expressions and compiled at run time,
 * the exact discrete adjoint of the RK4 map, and a batched launch over ragged
 * groups of different systems.
 *
 * Conventions for every function below.
 *   - Device memory: every array argument documented as "device" is memory
 *     of the current HIP device, owned by the caller (typically a torch
 *     tensor).  The library never frees caller memory.
 *   - Layout: structure of arrays.  Component d of particle i is
 *     state[d*ld + i]; per-particle parameter k of particle i is
 *     pparams[k*ld + i]; ld >= n.
 *   - Element type follows ff_batch.prec: float for FF_FP32 and
 *     FF_FP32_KAHAN, double for FF_FP64.
 *   - Streams: `stream` is a hipStream_t (NULL = the legacy default stream).
 *     Calls only enqueue work, with three exceptions stated where they
 *     apply: ff_autotune times launches (it synchronises its stream), growing
 *     library-owned scratch synchronises the stream before the old buffer is
 *     freed, and ff_system_destroy of an expression system waits for the
 *     device before unloading its kernels.
 *   - Errors: arguments are validated on the host before anything is
 *     enqueued; on failure nothing was enqueued and ff_last_error() explains
 *     why.  FF_E_DEVICE reports a HIP error (its text in ff_last_error()).
 *     No call aborts the process.  NaN/Inf in the data are not errors: they
 *     propagate through the arithmetic as IEEE values.
 */
#ifndef FIREFLIES_H
#define FIREFLIES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FF_ABI_VERSION 2
#define FF_MAX_PP 4 /* per-particle parameters per batch */
/* bytes of device scratch held by ff_project_histogram_noalloc (per GPU) */
#define FF_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)

typedef enum {
    FF_OK = 0,
    FF_E_INVALID = 1,     /* bad argument; nothing enqueued */
    FF_E_UNSUPPORTED = 2, /* valid request this build does not implement */
    FF_E_NOMEM = 3,       /* host or device allocation failed, or workspace too small */
    FF_E_DEVICE = 4       /* HIP runtime error */
} ff_status;

typedef enum {
    FF_FP32 = 0,       /* single precision */
    FF_FP32_KAHAN = 1, /* single precision, Kahan-compensated state update */
    FF_FP64 = 2        /* double precision */
} ff_prec;

/* Right-hand sides (all autonomous).  Parameter vectors, in order:
 *   FF_RHS_LINEAR        x' = A x, dim 1..4; params = A row-major (dim*dim).
 *   FF_RHS_LORENZ        Section 2.2, Eqs. lorenz_x/y/z; dim 3;
 *                        params = [sigma, r, beta].
 *   FF_RHS_WILSON_COWAN  E' = -E + S_E(c1 E - c2 I + P),
 *                        I' = -I + S_I(c3 E - c4 I + Q),
 *                        S(u) = 1/(1 + exp(-a (u - theta))): the
 *                        sigmoid-coupled pair of Section 2.1 (Eqs.
 *                        stn_gpe/eqnGPe) with unit time constants; dim 2;
 *                        params = [c1, c2, c3, c4, aE, thetaE, aI, thetaI, P, Q].
 *   FF_RHS_HH_RING       ring of N = dim/5 Hodgkin-Huxley neurons (Section 3,
 *                        Eqs. hh_v, hh_h, hh_m, hh_n, hh_isyn, hh_s); neuron j
 *                        is [V, m, h, n, s] at 5j and receives the synapse of
 *                        neuron (j - 1) mod N; dim 5 or 15 in this build;
 *                        params = [gNa, gK, gL, ENa, EK, EL, C, Iext, gsyn,
 *                        Esyn, r_rise, r_decay, theta_syn, sigma_syn].
 *   FF_RHS_EXPR          a right-hand side given as expressions; made only by
 *                        ff_system_create_expr, reported by ff_system_info. */
typedef enum {
    FF_RHS_LINEAR = 0,
    FF_RHS_LORENZ = 1,
    FF_RHS_WILSON_COWAN = 2,
    FF_RHS_HH_RING = 3,
    FF_RHS_EXPR = 16
} ff_rhs;

typedef struct ff_system_s* ff_system_t; /* opaque, library-owned */

/* One slice of particles (a "Particle Group" of Appendix A without its
 * initial-condition box, which is the caller's business). */
typedef struct {
    int32_t prec;                /* ff_prec */
    void* state;                 /* device [dim][ld], in/out */
    int64_t n;                   /* particles */
    int64_t ld;                  /* leading dimension, >= n */
    const void* pparams;         /* device [n_pp][ld], or NULL when n_pp == 0 */
    int32_t n_pp;                /* 0..FF_MAX_PP per-particle parameters */
    int32_t pp_slot[FF_MAX_PP];  /* pparams row k replaces global parameter pp_slot[k] */
    void* comp;                  /* device [dim][ld] Kahan compensation (FF_FP32_KAHAN
                                    only; carried across calls; start it at 0) */
} ff_batch;

/* Launch shape.  steps_per_launch: RK4 steps fused per kernel launch (the
 * state stays in registers between them); particles_per_thread: 1, 2 or 4
 * (the Hodgkin-Huxley rings are limited to 2; larger requests are clamped);
 * block: threads per block, a multiple of 64 in [64, 256].  Results are
 * bitwise independent of all three. */
typedef struct {
    int32_t steps_per_launch;
    int32_t particles_per_thread;
    int32_t block;
} ff_tuning;

/* Library plumbing, not part of the paper's method: the ABI version this
 * header describes (FF_ABI_VERSION), and the text of the last error on the
 * calling thread (valid until the next ff_* call on this thread; never
 * NULL). */
int32_t ff_abi_version(void);
const char* ff_last_error(void);

/* Create a system (Appendix A, "State Variables" and "Parameters": the N
 * state variables each with the right-hand side of its ODE, and the
 * parameters each with a default value).  rhs selects a compiled-in
 * right-hand side (ff_rhs; expression systems come from
 * ff_system_create_expr), dim is N, params holds the n_params default global
 * values (host, copied).  The variables' bounds and the parameters' allowed
 * ranges are not part of a system: the bounds are arguments of
 * ff_integrate_reset, and ranges are the caller's business.  FF_E_INVALID
 * when rhs is unknown, dim or n_params does not fit rhs (see ff_rhs above),
 * or params or out is NULL; FF_E_UNSUPPORTED for a Hodgkin-Huxley ring of
 * other than 1 or 3 neurons.  Host-only: touches no device.  *out receives
 * the handle (NULL on failure), owned by the library until
 * ff_system_destroy releases it; destroying NULL does nothing and returns
 * FF_OK, and a handle must not be used after it is destroyed. */
ff_status ff_system_create(int32_t rhs, int32_t dim, int32_t n_params, const double* params,
                           ff_system_t* out);
ff_status ff_system_destroy(ff_system_t sys);

/* Replace the global parameter values (host array of n_params doubles): the
 * paper's live slider (Appendix A.2).  Takes effect for calls enqueued
 * afterwards. */
ff_status ff_system_set_params(ff_system_t sys, const double* params, int32_t n_params);
/* Read back the current global parameter values (host array of n_params
 * doubles, n_params equal to the system's count) and the system's kind,
 * dimension and parameter count (Appendix A, "State Variables" and
 * "Parameters"); host-only. */
ff_status ff_system_get_params(ff_system_t sys, double* params, int32_t n_params);
ff_status ff_system_info(ff_system_t sys, int32_t* rhs, int32_t* dim, int32_t* n_params);

/* A system whose right-hand side is given as text, one expression per state
 * variable (Appendix A: a State Variable holds the expression of its time
 * derivative; Appendix A.1: the step kernel is the general RK4 template with
 * that right-hand side filled in, compiled at run time).  exprs[d] (host,
 * NUL-terminated, copied) is x_d' over the names x0..x{dim-1} and
 * p0..p{n_params-1}:
 *   sum := product (('+'|'-') product)*   product := prefix (('*'|'/') prefix)*
 *   prefix := '-' prefix | '+' prefix | atom
 *   atom := number | name | func '(' sum (',' sum)* ')' | '(' sum ')'
 * Binary operators associate to the left and a sign binds tighter than any of
 * them.  A number starts with a digit or '.' and is read by strtod (decimal or
 * hexadecimal, exponent allowed) into a double, which is then rounded to the
 * working precision; names are x or p followed by an index without leading
 * zeros; functions: exp expm1 log log1p sqrt sin cos tan tanh sinh cosh atan
 * fabs (one argument), pow fmin fmax (two), fma (three: a*b+c rounded once).
 * Every operation rounds to the working precision (no contraction, no fast
 * math; the device math library's functions for the named functions).
 * flags: 0, or FF_EXPR_FAST_F32: in single precision exp(x) is the hardware
 * 2^(x log2 e) and a / b is a * rcp(b) (about 1 ulp each: the single-precision
 * policy of the built-in systems) instead of the library expf and a correctly
 * rounded division; double precision is not affected.  Unknown bits:
 * FF_E_INVALID.
 * dim 1..15, n_params 0..16 (params: host array, copied; may be NULL when
 * n_params == 0), at most 65536 characters per expression, 256 levels of
 * nesting and 4096 distinct operations per system.  A syntax error returns
 * FF_E_INVALID with the state variable, column and reason in ff_last_error().
 * Nothing is compiled here: ff_integrate, ff_integrate_reset and
 * ff_integrate_record compile the kernels of the batch's precision for the
 * current device on first use (hipRTC; about a second) and keep them with the
 * handle (ff_system_destroy waits for the device before unloading them).
 * ff_integrate_checkpointed and ff_adjoint work as for the built-in systems:
 * the vector-Jacobian product is generated by reverse-mode differentiation of
 * the expressions (fabs has slope +1 at 0; fmin/fmax pass the adjoint to the
 * argument they return, the first on a tie), and the adjoint kernel is
 * compiled on the first ff_adjoint call of a precision.  The ragged-batch
 * calls (ff_integrate_groups, ff_autotune) hold compiled-in right-hand sides
 * only and return FF_E_UNSUPPORTED for such a system. */
#define FF_EXPR_FAST_F32 1u
ff_status ff_system_create_expr(int32_t dim, const char* const* exprs, int32_t n_params,
                                const double* params, uint32_t flags, ff_system_t* out);

/* Compile the kernels of an expression system for precision prec (ff_prec).
 * arch == NULL: for the current device, and load them there (do this before
 * capturing a stream into a graph, since the first integration of a
 * precision otherwise compiles and loads during the call).  arch != NULL
 * (e.g. "gfx950"): compile only, with no device needed (a check that the
 * generated code builds).  Both the integration kernels and the adjoint
 * kernel are compiled.  FF_E_INVALID for a built-in system. */
ff_status ff_system_compile(ff_system_t sys, int32_t prec, const char* arch);

/* The generated system (derived constants, right-hand side and its
 * vector-Jacobian product) of an expression system for precision prec:
 * *len receives its size including the NUL; up to cap bytes are written to
 * buf (NUL-terminated; FF_E_NOMEM if cap is too small; buf may be NULL to
 * ask for the size). */
ff_status ff_system_source(ff_system_t sys, int32_t prec, char* buf, size_t cap, size_t* len);

/* Advance every particle of the batch by nsteps classical RK4 steps of size
 * dt_signed (Section 2.1; Appendix A.1-A.2).  In single precision the step is
 * rounded to float once, and h/2 and h/6 are formed in float.  dt_signed == 0
 * or nsteps == 0 (the paper's paused state) or n == 0 enqueue nothing.
 * tuning may be NULL (defaults: up to 4096 steps per launch, particles per
 * thread and block size chosen per system and precision from measurement). */
ff_status ff_integrate(ff_system_t sys, const ff_batch* b, double dt_signed, int64_t nsteps,
                       const ff_tuning* tuning, void* stream);

/* The paper's reset rule (Section 2.1: a trajectory that leaves the region,
 * or that has not been reset for more than a time T_max, restarts from new
 * random initial conditions; Appendix A: the bounds of each state variable and
 * the group's initial-condition box), applied on the device after every RK4
 * step rather than lagged on the host (Appendix A.2):
 *   age += 1; if some component x_d is outside [bound_lo[d], bound_hi[d]]
 *   (NaN counts as outside) or age > max_age (max_age < 0: no age limit; the
 *   paper's T_max in steps), the particle is redrawn uniformly in
 *   [box_lo, box_hi), its Kahan compensation and age are set to 0 and
 *   n_resets += 1.
 * Draw number r (the particle's n_resets before the reset) of particle i uses
 * Philox4x32-10 (Salmon et al., SC'11) with key (seed low 32 bits, seed high
 * 32 bits) and counter (g low, g high, r, j), g = id_offset + i, block j:
 *   FP64: component d takes words 2d, 2d+1 (a, b) of the stream,
 *         u = ((a >> 5) * 2^26 + (b >> 6)) * 2^-53, x = fma(box_hi - box_lo, u, box_lo);
 *   FP32: component d takes word d, u = (a >> 8) * 2^-24,
 *         x = fmaf((float)(box_hi - box_lo), u, (float)box_lo).
 * bound_* and box_* are host arrays of dim doubles; age (int32) and n_resets
 * (uint32) are device arrays of n entries (particle i at index i), read and
 * written.  Results are bitwise independent of the launch shape. */
typedef struct {
    const double* bound_lo;
    const double* bound_hi;
    const double* box_lo;
    const double* box_hi;
    int64_t max_age;
    uint64_t seed;
    uint64_t id_offset;
    int32_t* age;
    uint32_t* n_resets;
} ff_reset;

ff_status ff_integrate_reset(ff_system_t sys, const ff_batch* b, double dt_signed, int64_t nsteps,
                             const ff_reset* reset, const ff_tuning* tuning, void* stream);

/* Trajectory recording (Section 4 names it as future work: record a subset of
 * trajectories, or all of them at an interval longer than the step).  Advances
 * the batch like ff_integrate (or like ff_integrate_reset when `reset` is not
 * NULL) and, after global steps every, 2*every, ..., stores the state of
 * particles 0, stride, 2*stride, ... of the batch:
 *   out[k][d][j] = component d of particle j*stride after step (k+1)*every,
 * k = 0 .. nsteps/every - 1, j = 0 .. ceil(n/stride) - 1.  out: device array
 * of the batch's element type, caller-owned, (nsteps/every)*dim*ceil(n/stride)
 * elements.  The integration itself is bitwise that of ff_integrate. */
ff_status ff_integrate_record(ff_system_t sys, const ff_batch* b, double dt_signed, int64_t nsteps,
                              int64_t every, int64_t stride, void* out, const ff_reset* reset,
                              const ff_tuning* tuning, void* stream);

/* 2D density projection (Appendix A "Render Technique", Appendix A.1:
 * additive accumulation of unit-weight points).  axis >= 0 selects state
 * component axis; axis = -1 - k selects per-particle parameter row k.  The
 * bin of a particle is ix = floor((a - x_lo) * (nx / (x_hi - x_lo))) (and
 * likewise iy), computed in double precision; it is kept iff 0 <= ix < nx and
 * 0 <= iy < ny (NaN fails), and then hist[iy*nx + ix] += 1; otherwise
 * *n_dropped += 1.  Counts are exact.  hist: device uint32 [ny][nx];
 * n_dropped: device uint64 or NULL (not counted); accumulate == 0 first sets
 * hist (and *n_dropped) to zero.  workspace: device scratch of at least
 * ff_histogram_workspace_size() bytes, or NULL to use library-owned scratch
 * (one buffer per device, allocated on first use and grown when needed: calls
 * that use it concurrently on different streams of one device race, and
 * under stream capture a workspace must be passed).  At most 2^31 - 1
 * particles per call (FF_E_UNSUPPORTED beyond), grids up to 64M bins. */
ff_status ff_histogram_workspace_size(int64_t n, int32_t nx, int32_t ny, size_t* bytes);
ff_status ff_project_histogram(ff_system_t sys, const ff_batch* b, int32_t axis_x, int32_t axis_y,
                               double x_lo, double x_hi, double y_lo, double y_hi, int32_t nx,
                               int32_t ny, uint32_t* hist, uint64_t* n_dropped, int32_t accumulate,
                               void* workspace, size_t workspace_bytes, void* stream);

/* The same projection for callers that cannot allocate device memory (code
 * under stream or graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): arguments and results as ff_project_histogram without a
 * workspace, and no call of this function allocates.  Its scratch is a static
 * device array of FF_NOALLOC_SCRATCH_BYTES per GPU, part of the library's code
 * object and held until the process ends; a projection needing more
 * (ff_histogram_workspace_size() > FF_NOALLOC_SCRATCH_BYTES: beyond about
 * 11M particles on a 1024 x 1024 grid, fewer on larger grids; grids of at
 * most 16384 bins need no scratch at all) returns
 * FF_E_NOMEM before anything is enqueued.  Every call on one GPU shares that
 * array: calls that overlap on one device (different streams, host threads)
 * race and must be ordered by the caller.  Nothing in it needs to start at
 * zero.  The first call on a device looks the array's address up there
 * (hipGetSymbolAddress, which loads the library's code object on that device
 * if nothing has yet): make that first call outside stream capture. */
ff_status ff_project_histogram_noalloc(ff_system_t sys, const ff_batch* b, int32_t axis_x, int32_t axis_y,
                                       double x_lo, double x_hi, double y_lo, double y_hi, int32_t nx,
                                       int32_t ny, uint32_t* hist, uint64_t* n_dropped, int32_t accumulate,
                                       void* stream);

/* Particle image: the paper's render technique (Appendix A "Render
 * Technique": 2D or perspective 3D projection onto chosen axes, colour fixed
 * or varying linearly with position; Appendix A.1: model-view and
 * view-projection transforms, a square sprite whose intensity falls off with
 * the distance from its centre, additive blending GL_SRC_ALPHA/GL_ONE).  For
 * each particle, with a = the three axis values (state component axis[i] >= 0
 * or per-particle parameter -1 - axis[i]), all in double precision:
 *   c = mvp (a0, a1, a2, 1), mvp row-major 4x4 = projection * view * model;
 *   culled (counted in *n_culled) if c3 <= 0 or some c_i / c3 (i < 3) is
 *   outside [-1, 1] or NaN; else px = (c0/c3 + 1) W/2, py = (1 - c1/c3) H/2;
 *   rgb_k = min(max(base_k + sum_i grad[3k + i] (a_i - origin_i), 0), 1);
 *   radius 0: pixel (floor px, floor py) gets w = weight; radius R > 0: every
 *   pixel ix in floor(px - R - 1) .. floor(px + R + 1) (likewise iy) whose
 *   centre is at distance d < R + 1 from (px, py) gets
 *   w = weight (1 - d/(R + 1))^2;
 *   img[(iy W + ix) 3 + k] += rint(256 * (w * rgb_k))  (pixels outside skipped).
 * A 2D orthographic view is an mvp whose last row is (0, 0, 0, 1).  img:
 * device uint32 [height][width][3], fixed point with 8 fractional bits, exact
 * and independent of particle order; a channel's sum wraps modulo 2^32 (after
 * 2^24 full-weight, full-colour hits of one pixel), so weight should keep the
 * densest pixel below that; n_culled: device uint64 or NULL; accumulate == 0
 * clears both first.  width * height <= 2^28, radius <= 64.
 * workspace: device scratch of at least ff_render_workspace_size() bytes (0
 * when the call needs none: sprites of radius > 8, images of more than 4096
 * tiles of 64 x 32 pixels, or more than 2^29 particles), or NULL to use
 * library-owned scratch (one buffer per device, allocated on first use and
 * grown when needed: calls that use it concurrently on different streams of
 * one device race, and under stream capture a workspace must be passed). */
typedef struct {
    int32_t axis[3];
    double mvp[16];
    int32_t width, height;
    double base[3];
    double grad[9];
    double origin[3];
    double weight;
    int32_t radius;
} ff_render;

ff_status ff_render_workspace_size(int64_t n, const ff_render* r, size_t* bytes);
ff_status ff_render_image(ff_system_t sys, const ff_batch* b, const ff_render* r, uint32_t* img,
                          uint64_t* n_culled, int32_t accumulate, void* workspace,
                          size_t workspace_bytes, void* stream);

/* Discrete adjoint.  The paper defines no adjoint or gradient: these three
 * calls extend its method with the exact gradient of the RK4 map above
 * (Section 2.1; Appendix A.1) with respect to the initial state and the
 * parameters, for sensitivities of quantities read off the ensemble (e.g.
 * how the mean of a state variable at time T changes with each particle's
 * bifurcation parameter).  The Kahan update is differentiated as exact
 * addition.  Usage: ff_integrate_checkpointed() advances the batch
 * like ff_integrate() and stores the state (and compensation) every K steps
 * in `workspace`; then ff_adjoint() walks the segments backwards, recomputing
 * each segment from its checkpoint.
 *   lambda:    device [dim][ld]; in dL/dx(T), out dL/dx(0)
 *   mu:        device [n_pp][ld]; out dL/d(per-particle parameter k)
 *              (NULL allowed when n_pp == 0)
 *   mu_global: device double [n_params]; out sum over particles of
 *              dL/d(parameter j) for every parameter (FP64 reduction), or NULL
 * The batch passed to ff_adjoint must describe the same particles (its state
 * pointer is not read).  workspace_bytes must be >= the size returned by
 * ff_adjoint_workspace_size for the same arguments. */
ff_status ff_adjoint_workspace_size(ff_system_t sys, const ff_batch* b, int64_t nsteps, int32_t K,
                                    size_t* bytes);
ff_status ff_integrate_checkpointed(ff_system_t sys, const ff_batch* b, double dt_signed,
                                    int64_t nsteps, int32_t K, void* workspace,
                                    size_t workspace_bytes, void* stream);
ff_status ff_adjoint(ff_system_t sys, const ff_batch* b, double dt_signed, int64_t nsteps,
                     int32_t K, void* workspace, size_t workspace_bytes, void* lambda, void* mu,
                     double* mu_global, void* stream);

/* Ragged batch (Appendix A, "Particle Group": a system holds one or more
 * groups, each with its own particle count and direction in time, forward or
 * backward; Appendix A.2: the main loop advances every group once per frame
 * before rendering): several groups (each with its own system, slice,
 * precision and signed step) advanced nsteps in one persistent launch per
 * steps_per_launch.  Every group must use FF_FP32 or FF_FP32_KAHAN or every
 * group FF_FP64.  Results are bitwise equal to ff_integrate on each group.
 * workspace: device scratch of at least ff_groups_workspace_size() bytes (it
 * holds the tile counter of the launch), or NULL for a library-owned counter
 * (one per device: launches that use it concurrently on different streams of
 * one device race, and under stream capture a workspace must be passed).
 * tuning: NULL takes the choice an earlier ff_autotune call in this process
 * made for the same list (the same systems' kinds and sizes, precisions,
 * particle counts, per-particle parameter counts and nsteps), and otherwise
 * steps_per_launch = min(nsteps, 4096), one particle per thread, 256 threads. */
typedef struct {
    ff_system_t sys;
    ff_batch b;
    double dt_signed;
} ff_group;

ff_status ff_groups_workspace_size(int32_t n_groups, size_t* bytes);
ff_status ff_integrate_groups(const ff_group* groups, int32_t n_groups, int64_t nsteps,
                              const ff_tuning* tuning, void* workspace, size_t workspace_bytes,
                              void* stream);

/* Launch-shape search for ff_integrate_groups.  Not part of the paper's
 * method (it changes no result: every shape gives the same bits), only of how
 * fast this library runs it.  Picks steps_per_launch, particles_per_thread and
 * block for a group list by timing candidate launches (on copies of the groups' state, which is left
 * unchanged).  steps_per_launch is searched in [10, min(500, nsteps)].
 * Synchronises the stream.  *out receives the choice.  Choices are cached
 * per list for the process; a list already tuned returns at once.  When the
 * environment variable FF_AUTOTUNE_CACHE names a file, the cache is also
 * read from it (at the first lookup of the process) and each new choice is
 * appended to it as a line "<signature> <steps_per_launch>
 * <particles_per_thread> <block>", where the signature is nsteps followed,
 * per group, by "|rhs,dim,prec,n,n_pp" (decimal).  The file is meant for one
 * kind of GPU; unreadable or malformed lines are skipped, and a failed write
 * is ignored. */
ff_status ff_autotune(const ff_group* groups, int32_t n_groups, int64_t nsteps, ff_tuning* out,
                      void* stream);

/* Accuracy check of the double-precision elementary kernels the built-in
 * Wilson-Cowan and Hodgkin-Huxley right-hand sides evaluate (the paper fixes
 * no exponential or division; these are the library's own, Cody-Waite
 * reductions and Chebyshev interpolants): y[i] = fn(x[i]) for i < n, with x
 * and y device arrays of n doubles (caller-owned; y may equal x).  fn is one
 * of ff_math; the argument ranges each kernel is valid for:
 *   FF_MATH_EXP       e^x, |x| <= 708 (gradual underflow included)
 *   FF_MATH_EXP2      2^x, |x| <= 2^31 (inf above 1024, 0 below -1075)
 *   FF_MATH_EXPM1     e^x - 1, |x| <= 708
 *   FF_MATH_RCP       1/x, 2^-1022 <= |x| <= 2^1022
 *   FF_MATH_LOGISTIC  1/(1 + e^x) with x clamped to [-700, 700], any x; NaN
 *                     for a NaN or infinite x
 *   FF_MATH_LOGISTIC2 1/(1 + 2^x) with x clamped to [-1000, 1000], any x; NaN
 *                     for a NaN or infinite x
 *   FF_MATH_PSI       x/(e^x - 1) (1 at x = 0) with e^x - 1 taken at
 *                     min(x, 700), for x >= -708
 * Enqueues one launch on stream.  FF_E_INVALID for an unknown fn, n < 0, or
 * x or y NULL with n > 0; n == 0 launches nothing. */
enum {
    FF_MATH_EXP = 0,
    FF_MATH_EXP2 = 1,
    FF_MATH_EXPM1 = 2,
    FF_MATH_RCP = 3,
    FF_MATH_LOGISTIC = 4,
    FF_MATH_LOGISTIC2 = 5,
    FF_MATH_PSI = 6
};
ff_status ff_math_eval(int32_t fn, const double* x, double* y, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FIREFLIES_H */
