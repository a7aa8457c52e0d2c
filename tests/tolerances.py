"""Numerical tolerances, fixed from the arithmetic before any GPU result.

Error metric for a particle: e = ||x - x_ref||_2 / max(||x_ref||_2, 1) over its
state components (a relative error that does not blow up as a trajectory
approaches the origin).

FP64 path vs the FP64 oracle (the hot-path contract: 1e-12 relative):
  * systems without transcendental functions (Lorenz, linear) evaluate the
    same correctly rounded operations in the same order: bit-identical;
  * Wilson-Cowan / Hodgkin-Huxley call exp/expm1 from two different math
    libraries (each within 1 ulp), so results differ by a few ulp per step,
    amplified by the local expansion rate of the flow.  Forward (contracting)
    runs: max 1e-12.  Backward Wilson-Cowan (expanding, e^|t| growth) stays
    at the 1e-12 level at p99 and below 1e-11 at the max.
FP32 vs FP64 (per-system bounds; Kahan must also beat plain FP32): see the
constants below.  Histogram counts from identical positions: exact.
Adjoint: FP64 vs the oracle's adjoint and complex-step 1e-10 relative (floor
1e-3 on |g|); vs central differences with h = 1e-4: p99 1e-6, max 1e-4.
"""

FP64_EXACT = 0.0
FP64_REL = 1e-12
FP64_WC_BACKWARD_P99 = 1e-12
FP64_WC_BACKWARD_MAX = 1e-11

# FP32 (plain / Kahan) vs FP64, mixed metric.
FP32_NONCHAOTIC_MAX = 1e-5           # linear, Lorenz r<1, z-axis; 500 steps
FP32_LORENZ28_100_P99 = 1e-5         # Lorenz r = 28, 100 steps
FP32_LORENZ_BIF_MEDIAN = 1e-5        # per-particle r ~ U[0,50], 500 steps, plain
FP32_LORENZ_BIF_P99 = 1e-3
KAHAN_LORENZ_BIF_MEDIAN = 1e-6
KAHAN_LORENZ_BIF_P99 = 1e-4
FP32_WC_P99 = 1e-4                   # Wilson-Cowan, 1000 steps
KAHAN_WC_MEDIAN = 1e-7              # contracting (forward) groups only
KAHAN_WC_P99 = 1e-5
# Expanding (backward) Wilson-Cowan groups.  Integrated backward, the flow
# expands areas: most particles leave the unit square, both sigmoids saturate
# to exactly 0 or 1, the right-hand side becomes affine and the state grows
# like e^{|t|}.  The relative error of such a particle is then set by the
# single-precision rounding of the step weight h/6 (relative rho,
# |rho| <= u = 2^-24), which every step's growth factor carries: after the
# elapsed time T = nsteps*|h| it is T*|rho| plus smaller terms (h = -0.01,
# 1000 steps: rho = -2.33e-8, T*|rho| = 2.33e-7).  The median bound is the
# worst case over h, T*u (5.96e-7 at T = 10); the contracting groups' median
# bound does not apply.  The p99 bound stays KAHAN_WC_P99, plain FP32 keeps
# FP32_WC_P99, and Kahan must halve plain FP32's median (KAHAN_GAIN).
UNIT_ROUNDOFF_F32 = 2.0 ** -24


def kahan_wc_expanding_median(nsteps, h):
    """Median bound of FP32-Kahan vs FP64 on an expanding Wilson-Cowan group."""
    return nsteps * abs(h) * UNIT_ROUNDOFF_F32


KAHAN_HH_MEDIAN = 1e-6               # HH ring, 2000 steps
KAHAN_HH_P99 = 1e-4
KAHAN_HH_MAX = 1e-3
# median(Kahan) <= KAHAN_GAIN * median(plain).  On Lorenz the update rounding
# dominates and compensation removes most of it.  On the contracting
# Wilson-Cowan forward group the particles sit at attracting equilibria whose
# FP32 position is set by the rounding of the right-hand side itself, which a
# compensated update cannot remove; a CPU probe of this case in NumPy measured
# a ratio of 0.54.
KAHAN_GAIN = 0.5
KAHAN_GAIN_WC = 0.75

# Adjoint.
ADJ_REL = 1e-10
ADJ_FLOOR = 1e-3
ADJ_FD_P99 = 1e-6
ADJ_FD_MAX = 1e-4
ADJ_FP32_P99 = 1e-3
