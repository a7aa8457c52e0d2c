"""The oracle's own FP64 rounding error, bounded against the exact result.

The same RK4 map (Section 2.1, Appendix A.1) is run in 50-digit decimal
arithmetic (Python's ``decimal``, with ``Decimal.exp``), from the same FP64
inputs, on a few particles over short horizons.  The FP64 oracle must agree
to 1e-13 (mixed relative metric): this bounds the rounding of the oracle's
evaluation order and of its libm exp/expm1.  (It checks rounding, not the
formulas; the formulas are pinned in the per-system tests.)
"""
from decimal import Decimal as D, getcontext

import numpy as np
import pytest

from paper_1505_00344_amd.inputs import HH_PARAMS, LORENZ_PARAMS, WC_PARAMS

getcontext().prec = 50


def lorenz(p, x):
    s, r, b = p
    return [s * (x[1] - x[0]), x[0] * (r - x[2]) - x[1], x[0] * x[1] - b * x[2]]


def sig(u, a, th):
    return 1 / (1 + (-(a * (u - th))).exp())


def wc(p, x):
    c1, c2, c3, c4, aE, thE, aI, thI, P, Q = p
    E, I = x
    return [sig(c1 * E - c2 * I + P, aE, thE) - E, sig(c3 * E - c4 * I + Q, aI, thI) - I]


def psi(u):
    return D(1) if u == 0 else u / (u.exp() - 1)


def hh(p, x):
    gNa, gK, gL, ENa, EK, EL, C, Iext, gsyn, Esyn, rr, rd, th, sg = p
    N = len(x) // 5
    f = []
    for j in range(N):
        V, m, h, n, s = x[5 * j:5 * j + 5]
        sp = x[5 * ((j - 1) % N) + 4]
        am = psi(-(V + 40) / 10)
        bm = 4 * (-(V + 65) / 18).exp()
        ah = D("0.07") * (-(V + 65) / 20).exp()
        bh = 1 / (1 + (-(V + 35) / 10).exp())
        an = D("0.1") * psi(-(V + 55) / 10)
        bn = D("0.125") * (-(V + 65) / 80).exp()
        T = 1 / (1 + (-sg * (V - th)).exp())
        dV = (gL * (EL - V) + gNa * m ** 3 * h * (ENa - V) + gK * n ** 4 * (EK - V)
              + gsyn * sp * (Esyn - V) + Iext) / C
        f += [dV, am * (1 - m) - bm * m, ah * (1 - h) - bh * h, an * (1 - n) - bn * n,
              rr * T * (1 - s) - rd * s]
    return f


def rk4_decimal(f, p, x, h, n):
    p = [D(v) for v in p]
    x = [D(v) for v in x]
    h = D(h)
    for _ in range(n):
        k1 = f(p, x)
        k2 = f(p, [xi + h / 2 * ki for xi, ki in zip(x, k1)])
        k3 = f(p, [xi + h / 2 * ki for xi, ki in zip(x, k2)])
        k4 = f(p, [xi + h * ki for xi, ki in zip(x, k3)])
        x = [xi + h / 6 * (a + 2 * b + 2 * c + d) for xi, a, b, c, d in zip(x, k1, k2, k3, k4)]
    return np.array([float(v) for v in x])


# The oracle's HH rates use the doubles nearest to -1/10, -1/18, ... and to the
# decimal constants 0.07, 0.1, 0.125; the decimal run uses the exact values,
# so its "p" must be the exact decimal values of the FP64 parameter inputs.
@pytest.mark.parametrize("name,sysid,p,box,h,n", [
    ("lorenz28", 1, LORENZ_PARAMS, [(-20, 20), (-30, 30), (0, 50)], 0.005, 100),
    ("lorenz28_back", 1, LORENZ_PARAMS, [(-20, 20), (-30, 30), (0, 50)], -0.005, 40),
    ("wc", 2, WC_PARAMS[:8] + [1.5, 0.0], [(0, 1), (0, 1)], 0.01, 200),
    ("wc_back", 2, WC_PARAMS[:8] + [1.5, 0.0], [(0, 1), (0, 1)], -0.01, 200),
    ("hh", 3, HH_PARAMS, [(-80, 40), (0, 1), (0, 1), (0, 1), (0, 1)] * 3, 0.01, 100),
])
def test_fp64_oracle_within_1e13_of_exact(ora, name, sysid, p, box, h, n):
    rng = np.random.default_rng(123)
    x0 = np.stack([rng.uniform(lo, hi, 4) for lo, hi in box])
    got = ora.rk4(sysid, p, x0, h, n)
    f = {1: lorenz, 2: wc, 3: hh}[sysid]
    for i in range(x0.shape[1]):
        want = rk4_decimal(f, p, x0[:, i], h, n)
        e = np.linalg.norm(got[:, i] - want) / max(np.linalg.norm(want), 1.0)
        assert e < 1e-13, (name, i, e)
