"""Pins of the oracle's Runge-Kutta stepper.

The paper integrates every particle with "4th order Runge-Kutta" at a constant
step (Section 2.1; Appendix A.1).  The reading taken is the classical (Kutta)
tableau.  These tests compare the oracle with an exact-arithmetic brute force
of a generic explicit Runge-Kutta step driven by a Butcher tableau (a
different formulation from the oracle's hand-written stages), on the scalar
Riccati equation y' = y^2 whose exact solution is y0 / (1 - y0 t).
"""
from fractions import Fraction as F

import numpy as np

CLASSICAL = dict(A=[[], [F(1, 2)], [F(0), F(1, 2)], [F(0), F(0), F(1)]],
                 b=[F(1, 6), F(1, 3), F(1, 3), F(1, 6)])
THREE_EIGHTHS = dict(A=[[], [F(1, 3)], [F(-1, 3), F(1)], [F(1), F(-1), F(1)]],
                     b=[F(1, 8), F(3, 8), F(3, 8), F(1, 8)])


def tableau_step(f, y, h, A, b):
    ks = []
    for i in range(len(b)):
        yi = y + h * sum((A[i][j] * ks[j] for j in range(i)), F(0))
        ks.append(f(yi))
    return y + h * sum((b[i] * ks[i] for i in range(len(b))), F(0))


def sq(y):
    return y * y


def test_one_step_matches_classical_tableau(ora):
    # h = 1/8 and y0 = 1 are exact binary fractions, so the only error of the
    # oracle is its own rounding.
    h, y0 = F(1, 8), F(1)
    exact = tableau_step(sq, y0, h, **CLASSICAL)
    other = tableau_step(sq, y0, h, **THREE_EIGHTHS)
    got = ora.rk4(ora.RICCATI, [], np.array([[1.0]]), 0.125, 1)[0, 0]
    assert abs(F(got) - exact) <= 4 * abs(exact) * F(2) ** -52
    # the 3/8 rule is also fourth order; the test must tell the two apart
    assert abs(float(other - exact)) > 1e3 * abs(float(exact)) * 2.0 ** -52


def test_known_classical_value_h_tenth(ora):
    # one classical step from y0 = 1 with h = 1/10 (exact rational value of the
    # tableau), in the double nearest to 0.1
    exact = tableau_step(sq, F(1), F(1, 10), **CLASSICAL)
    got = ora.rk4(ora.RICCATI, [], np.array([[1.0]]), 0.1, 1)[0, 0]
    assert abs(got - float(exact)) < 1e-15


def test_many_steps_exact_arithmetic(ora):
    h, y = F(1, 16), F(1, 2)
    for _ in range(3):
        y = tableau_step(sq, y, h, **CLASSICAL)
    got = ora.rk4(ora.RICCATI, [], np.array([[0.5]]), 1.0 / 16, 3)[0, 0]
    assert abs(got - float(y)) <= 1e-14 * abs(float(y))


def test_fourth_order_local_error_riccati(ora):
    # local error of one step ~ C h^5: halving h divides it by ~32
    errs = []
    for h in (0.02, 0.01, 0.005):
        got = ora.rk4(ora.RICCATI, [], np.array([[1.0]]), h, 1)[0, 0]
        errs.append(abs(got - 1.0 / (1.0 - h)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 30 < r1 < 34 and 30 < r2 < 34, (r1, r2)


def test_global_order_four_riccati(ora):
    # global error at t = 0.5 from y0 = 1 (exact value 2): ratio -> 16
    errs = []
    for k in (1, 2, 3):
        n = 10 * 2 ** k
        got = ora.rk4(ora.RICCATI, [], np.array([[1.0]]), 0.5 / n, n)[0, 0]
        errs.append(abs(got - 2.0))
    assert abs(errs[0] / errs[1] - 16) < 1.0 and abs(errs[1] / errs[2] - 16) < 0.7


def test_zero_steps_and_zero_step_size(ora):
    x = np.array([[1.25], [-3.0], [7.5]])
    assert np.array_equal(ora.rk4(ora.LORENZ, [10, 28, 8 / 3], x, 0.01, 0), x)
    assert np.array_equal(ora.rk4(ora.LORENZ, [10, 28, 8 / 3], x, 0.0, 10), x)
