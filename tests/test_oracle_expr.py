"""Pins of the oracle's expression right-hand sides (Appendix A: a State
Variable holds the expression of its time derivative; Appendix A.1: that
expression fills in the general RK4 step).

The evaluator is pinned against things it does not share code with: the
built-in oracle systems (pinned on their own by closed forms and
convergence), hand-evaluated constant expressions, RK4 on quadratures whose
integrals are known in closed form (RK4 on x' = g(t) is Simpson's rule), and
the exact RK4 amplification matrix of a linear system."""
import math

import numpy as np
import pytest

from expr_cases import BAD, CONSTANTS, LORENZ_EXPR, QUAD_EXPRS, WC_EXPR
from paper_1505_00344_amd import inputs as I


def lorenz_start(n=300, seed=3):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-15, 15, (3, n))
    x[2] += 25
    return x


def test_lorenz_expressions_equal_builtin_bitwise(ora):
    x = lorenz_start()
    P = I.LORENZ_PARAMS
    rng = np.random.default_rng(4)
    pp = np.stack([rng.uniform(9, 11, x.shape[1]), rng.uniform(26, 30, x.shape[1])])
    a = ora.rk4(ora.LORENZ, P, x, 0.004, 400, pp_slot=[0, 1], pparams=pp)
    b = ora.expr_rk4(LORENZ_EXPR, P, x, 0.004, 400, pp_slot=[0, 1], pparams=pp)
    assert np.array_equal(a, b)
    for kahan in (False, True):
        for h, n in ((0.004, 400), (-0.002, 40)):  # backward in time blows up sooner
            a, ca = ora.rk4_f32(ora.LORENZ, P, x, h, n, pp_slot=[1], pparams=pp[1:], kahan=kahan)
            b, cb = ora.expr_rk4_f32(LORENZ_EXPR, P, x, h, n, pp_slot=[1], pparams=pp[1:], kahan=kahan)
            assert np.isfinite(a).all() and np.array_equal(a, b)
            if kahan:
                assert np.array_equal(ca, cb)


def test_wilson_cowan_expressions_equal_builtin_bitwise(ora):
    w = I.wilson_cowan_4m(n=2000)
    e = I.generate(w)
    a = ora.rk4(ora.WILSON_COWAN, w.params, e.state, 0.01, 200, pp_slot=w.pp_slot, pparams=e.pparams)
    b = ora.expr_rk4(WC_EXPR, w.params, e.state, 0.01, 200, pp_slot=w.pp_slot, pparams=e.pparams)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("expr,value", CONSTANTS)
def test_constant_expressions(ora, expr, value):
    # x' = c from x = 0 with h = 6: s = 6c and x = (h/6) s = 6c exactly
    for prec in ("fp64", "fp32"):
        if prec == "fp64":
            x = ora.expr_rk4([expr], [], np.zeros((1, 1)), 6.0, 1)
        else:
            x, _ = ora.expr_rk4_f32([expr], [], np.zeros((1, 1)), 6.0, 1)
        assert x[0, 0] == 6 * value, (expr, prec)


def test_literal_rounds_once_to_float(ora):
    # 0.1 is read as the nearest double, then rounded to float: the float
    # nearest 0.1 (a literal read straight as float gives the same here)
    x, _ = ora.expr_rk4_f32(["0.1"], [], np.zeros((1, 1)), 6.0, 1)
    assert x[0, 0] == np.float32(6) * np.float32(0.1)


CLOSED_FORMS = [  # the integral from 0 to t of each integrand in QUAD_EXPRS
    lambda t: math.exp(t) - 1,
    lambda t: math.exp(t) - 1 - t,
    lambda t: (1 + t) * math.log(1 + t) - t,
    lambda t: (1 + t) * math.log(1 + t) - t,
    lambda t: 1 - math.cos(t),
    lambda t: math.sin(t),
    lambda t: -math.log(math.cos(t)),
    lambda t: math.log(math.cosh(t)),
    lambda t: math.cosh(t) - 1,
    lambda t: math.sinh(t),
    lambda t: t * math.atan(t) - 0.5 * math.log(1 + t * t),
    lambda t: t ** 4 / 4,
    lambda t: math.atan(t),
    lambda t: (2 / 3) * ((1 + t) ** 1.5 - 1),
]


def quad_system():
    return ["1"] + QUAD_EXPRS


@pytest.mark.parametrize("T", [1.0, 0.5])
def test_functions_by_quadrature(ora, T):
    # dim 15: x0' = 1 is time, x_k' = g_k(x0); RK4 is Simpson's rule on each
    n = 100
    x = ora.expr_rk4(quad_system(), [], np.zeros((15, 1)), T / n, n)
    assert x[0, 0] == pytest.approx(T, abs=1e-14)
    for k, (g, F) in enumerate(zip(QUAD_EXPRS, CLOSED_FORMS), start=1):
        assert x[k, 0] == pytest.approx(F(T), rel=2e-9, abs=1e-12), g


def test_linear_system_equals_rk4_amplification(ora):
    # x' = A x: one RK4 step multiplies by R(hA) = I + hA + (hA)^2/2 + (hA)^3/6 + (hA)^4/24
    A = np.array([[-0.5, 2.0, 0.0], [-2.0, -0.5, 0.3], [0.1, 0.0, -1.0]])
    exprs = ["p0*x0 + p1*x1 + p2*x2", "p3*x0 + p4*x1 + p5*x2", "p6*x0 + p7*x1 + p8*x2"]
    rng = np.random.default_rng(5)
    x0 = rng.normal(size=(3, 8))
    h, n = 0.01, 500
    Z = h * A
    R = np.eye(3) + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + Z @ Z @ Z @ Z / 24
    want = np.linalg.matrix_power(R, n) @ x0
    got = ora.expr_rk4(exprs, A.ravel(), x0, h, n)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-13)
    # a per-particle value replaces one global parameter
    pp = rng.uniform(-1, 1, (1, 8))
    got = ora.expr_rk4(exprs, A.ravel(), x0, h, n, pp_slot=[8], pparams=pp)
    for i in range(8):
        Ai = A.copy()
        Ai[2, 2] = pp[0, i]
        Zi = h * Ai
        Ri = np.eye(3) + Zi + Zi @ Zi / 2 + Zi @ Zi @ Zi / 6 + Zi @ Zi @ Zi @ Zi / 24
        np.testing.assert_allclose(got[:, i], np.linalg.matrix_power(Ri, n) @ x0[:, i], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("text", BAD)
def test_malformed_expressions_are_rejected(ora, text):
    with pytest.raises(ValueError):
        ora.expr_rk4([text, "x0", "x1"], [], np.zeros((3, 1)), 0.1, 1)


# --- forward-mode derivative of the expression map (the adjoint's reference) ---

def test_dual_value_part_is_the_map(ora):
    x = lorenz_start(200)
    P = I.LORENZ_PARAMS
    a = ora.expr_rk4(LORENZ_EXPR, P, x, 0.004, 300)
    b, _ = ora.expr_rk4_dual(LORENZ_EXPR, P, x, 0.004, 300, dx0=np.ones_like(x))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("which", ["lorenz", "wc"])
def test_dual_derivative_equals_builtin_complex_step(ora, which):
    # the same maps written as expressions; derivative along random directions
    # of the state, the global parameters and a per-particle parameter
    rng = np.random.default_rng(9)
    if which == "lorenz":
        exprs, sysid, P, x, h, n = LORENZ_EXPR, ora.LORENZ, I.LORENZ_PARAMS, lorenz_start(200), 0.004, 150
        slots, pp = [1], rng.uniform(20, 30, (1, 200))
    else:
        w = I.wilson_cowan_4m(n=400)
        e = I.generate(w)
        exprs, sysid, P, x, h, n = WC_EXPR, ora.WILSON_COWAN, w.params, e.state, -0.01, 200
        slots, pp = w.pp_slot, e.pparams
    dx0 = rng.normal(size=x.shape)
    dparams = rng.normal(size=len(P))
    dpp = rng.normal(size=pp.shape)
    _, want = ora.rk4_cstep(sysid, P, x, h, n, pp_slot=slots, pparams=pp, dx0=dx0, dparams=dparams, dpp=dpp)
    _, got = ora.expr_rk4_dual(exprs, P, x, h, n, pp_slot=slots, pparams=pp, dx0=dx0, dparams=dparams, dpp=dpp)
    scale = np.maximum(np.abs(want), 1e-3 * np.abs(want).max())
    assert (np.abs(got - want) / scale).max() <= 1e-10


INTEGRANDS = [  # each expression of QUAD_EXPRS as a function of time
    math.exp, math.expm1, lambda t: math.log(1 + t), math.log1p, math.sin, math.cos, math.tan, math.tanh,
    math.sinh, math.cosh, math.atan, lambda t: t ** 3, lambda t: 1 / (1 + t * t), lambda t: math.sqrt(1 + t),
]


def test_dual_derivative_of_every_function(ora):
    # x_k(T) = x_k(0) + int_{t0}^{t0+T} g_k(t) dt, so d x_k(T) / d t0 = g_k(t0 + T) - g_k(t0);
    # RK4 integrates g_k' by Simpson's rule (error ~h^4), which tests every derivative rule
    t0, T, n = 0.1, 0.5, 100
    x = np.zeros((15, 1))
    x[0] = t0
    dx0 = np.zeros((15, 1))
    dx0[0] = 1.0
    _, d = ora.expr_rk4_dual(quad_system(), [], x, T / n, n, dx0=dx0)
    assert d[0, 0] == 1.0
    for k, (text, g) in enumerate(zip(QUAD_EXPRS, INTEGRANDS), start=1):
        assert d[k, 0] == pytest.approx(g(t0 + T) - g(t0), rel=1e-9, abs=1e-12), text


@pytest.mark.parametrize("exprs,params", [
    (["pow(fabs(x1) + 1, p0) - x0", "fmin(x0, p1) - fmax(x1, -p1) * 0.5"], [1.5, 0.3]),
    (["x1 / (1 + x0*x0)", "-p0 * x0 + p1 * fma(x0, x1, -x1)"], [0.8, 0.4]),
])
def test_dual_derivative_against_central_differences(ora, exprs, params):
    rng = np.random.default_rng(4)
    x = rng.uniform(-1.5, 1.5, (2, 64))
    dx0 = rng.normal(size=x.shape)
    dparams = rng.normal(size=len(params))
    _, d = ora.expr_rk4_dual(exprs, params, x, 0.01, 100, dx0=dx0, dparams=dparams)
    eps = 1e-6
    xp = ora.expr_rk4(exprs, np.add(params, eps * dparams), x + eps * dx0, 0.01, 100)
    xm = ora.expr_rk4(exprs, np.subtract(params, eps * dparams), x - eps * dx0, 0.01, 100)
    fd = (xp - xm) / (2 * eps)
    assert np.abs(d - fd).max() <= 1e-6 * max(1.0, np.abs(fd).max())
