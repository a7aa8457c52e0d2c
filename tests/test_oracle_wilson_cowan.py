"""Pins of the oracle's Wilson-Cowan pair (the sigmoid-coupled structure of
Section 2.1, Eqs. stn_gpe/eqnGPe, with the published Wilson-Cowan constants
c1..c4 = 16, 12, 15, 3, aE = 1.3, thetaE = 4, aI = 2, thetaI = 3.7)."""
import numpy as np
from scipy.optimize import fsolve

from paper_1505_00344_amd.inputs import WC_PARAMS


def params(**kw):
    names = ["c1", "c2", "c3", "c4", "aE", "thE", "aI", "thI", "P", "Q"]
    p = list(WC_PARAMS)
    for k, v in kw.items():
        p[names.index(k)] = v
    return p


def R4(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def test_saturated_regime_is_linear_closed_form(ora):
    # with huge opposite inputs S_E = 1 and S_I = 0 exactly (exp under/overflow),
    # so E' = 1 - E and I' = -I: E_n = 1 + (E0 - 1) R(-h)^n, I_n = I0 R(-h)^n
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, size=(2, 64))
    h, n = 0.01, 1000
    p = params(P=1000.0, Q=-1000.0)
    got = ora.rk4(ora.WILSON_COWAN, p, x, h, n)
    r = R4(-h) ** n
    assert np.allclose(got[0], 1 + (x[0] - 1) * r, rtol=1e-13, atol=1e-15)
    assert np.allclose(got[1], x[1] * r, rtol=1e-13, atol=1e-300)
    # backward: the same closed form with -h, and no NaN even when saturated
    gotb = ora.rk4(ora.WILSON_COWAN, p, x, -h, 300)
    rb = R4(h) ** 300
    assert np.allclose(gotb[0], 1 + (x[0] - 1) * rb, rtol=1e-12)
    f = ora.rhs(ora.WILSON_COWAN, params(P=1e6, Q=-1e6), x.T)
    assert np.all(np.isfinite(f))


def test_half_activation_point(ora):
    # at u = theta the sigmoid is exactly 1/2.  With thetaI = 3.75, Q = -2.25,
    # P = 2 the point (E, I) = (1/2, 1/2) has uE = 4 and uI = 3.75 exactly, so it
    # is an exact equilibrium and the RK4 map leaves it untouched.
    p = params(thI=3.75, Q=-2.25, P=2.0)
    x = np.array([[0.5], [0.5]])
    assert np.array_equal(ora.rhs(ora.WILSON_COWAN, p, x.T), np.zeros((1, 2)))
    assert np.array_equal(ora.rk4(ora.WILSON_COWAN, p, x, 0.01, 1000), x)
    assert np.array_equal(ora.rk4(ora.WILSON_COWAN, p, x, -0.01, 1000), x)
    # off the point: f = (1/2 - E, 1/2 - I) whenever both inputs sit at threshold
    E, I = 0.25, 0.75
    p2 = params(P=4 - 16 * E + 12 * I, Q=3.7 - 15 * E + 3 * I)
    f = ora.rhs(ora.WILSON_COWAN, p2, np.array([[E, I]]))[0]
    assert np.allclose(f, [0.5 - E, 0.5 - I], atol=1e-15)


def test_sigmoid_gain_and_threshold(ora):
    # dS/du at u = theta is a/4; and S(theta + 1/a) = 1/(1 + e^-1)
    E, I = 0.3, 0.6
    base = dict(P=4 - 16 * E + 12 * I)
    eps = 1e-6
    fp = ora.rhs(ora.WILSON_COWAN, params(P=base["P"] + eps), np.array([[E, I]]))[0, 0]
    fm = ora.rhs(ora.WILSON_COWAN, params(P=base["P"] - eps), np.array([[E, I]]))[0, 0]
    assert abs((fp - fm) / (2 * eps) - 1.3 / 4) < 1e-8
    f = ora.rhs(ora.WILSON_COWAN, params(P=base["P"] + 1 / 1.3), np.array([[E, I]]))[0, 0]
    assert abs(f - (1 / (1 + np.exp(-1)) - E)) < 1e-15


def test_forward_particles_reach_the_stable_equilibrium(ora):
    # forward-time particles reveal stable attractors (Section 1); at low input
    # P = -2 the pair has a single stable equilibrium (low activity), found here
    # with a library root finder
    p = params(P=-2.0)
    f = lambda v: ora.rhs(ora.WILSON_COWAN, p, np.array([v]))[0]
    root = fsolve(f, [0.01, 0.01], xtol=1e-14)
    J = np.array([[(f(root + e)[r] - f(root - e)[r]) / 2e-7 for e in np.eye(2) * 1e-7] for r in range(2)])
    assert np.all(np.linalg.eigvals(J).real < 0)
    x = np.random.default_rng(2).uniform(0, 1, size=(2, 500))
    got = ora.rk4(ora.WILSON_COWAN, p, x, 0.01, 5000)
    assert np.abs(got - root[:, None]).max() < 1e-9


def test_fourth_order_convergence(ora):
    x0 = np.random.default_rng(3).uniform(0, 1, size=(2, 16))
    p = params(P=1.25)
    ref = ora.rk4(ora.WILSON_COWAN, p, x0, 4.0 / 3200, 3200)
    errs = [np.abs(ora.rk4(ora.WILSON_COWAN, p, x0, 4.0 / n, n) - ref).max() for n in (50, 100, 200)]
    assert abs(errs[0] / errs[1] - 16) < 1.5 and abs(errs[1] / errs[2] - 16) < 1.0


def test_per_particle_P_equals_separate_runs(ora):
    x = np.random.default_rng(4).uniform(0, 1, size=(2, 12))
    Pv = np.random.default_rng(5).uniform(-2, 4, 12)
    got = ora.rk4(ora.WILSON_COWAN, WC_PARAMS, x, -0.01, 300, pp_slot=[8], pparams=Pv[None])
    for i in range(12):
        want = ora.rk4(ora.WILSON_COWAN, params(P=Pv[i]), x[:, i:i + 1], -0.01, 300)
        assert np.array_equal(got[:, i:i + 1], want)
