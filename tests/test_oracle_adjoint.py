"""Pins of the oracle's discrete adjoint (exact reverse-mode gradient of the
RK4 map of Section 2.1 / Appendix A.1 with respect to initial states and
parameters).

Independent references: the complex-step derivative of the oracle's forward
map (forward mode in complex arithmetic, Squire & Trapp 1998), central finite
differences, the closed form (T4(hA)^T)^n for linear systems, and a
dot-product test.  The Jacobians themselves are checked against central
differences of the right-hand side.
"""
import numpy as np
import pytest

from paper_1505_00344_amd.inputs import HH_PARAMS, LORENZ_BOX, LORENZ_PARAMS, WC_PARAMS


def cases(ora):
    rng = np.random.default_rng(42)
    lor = rng.uniform([[-20], [-30], [0]], [[20], [30], [50]], size=(3, 8))
    wc = rng.uniform(0, 1, size=(2, 8))
    hh = rng.uniform(0, 1, size=(15, 4))
    hh[0::5] = rng.uniform(-80, 40, size=(3, 4))
    A = rng.normal(size=(3, 3)) * 0.5
    lin = rng.uniform(-1, 1, size=(3, 6))
    return {
        "linear": (ora.LINEAR, A.ravel(), lin, 0.05, 60, [4], rng.uniform(-1, 1, (1, 6))),
        "lorenz": (ora.LORENZ, LORENZ_PARAMS, lor, 0.005, 200, [1], rng.uniform(0, 50, (1, 8))),
        "lorenz_back": (ora.LORENZ, LORENZ_PARAMS, lor, -0.005, 40, [], None),
        "wc": (ora.WILSON_COWAN, WC_PARAMS, wc, 0.01, 300, [8], rng.uniform(-2, 4, (1, 8))),
        "wc_back": (ora.WILSON_COWAN, WC_PARAMS, wc, -0.01, 300, [8], rng.uniform(-2, 4, (1, 8))),
        "hh": (ora.HH_RING, HH_PARAMS, hh, 0.01, 300, [8, 7], np.array([[0.5] * 4, [10.0] * 4])),
    }


CASES = ["linear", "lorenz", "lorenz_back", "wc", "wc_back", "hh"]


def rel(a, b, floor=1e-3):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


@pytest.mark.parametrize("name", CASES)
def test_jacobians_match_differences(ora, name):
    sysid, p, x0, *_ = cases(ora)[name]
    pts = x0.T[:3]
    J, Fp = ora.jacobians(sysid, p, pts)
    dim = pts.shape[1]
    for k, x in enumerate(pts):
        for c in range(dim):
            e = np.zeros(dim)
            e[c] = 1e-6 * max(1.0, abs(x[c]))
            fd = (ora.rhs(sysid, p, x + e)[0] - ora.rhs(sysid, p, x - e)[0]) / (2 * e[c])
            assert np.allclose(J[k][:, c], fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max() + 1e-9)
        for q in range(len(p)):
            dp = np.zeros(len(p))
            dp[q] = 1e-6 * max(1.0, abs(p[q]))
            fd = (ora.rhs(sysid, np.add(p, dp), x)[0] - ora.rhs(sysid, np.subtract(p, dp), x)[0]) / (2 * dp[q])
            assert np.allclose(Fp[k][:, q], fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max() + 1e-9)


@pytest.mark.parametrize("name", CASES)
def test_adjoint_matches_complex_step(ora, name):
    sysid, p, x0, h, n, slots, pp = cases(ora)[name]
    dim, npart = x0.shape
    rng = np.random.default_rng(1)
    w = rng.normal(size=(dim, npart))   # loss L = sum_i <w_i, x_i(T)>
    lam0, mu_pp, mu_g = ora.adjoint(sysid, p, x0, w, h, n, pp_slot=slots, pparams=pp)
    # d/dx0 along every unit direction, one component at a time
    for c in range(dim):
        dx = np.zeros_like(x0)
        dx[c] = 1.0
        _, dxT = ora.rk4_cstep(sysid, p, x0, h, n, pp_slot=slots, pparams=pp, dx0=dx)
        g = np.sum(w * dxT, axis=0)
        assert rel(lam0[c], g).max() < 1e-10, (c, rel(lam0[c], g).max())
    # per-particle parameters
    for k in range(len(slots)):
        dpp = np.zeros_like(pp)
        dpp[k] = 1.0
        _, dxT = ora.rk4_cstep(sysid, p, x0, h, n, pp_slot=slots, pparams=pp, dpp=dpp)
        g = np.sum(w * dxT, axis=0)
        assert rel(mu_pp[k], g).max() < 1e-10
    # global parameters (summed over particles)
    for q in range(len(p)):
        if q in slots:
            continue
        dp = np.zeros(len(p))
        dp[q] = 1.0
        _, dxT = ora.rk4_cstep(sysid, p, x0, h, n, pp_slot=slots, pparams=pp, dparams=dp)
        g = np.sum(w * dxT)
        assert rel(mu_g[q], g, floor=1e-3 * max(1.0, abs(g))) < 1e-10, q


def test_adjoint_linear_closed_form(ora):
    rng = np.random.default_rng(5)
    A = rng.normal(size=(4, 4)) * 0.3
    Z = 0.05 * A
    Z2 = Z @ Z
    T = np.eye(4) + Z + Z2 / 2 + Z2 @ Z / 6 + Z2 @ Z2 / 24
    lamT = rng.normal(size=(4, 5))
    lam0, _, _ = ora.adjoint(ora.LINEAR, A.ravel(), rng.normal(size=(4, 5)), lamT, 0.05, 100)
    want = np.linalg.matrix_power(T.T, 100) @ lamT
    assert np.allclose(lam0, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_adjoint_central_differences_lorenz_r(ora):
    # d(mean z(T))/d r_i for per-particle r, 200 steps, against central
    # differences with h = 1e-4 in FP64
    rng = np.random.default_rng(8)
    n = 64
    x0 = np.stack([rng.uniform(lo, hi, n) for lo, hi in LORENZ_BOX])
    r = rng.uniform(0, 50, (1, n))
    lamT = np.zeros((3, n))
    lamT[2] = 1.0 / n
    _, mu, _ = ora.adjoint(ora.LORENZ, LORENZ_PARAMS, x0, lamT, 0.005, 200, pp_slot=[1], pparams=r)
    zp = ora.rk4(ora.LORENZ, LORENZ_PARAMS, x0, 0.005, 200, pp_slot=[1], pparams=r + 1e-4)[2]
    zm = ora.rk4(ora.LORENZ, LORENZ_PARAMS, x0, 0.005, 200, pp_slot=[1], pparams=r - 1e-4)[2]
    fd = (zp - zm) / (2e-4) / n
    e = rel(mu[0], fd, floor=1e-3 / n)
    assert np.quantile(e, 0.99) < 1e-6 and e.max() < 1e-4


def test_dot_product(ora):
    # <w, J v> = <J^T w, v> for the Jacobian of the whole n-step map
    rng = np.random.default_rng(9)
    x0 = rng.uniform(0, 1, size=(2, 10))
    P = rng.uniform(-2, 4, (1, 10))
    v = rng.normal(size=x0.shape)
    w = rng.normal(size=x0.shape)
    _, Jv = ora.rk4_cstep(ora.WILSON_COWAN, WC_PARAMS, x0, 0.01, 500, pp_slot=[8], pparams=P, dx0=v)
    JTw, _, _ = ora.adjoint(ora.WILSON_COWAN, WC_PARAMS, x0, w, 0.01, 500, pp_slot=[8], pparams=P)
    lhs = np.sum(w * Jv, axis=0)
    rhs = np.sum(JTw * v, axis=0)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-14)
