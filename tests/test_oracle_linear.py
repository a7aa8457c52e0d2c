"""Pins of the oracle on linear systems x' = A x.

Classical RK4 applied to x' = A x is x_{n+1} = T4(hA) x_n with
T4(Z) = I + Z + Z^2/2 + Z^3/6 + Z^4/24 (closed form; the method of Section 2.1
and Appendix A.1 applied to a linear right-hand side).
"""
import numpy as np
import pytest
from scipy.linalg import expm


def T4(Z):
    I = np.eye(Z.shape[0])
    Z2 = Z @ Z
    return I + Z + Z2 / 2 + Z2 @ Z / 6 + Z2 @ Z2 / 24


def rand_A(rng, dim):
    A = rng.normal(size=(dim, dim))
    return A / max(1.0, np.max(np.abs(np.linalg.eigvals(A))))


@pytest.mark.parametrize("dim", [1, 2, 3, 4])
def test_matches_T4_power(ora, dim):
    rng = np.random.default_rng(dim)
    A = rand_A(rng, dim)
    x0 = rng.uniform(-1, 1, size=(dim, 64))
    h, n = 0.05, 200
    got = ora.rk4(ora.LINEAR, A.ravel(), x0, h, n)
    want = np.linalg.matrix_power(T4(h * A), n) @ x0
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err < 1e-12, err


def test_converges_to_exponential_fourth_order(ora):
    rng = np.random.default_rng(7)
    A = rand_A(rng, 3)
    x0 = rng.uniform(-1, 1, size=(3, 16))
    t = 2.0
    exact = expm(A * t) @ x0
    errs = []
    for n in (20, 40, 80):
        got = ora.rk4(ora.LINEAR, A.ravel(), x0, t / n, n)
        errs.append(np.abs(got - exact).max())
    assert abs(errs[0] / errs[1] - 16) < 1.5 and abs(errs[1] / errs[2] - 16) < 1.0


def test_harmonic_oscillator_norm_factor(ora):
    # A = [[0, -w], [w, 0]]: |R(i w h)|^2 = 1 - (wh)^6/72 + (wh)^8/576 per step
    w, h, n = 1.0, 0.1, 1000
    A = np.array([[0.0, -w], [w, 0.0]])
    x0 = np.array([[1.0, 0.3], [0.0, -2.0]])
    got = ora.rk4(ora.LINEAR, A.ravel(), x0, h, n)
    th = w * h
    factor = 1 - th ** 6 / 72 + th ** 8 / 576
    ratio = np.sum(got ** 2, axis=0) / np.sum(x0 ** 2, axis=0)
    assert np.allclose(ratio, factor ** n, rtol=1e-12, atol=0)
    assert abs(factor - (1 - 1.38715e-8)) < 1e-13


def test_forward_then_backward(ora):
    # forward n steps then backward n steps equals R(-hA)^n R(hA)^n x0
    rng = np.random.default_rng(11)
    A = rand_A(rng, 4)
    x0 = rng.uniform(-1, 1, size=(4, 32))
    h, n = 0.05, 100
    fwd = ora.rk4(ora.LINEAR, A.ravel(), x0, h, n)
    back = ora.rk4(ora.LINEAR, A.ravel(), fwd, -h, n)
    want = np.linalg.matrix_power(T4(-h * A), n) @ np.linalg.matrix_power(T4(h * A), n) @ x0
    assert np.abs(back - want).max() < 1e-12 * np.abs(want).max()
    # and it is not the identity: R(z)R(-z) = 1 + z^6/72 + O(z^8)
    assert np.abs(back - x0).max() > 1e-11


def test_per_particle_matrix_entry(ora):
    # a per-particle parameter replaces one entry of A for that particle only
    rng = np.random.default_rng(3)
    A = rand_A(rng, 2)
    x0 = rng.uniform(-1, 1, size=(2, 8))
    a01 = rng.uniform(-1, 1, size=8)
    got = ora.rk4(ora.LINEAR, A.ravel(), x0, 0.1, 30, pp_slot=[1], pparams=a01[None, :])
    for i in range(8):
        Ai = A.copy()
        Ai[0, 1] = a01[i]
        want = np.linalg.matrix_power(T4(0.1 * Ai), 30) @ x0[:, i]
        assert np.allclose(got[:, i], want, rtol=1e-13, atol=1e-15)
