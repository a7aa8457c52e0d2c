"""Accuracy of the library's double-precision elementary kernels on the device
(ff_math_eval): the exp, exp2 and expm1 kernels (Cody-Waite reduction and
Chebyshev interpolants), the refined reciprocal, the clamped
logistics of the Wilson-Cowan and Hodgkin-Huxley right-hand sides and the
HH rate function psi(u) = u/(e^u - 1) (Section 3's rates; the paper fixes no
exponential of its own).  The reference is the same function in 80-bit long
double (numpy.longdouble), an independent implementation with 11 more
mantissa bits; errors are in units in the last place of the double nearest
the reference."""
import numpy as np
import pytest

from helpers import api, record, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LD = np.longdouble
N = 1 << 20


@pytest.fixture(scope="module")
def A():
    assert np.finfo(LD).nmant >= 63, "the reference needs 80-bit long double"
    return api()


def ulp_error(got, ref):
    """|got - ref| in units of the spacing of the double nearest ref (ref
    finite and nonzero)."""
    ref64 = ref.astype(np.float64)
    return (np.abs(got.astype(LD) - ref) / np.spacing(np.abs(ref64)).astype(LD)).astype(np.float64)


def draw(lo, hi, seed):
    return np.random.default_rng(seed).uniform(lo, hi, N)


def run(A, fn, x):
    y = A.math_eval(fn, to_dev(x, torch.float64))
    torch.cuda.synchronize()
    return to_host(y)


def reference(fn, x):
    xl = x.astype(LD)
    if fn == "exp":
        return np.exp(xl)
    if fn == "exp2":
        return np.exp2(xl)
    if fn == "expm1":
        return np.expm1(xl)
    if fn == "rcp":
        return LD(1) / xl
    if fn == "logistic":
        return LD(1) / (LD(1) + np.exp(np.clip(xl, LD(-700), LD(700))))
    if fn == "logistic2":
        return LD(1) / (LD(1) + np.exp2(np.clip(xl, LD(-1000), LD(1000))))
    if fn == "psi":
        with np.errstate(invalid="ignore", divide="ignore"):
            r = xl / np.expm1(np.minimum(xl, LD(700)))
        return np.where(xl == 0, LD(1), r)
    raise ValueError(fn)


# (function, argument range, bound in ulp).  The first four bounds are the
# kernels' accuracy as measured on the CPU against long-double references
# (within 0.94, 0.89, 1.10 ulp; the reciprocal within 1 ulp) rounded up; the
# composed functions add the rounding of 1 + e and the reciprocal's, or the
# quotient's, error to the exponential's: the logistic up to 0.9 + 0.5 + 1
# ulp relative (about 2.4 ulp of the result), psi = u/expm1(u) up to
# 1.1 + 1 (measured on the device: 2.41 and 1.59).
CASES = [
    ("exp", (-708.0, 708.0), 1.0), ("exp", (-1.0, 1.0), 1.0), ("exp", (-1e-3, 1e-3), 1.0),
    ("exp2", (-1070.0, 1023.0), 1.0), ("exp2", (-1.0, 1.0), 1.0), ("exp2", (-1e-3, 1e-3), 1.0),
    ("expm1", (-708.0, 708.0), 1.2), ("expm1", (-40.0, 40.0), 1.2), ("expm1", (-1.0, 1.0), 1.2),
    ("expm1", (-1e-3, 1e-3), 1.2),
    ("logistic", (-800.0, 800.0), 3.0), ("logistic", (-40.0, 40.0), 3.0),
    ("logistic2", (-1100.0, 1100.0), 3.0), ("logistic2", (-60.0, 60.0), 3.0),
    ("psi", (-700.0, 720.0), 2.5), ("psi", (-30.0, 30.0), 2.5), ("psi", (-1e-3, 1e-3), 2.5),
]


@pytest.mark.parametrize("fn,rng,bound", CASES, ids=[f"{c[0]}[{c[1][0]:g},{c[1][1]:g}]" for c in CASES])
def test_kernel_ulp_error(A, fn, rng, bound):
    x = draw(*rng, seed=1000 + CASES.index((fn, rng, bound)))
    got = run(A, fn, x)
    ref = reference(fn, x)
    ok = np.isfinite(ref) & (ref != 0)
    assert np.isfinite(got[ok]).all()
    e = ulp_error(got[ok], ref[ok])
    record(f"math_{fn}_{rng[0]:g}_{rng[1]:g}", ulp={"max": float(e.max()), "mean": float(e.mean()),
                                                  "p999": float(np.quantile(e, 0.999))})
    assert e.max() <= bound, (fn, rng, float(e.max()), float(x[ok][np.argmax(e)]))


def test_reciprocal_over_the_exponent_range(A):
    r = np.random.default_rng(11)
    x = np.ldexp(r.uniform(1.0, 2.0, N), r.integers(-1022, 1022, N).astype(np.int32)) * r.choice([-1.0, 1.0], N)
    got = run(A, "rcp", x)
    e = ulp_error(got, reference("rcp", x))
    record("math_rcp_exponent_range", ulp={"max": float(e.max()), "mean": float(e.mean())})
    assert e.max() <= 1.0
    assert np.array_equal(run(A, "rcp", np.array([1.0, -2.0, 0.25, 2.0 ** 1022])),
                          np.array([1.0, -0.5, 4.0, 2.0 ** -1022]))


def test_special_values(A):
    k = np.arange(-1074, 1024, dtype=np.float64)
    assert np.array_equal(run(A, "exp2", k), np.ldexp(1.0, k.astype(np.int32)))   # exact powers of two
    assert np.array_equal(run(A, "exp2", np.array([1024.0, 1100.0, -1076.0, -2000.0])),
                          np.array([np.inf, np.inf, 0.0, 0.0]))
    assert run(A, "exp", np.array([0.0]))[0] == 1.0
    tiny = np.array([1e-300, -1e-300, 2.0 ** -1074, 1e-20])
    assert np.array_equal(run(A, "expm1", tiny), tiny)      # e^x - 1 = x below half an ulp of x
    assert np.array_equal(run(A, "psi", np.array([0.0])), np.array([1.0]))
    for fn in ("logistic", "logistic2"):
        y = run(A, fn, np.array([np.nan, np.inf, -np.inf, -5000.0, 0.0]))
        assert np.isnan(y[:3]).all()                          # a NaN or infinite argument stays visible
        assert y[3] == 1.0 and y[4] == 0.5
    assert run(A, "logistic2", np.array([5000.0]))[0] == pytest.approx(2.0 ** -1000, rel=1e-15)
    assert run(A, "logistic", np.array([5000.0]))[0] == pytest.approx(np.exp(-700.0), rel=1e-15)
    assert np.isnan(run(A, "psi", np.array([np.nan]))[0])

