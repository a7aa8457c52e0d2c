"""GPU parity of expression systems (Appendix A: a State Variable's
right-hand side is an expression; Appendix A.1: it is filled into the step
kernel, compiled at run time) against the oracle's expression evaluator.

Expressions made of +, -, *, / and fma are correctly rounded operations on
both sides: identical bits.  Expressions with exp, sin, ... compare two math
libraries (each within a few ulp): the tolerances of the built-in systems
that call exp apply."""
import numpy as np
import pytest

import tolerances as tol
from expr_cases import LORENZ_EXPR, QUAD_EXPRS, WC_EXPR
from helpers import api, f32_inputs, finite_cols, mixed_error, quantiles, record, to_dev, to_host
from paper_1505_00344_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# a rational system (van der Pol with a saturating drive): arithmetic only
RATIONAL = ["x1", "p0*(1 - x0*x0)*x1 - x0 + p1*x2/(1 + x2*x2)", "-x2/p2 + x0*x1/(3 + x0*x0)"]


@pytest.fixture(scope="module")
def A():
    return api()


def run(A, sysobj, x, dt, nsteps, dtype, pp=None, pp_slot=(), kahan=False, tuning=None, n=None, offset=0):
    st = to_dev(x, dtype)
    ppt = None if pp is None else to_dev(pp, dtype)
    comp = torch.zeros_like(st) if kahan else None
    A.integrate(sysobj, st, dt, nsteps, pparams=ppt, pp_slot=pp_slot, comp=comp, tuning=tuning, n=n,
                offset=offset)
    torch.cuda.synchronize()
    return to_host(st), (None if comp is None else to_host(comp))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_kahan"])
@pytest.mark.parametrize("tuning", [None, (37, 2, 128), (200, 1, 64)])
def test_lorenz_expressions_bitwise(A, ora, prec, tuning):
    w = I.lorenz_4096()
    e = I.generate(w)
    nf = e.counts[0]
    x = e.state[:, :nf]
    rng = np.random.default_rng(7)
    pp = rng.uniform(24.0, 32.0, (1, nf))
    s_expr = A.System.from_exprs(LORENZ_EXPR, w.params)
    s_builtin = A.System("lorenz", 3, w.params)
    if prec == "fp64":
        got, _ = run(A, s_expr, x, 0.005, 400, torch.float64, pp=pp, pp_slot=[1], tuning=tuning)
        ref = ora.expr_rk4(LORENZ_EXPR, w.params, x, 0.005, 400, pp_slot=[1], pparams=pp)
        same, _ = run(A, s_builtin, x, 0.005, 400, torch.float64, pp=pp, pp_slot=[1], tuning=tuning)
        assert np.array_equal(got, ref) and np.array_equal(got, same)
    else:
        kahan = prec == "fp32_kahan"
        x32, pp32 = x.astype(np.float32), pp.astype(np.float32)
        got, c = run(A, s_expr, x32, 0.005, 400, torch.float32, pp=pp32, pp_slot=[1], kahan=kahan, tuning=tuning)
        ref, cref = ora.expr_rk4_f32(LORENZ_EXPR, w.params, x32, 0.005, 400, pp_slot=[1], pparams=pp32, kahan=kahan)
        same, csame = run(A, s_builtin, x32, 0.005, 400, torch.float32, pp=pp32, pp_slot=[1], kahan=kahan,
                          tuning=tuning)
        assert np.array_equal(got, ref) and np.array_equal(got, same)
        if kahan:
            assert np.array_equal(c, cref) and np.array_equal(c, csame)


@pytest.mark.parametrize("n", [1, 255, 256 * 3 + 17])
def test_rational_system_bitwise(A, ora, n):
    rng = np.random.default_rng(n)
    x = rng.uniform(-2, 2, (3, n))
    params = [1.5, 0.7, 2.0]
    s = A.System.from_exprs(RATIONAL, params)
    got, _ = run(A, s, x, 0.01, 300, torch.float64)
    assert np.array_equal(got, ora.expr_rk4(RATIONAL, params, x, 0.01, 300))
    for kahan in (False, True):
        x32 = x.astype(np.float32)
        got, c = run(A, s, x32, -0.01, 300, torch.float32, kahan=kahan)
        ref, cref = ora.expr_rk4_f32(RATIONAL, params, x32, -0.01, 300, kahan=kahan)
        assert np.array_equal(finite_cols(got), finite_cols(ref))
        fin = finite_cols(ref)
        assert np.array_equal(got[:, fin], ref[:, fin])
        if kahan:
            assert np.array_equal(c[:, fin], cref[:, fin])


def test_slice_with_offset_and_ld(A, ora):
    # particles 100..899 of a (3, 1000) array; the rest stay untouched
    rng = np.random.default_rng(11)
    x = rng.uniform(-2, 2, (3, 1000))
    params = [1.5, 0.7, 2.0]
    s = A.System.from_exprs(RATIONAL, params)
    got, _ = run(A, s, x, 0.01, 50, torch.float64, n=800, offset=100)
    assert np.array_equal(got[:, :100], x[:, :100]) and np.array_equal(got[:, 900:], x[:, 900:])
    assert np.array_equal(got[:, 100:900], ora.expr_rk4(RATIONAL, params, x[:, 100:900], 0.01, 50))


def test_wilson_cowan_expressions_fp64(A, ora):
    w = I.wilson_cowan_4m(n=8192 + 77)
    e = I.generate(w)
    nf = e.counts[0]
    s = A.System.from_exprs(WC_EXPR, w.params)
    x, pp = e.state[:, :nf], e.pparams[:, :nf]
    got, _ = run(A, s, x, e.dts[0], w.nsteps, torch.float64, pp=pp, pp_slot=w.pp_slot)
    ref = ora.expr_rk4(WC_EXPR, w.params, x, e.dts[0], w.nsteps, pp_slot=w.pp_slot, pparams=pp)
    err = mixed_error(got, ref)
    record("expr_wc_fp64_forward", err=quantiles(err))
    assert err.max() <= tol.FP64_REL, quantiles(err)


def test_wilson_cowan_expressions_fp32_vs_fp64(A, ora):
    w = I.wilson_cowan_4m(n=20000)
    e = I.generate(w)
    nf = e.counts[0]
    x, pp = f32_inputs(e.state[:, :nf]), f32_inputs(e.pparams[:, :nf])
    h = float(np.float32(0.01))
    ref = ora.expr_rk4(WC_EXPR, w.params, x, h, w.nsteps, pp_slot=w.pp_slot, pparams=pp)
    s = A.System.from_exprs(WC_EXPR, w.params)
    errs = {}
    for kahan in (False, True):
        got, _ = run(A, s, x.astype(np.float32), h, w.nsteps, torch.float32, pp=pp.astype(np.float32),
                     pp_slot=w.pp_slot, kahan=kahan)
        errs[kahan] = mixed_error(got, ref)
    record("expr_wc_fp32_vs_fp64", plain=quantiles(errs[False]), kahan=quantiles(errs[True]))
    assert np.quantile(errs[False], 0.99) <= tol.FP32_WC_P99, quantiles(errs[False])
    assert np.median(errs[True]) <= tol.KAHAN_WC_MEDIAN, quantiles(errs[True])
    assert np.quantile(errs[True], 0.99) <= tol.KAHAN_WC_P99, quantiles(errs[True])


def test_every_function_fp64_and_fp32(A, ora):
    # x0' = 1 is time and x_k' = g_k(x0): 15 components, each function once;
    # particles start at different times in [0, 0.5]
    exprs = ["1"] + QUAD_EXPRS
    n = 1000
    x = np.zeros((15, n))
    x[0] = np.linspace(0.0, 0.5, n)
    s = A.System.from_exprs(exprs)
    got, _ = run(A, s, x, 0.005, 100, torch.float64)
    ref = ora.expr_rk4(exprs, [], x, 0.005, 100)
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
    record("expr_functions_fp64", err=quantiles(err.ravel()))
    assert err.max() <= tol.FP64_REL
    x32 = x.astype(np.float32)
    got, _ = run(A, s, x32, 0.005, 100, torch.float32)
    ref32, _ = ora.expr_rk4_f32(exprs, [], x32, 0.005, 100)
    err = np.abs(got - ref32) / np.maximum(np.abs(ref32), 1.0)
    record("expr_functions_fp32", err=quantiles(err.ravel()))
    # 100 steps, each adding h/6-weighted values that differ by a few float ulp
    assert err.max() <= 1e-5


def test_reset_and_record_with_expressions(A, ora):
    w = I.lorenz_4096()
    e = I.generate(w)
    nf = e.counts[0]
    x0 = e.state[:, nf:]
    n = x0.shape[1]
    bounds = [(-40.0, 40.0), (-60.0, 60.0), (-10.0, 80.0)]
    s = A.System.from_exprs(LORENZ_EXPR, w.params)
    st = to_dev(x0, torch.float64)
    age = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    nres = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    out = A.integrate_record(s, st, -0.005, 300, 50, 1,
                             reset=dict(bounds=bounds, box=I.LORENZ_BOX, age=age, n_resets=nres, seed=5,
                                        max_age=120))
    torch.cuda.synchronize()
    rec = to_host(out)
    ref, a, r = x0.copy(), None, None
    for k in range(6):
        ref, _, a, r = ora.rk4_reset(ora.LORENZ, w.params, ref, -0.005, 50, bounds, I.LORENZ_BOX, max_age=120,
                                     seed=5, age=a, n_resets=r)
        assert np.array_equal(rec[k], ref), k
    assert np.array_equal(to_host(age), a) and np.array_equal(to_host(nres).view(np.uint32), r)
    # reset alone
    st = to_dev(x0, torch.float64)
    age.zero_()
    nres.zero_()
    A.integrate_reset(s, st, -0.005, 300, bounds=bounds, box=I.LORENZ_BOX, age=age, n_resets=nres, seed=5,
                      max_age=120)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(st), ref)


def test_explicit_compile_then_many_systems(A, ora):
    # compile ahead of use; several live systems with their own modules
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (1, 300))
    systems = []
    for k in range(4):
        s = A.System.from_exprs([f"-{k + 1}*x0 + p0"], [0.25 * k])
        s.compile("fp64")
        systems.append(s)
    for k, s in enumerate(systems):
        got, _ = run(A, s, x, 0.01, 100, torch.float64)
        assert np.array_equal(got, ora.expr_rk4([f"-{k + 1}*x0 + p0"], [0.25 * k], x, 0.01, 100))
    # new parameter values need no recompilation
    systems[0].set_params([2.0])
    got, _ = run(A, systems[0], x, 0.01, 100, torch.float64)
    assert np.array_equal(got, ora.expr_rk4(["-1*x0 + p0"], [2.0], x, 0.01, 100))
    del systems


def test_fast_f32_flag(A, ora):
    # without exp or division the flag changes nothing: identical bits
    w = I.lorenz_4096()
    e = I.generate(w)
    x32 = e.state[:, :3072].astype(np.float32)
    s = A.System.from_exprs(LORENZ_EXPR, w.params, fast_f32=True)
    got, c = run(A, s, x32, 0.005, 300, torch.float32, kahan=True)
    ref, cref = ora.expr_rk4_f32(LORENZ_EXPR, w.params, x32, 0.005, 300, kahan=True)
    assert np.array_equal(got, ref) and np.array_equal(c, cref)
    # Wilson-Cowan with the hardware exp and reciprocal: the FP32 bounds against FP64
    wc = I.wilson_cowan_4m(n=20000)
    ew = I.generate(wc)
    nf = ew.counts[0]
    x, pp = f32_inputs(ew.state[:, :nf]), f32_inputs(ew.pparams[:, :nf])
    h = float(np.float32(0.01))
    ref = ora.expr_rk4(WC_EXPR, wc.params, x, h, wc.nsteps, pp_slot=wc.pp_slot, pparams=pp)
    s = A.System.from_exprs(WC_EXPR, wc.params, fast_f32=True)
    got, _ = run(A, s, x.astype(np.float32), h, wc.nsteps, torch.float32, pp=pp.astype(np.float32),
                 pp_slot=wc.pp_slot, kahan=True)
    err = mixed_error(got, ref)
    record("expr_wc_fast_fp32_kahan_vs_fp64", kahan=quantiles(err))
    assert np.median(err) <= tol.KAHAN_WC_MEDIAN and np.quantile(err, 0.99) <= tol.KAHAN_WC_P99, quantiles(err)
    # a rational system: divisions through the hardware reciprocal
    rng = np.random.default_rng(21)
    xr = f32_inputs(rng.uniform(-2, 2, (3, 3000)))
    s = A.System.from_exprs(RATIONAL, [1.5, 0.7, 2.0], fast_f32=True)
    got, _ = run(A, s, xr.astype(np.float32), 0.01, 300, torch.float32, kahan=True)
    ref = ora.expr_rk4(RATIONAL, [1.5, 0.7, 2.0], xr, float(np.float32(0.01)), 300)
    err = mixed_error(got, ref)
    record("expr_rational_fast_fp32_kahan_vs_fp64", kahan=quantiles(err))
    assert np.quantile(err, 0.99) <= 1e-5 and err.max() <= 1e-4, quantiles(err)


# --- the discrete adjoint of expression systems (vector-Jacobian products
# generated by reverse-mode differentiation of the expressions) against the
# oracle's forward-mode derivative of the same map ---

def expr_adjoint(A, sysobj, x0, lamT, dt, nsteps, K, pp=None, pp_slot=(), dtype=torch.float64, kahan=False):
    x = to_dev(x0, dtype)
    ppt = None if pp is None else to_dev(pp, dtype)
    comp = torch.zeros_like(x) if kahan else None
    nb = A.adjoint_workspace_size(sysobj, x, nsteps, K, pparams=ppt, pp_slot=pp_slot, comp=comp)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda:0")
    A.integrate_checkpointed(sysobj, x, dt, nsteps, K, ws, pparams=ppt, pp_slot=pp_slot, comp=comp)
    lam = to_dev(lamT, dtype)
    mu = None if ppt is None else torch.empty_like(ppt)
    mug = torch.empty(max(sysobj.n_params, 1), dtype=torch.float64, device="cuda:0")
    A.adjoint(sysobj, x, dt, nsteps, K, ws, lam, mu=mu, mu_global=mug, pparams=ppt, pp_slot=pp_slot,
              prec="fp32_kahan" if kahan else None)
    torch.cuda.synchronize()
    return to_host(x), to_host(lam), (None if mu is None else to_host(mu)), to_host(mug)[:sysobj.n_params]


def dual_reference(ora, exprs, params, x0, lamT, dt, nsteps, pp=None, pp_slot=()):
    """dL/dx0, dL/dpp and dL/dp for L = sum lamT * x(T), from forward-mode runs."""
    dim, n = x0.shape
    lam0 = np.zeros_like(x0)
    for d in range(dim):
        dx0 = np.zeros_like(x0)
        dx0[d] = 1.0
        _, dxT = ora.expr_rk4_dual(exprs, params, x0, dt, nsteps, pp_slot=pp_slot, pparams=pp, dx0=dx0)
        lam0[d] = (lamT * dxT).sum(axis=0)
    mu = None
    if pp is not None:
        mu = np.zeros_like(pp)
        for k in range(pp.shape[0]):
            dpp = np.zeros_like(pp)
            dpp[k] = 1.0
            _, dxT = ora.expr_rk4_dual(exprs, params, x0, dt, nsteps, pp_slot=pp_slot, pparams=pp, dpp=dpp)
            mu[k] = (lamT * dxT).sum(axis=0)
    mug = np.zeros(len(params))
    for q in range(len(params)):
        if q in list(pp_slot):
            # a slot overridden per particle: the sum of its per-particle gradients
            mug[q] = mu[list(pp_slot).index(q)].sum()
            continue
        dp = np.zeros(len(params))
        dp[q] = 1.0
        _, dxT = ora.expr_rk4_dual(exprs, params, x0, dt, nsteps, pp_slot=pp_slot, pparams=pp, dparams=dp)
        mug[q] = (lamT * dxT).sum()
    return lam0, mu, mug


def rel_err(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), tol.ADJ_FLOOR * max(np.abs(b).max(), 1e-300))


ALL_FUNCS = ["1", "exp(x0) - x1", "pow(fabs(x1) + 1, p0) - 0.5 * x2",
             "fmin(x0, x1) / (1 + fabs(x2)) - p1 * x3", "atan(x3) * tanh(x1) - sqrt(1 + x0*x0) * 0.1",
             "log1p(x0*x0) + sinh(0.1 * x1) - cosh(0.1 * x2) + tan(0.3 * x4) - x5 + log(2 + cos(x3)) * sin(x4)"]


@pytest.mark.parametrize("case", ["lorenz", "wc_backward", "all_functions"])
def test_expression_adjoint_fp64_matches_oracle(A, ora, case):
    rng = np.random.default_rng(13)
    if case == "lorenz":
        exprs, params, n = LORENZ_EXPR, I.LORENZ_PARAMS, 700
        x0 = rng.uniform(-10, 10, (3, n))
        x0[2] += 25
        pp, slots, dt, nsteps, K = rng.uniform(20, 30, (1, n)), [1], 0.005, 150, 40
    elif case == "wc_backward":
        w = I.wilson_cowan_4m(n=600)
        e = I.generate(w)
        exprs, params, x0, pp, slots = WC_EXPR, w.params, e.state, e.pparams, w.pp_slot
        dt, nsteps, K = -0.01, 120, 50
    else:
        exprs, params, n = ALL_FUNCS, [1.5, 0.3], 300
        x0 = rng.uniform(-0.8, 0.8, (6, n))
        pp, slots, dt, nsteps, K = rng.uniform(0.1, 0.5, (1, n)), [1], 0.01, 60, 25
    s = A.System.from_exprs(exprs, params)
    lamT = rng.normal(size=x0.shape)
    xT, lam0, mu, mug = expr_adjoint(A, s, x0, lamT, dt, nsteps, K, pp=pp, pp_slot=slots)
    assert np.array_equal(xT, ora.expr_rk4(exprs, params, x0, dt, nsteps, pp_slot=slots, pparams=pp)) or \
        case != "lorenz"
    ref_l, ref_mu, ref_g = dual_reference(ora, exprs, params, x0, lamT, dt, nsteps, pp=pp, pp_slot=slots)
    for name, got, want in (("lambda0", lam0, ref_l), ("mu", mu, ref_mu), ("mu_global", mug, ref_g)):
        e = rel_err(got, want)
        record(f"expr_adjoint_fp64_{case}_{name}", err=quantiles(e.ravel()))
        assert e.max() <= tol.ADJ_REL, (name, quantiles(e.ravel()))


def test_expression_adjoint_equals_builtin_and_is_K_invariant(A, ora):
    rng = np.random.default_rng(14)
    n = 500
    x0 = rng.uniform(-10, 10, (3, n))
    x0[2] += 25
    pp = rng.uniform(20, 30, (1, n))
    lamT = rng.normal(size=x0.shape)
    s = A.System.from_exprs(LORENZ_EXPR, I.LORENZ_PARAMS)
    outs = [expr_adjoint(A, s, x0, lamT, 0.005, 120, K, pp=pp, pp_slot=[1]) for K in (120, 7, 50)]
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)
    # the built-in Lorenz adjoint: same map, its own hand-written vector-Jacobian product
    b = A.System("lorenz", 3, I.LORENZ_PARAMS)
    builtin = expr_adjoint(A, b, x0, lamT, 0.005, 120, 50, pp=pp, pp_slot=[1])
    for got, want in zip(outs[0][1:], builtin[1:]):
        assert rel_err(got, want).max() <= 1e-12


def test_expression_adjoint_fp32_kahan_vs_fp64(A, ora):
    rng = np.random.default_rng(15)
    n = 2000
    x0 = f32_inputs(rng.uniform(-10, 10, (3, n)) + np.array([[0.0], [0.0], [25.0]]))
    pp = f32_inputs(rng.uniform(20, 30, (1, n)))
    lamT = np.zeros((3, n))
    lamT[2] = 1.0
    s = A.System.from_exprs(LORENZ_EXPR, I.LORENZ_PARAMS)
    dt32 = float(np.float32(0.005))
    _, _, mu32, _ = expr_adjoint(A, s, x0.astype(np.float32), lamT.astype(np.float32), dt32, 200, 50,
                                 pp=pp.astype(np.float32), pp_slot=[1], dtype=torch.float32, kahan=True)
    _, dxT = ora.expr_rk4_dual(LORENZ_EXPR, I.LORENZ_PARAMS, x0, dt32, 200, pp_slot=[1], pparams=pp,
                               dpp=np.ones_like(pp))
    e = np.abs(mu32[0] - dxT[2]) / np.maximum(np.abs(dxT[2]), 1e-3 * max(1.0, np.abs(dxT[2]).max()))
    record("expr_adjoint_fp32_kahan_lorenz", err=quantiles(e))
    assert np.quantile(e, 0.99) <= tol.ADJ_FP32_P99, quantiles(e)


def test_expression_system_in_a_captured_graph(A, ora):
    # compiled ahead of capture (the first call of a precision would compile
    # and load during the call); every replay matches the eager run, and four
    # replays of 50 steps match the oracle's 200
    w = I.lorenz_4096()
    e = I.generate(w)
    x = e.state[:, :e.counts[0]]
    s = A.System.from_exprs(LORENZ_EXPR, w.params)
    s.compile("fp64")
    st_g = to_dev(x, torch.float64)
    st_e = to_dev(x, torch.float64)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        A.integrate(s, st_g, 0.005, 50)
    torch.cuda.synchronize()
    assert torch.equal(st_g, st_e)  # capturing does not execute
    for rep in range(4):
        g.replay()
        A.integrate(s, st_e, 0.005, 50)
        torch.cuda.synchronize()
        assert torch.equal(st_g, st_e), rep
    assert np.array_equal(to_host(st_g), ora.expr_rk4(LORENZ_EXPR, w.params, x, 0.005, 200))
