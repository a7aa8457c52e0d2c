"""CPU checks of the library's expression systems (ff_system_create_expr,
ff_system_source, ff_system_compile with an explicit architecture): parsing
and its errors, the generated kernel source, and a gfx950 compilation that
needs no device.  The kernels themselves run in the GPU tests."""
import ctypes

import numpy as np
import pytest

from expr_cases import BAD, CONSTANTS, LORENZ_EXPR, QUAD_EXPRS, WC_EXPR


@pytest.fixture(scope="module")
def A():
    from paper_1505_00344_amd import api
    api._ffi.lib()
    return api


def test_info_and_params(A):
    s = A.System.from_exprs(LORENZ_EXPR, [10.0, 28.0, 8 / 3])
    rhs, dim, npar = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    A.call("ff_system_info", s.handle, ctypes.byref(rhs), ctypes.byref(dim), ctypes.byref(npar))
    assert (rhs.value, dim.value, npar.value) == (A._ffi.FF_RHS_EXPR, 3, 3)
    s.set_params([1.0, 2.0, 3.0])
    assert s.get_params() == [1.0, 2.0, 3.0]


@pytest.mark.parametrize("text", BAD)
def test_library_rejects_what_the_oracle_rejects(A, ora, text):
    with pytest.raises(ValueError):
        ora.expr_rk4([text, "x0", "x1"], [], np.zeros((3, 1)), 0.1, 1)
    with pytest.raises(A._ffi.FirefliesError, match="FF_E_INVALID.*column"):
        A.System.from_exprs([text, "x0", "x1"])


@pytest.mark.parametrize("text", [e for e, _ in CONSTANTS] + QUAD_EXPRS + LORENZ_EXPR)
def test_library_accepts_what_the_oracle_accepts(A, ora, text):
    ora.expr_rk4([text, "x0", "x1"], [1.0, 2.0, 3.0], np.zeros((3, 1)), 0.1, 1)
    A.System.from_exprs([text, "x0", "x1"], [1.0, 2.0, 3.0])


def test_error_names_variable_and_column(A):
    with pytest.raises(A._ffi.FirefliesError, match=r"x1, column 6: unknown name 'foo'"):
        A.System.from_exprs(["x0", "1 + (foo(x0))"])


@pytest.mark.parametrize("dim,npar,exprs,params", [
    (0, 0, [], []), (16, 0, ["1"] * 16, []), (1, 17, ["1"], [0.0] * 17)])
def test_size_limits(A, dim, npar, exprs, params):
    arr = (ctypes.c_char_p * max(len(exprs), 1))(*[e.encode() for e in exprs])
    p = (ctypes.c_double * max(len(params), 1))(*params)
    h = ctypes.c_void_p()
    assert A._ffi.lib().ff_system_create_expr(dim, arr, npar, p, 0, ctypes.byref(h)) == A._ffi.FF_E_INVALID


def test_unknown_flags_rejected(A):
    arr = (ctypes.c_char_p * 1)(b"x0")
    h = ctypes.c_void_p()
    assert A._ffi.lib().ff_system_create_expr(1, arr, 0, None, 2, ctypes.byref(h)) == A._ffi.FF_E_INVALID
    assert A._ffi.lib().ff_system_create_expr(1, arr, 0, None, 1, ctypes.byref(h)) == 0
    A._ffi.lib().ff_system_destroy(h)


def test_fast_f32_source(A):
    s = A.System.from_exprs(["exp(x0) / (1 + x1)", "x0 - x1"], fast_f32=True)
    f32 = s.source("fp32")
    assert "__builtin_amdgcn_exp2f(" in f32 and "__builtin_amdgcn_rcpf(" in f32 and "expf(" not in f32
    f64 = s.source("fp64")
    assert "exp(" in f64 and " / " in f64 and "amdgcn" not in f64
    s.compile("fp32_kahan", arch="gfx950")


def test_nesting_and_size_limits(A):
    with pytest.raises(A._ffi.FirefliesError, match="nested deeper"):
        A.System.from_exprs(["(" * 300 + "x0" + ")" * 300])
    A.System.from_exprs(["(" * 200 + "x0" + ")" * 200])
    big = " + ".join(f"{k}*x0" for k in range(3000))  # 6000 distinct operations
    with pytest.raises(A._ffi.FirefliesError, match="too large"):
        A.System.from_exprs([big])


def test_builtin_create_refuses_expr_kind(A):
    h = ctypes.c_void_p()
    p = (ctypes.c_double * 1)(0.0)
    assert A._ffi.lib().ff_system_create(A._ffi.FF_RHS_EXPR, 1, 0, p, ctypes.byref(h)) == A._ffi.FF_E_INVALID


def test_source_shares_subtrees_and_hoists_parameter_terms(A):
    s = A.System.from_exprs(["exp(p0*p1) * x0 + exp(p0*p1)", "sin(x0)*sin(x0) - p1"], [0.5, 2.0])
    src = s.source("fp64")
    # exp(p0*p1) is state-free: computed once per particle in derive()
    derive, rest = src.split("void f(")
    f, vjp = rest.split("void vjp(")
    assert derive.count("exp(") == 1 and "exp(" not in f
    # the vector-Jacobian product differentiates sin(x0)^2 through cos
    assert "cos(" in vjp and "gx[0]" in vjp and "gp[0]" in vjp and "gp[1]" in vjp
    # sin(x0) appears twice in the text and once in the code
    assert f.count("sin(") == 1
    assert "sinf(" in s.source("fp32") and "sinf(" in s.source("fp32_kahan")
    assert "ff::k_rk4" not in src  # instances are requested by name at compile time


def test_literals_are_exact(A):
    s = A.System.from_exprs(["0.1 * x0 + 1e999 - 5e-324"])
    src = s.source("fp64")
    assert "0x1.999999999999ap-4" in src and "__builtin_huge_val()" in src
    assert "0x0.0000000000001p-1022" in src or "0x1p-1074" in src
    assert "((float)(0x1.999999999999ap-4))" in s.source("fp32")


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_compiles_for_gfx950_without_a_device(A, prec):
    s = A.System.from_exprs(WC_EXPR, [1.0] * 10)
    s.compile(prec, arch="gfx950")
    q = A.System.from_exprs(["1"] + QUAD_EXPRS)
    q.compile(prec, arch="gfx950")


def test_groups_refuse_expression_systems_and_adjoint_layout(A):
    from paper_1505_00344_amd import _ffi
    L = _ffi.lib()
    s = A.System.from_exprs(LORENZ_EXPR, [10.0, 28.0, 8 / 3])
    b = _ffi.Batch()
    b.prec, b.state, b.n, b.ld = _ffi.FF_FP64, 4096, 10, 10
    g = A.make_groups([(s, b, 0.01)])
    assert L.ff_integrate_groups(g, 1, 10, None, None, 0, None) == _ffi.FF_E_UNSUPPORTED
    # the adjoint workspace of a small expression system is laid out like the
    # built-in system of the same size with a tape of eight steps (the
    # built-in Lorenz keeps four in double precision: one more sub-checkpoint
    # for a 10-step segment)
    builtin = A.System("lorenz", 3, [10.0, 28.0, 8 / 3])
    sz, sz2 = ctypes.c_size_t(), ctypes.c_size_t()
    b32 = _ffi.Batch()
    b32.prec, b32.state, b32.n, b32.ld = _ffi.FF_FP32, 4096, 10, 10
    assert L.ff_adjoint_workspace_size(s.handle, ctypes.byref(b32), 100, 10, ctypes.byref(sz)) == 0
    assert L.ff_adjoint_workspace_size(builtin.handle, ctypes.byref(b32), 100, 10, ctypes.byref(sz2)) == 0
    assert sz.value == sz2.value
    assert L.ff_adjoint_workspace_size(s.handle, ctypes.byref(b), 100, 10, ctypes.byref(sz)) == 0
    assert L.ff_adjoint_workspace_size(builtin.handle, ctypes.byref(b), 100, 10, ctypes.byref(sz2)) == 0
    sub = 10 * 3 * 8    # one sub-checkpoint of 10 particles x 3 doubles
    assert sz2.value - sz.value == (sub + 255) // 256 * 256


def test_noop_calls_compile_nothing(A):
    # n == 0, nsteps == 0 or dt == 0 return before any compilation or device use
    from paper_1505_00344_amd import _ffi
    L = _ffi.lib()
    s = A.System.from_exprs(LORENZ_EXPR, [10.0, 28.0, 8 / 3])
    b = _ffi.Batch()
    b.prec, b.state, b.n, b.ld = _ffi.FF_FP64, 4096, 10, 10
    assert L.ff_integrate(s.handle, ctypes.byref(b), 0.0, 100, None, None) == 0
    assert L.ff_integrate(s.handle, ctypes.byref(b), 0.01, 0, None, None) == 0


def test_make_reset_checks_tensor_sizes_and_device(A):
    import torch
    age = torch.zeros(10, dtype=torch.int32)
    nres = torch.zeros(10, dtype=torch.int32)
    box = [(-1.0, 1.0)] * 3
    with pytest.raises(ValueError, match="covering"):
        A.make_reset(box, box, age, nres, 5, offset=6)
    with pytest.raises(ValueError, match="covering"):
        A.make_reset(box, box, age.to(torch.int64), nres, 10)
    # right sizes, but host memory: refused before any pointer reaches a kernel
    with pytest.raises(ValueError, match="GPU tensor"):
        A.make_reset(box, box, age, nres, 10)


def test_host_tensors_are_refused_before_any_call(A):
    import torch
    s = A.System("lorenz", 3, [10.0, 28.0, 8 / 3])
    x = torch.zeros((3, 16), dtype=torch.float64)
    for call in (lambda: A.integrate(s, x, 0.01, 10),
                 lambda: A.project_histogram(s, x, 0, 1, (0.0, 1.0), (0.0, 1.0), 8, 8),
                 lambda: A.render_image(s, x, (0, 1, 2), [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]],
                                        8, 8),
                 lambda: A.integrate_record(s, x, 0.01, 10, 5),
                 lambda: A.adjoint_workspace_size(s, x, 10, 5)):
        with pytest.raises(ValueError, match="GPU tensor"):
            call()
