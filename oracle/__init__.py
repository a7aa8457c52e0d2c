"""CPU oracle for the Fireflies particle-RK4 hot path (arXiv:1505.00344).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library ``paper_1505_00344_amd`` and neither imports the
other.  Everything here is a thin numpy/ctypes wrapper around ``ffo.cpp``; see
``ffo.h`` for what each function computes and which passage of the paper it
follows.

Arrays are structure-of-arrays: ``state`` has shape ``(dim, n)`` (component d
of particle i is ``state[d, i]``), per-particle parameters have shape
``(n_pp, n)`` and replace global parameter ``pp_slot[k]``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# FFO_LIB points the wrapper at another build of ffo.cpp (the mutation test
# uses it to load deliberately broken copies and check that the pins fail).
LIB_PATH = os.environ.get("FFO_LIB") or os.path.join(HERE, "libffo.so")

LINEAR, LORENZ, WILSON_COWAN, HH_RING, RICCATI = 0, 1, 2, 3, 100

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_ip = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64 = ctypes.c_int64
_int = ctypes.c_int


def lib():
    """Load libffo.so (building it first if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        L.ffo_n_params.argtypes = [_int, _int]
        L.ffo_rhs.argtypes = [_int, _int, _dp, _int, _dp, _dp, _i64]
        L.ffo_jacobians.argtypes = [_int, _int, _dp, _int, _dp, _dp, _dp, _i64]
        L.ffo_rk4.argtypes = [_int, _int, _dp, _int, _ip, _int, _dp, _dp, _i64, _i64,
                              ctypes.c_double, _i64, _int]
        L.ffo_rk4_f32.argtypes = [_int, _int, _dp, _int, _ip, _int, _fp, _fp, _fp, _int,
                                  _i64, _i64, ctypes.c_float, _i64, _int]
        L.ffo_rk4_cstep.argtypes = [_int, _int, _dp, _int, _ip, _int, _dp, _dp, _dp, _dp,
                                    _dp, ctypes.c_double, _dp, _dp, _i64, _i64,
                                    ctypes.c_double, _i64, _int]
        L.ffo_adjoint.argtypes = [_int, _int, _dp, _int, _ip, _int, _dp, _dp, _dp, _dp,
                                  _dp, _i64, _i64, ctypes.c_double, _i64, _int]
        L.ffo_histogram.argtypes = [_int, _dp, _int, _dp, _i64, _i64, _int, _int,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, _int, _int, _u32p, _u64p, _int]
        _u32a = ctypes.POINTER(ctypes.c_uint32)
        _i32a = ctypes.POINTER(ctypes.c_int32)
        L.ffo_philox4x32_10.argtypes = [_u32a, _u32a, _u32a]
        L.ffo_rk4_reset.argtypes = [_int, _int, _dp, _int, _ip, _int, _dp, _dp, _i64, _i64,
                                    ctypes.c_double, _i64, _dp, _dp, _dp, _dp, _i64,
                                    ctypes.c_uint64, ctypes.c_uint64, _i32a, _u32a, _int]
        L.ffo_rk4_reset_f32.argtypes = [_int, _int, _dp, _int, _ip, _int, _fp, _fp, _fp, _int,
                                        _i64, _i64, ctypes.c_float, _i64, _dp, _dp, _dp, _dp,
                                        _i64, ctypes.c_uint64, ctypes.c_uint64, _i32a, _u32a,
                                        _int]
        L.ffo_render.argtypes = [_int, _dp, _int, _dp, _i64, _i64, ctypes.c_void_p, _u32p, _u64p,
                                 _int]
        _cpp = ctypes.POINTER(ctypes.c_char_p)
        L.ffo_expr_rk4.argtypes = [_int, _cpp, _dp, _int, _ip, _int, _dp, _dp, _i64, _i64,
                                   ctypes.c_double, _i64]
        L.ffo_expr_rk4_f32.argtypes = [_int, _cpp, _dp, _int, _ip, _int, _fp, _fp, _fp, _i64,
                                       _i64, ctypes.c_float, _i64]
        L.ffo_expr_rk4_dual.argtypes = [_int, _cpp, _dp, _int, _ip, _int, _dp, _dp, _dp, _dp, _dp,
                                        _dp, _dp, _i64, _i64, ctypes.c_double, _i64]
        L.ffo_expr_error.restype = ctypes.c_char_p
        for f in ("ffo_expr_rk4", "ffo_expr_rk4_f32", "ffo_expr_rk4_dual", "ffo_n_params", "ffo_rhs", "ffo_jacobians", "ffo_rk4", "ffo_rk4_f32", "ffo_render",
                  "ffo_rk4_cstep", "ffo_adjoint", "ffo_histogram", "ffo_philox4x32_10",
                  "ffo_rk4_reset", "ffo_rk4_reset_f32"):
            getattr(L, f).restype = _int
        _lib = L
    return _lib


def _ptr(a, typ):
    if a is None:
        return ctypes.cast(None, typ)
    return a.ctypes.data_as(typ)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what}: invalid arguments (code {rc})")


def n_params(sys: int, dim: int) -> int:
    return lib().ffo_n_params(sys, dim)


def _pp(pp_slot, pparams, n, conv):
    if pp_slot is None or len(pp_slot) == 0:
        return None, 0, None
    slots = np.ascontiguousarray(pp_slot, dtype=np.int32)
    pp = conv(pparams).reshape(len(slots), n)
    return slots, len(slots), pp


def rhs(sys, params, x):
    """f(x) at points x of shape (m, dim)."""
    x = _f64(np.atleast_2d(x))
    m, dim = x.shape
    p = _f64(params)
    f = np.empty_like(x)
    _check(lib().ffo_rhs(sys, dim, _ptr(p, _dp), len(p), _ptr(x, _dp), _ptr(f, _dp), m), "rhs")
    return f


def jacobians(sys, params, x):
    """(J, Fp) at points x of shape (m, dim): J (m, dim, dim), Fp (m, dim, n_params)."""
    x = _f64(np.atleast_2d(x))
    m, dim = x.shape
    p = _f64(params)
    J = np.empty((m, dim, dim))
    Fp = np.empty((m, dim, max(len(p), 1)))
    _check(lib().ffo_jacobians(sys, dim, _ptr(p, _dp), len(p), _ptr(x, _dp), _ptr(J, _dp),
                               _ptr(Fp, _dp), m), "jacobians")
    return J, Fp[:, :, :len(p)]


def rk4(sys, params, state, h, nsteps, pp_slot=None, pparams=None, nthreads=0):
    """FP64 classical RK4; returns the final state (a new (dim, n) array)."""
    st = _f64(state).copy()
    dim, n = st.shape
    p = _f64(params)
    slots, npp, pp = _pp(pp_slot, pparams, n, _f64)
    _check(lib().ffo_rk4(sys, dim, _ptr(p, _dp), len(p), _ptr(slots, _ip), npp, _ptr(pp, _dp),
                         _ptr(st, _dp), n, n, float(h), int(nsteps), nthreads), "rk4")
    return st


def rk4_f32(sys, params, state, h, nsteps, pp_slot=None, pparams=None, kahan=False,
            comp=None, nthreads=0):
    """Single-precision RK4 (params rounded to float); returns (state, comp)."""
    st = _f32(state).copy()
    dim, n = st.shape
    p = _f64(params)
    slots, npp, pp = _pp(pp_slot, pparams, n, _f32)
    c = None
    if kahan:
        c = np.zeros_like(st) if comp is None else _f32(comp).copy()
    _check(lib().ffo_rk4_f32(sys, dim, _ptr(p, _dp), len(p), _ptr(slots, _ip), npp,
                             _ptr(pp, _fp), _ptr(st, _fp), _ptr(c, _fp), int(bool(kahan)), n,
                             n, float(np.float32(h)), int(nsteps), nthreads), "rk4_f32")
    return st, c


def rk4_cstep(sys, params, x0, h, nsteps, pp_slot=None, pparams=None, dx0=None,
              dparams=None, dpp=None, eps=1e-30, nthreads=0):
    """Complex-step directional derivative of the FP64 map: returns (xT, dxT)."""
    x0 = _f64(x0)
    dim, n = x0.shape
    p = _f64(params)
    slots, npp, pp = _pp(pp_slot, pparams, n, _f64)
    dx0 = None if dx0 is None else _f64(dx0).reshape(dim, n)
    dparams = None if dparams is None else _f64(dparams)
    dpp = None if dpp is None else _f64(dpp).reshape(npp, n)
    xT = np.empty_like(x0)
    dxT = np.empty_like(x0)
    _check(lib().ffo_rk4_cstep(sys, dim, _ptr(p, _dp), len(p), _ptr(slots, _ip), npp,
                               _ptr(pp, _dp), _ptr(x0, _dp), _ptr(dx0, _dp), _ptr(dparams, _dp),
                               _ptr(dpp, _dp), float(eps), _ptr(xT, _dp), _ptr(dxT, _dp), n, n,
                               float(h), int(nsteps), nthreads), "rk4_cstep")
    return xT, dxT


def adjoint(sys, params, x0, lamT, h, nsteps, pp_slot=None, pparams=None, nthreads=0):
    """Exact gradient of the FP64 map.  Returns (lam0, mu_pp, mu_global)."""
    x0 = _f64(x0)
    dim, n = x0.shape
    p = _f64(params)
    slots, npp, pp = _pp(pp_slot, pparams, n, _f64)
    lam = _f64(lamT).reshape(dim, n).copy()
    mu_pp = np.zeros((npp, n)) if npp else None
    mu_g = np.zeros(len(p))
    _check(lib().ffo_adjoint(sys, dim, _ptr(p, _dp), len(p), _ptr(slots, _ip), npp,
                             _ptr(pp, _dp), _ptr(x0, _dp), _ptr(lam, _dp), _ptr(mu_pp, _dp),
                             _ptr(mu_g, _dp), n, n, float(h), int(nsteps), nthreads), "adjoint")
    return lam, mu_pp, mu_g


def histogram(state, axis_x, axis_y, x_range, y_range, nx, ny, pparams=None,
              hist=None, n_dropped=0):
    """2D density projection; returns (hist[ny, nx] uint32, n_dropped).

    Single-precision positions are converted exactly to double first.  Pass a
    previous ``hist`` and ``n_dropped`` to accumulate."""
    st = _f64(state)
    dim, n = st.shape
    pp = None if pparams is None else _f64(pparams).reshape(-1, n)
    npp = 0 if pp is None else pp.shape[0]
    acc = hist is not None
    h = np.zeros((ny, nx), dtype=np.uint32) if hist is None else np.array(hist, dtype=np.uint32)
    d = np.array([n_dropped], dtype=np.uint64)
    _check(lib().ffo_histogram(dim, _ptr(st, _dp), npp, _ptr(pp, _dp), n, n, axis_x, axis_y,
                               float(x_range[0]), float(x_range[1]), float(y_range[0]),
                               float(y_range[1]), nx, ny, _ptr(h, _u32p), _ptr(d, _u64p),
                               int(acc)), "histogram")
    return h, int(d[0])


def philox4x32_10(ctr, key):
    """Philox4x32-10 of counter ctr[4] under key key[2] (uint32 words)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    _check(lib().ffo_philox4x32_10(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(out, _u32p)), "philox")
    return out


def rk4_reset(sys, params, state, h, nsteps, bounds, box, max_age=-1, seed=0, id_offset=0,
              age=None, n_resets=None, pp_slot=None, pparams=None, prec="fp64", comp=None,
              nthreads=0):
    """RK4 with the reset rule; returns (state, comp, age, n_resets).

    bounds, box: sequences of (lo, hi) per state component.  prec: "fp64",
    "fp32" or "fp32_kahan" (state/pparams are then float32)."""
    f64 = prec == "fp64"
    st = (_f64(state) if f64 else _f32(state)).copy()
    dim, n = st.shape
    p = _f64(params)
    slots, npp, pp = _pp(pp_slot, pparams, n, _f64 if f64 else _f32)
    blo = _f64([b[0] for b in bounds])
    bhi = _f64([b[1] for b in bounds])
    xlo = _f64([b[0] for b in box])
    xhi = _f64([b[1] for b in box])
    a = np.zeros(n, dtype=np.int32) if age is None else np.array(age, dtype=np.int32)
    r = np.zeros(n, dtype=np.uint32) if n_resets is None else np.array(n_resets, dtype=np.uint32)
    _i32p = ctypes.POINTER(ctypes.c_int32)
    if f64:
        _check(lib().ffo_rk4_reset(sys, dim, _ptr(p, _dp), len(p), _ptr(slots, _ip), npp, _ptr(pp, _dp),
                                   _ptr(st, _dp), n, n, float(h), int(nsteps), _ptr(blo, _dp),
                                   _ptr(bhi, _dp), _ptr(xlo, _dp), _ptr(xhi, _dp), int(max_age),
                                   int(seed), int(id_offset), _ptr(a, _i32p), _ptr(r, _u32p),
                                   nthreads), "rk4_reset")
        return st, None, a, r
    kahan = prec == "fp32_kahan"
    c = None
    if kahan:
        c = np.zeros_like(st) if comp is None else _f32(comp).copy()
    _check(lib().ffo_rk4_reset_f32(sys, dim, _ptr(p, _dp), len(p), _ptr(slots, _ip), npp, _ptr(pp, _fp),
                                   _ptr(st, _fp), _ptr(c, _fp), int(kahan), n, n,
                                   float(np.float32(h)), int(nsteps), _ptr(blo, _dp), _ptr(bhi, _dp),
                                   _ptr(xlo, _dp), _ptr(xhi, _dp), int(max_age), int(seed),
                                   int(id_offset), _ptr(a, _i32p), _ptr(r, _u32p), nthreads),
           "rk4_reset_f32")
    return st, c, a, r


class RenderSpec(ctypes.Structure):
    _fields_ = [("axis", ctypes.c_int * 3), ("mvp", ctypes.c_double * 16), ("width", ctypes.c_int),
                ("height", ctypes.c_int), ("base", ctypes.c_double * 3), ("grad", ctypes.c_double * 9),
                ("origin", ctypes.c_double * 3), ("weight", ctypes.c_double), ("radius", ctypes.c_int)]


def render_spec(axis, mvp, width, height, base=(1.0, 1.0, 1.0), grad=None, origin=(0.0, 0.0, 0.0),
                weight=1.0, radius=0):
    r = RenderSpec()
    for i in range(3):
        r.axis[i] = int(axis[i])
    m = np.asarray(mvp, dtype=np.float64).reshape(16)
    for i in range(16):
        r.mvp[i] = float(m[i])
    r.width, r.height = int(width), int(height)
    g = np.zeros(9) if grad is None else np.asarray(grad, dtype=np.float64).reshape(9)
    for i in range(3):
        r.base[i] = float(base[i])
        r.origin[i] = float(origin[i])
    for i in range(9):
        r.grad[i] = float(g[i])
    r.weight = float(weight)
    r.radius = int(radius)
    return r


def render(state, spec, pparams=None, img=None, n_culled=0):
    """Particle image as fixed-point uint32 [H, W, 3]; returns (img, n_culled)."""
    st = _f64(state)
    dim, n = st.shape
    pp = None if pparams is None else _f64(pparams).reshape(-1, n)
    npp = 0 if pp is None else pp.shape[0]
    acc = img is not None
    im = np.zeros((spec.height, spec.width, 3), dtype=np.uint32) if img is None else np.array(img, dtype=np.uint32)
    d = np.array([n_culled], dtype=np.uint64)
    _check(lib().ffo_render(dim, _ptr(st, _dp), npp, _ptr(pp, _dp), n, n, ctypes.byref(spec),
                            _ptr(im, _u32p), _ptr(d, _u64p), int(acc)), "render")
    return im, int(d[0])


def _exprs(exprs):
    arr = (ctypes.c_char_p * len(exprs))(*[e.encode() for e in exprs])
    return ctypes.cast(arr, ctypes.POINTER(ctypes.c_char_p)), arr


def _expr_check(rc):
    if rc == -2:
        raise ValueError("oracle expr_rk4: " + lib().ffo_expr_error().decode())
    _check(rc, "expr_rk4")


def expr_rk4(exprs, params, state, h, nsteps, pp_slot=None, pparams=None):
    """FP64 RK4 of the system x_d' = exprs[d] (names x0.., p0..); returns the final state."""
    st = _f64(state).copy()
    dim, n = st.shape
    if len(exprs) != dim:
        raise ValueError("one expression per state variable")
    p = _f64(params)
    slots, npp, pp = _pp(pp_slot, pparams, n, _f64)
    ex, _keep = _exprs(exprs)
    _expr_check(lib().ffo_expr_rk4(dim, ex, _ptr(p, _dp), len(p), _ptr(slots, _ip), npp,
                                   _ptr(pp, _dp), _ptr(st, _dp), n, n, float(h), int(nsteps)))
    return st


def expr_rk4_f32(exprs, params, state, h, nsteps, pp_slot=None, pparams=None, kahan=False,
                 comp=None):
    """Single-precision form of :func:`expr_rk4` (params and literals rounded to
    float); returns (state, comp)."""
    st = _f32(state).copy()
    dim, n = st.shape
    if len(exprs) != dim:
        raise ValueError("one expression per state variable")
    p = _f64(params)
    slots, npp, pp = _pp(pp_slot, pparams, n, _f32)
    c = None
    if kahan:
        c = np.zeros_like(st) if comp is None else _f32(comp).copy()
    ex, _keep = _exprs(exprs)
    _expr_check(lib().ffo_expr_rk4_f32(dim, ex, _ptr(p, _dp), len(p), _ptr(slots, _ip), npp,
                                       _ptr(pp, _fp), _ptr(st, _fp), _ptr(c, _fp), n, n,
                                       float(np.float32(h)), int(nsteps)))
    return st, c


def expr_rk4_dual(exprs, params, x0, h, nsteps, pp_slot=None, pparams=None, dx0=None, dparams=None,
                  dpp=None):
    """FP64 expression map and its directional derivative: returns (xT, dxT)."""
    x0 = _f64(x0)
    dim, n = x0.shape
    if len(exprs) != dim:
        raise ValueError("one expression per state variable")
    p = _f64(params)
    slots, npp, pp = _pp(pp_slot, pparams, n, _f64)
    dx0 = None if dx0 is None else _f64(dx0).reshape(dim, n)
    dparams = None if dparams is None else _f64(dparams)
    dpp = None if dpp is None else _f64(dpp).reshape(npp, n)
    xT = np.empty_like(x0)
    dxT = np.empty_like(x0)
    ex, _keep = _exprs(exprs)
    _expr_check(lib().ffo_expr_rk4_dual(dim, ex, _ptr(p, _dp), len(p), _ptr(slots, _ip), npp,
                                        _ptr(pp, _dp), _ptr(x0, _dp), _ptr(dx0, _dp),
                                        _ptr(dparams, _dp), _ptr(dpp, _dp), _ptr(xT, _dp),
                                        _ptr(dxT, _dp), n, n, float(h), int(nsteps)))
    return xT, dxT
