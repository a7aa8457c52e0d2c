"""ctypes declarations of libfireflies.so (the C ABI of include/fireflies.h).

Argument marshalling only.  Loading fails loudly (RuntimeError) when the
library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# FF_LIB selects another build of the library (for A/B measurements).
LIB_PATH = os.environ.get("FF_LIB") or os.path.join(HERE, "libfireflies.so")

FF_OK, FF_E_INVALID, FF_E_UNSUPPORTED, FF_E_NOMEM, FF_E_DEVICE = range(5)
FF_FP32, FF_FP32_KAHAN, FF_FP64 = 0, 1, 2
FF_RHS_LINEAR, FF_RHS_LORENZ, FF_RHS_WILSON_COWAN, FF_RHS_HH_RING = 0, 1, 2, 3
FF_RHS_EXPR = 16
FF_EXPR_FAST_F32 = 1
FF_MAX_PP = 4
ABI_VERSION = 2

_c = ctypes
_vp = _c.c_void_p
_i32 = _c.c_int32
_i64 = _c.c_int64
_dbl = _c.c_double
_sz = _c.c_size_t


class Batch(_c.Structure):
    _fields_ = [("prec", _i32), ("state", _vp), ("n", _i64), ("ld", _i64),
                ("pparams", _vp), ("n_pp", _i32), ("pp_slot", _i32 * FF_MAX_PP),
                ("comp", _vp)]


class Tuning(_c.Structure):
    _fields_ = [("steps_per_launch", _i32), ("particles_per_thread", _i32), ("block", _i32)]


class Reset(_c.Structure):
    _fields_ = [("bound_lo", _c.POINTER(_dbl)), ("bound_hi", _c.POINTER(_dbl)), ("box_lo", _c.POINTER(_dbl)),
                ("box_hi", _c.POINTER(_dbl)), ("max_age", _i64), ("seed", _c.c_uint64), ("id_offset", _c.c_uint64),
                ("age", _vp), ("n_resets", _vp)]


class Render(_c.Structure):
    _fields_ = [("axis", _i32 * 3), ("mvp", _dbl * 16), ("width", _i32), ("height", _i32), ("base", _dbl * 3),
                ("grad", _dbl * 9), ("origin", _dbl * 3), ("weight", _dbl), ("radius", _i32)]


class Group(_c.Structure):
    _fields_ = [("sys", _vp), ("b", Batch), ("dt_signed", _dbl)]


# name -> (restype, argtypes); every exported symbol of include/fireflies.h
SIGNATURES = {
    "ff_abi_version": (_i32, []),
    "ff_last_error": (_c.c_char_p, []),
    "ff_system_create": (_i32, [_i32, _i32, _i32, _c.POINTER(_dbl), _c.POINTER(_vp)]),
    "ff_system_destroy": (_i32, [_vp]),
    "ff_system_set_params": (_i32, [_vp, _c.POINTER(_dbl), _i32]),
    "ff_system_get_params": (_i32, [_vp, _c.POINTER(_dbl), _i32]),
    "ff_system_info": (_i32, [_vp, _c.POINTER(_i32), _c.POINTER(_i32), _c.POINTER(_i32)]),
    "ff_system_create_expr": (_i32, [_i32, _c.POINTER(_c.c_char_p), _i32, _c.POINTER(_dbl), _c.c_uint32,
                                     _c.POINTER(_vp)]),
    "ff_system_compile": (_i32, [_vp, _i32, _c.c_char_p]),
    "ff_system_source": (_i32, [_vp, _i32, _c.c_char_p, _sz, _c.POINTER(_sz)]),
    "ff_integrate": (_i32, [_vp, _c.POINTER(Batch), _dbl, _i64, _c.POINTER(Tuning), _vp]),
    "ff_integrate_reset": (_i32, [_vp, _c.POINTER(Batch), _dbl, _i64, _c.POINTER(Reset), _c.POINTER(Tuning), _vp]),
    "ff_integrate_record": (_i32, [_vp, _c.POINTER(Batch), _dbl, _i64, _i64, _i64, _vp, _c.POINTER(Reset),
                                   _c.POINTER(Tuning), _vp]),
    "ff_render_workspace_size": (_i32, [_i64, _c.POINTER(Render), _c.POINTER(_sz)]),
    "ff_render_image": (_i32, [_vp, _c.POINTER(Batch), _c.POINTER(Render), _vp, _vp, _i32, _vp, _sz, _vp]),
    "ff_histogram_workspace_size": (_i32, [_i64, _i32, _i32, _c.POINTER(_sz)]),
    "ff_project_histogram": (_i32, [_vp, _c.POINTER(Batch), _i32, _i32, _dbl, _dbl, _dbl, _dbl,
                                    _i32, _i32, _vp, _vp, _i32, _vp, _sz, _vp]),
    "ff_project_histogram_noalloc": (_i32, [_vp, _c.POINTER(Batch), _i32, _i32, _dbl, _dbl, _dbl, _dbl,
                                            _i32, _i32, _vp, _vp, _i32, _vp]),
    "ff_adjoint_workspace_size": (_i32, [_vp, _c.POINTER(Batch), _i64, _i32, _c.POINTER(_sz)]),
    "ff_integrate_checkpointed": (_i32, [_vp, _c.POINTER(Batch), _dbl, _i64, _i32, _vp, _sz, _vp]),
    "ff_adjoint": (_i32, [_vp, _c.POINTER(Batch), _dbl, _i64, _i32, _vp, _sz, _vp, _vp, _vp, _vp]),
    "ff_groups_workspace_size": (_i32, [_i32, _c.POINTER(_sz)]),
    "ff_integrate_groups": (_i32, [_c.POINTER(Group), _i32, _i64, _c.POINTER(Tuning), _vp, _sz, _vp]),
    "ff_autotune": (_i32, [_c.POINTER(Group), _i32, _i64, _c.POINTER(Tuning), _vp]),
    "ff_math_eval": (_i32, [_i32, _vp, _vp, _i64, _vp]),
}

_lib = None


class FirefliesError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        names = {1: "FF_E_INVALID", 2: "FF_E_UNSUPPORTED", 3: "FF_E_NOMEM", 4: "FF_E_DEVICE"}
        super().__init__(f"{where}: {names.get(status, status)}: {msg}")
        self.status = status


def lib(required_symbols=None):
    """Load libfireflies.so and declare every signature it exports."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1505_00344_amd.build` "
                "(there is no CPU fallback)")
        L = _c.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        if L.ff_abi_version() != ABI_VERSION:
            raise RuntimeError("libfireflies.so ABI version mismatch")
        _lib = L
    return _lib


def call(name: str, *args) -> None:
    """Call an ff_* function and raise FirefliesError on a non-OK status."""
    L = lib()
    fn = getattr(L, name, None)
    if fn is None:
        raise RuntimeError(f"libfireflies.so does not export {name}")
    st = fn(*args)
    if st != FF_OK:
        raise FirefliesError(st, name, L.ff_last_error().decode(errors="replace"))
