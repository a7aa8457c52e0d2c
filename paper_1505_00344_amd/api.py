"""Python binding of libfireflies.so with the C ABI's names.

Only argument marshalling happens here: torch tensors provide device memory
and the current stream; every step of the computation runs in the HIP
kernels behind the C ABI.  State tensors are structure-of-arrays with shape
``(dim, ld)`` (``ld`` >= the particle count ``n``), per-particle parameters
``(n_pp, ld)``; float32 or float64 on a CUDA (HIP) device.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _ffi
from ._ffi import (FF_FP32, FF_FP32_KAHAN, FF_FP64, FF_RHS_EXPR, FF_RHS_HH_RING, FF_RHS_LINEAR,
                   FF_RHS_LORENZ, FF_RHS_WILSON_COWAN, Batch, Group, Tuning, call)

RHS = {"linear": FF_RHS_LINEAR, "lorenz": FF_RHS_LORENZ, "wilson_cowan": FF_RHS_WILSON_COWAN,
       "hh_ring": FF_RHS_HH_RING}
PREC = {"fp32": FF_FP32, "fp32_kahan": FF_FP32_KAHAN, "fp64": FF_FP64}


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream if hasattr(s, "cuda_stream") else int(s)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _check_out(t: torch.Tensor, name: str, shape, dtypes, min_numel: bool = False) -> None:
    """A tensor the library writes: its dtype, contiguity and shape (or, with
    min_numel, at least that many elements) must match what the call writes."""
    if t.dtype not in dtypes or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {' or '.join(map(str, dtypes))} tensor")
    if min_numel:
        if t.numel() < shape:
            raise ValueError(f"{name} needs at least {shape} elements")
    elif tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, not {tuple(t.shape)}")


def _check_gpu(like: Optional[torch.Tensor], **tensors) -> None:
    """Every tensor whose memory the library reads or writes must live on a GPU
    (the one of the state, ``like``): a host pointer would reach a kernel."""
    for name, t in tensors.items():
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError(f"{name} must be a GPU tensor, not on {t.device}")
        if like is not None and t.device != like.device:
            raise ValueError(f"{name} is on {t.device} but the state is on {like.device}")


class System:
    """An ODE system handle (ff_system_create)."""

    def __init__(self, rhs, dim: int, params: Sequence[float]):
        self.rhs = RHS[rhs] if isinstance(rhs, str) else int(rhs)
        self.dim = int(dim)
        p = (ctypes.c_double * len(params))(*map(float, params))
        h = ctypes.c_void_p()
        call("ff_system_create", self.rhs, self.dim, len(params), p, ctypes.byref(h))
        self.handle = h
        self.n_params = len(params)

    @classmethod
    def from_exprs(cls, exprs: Sequence[str], params: Sequence[float] = (), fast_f32: bool = False) -> "System":
        """A system whose right-hand side is given as text (ff_system_create_expr):
        ``exprs[d]`` is x_d' over ``x0..`` and ``p0..``; ``fast_f32`` selects the
        hardware exp and reciprocal in single precision."""
        self = cls.__new__(cls)
        arr = (ctypes.c_char_p * len(exprs))(*[e.encode() for e in exprs])
        p = (ctypes.c_double * max(len(params), 1))(*map(float, params))
        h = ctypes.c_void_p()
        call("ff_system_create_expr", len(exprs), arr, len(params), p, _ffi.FF_EXPR_FAST_F32 if fast_f32 else 0,
             ctypes.byref(h))
        self.handle = h
        self.rhs = FF_RHS_EXPR
        self.dim = len(exprs)
        self.n_params = len(params)
        self.exprs = list(exprs)
        return self

    def compile(self, prec: str = "fp64", arch: Optional[str] = None) -> None:
        """Compile (and, without ``arch``, load) the kernels of one precision."""
        call("ff_system_compile", self.handle, PREC[prec], None if arch is None else arch.encode())

    def source(self, prec: str = "fp64") -> str:
        """The generated kernel source of an expression system."""
        n = ctypes.c_size_t()
        call("ff_system_source", self.handle, PREC[prec], None, 0, ctypes.byref(n))
        buf = ctypes.create_string_buffer(n.value)
        call("ff_system_source", self.handle, PREC[prec], buf, n.value, ctypes.byref(n))
        return buf.value.decode()

    def set_params(self, params: Sequence[float]) -> None:
        p = (ctypes.c_double * len(params))(*map(float, params))
        call("ff_system_set_params", self.handle, p, len(params))

    def get_params(self):
        p = (ctypes.c_double * self.n_params)()
        call("ff_system_get_params", self.handle, p, self.n_params)
        return list(p)

    def __del__(self):
        h = getattr(self, "handle", None)
        L = getattr(_ffi, "_lib", None) if _ffi is not None else None
        if h is not None and L is not None:
            L.ff_system_destroy(h)
            self.handle = None


def make_batch(state: torch.Tensor, n: Optional[int] = None, pparams: Optional[torch.Tensor] = None,
               pp_slot: Sequence[int] = (), comp: Optional[torch.Tensor] = None,
               prec: Optional[str] = None, offset: int = 0) -> Batch:
    """Describe a particle slice for the C ABI (no copies): particles
    ``offset .. offset + n - 1`` of the (dim, ld) arrays."""
    _check_gpu(None, state=state)
    _check_gpu(state, pparams=pparams, comp=comp)
    if state.dim() != 2:
        raise ValueError("state must have shape (dim, ld)")
    if not state.is_contiguous():
        raise ValueError("state must be contiguous")
    ld = state.shape[1]
    offset = int(offset)
    n = ld - offset if n is None else int(n)
    if offset < 0 or n < 0 or offset + n > ld:
        raise ValueError("slice outside the arrays")
    if prec is None:
        if state.dtype == torch.float64:
            prec = "fp64"
        elif state.dtype == torch.float32:
            prec = "fp32_kahan" if comp is not None else "fp32"
        else:
            raise ValueError("state must be float32 or float64")
    pc = PREC[prec]
    want = torch.float64 if pc == FF_FP64 else torch.float32
    for name, t in (("state", state), ("pparams", pparams), ("comp", comp)):
        if t is not None and (t.dtype != want or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {want} tensor")
    b = Batch()
    b.prec = pc
    esz = state.element_size()
    b.state = state.data_ptr() + offset * esz
    b.n = n
    b.ld = ld
    slots = list(pp_slot)
    if pparams is not None:
        if pparams.dim() != 2 or pparams.shape[1] != ld or pparams.shape[0] != len(slots):
            raise ValueError("pparams must have shape (len(pp_slot), ld)")
        b.pparams = pparams.data_ptr() + offset * esz
    elif slots:
        raise ValueError("pp_slot given without pparams")
    b.n_pp = len(slots)
    for k, s in enumerate(slots):
        b.pp_slot[k] = int(s)
    if comp is not None:
        if comp.shape != state.shape:
            raise ValueError("comp must have the shape of state")
        b.comp = comp.data_ptr() + offset * esz
    b._keep = (state, pparams, comp)  # the tensors behind the pointers live as long as the batch
    return b


def make_tuning(tuning) -> Optional[Tuning]:
    if tuning is None:
        return None
    if isinstance(tuning, Tuning):
        return tuning
    s, ppt, blk = tuning
    return Tuning(int(s), int(ppt), int(blk))


def integrate(sys: System, state: torch.Tensor, dt: float, nsteps: int, *, n=None, pparams=None,
              pp_slot=(), comp=None, prec=None, tuning=None, stream=None, offset=0) -> None:
    """ff_integrate: advance ``state`` in place by ``nsteps`` RK4 steps."""
    b = make_batch(state, n, pparams, pp_slot, comp, prec, offset)
    t = make_tuning(tuning)
    call("ff_integrate", sys.handle, ctypes.byref(b), float(dt), int(nsteps),
         ctypes.byref(t) if t is not None else None, _stream(stream))


def make_reset(bounds, box, age: torch.Tensor, n_resets: torch.Tensor, n: int, max_age: int = -1, seed: int = 0,
               id_offset: int = 0, offset: int = 0):
    """Describe the reset rule for the C ABI (host arrays are kept alive on
    the returned object)."""
    d = len(bounds)
    arr = lambda v: (ctypes.c_double * d)(*map(float, v))
    r = _ffi.Reset()
    r.bound_lo = arr([x[0] for x in bounds])
    r.bound_hi = arr([x[1] for x in bounds])
    r.box_lo = arr([x[0] for x in box])
    r.box_hi = arr([x[1] for x in box])
    r.max_age = int(max_age)
    r.seed = int(seed)
    r.id_offset = int(id_offset)
    for name, t in (("age", age), ("n_resets", n_resets)):
        if t.dtype != torch.int32 or not t.is_contiguous() or t.numel() < offset + int(n):
            raise ValueError(f"{name} must be a contiguous int32 tensor covering the particles")
    _check_gpu(None, age=age, n_resets=n_resets)
    r.age = age.data_ptr() + 4 * int(offset)
    r.n_resets = n_resets.data_ptr() + 4 * int(offset)
    return r


def integrate_reset(sys: System, state: torch.Tensor, dt: float, nsteps: int, *, bounds, box, age: torch.Tensor,
                    n_resets: torch.Tensor, max_age: int = -1, seed: int = 0, id_offset: int = 0, n=None,
                    pparams=None, pp_slot=(), comp=None, prec=None, tuning=None, stream=None, offset=0) -> None:
    """ff_integrate_reset: RK4 with the reset rule.  bounds/box: (lo, hi) per
    state component; age (int32) and n_resets (int32 storage of uint32
    counts) are device tensors indexed like the particles of the slice
    (``offset`` applies to them too)."""
    b = make_batch(state, n, pparams, pp_slot, comp, prec, offset)
    r = make_reset(bounds, box, age, n_resets, b.n, max_age, seed, id_offset, offset)
    t = make_tuning(tuning)
    call("ff_integrate_reset", sys.handle, ctypes.byref(b), float(dt), int(nsteps), ctypes.byref(r),
         ctypes.byref(t) if t is not None else None, _stream(stream))


def integrate_record(sys: System, state: torch.Tensor, dt: float, nsteps: int, every: int, stride: int = 1, *,
                     out: Optional[torch.Tensor] = None, reset: Optional[dict] = None, n=None, pparams=None,
                     pp_slot=(), comp=None, prec=None, tuning=None, stream=None, offset=0) -> torch.Tensor:
    """ff_integrate_record: returns out of shape (nsteps // every, dim,
    ceil(n / stride)); ``reset`` (optional) holds make_reset's keywords."""
    b = make_batch(state, n, pparams, pp_slot, comp, prec, offset)
    m = (b.n + stride - 1) // stride if stride >= 1 else 0
    shape = (int(nsteps) // int(every) if every >= 1 else 0, state.shape[0], m)
    if out is None:
        out = torch.empty(shape, dtype=state.dtype, device=state.device)
    elif tuple(out.shape) != shape or out.dtype != state.dtype or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous {state.dtype} tensor of shape {shape}")
    _check_gpu(state, out=out)
    r = None if reset is None else make_reset(n=b.n, offset=offset, **reset)
    t = make_tuning(tuning)
    call("ff_integrate_record", sys.handle, ctypes.byref(b), float(dt), int(nsteps), int(every), int(stride),
         out.data_ptr() if out.numel() else None, ctypes.byref(r) if r is not None else None,
         ctypes.byref(t) if t is not None else None, _stream(stream))
    return out


def histogram_workspace_size(n: int, nx: int, ny: int) -> int:
    out = ctypes.c_size_t()
    call("ff_histogram_workspace_size", int(n), int(nx), int(ny), ctypes.byref(out))
    return out.value


def project_histogram(sys: System, state: torch.Tensor, axis_x: int, axis_y: int, x_range, y_range,
                      nx: int, ny: int, *, hist: Optional[torch.Tensor] = None,
                      n_dropped: Optional[torch.Tensor] = None, accumulate: bool = False, n=None,
                      pparams=None, pp_slot=(), prec=None, workspace: Optional[torch.Tensor] = None,
                      stream=None, offset=0):
    """ff_project_histogram: returns (hist uint32 (ny, nx) as int32 view, n_dropped)."""
    b = make_batch(state, n, pparams, pp_slot, None, prec if prec != "fp32_kahan" else "fp32", offset)
    dev = state.device
    if hist is None:
        hist = torch.empty((ny, nx), dtype=torch.int32, device=dev)
    if n_dropped is None:
        n_dropped = torch.empty(1, dtype=torch.int64, device=dev)
    _check_out(hist, "hist", (ny, nx), (torch.int32,))
    _check_out(n_dropped, "n_dropped", 1, (torch.int64,), min_numel=True)
    _check_gpu(state, hist=hist, n_dropped=n_dropped, workspace=workspace)
    ws_ptr, ws_bytes = (None, 0) if workspace is None else (workspace.data_ptr(), workspace.numel() * workspace.element_size())
    call("ff_project_histogram", sys.handle, ctypes.byref(b), int(axis_x), int(axis_y),
         float(x_range[0]), float(x_range[1]), float(y_range[0]), float(y_range[1]), int(nx), int(ny),
         hist.data_ptr(), n_dropped.data_ptr(), int(bool(accumulate)), ws_ptr, ws_bytes, _stream(stream))
    return hist, n_dropped


def project_histogram_noalloc(sys: System, state: torch.Tensor, axis_x: int, axis_y: int, x_range, y_range,
                              nx: int, ny: int, *, hist: Optional[torch.Tensor] = None,
                              n_dropped: Optional[torch.Tensor] = None, accumulate: bool = False, n=None,
                              pparams=None, pp_slot=(), prec=None, stream=None, offset=0):
    """ff_project_histogram_noalloc: as project_histogram, with the library's
    static scratch instead of a workspace (hist and n_dropped must be passed
    in for a call that allocates nothing at all)."""
    b = make_batch(state, n, pparams, pp_slot, None, prec if prec != "fp32_kahan" else "fp32", offset)
    dev = state.device
    if hist is None:
        hist = torch.empty((ny, nx), dtype=torch.int32, device=dev)
    if n_dropped is None:
        n_dropped = torch.empty(1, dtype=torch.int64, device=dev)
    _check_out(hist, "hist", (ny, nx), (torch.int32,))
    _check_out(n_dropped, "n_dropped", 1, (torch.int64,), min_numel=True)
    _check_gpu(state, hist=hist, n_dropped=n_dropped)
    call("ff_project_histogram_noalloc", sys.handle, ctypes.byref(b), int(axis_x), int(axis_y),
         float(x_range[0]), float(x_range[1]), float(y_range[0]), float(y_range[1]), int(nx), int(ny),
         hist.data_ptr(), n_dropped.data_ptr(), int(bool(accumulate)), _stream(stream))
    return hist, n_dropped


def _render_desc(axis, mvp, width, height, base, grad, origin, weight, radius):
    r = _ffi.Render()
    for i in range(3):
        r.axis[i] = int(axis[i])
    m = [float(v) for row in mvp for v in row] if hasattr(mvp[0], "__len__") else [float(v) for v in mvp]
    for i in range(16):
        r.mvp[i] = m[i]
    r.width, r.height = int(width), int(height)
    g = [0.0] * 9 if grad is None else [float(v) for row in grad for v in row]
    for i in range(3):
        r.base[i] = float(base[i])
        r.origin[i] = float(origin[i])
    for i in range(9):
        r.grad[i] = g[i]
    r.weight = float(weight)
    r.radius = int(radius)
    return r


def render_workspace_size(n: int, width: int, height: int, radius: int = 0) -> int:
    """ff_render_workspace_size: scratch bytes of a render of n particles."""
    r = _render_desc((0, 0, 0), [0.0] * 16, width, height, (1.0, 1.0, 1.0), None, (0.0, 0.0, 0.0), 1.0, radius)
    out = ctypes.c_size_t()
    call("ff_render_workspace_size", int(n), ctypes.byref(r), ctypes.byref(out))
    return out.value


def render_image(sys: System, state: torch.Tensor, axis, mvp, width: int, height: int, *, base=(1.0, 1.0, 1.0),
                 grad=None, origin=(0.0, 0.0, 0.0), weight: float = 1.0, radius: int = 0,
                 img: Optional[torch.Tensor] = None, n_culled: Optional[torch.Tensor] = None,
                 accumulate: bool = False, n=None, pparams=None, pp_slot=(), prec=None, stream=None, offset=0,
                 workspace: Optional[torch.Tensor] = None):
    """ff_render_image: returns (img int32 view of uint32 [H, W, 3] with 8
    fractional bits, n_culled).  workspace: None (library-owned scratch) or a
    device uint8 tensor of at least render_workspace_size() bytes."""
    b = make_batch(state, n, pparams, pp_slot, None, prec if prec != "fp32_kahan" else "fp32", offset)
    r = _render_desc(axis, mvp, width, height, base, grad, origin, weight, radius)
    if img is None:
        img = torch.empty((int(height), int(width), 3), dtype=torch.int32, device=state.device)
    if n_culled is None:
        n_culled = torch.empty(1, dtype=torch.int64, device=state.device)
    _check_out(img, "img", (int(height), int(width), 3), (torch.int32,))
    _check_out(n_culled, "n_culled", 1, (torch.int64,), min_numel=True)
    _check_gpu(state, img=img, n_culled=n_culled, workspace=workspace)
    ws_ptr, ws_bytes = (None, 0) if workspace is None else (workspace.data_ptr(), workspace.numel() * workspace.element_size())
    call("ff_render_image", sys.handle, ctypes.byref(b), ctypes.byref(r), img.data_ptr(), n_culled.data_ptr(),
         int(bool(accumulate)), ws_ptr, ws_bytes, _stream(stream))
    return img, n_culled


def adjoint_workspace_size(sys: System, state: torch.Tensor, nsteps: int, K: int, *, n=None,
                           pparams=None, pp_slot=(), comp=None, prec=None) -> int:
    b = make_batch(state, n, pparams, pp_slot, comp, prec)
    out = ctypes.c_size_t()
    call("ff_adjoint_workspace_size", sys.handle, ctypes.byref(b), int(nsteps), int(K), ctypes.byref(out))
    return out.value


def integrate_checkpointed(sys: System, state: torch.Tensor, dt: float, nsteps: int, K: int,
                           workspace: torch.Tensor, *, n=None, pparams=None, pp_slot=(), comp=None,
                           prec=None, stream=None) -> None:
    b = make_batch(state, n, pparams, pp_slot, comp, prec)
    _check_gpu(state, workspace=workspace)
    call("ff_integrate_checkpointed", sys.handle, ctypes.byref(b), float(dt), int(nsteps), int(K),
         workspace.data_ptr(), workspace.numel() * workspace.element_size(), _stream(stream))


def adjoint(sys: System, state: torch.Tensor, dt: float, nsteps: int, K: int, workspace: torch.Tensor,
            lam: torch.Tensor, *, mu: Optional[torch.Tensor] = None,
            mu_global: Optional[torch.Tensor] = None, n=None, pparams=None, pp_slot=(), comp=None,
            prec=None, stream=None) -> None:
    """ff_adjoint: ``lam`` holds dL/dx(T) on entry and dL/dx(0) on exit."""
    b = make_batch(state, n, pparams, pp_slot, comp, prec)
    _check_out(lam, "lam", tuple(state.shape), (state.dtype,))
    if mu is not None:
        if pparams is None:
            raise ValueError("mu is given but the batch has no per-particle parameters")
        _check_out(mu, "mu", tuple(pparams.shape), (pparams.dtype,))
    if mu_global is not None:
        _check_out(mu_global, "mu_global", sys.n_params, (torch.float64,), min_numel=True)
    _check_gpu(state, workspace=workspace, lam=lam, mu=mu, mu_global=mu_global)
    call("ff_adjoint", sys.handle, ctypes.byref(b), float(dt), int(nsteps), int(K), workspace.data_ptr(),
         workspace.numel() * workspace.element_size(), lam.data_ptr(), _ptr(mu), _ptr(mu_global),
         _stream(stream))


def make_groups(specs) -> "ctypes.Array":
    """specs: iterable of (System, Batch, dt).  The array keeps the systems
    (whose handles it holds) and the batches' tensors alive."""
    specs = list(specs)
    arr = (Group * len(specs))()
    for g, (sys, b, dt) in zip(arr, specs):
        g.sys = sys.handle
        g.b = b
        g.dt_signed = float(dt)
    arr._keep = [(sys, getattr(b, "_keep", None)) for sys, b, _ in specs]
    return arr


def groups_workspace_size(n_groups: int) -> int:
    out = ctypes.c_size_t()
    call("ff_groups_workspace_size", int(n_groups), ctypes.byref(out))
    return out.value


def integrate_groups(groups, nsteps: int, *, tuning=None, workspace: Optional[torch.Tensor] = None,
                     stream=None) -> None:
    t = make_tuning(tuning)
    _check_gpu(None, workspace=workspace)
    ws_ptr, ws_bytes = (None, 0) if workspace is None else (workspace.data_ptr(), workspace.numel() * workspace.element_size())
    call("ff_integrate_groups", groups, len(groups), int(nsteps),
         ctypes.byref(t) if t is not None else None, ws_ptr, ws_bytes, _stream(stream))


def autotune(groups, nsteps: int, stream=None) -> Tuning:
    out = Tuning()
    call("ff_autotune", groups, len(groups), int(nsteps), ctypes.byref(out), _stream(stream))
    return out


MATH = {"exp": 0, "exp2": 1, "expm1": 2, "rcp": 3, "logistic": 4, "logistic2": 5, "psi": 6}


def math_eval(fn: str, x: torch.Tensor, *, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """ff_math_eval: the library's double-precision kernel ``fn`` (a key of
    MATH) applied elementwise to the float64 GPU tensor ``x``."""
    if x.dtype != torch.float64 or not x.is_contiguous():
        raise ValueError("x must be a contiguous float64 tensor")
    if out is None:
        out = torch.empty_like(x)
    _check_out(out, "out", tuple(x.shape), (torch.float64,))
    _check_gpu(x, x=x, out=out)
    call("ff_math_eval", MATH[fn], x.data_ptr(), out.data_ptr(), x.numel(), _stream(stream))
    return out
