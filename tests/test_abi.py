"""CPU checks of the C ABI: the library loads, exports every function that
include/fireflies.h declares, and validates arguments on the host (no GPU
needed: these calls fail before anything touches a device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fireflies.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ff_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_1505_00344_amd import _ffi
    return _ffi.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 16
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_1505_00344_amd import _ffi
    assert set(declared_functions()) == set(_ffi.SIGNATURES)


def test_abi_version(L):
    assert L.ff_abi_version() == 2


def test_system_create_validation(L):
    from paper_1505_00344_amd import _ffi
    h = ctypes.c_void_p()
    p = (ctypes.c_double * 16)(*range(16))
    cases = [
        (_ffi.FF_RHS_LORENZ, 3, 3, _ffi.FF_OK),
        (_ffi.FF_RHS_LORENZ, 4, 3, _ffi.FF_E_INVALID),
        (_ffi.FF_RHS_LORENZ, 3, 2, _ffi.FF_E_INVALID),
        (_ffi.FF_RHS_WILSON_COWAN, 2, 10, _ffi.FF_OK),
        (_ffi.FF_RHS_HH_RING, 15, 14, _ffi.FF_OK),
        (_ffi.FF_RHS_HH_RING, 5, 14, _ffi.FF_OK),
        (_ffi.FF_RHS_HH_RING, 10, 14, _ffi.FF_E_UNSUPPORTED),
        (_ffi.FF_RHS_LINEAR, 4, 16, _ffi.FF_OK),
        (_ffi.FF_RHS_LINEAR, 5, 25, _ffi.FF_E_INVALID),
        (9, 3, 3, _ffi.FF_E_INVALID),
    ]
    for rhs, dim, npar, want in cases:
        st = L.ff_system_create(rhs, dim, npar, p, ctypes.byref(h))
        assert st == want, (rhs, dim, npar, L.ff_last_error())
        if st == _ffi.FF_OK:
            assert h.value
            L.ff_system_destroy(h)
        else:
            assert L.ff_last_error()
    assert L.ff_system_create(_ffi.FF_RHS_LORENZ, 3, 3, None, ctypes.byref(h)) == _ffi.FF_E_INVALID


def test_params_roundtrip_and_info(L):
    from paper_1505_00344_amd import api as A
    s = A.System("wilson_cowan", 2, [16, 12, 15, 3, 1.3, 4, 2, 3.7, 0, 0])
    s.set_params([1.0] * 10)
    assert s.get_params() == [1.0] * 10
    rhs, dim, npar = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert L.ff_system_info(s.handle, ctypes.byref(rhs), ctypes.byref(dim), ctypes.byref(npar)) == 0
    assert (rhs.value, dim.value, npar.value) == (2, 2, 10)
    with pytest.raises(A._ffi.FirefliesError, match="FF_E_INVALID"):
        s.set_params([1.0] * 9)


def _batch(**kw):
    from paper_1505_00344_amd import _ffi
    b = _ffi.Batch()
    b.prec = kw.get("prec", _ffi.FF_FP64)
    b.state = kw.get("state", 4096)
    b.n = kw.get("n", 10)
    b.ld = kw.get("ld", 10)
    b.pparams = kw.get("pparams", None)
    b.n_pp = kw.get("n_pp", 0)
    for k, v in enumerate(kw.get("slots", [])):
        b.pp_slot[k] = v
    b.comp = kw.get("comp", None)
    return b


@pytest.mark.parametrize("kw,dt,nsteps", [
    (dict(ld=5), 0.01, 10),                       # ld < n
    (dict(n=-1), 0.01, 10),                       # n < 0
    (dict(prec=7), 0.01, 10),                     # bad precision
    (dict(n_pp=1, slots=[0]), 0.01, 10),          # pparams NULL
    (dict(n_pp=1, slots=[3], pparams=4096), 0.01, 10),   # slot out of range
    (dict(n_pp=2, slots=[1, 1], pparams=4096), 0.01, 10),  # repeated slot
    (dict(n_pp=5, pparams=4096), 0.01, 10),        # too many per-particle params
    (dict(prec=1), 0.01, 10),                     # Kahan without comp
    (dict(state=None), 0.01, 10),                 # NULL state
    (dict(), float("inf"), 10),                   # non-finite step
    (dict(), 0.01, -3),                           # negative steps
])
def test_integrate_rejects_bad_arguments_on_host(L, kw, dt, nsteps):
    from paper_1505_00344_amd import _ffi
    from paper_1505_00344_amd import api as A
    s = A.System("lorenz", 3, [10, 28, 8 / 3])
    b = _batch(**kw)
    st = L.ff_integrate(s.handle, ctypes.byref(b), dt, nsteps, None, None)
    assert st == _ffi.FF_E_INVALID, L.ff_last_error()
    assert L.ff_last_error()


def test_noops_touch_no_device(L):
    # n == 0, nsteps == 0 or dt == 0 return OK without launching (so they work
    # even on a machine without a GPU)
    from paper_1505_00344_amd import api as A
    s = A.System("lorenz", 3, [10, 28, 8 / 3])
    for b, dt, n in [(_batch(n=0), 0.01, 5), (_batch(), 0.0, 5), (_batch(), 0.01, 0)]:
        assert L.ff_integrate(s.handle, ctypes.byref(b), dt, n, None, None) == 0


def test_math_eval_validation_on_host(L):
    # rejected before any launch, so no device is needed; n == 0 launches nothing
    fake = ctypes.c_void_p(0x1000)
    assert L.ff_math_eval(7, fake, fake, 4, None) == 1
    assert L.ff_math_eval(-1, fake, fake, 4, None) == 1
    assert L.ff_math_eval(0, fake, fake, -1, None) == 1
    assert L.ff_math_eval(0, None, fake, 4, None) == 1
    assert L.ff_math_eval(6, fake, None, 4, None) == 1
    assert L.ff_math_eval(0, None, None, 0, None) == 0


def test_bad_tuning_rejected(L):
    from paper_1505_00344_amd import _ffi
    from paper_1505_00344_amd import api as A
    s = A.System("lorenz", 3, [10, 28, 8 / 3])
    b = _batch()
    for t in [(0, 1, 256), (10, 3, 256), (10, 1, 100), (10, 1, 512)]:
        tt = _ffi.Tuning(*t)
        assert L.ff_integrate(s.handle, ctypes.byref(b), 0.01, 5, ctypes.byref(tt), None) == _ffi.FF_E_INVALID


def test_histogram_and_adjoint_validation(L):
    from paper_1505_00344_amd import _ffi
    from paper_1505_00344_amd import api as A
    s = A.System("lorenz", 3, [10, 28, 8 / 3])
    b = _batch()
    sz = ctypes.c_size_t()
    assert L.ff_histogram_workspace_size(100, 1024, 1024, ctypes.byref(sz)) == 0 and sz.value > 0
    assert L.ff_histogram_workspace_size(100, 64, 64, ctypes.byref(sz)) == 0 and sz.value == 0
    bad = [(3, 0, 0.0, 1.0, 8), (0, -1, 0.0, 1.0, 8), (0, 1, 1.0, 1.0, 8), (0, 1, 0.0, 1.0, 0)]
    for ax, ay, lo, hi, nx in bad:
        st = L.ff_project_histogram(s.handle, ctypes.byref(b), ax, ay, lo, hi, 0.0, 1.0, nx, 8, 4096, None, 0,
                                    None, 0, None)
        assert st == _ffi.FF_E_INVALID
    # the allocation-free projection validates the same way, refuses a NULL grid, and refuses a projection
    # whose scratch would exceed its static buffer before touching a device
    for ax, ay, lo, hi, nx in bad:
        st = L.ff_project_histogram_noalloc(s.handle, ctypes.byref(b), ax, ay, lo, hi, 0.0, 1.0, nx, 8, 4096, None,
                                            0, None)
        assert st == _ffi.FF_E_INVALID
    assert L.ff_project_histogram_noalloc(s.handle, ctypes.byref(b), 0, 1, 0.0, 1.0, 0.0, 1.0, 8, 8, None, None, 0,
                                          None) == _ffi.FF_E_INVALID
    n = 12 * 1024 * 1024
    big = _batch(n=n, ld=n)
    assert L.ff_histogram_workspace_size(n, 1024, 1024, ctypes.byref(sz)) == 0 and sz.value > 64 * 1024 * 1024
    st = L.ff_project_histogram_noalloc(s.handle, ctypes.byref(big), 0, 2, -20.0, 20.0, 0.0, 50.0, 1024, 1024, 4096,
                                        None, 0, None)
    assert st == _ffi.FF_E_NOMEM and b"static" in L.ff_last_error()
    assert L.ff_adjoint_workspace_size(s.handle, ctypes.byref(b), 200, 50, ctypes.byref(sz)) == 0
    # 4 checkpoints + 7 sub-checkpoints of 3 x 10 doubles, + partial sums
    assert sz.value >= (4 + 7) * 3 * 10 * 8
    assert L.ff_adjoint_workspace_size(s.handle, ctypes.byref(b), 200, 0, ctypes.byref(sz)) == _ffi.FF_E_INVALID
    assert L.ff_integrate_checkpointed(s.handle, ctypes.byref(b), 0.01, 200, 50, None, 0, None) == _ffi.FF_E_NOMEM


def test_groups_validation(L):
    from paper_1505_00344_amd import _ffi
    from paper_1505_00344_amd import api as A
    s = A.System("lorenz", 3, [10, 28, 8 / 3])
    g = A.make_groups([(s, _batch(prec=_ffi.FF_FP64), 0.01), (s, _batch(prec=_ffi.FF_FP32), 0.01)])
    assert L.ff_integrate_groups(g, 2, 10, None, None, 0, None) == _ffi.FF_E_INVALID
    g = A.make_groups([(s, _batch(), float("nan"))])
    assert L.ff_integrate_groups(g, 1, 10, None, None, 0, None) == _ffi.FF_E_INVALID
    g = A.make_groups([(s, _batch(), 0.0)])
    assert L.ff_integrate_groups(g, 1, 10, None, None, 0, None) == 0  # nothing to do


def test_groups_keep_their_systems_alive(L):
    """The group array holds raw system handles: the System objects must live
    as long as the array, or a later call would use a destroyed handle."""
    import gc
    import weakref

    from paper_1505_00344_amd import api as A
    g = A.make_groups([(A.System("lorenz", 3, [10, 28, 8 / 3]), _batch(), 0.0)])
    ref = weakref.ref(g._keep[0][0])
    gc.collect()
    assert ref() is not None
    assert L.ff_integrate_groups(g, 1, 10, None, None, 0, None) == 0
    del g
    gc.collect()
    assert ref() is None


def test_autotune_reads_its_cache_file(tmp_path):
    """ff_autotune answers from the FF_AUTOTUNE_CACHE file when it holds the
    group list (a hit returns before any device call; malformed lines and
    invalid launch shapes are skipped).  Fresh process: the file is read once."""
    import subprocess
    import sys

    from paper_1505_00344_amd import _ffi
    key = f"50|{_ffi.FF_RHS_LORENZ},3,{_ffi.FF_FP64},10,0"
    cache = tmp_path / "tune.txt"
    cache.write_text("not a tuning line\n"
                     f"{key} 37 4 64\n"
                     f"7|9,9,9,9,9 20 2 100\n"   # block 100: invalid, skipped
                     f"{key} 37 3 64\n")         # 3 particles per thread: invalid, skipped (else it would win)
    code = (
        "import ctypes, sys\n"
        f"sys.path.insert(0, {os.path.join(ROOT, 'tests')!r})\n"
        "from test_abi import _batch\n"
        "from paper_1505_00344_amd import _ffi, api as A\n"
        "L = _ffi.lib()\n"
        "s = A.System('lorenz', 3, [10, 28, 8 / 3])\n"
        "g = A.make_groups([(s, _batch(), 0.01)])\n"
        "t = _ffi.Tuning()\n"
        "rc = L.ff_autotune(g, 1, 50, ctypes.byref(t), None)\n"
        "print(rc, t.steps_per_launch, t.particles_per_thread, t.block)\n")
    env = dict(os.environ, FF_AUTOTUNE_CACHE=str(cache), PYTHONPATH=ROOT)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["0", "37", "4", "64"]


def test_render_workspace_size_selects_the_path(L):
    from paper_1505_00344_amd import api as A
    size = A.render_workspace_size
    assert size(0, 1920, 1080, 2) == 0
    assert size(1000, 1920, 1080, 2) > 0           # tiled: sprites of radius <= 8
    assert size(1000, 1920, 1080, 8) > 0
    assert size(1000, 1920, 1080, 9) == 0          # larger sprites: one thread per particle
    assert size(1000, 3840, 2160, 1) > 0           # 4080 tiles of 64 x 32
    assert size(1000, 4096, 2100, 1) == 0          # 4224 tiles
    assert size(1 << 29, 64, 32, 0) > 0
    assert size((1 << 29) + 1, 64, 32, 0) == 0     # uint32 entry offsets
    # one entry per particle for points, up to four (2 x 2 tiles) for sprites
    n = 1 << 20
    assert size(n, 640, 480, 1) - size(n, 640, 480, 0) == 3 * 4 * n
    for bad in ((1000, 0, 1080, 0), (1000, 1920, 1080, 65), (-1, 1920, 1080, 0)):
        with pytest.raises(A._ffi.FirefliesError, match="FF_E_INVALID"):
            size(*bad)
    with pytest.raises(A._ffi.FirefliesError, match="FF_E_UNSUPPORTED"):
        size(10, 1 << 15, 1 << 14, 0)              # more than 2^28 pixels


def test_histogram_grid_limit(L):
    from paper_1505_00344_amd import api as A
    assert A.histogram_workspace_size(1000, 8192, 8192) > 0             # 64M bins: the largest grid
    with pytest.raises(A._ffi.FirefliesError, match="FF_E_UNSUPPORTED"):
        A.histogram_workspace_size(1000, 8192, 8193)
    assert A.histogram_workspace_size(1000, 128, 128) == 0              # one LDS histogram per block
    with pytest.raises(A._ffi.FirefliesError, match="FF_E_INVALID"):
        A.histogram_workspace_size(-1, 64, 64)
