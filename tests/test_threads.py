"""Host calls from several threads at once (ctypes releases the GIL during a
call, so the threads run inside the library together): the generated source of
one shared expression system is the same in every thread, and each thread's
error message is the one of its own last call."""
import ctypes
import threading

from paper_1505_00344_amd import _ffi
from paper_1505_00344_amd import api as A

LORENZ_EXPR = ["p0*(x1 - x0)", "x0*(p1 - x2) - x1", "x0*x1 - p2*x2"]


def test_concurrent_source_generation_and_error_messages():
    L = _ffi.lib()
    shared = A.System.from_exprs(LORENZ_EXPR, [10.0, 28.0, 8.0 / 3.0])
    fresh = A.System.from_exprs(LORENZ_EXPR, [10.0, 28.0, 8.0 / 3.0])
    want = {p: fresh.source(p) for p in ("fp32", "fp32_kahan", "fp64")}
    barrier = threading.Barrier(8)
    failures = []

    def worker(k):
        try:
            barrier.wait()
            for i in range(25):
                p = ("fp32", "fp32_kahan", "fp64")[(i + k) % 3]
                if shared.source(p) != want[p]:
                    failures.append(f"thread {k}: {p} source differs")
                h = ctypes.c_void_p()
                if k % 2:
                    rc, msg = L.ff_system_create(99, 3, 0, None, ctypes.byref(h)), L.ff_last_error()
                    expect = b"unknown right-hand side"
                else:
                    rc = L.ff_system_create(_ffi.FF_RHS_LORENZ, 4, 3, (ctypes.c_double * 3)(1, 2, 3), ctypes.byref(h))
                    msg, expect = L.ff_last_error(), b"dimension 4"
                if rc == 0 or expect not in msg:
                    failures.append(f"thread {k}: status {rc}, message {msg!r}")
                own = A.System("lorenz", 3, [10.0, 28.0 + k, 8.0 / 3.0])
                if own.get_params()[1] != 28.0 + k:
                    failures.append(f"thread {k}: parameters of its own system changed")
        except Exception as ex:  # reported by the main thread
            failures.append(f"thread {k}: {ex!r}")

    ts = [threading.Thread(target=worker, args=(k,)) for k in range(8)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not failures, failures[:5]
