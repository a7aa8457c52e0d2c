"""GPU check of ff_project_histogram_noalloc, the projection for callers that
cannot allocate device memory: through the C ABI, its counts and drop counts
equal ff_project_histogram's bit for bit on two calls in a row (the second
smaller, on another grid, so the static scratch holds the first call's
values), in both precisions and with accumulation; a projection that needs
more scratch than the static buffer holds is refused before anything runs."""
import ctypes

import numpy as np
import pytest

from helpers import api, to_dev, to_host
from paper_1505_00344_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def A():
    return api()


def positions(n, seed):
    """(E, I) positions of the Wilson-Cowan 4M workload's shape: half of them
    piled into a few bins, a few NaN and out-of-range values."""
    rng = np.random.default_rng(seed)
    st = np.empty((2, n))
    st[:, :] = rng.uniform(0.0, 1.0, (2, n))
    half = n // 2
    st[0, :half] = np.round(rng.uniform(0, 1, half) * 8) / 8 + 1 / 4096
    st[0, half:half + 100] = np.nan
    st[0, half + 100:half + 200] = 1.0
    st[1, half + 200:half + 300] = -0.5
    p = rng.uniform(-2.0, 4.0, (1, n))
    return st, p


def both(A, sysobj, st, pp, nx, ny, xr, yr, accumulate=False, seed_hist=None):
    """(noalloc counts, noalloc drops), (reference counts, reference drops)."""
    out = []
    for fn in (A.project_histogram_noalloc, A.project_histogram):
        hist = torch.zeros((ny, nx), dtype=torch.int32, device="cuda:0")
        dropped = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        if seed_hist is not None:
            hist.copy_(seed_hist)
            dropped.fill_(7)
        fn(sysobj, st, -1, 0, xr, yr, nx, ny, hist=hist, n_dropped=dropped, accumulate=accumulate,
           pparams=pp, pp_slot=[8])
        torch.cuda.synchronize()
        out.append((to_host(hist).view(np.uint32).copy(), int(dropped.item())))
    return out


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_equals_workspace_call_twice(A, ora, dtype):
    w = I.wilson_cowan_4m()
    sysobj = A.System("wilson_cowan", 2, w.params)
    hs = w.hist
    # first call: the full 4M ensemble on the 1024 x 1024 (P, E) grid
    st, p = positions(w.n, 3)
    dst, dpp = to_dev(st, dtype), to_dev(p, dtype)
    (h1, d1), (r1, e1) = both(A, sysobj, dst, dpp, hs["nx"], hs["ny"], hs["x_range"], hs["y_range"])
    assert d1 == e1 and np.array_equal(h1, r1)
    assert int(h1.sum(dtype=np.int64)) + d1 == w.n
    # second call: fewer particles (a ragged count) on a 700 x 300 grid
    n2 = 250_001
    st2, p2 = positions(n2, 4)
    dst2, dpp2 = to_dev(st2, dtype), to_dev(p2, dtype)
    (h2, d2), (r2, e2) = both(A, sysobj, dst2, dpp2, 700, 300, (-2.0, 4.0), (0.0, 1.0))
    assert d2 == e2 and np.array_equal(h2, r2)
    # and the oracle's binning of the same values
    s64 = st2 if dtype == torch.float64 else st2.astype(np.float32).astype(np.float64)
    p64 = p2 if dtype == torch.float64 else p2.astype(np.float32).astype(np.float64)
    want, wd = ora.histogram(s64, -1, 0, (-2.0, 4.0), (0.0, 1.0), 700, 300, pparams=p64)
    assert wd == d2 and np.array_equal(h2, want)


def test_noalloc_accumulate_and_small_grid(A):
    w = I.wilson_cowan_4m()
    sysobj = A.System("wilson_cowan", 2, w.params)
    st, p = positions(300_007, 5)
    dst, dpp = to_dev(st, torch.float32), to_dev(p, torch.float32)
    seed = torch.arange(1024 * 1024, dtype=torch.int32, device="cuda:0").reshape(1024, 1024) % 5
    (h, d), (r, e) = both(A, sysobj, dst, dpp, 1024, 1024, (-2.0, 4.0), (0.0, 1.0), accumulate=True,
                          seed_hist=seed)
    assert d == e and np.array_equal(h, r)
    # a grid of at most 16384 bins takes the path without scratch
    (h, d), (r, e) = both(A, sysobj, dst, dpp, 128, 128, (-2.0, 4.0), (0.0, 1.0))
    assert d == e and np.array_equal(h, r)


def test_noalloc_refuses_projection_beyond_its_scratch(A):
    from paper_1505_00344_amd import _ffi
    w = I.wilson_cowan_4m()
    sysobj = A.System("wilson_cowan", 2, w.params)
    n = 12 * 1024 * 1024
    need = ctypes.c_size_t()
    _ffi.call("ff_histogram_workspace_size", n, 1024, 1024, ctypes.byref(need))
    assert need.value > 64 * 1024 * 1024
    st = torch.zeros((2, n), dtype=torch.float32, device="cuda:0")
    pp = torch.zeros((1, n), dtype=torch.float32, device="cuda:0")
    hist = torch.full((1024, 1024), 3, dtype=torch.int32, device="cuda:0")
    dropped = torch.full((1,), 5, dtype=torch.int64, device="cuda:0")
    with pytest.raises(_ffi.FirefliesError) as ei:
        A.project_histogram_noalloc(sysobj, st, -1, 0, (-2.0, 4.0), (0.0, 1.0), 1024, 1024, hist=hist,
                                    n_dropped=dropped, pparams=pp, pp_slot=[8])
    assert ei.value.status == _ffi.FF_E_NOMEM and "static" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((hist == 3).all()) and int(dropped.item()) == 5  # nothing was enqueued


def test_noalloc_empty_batch_and_largest_accepted_size(A, ora):
    from paper_1505_00344_amd import _ffi
    w = I.wilson_cowan_4m()
    sysobj = A.System("wilson_cowan", 2, w.params)
    # an empty batch clears the grid and the drop count and touches nothing else
    st = torch.zeros((2, 0), dtype=torch.float32, device="cuda:0")
    pp = torch.zeros((1, 0), dtype=torch.float32, device="cuda:0")
    hist = torch.full((1024, 1024), 9, dtype=torch.int32, device="cuda:0")
    dropped = torch.full((1,), 9, dtype=torch.int64, device="cuda:0")
    A.project_histogram_noalloc(sysobj, st, -1, 0, (-2.0, 4.0), (0.0, 1.0), 1024, 1024, hist=hist,
                                n_dropped=dropped, pparams=pp, pp_slot=[8])
    torch.cuda.synchronize()
    assert bool((hist == 0).all()) and int(dropped.item()) == 0
    # the largest particle count whose workspace fits the static buffer (on the
    # 1024 x 1024 grid) is accepted and equals the workspace call; one more
    # count block is refused
    limit = 64 * 1024 * 1024

    def need(n):
        out = ctypes.c_size_t()
        _ffi.call("ff_histogram_workspace_size", n, 1024, 1024, ctypes.byref(out))
        return out.value

    lo, hi = 1, 16 * 1024 * 1024
    while hi - lo > 1:
        mid = (lo + hi) // 2
        lo, hi = (mid, hi) if need(mid) <= limit else (lo, mid)
    n_max = lo
    assert need(n_max) <= limit < need(n_max + 1)
    st, p = positions(n_max, 6)
    dst, dpp = to_dev(st, torch.float32), to_dev(p, torch.float32)
    (h, d), (r, e) = both(A, sysobj, dst, dpp, 1024, 1024, (-2.0, 4.0), (0.0, 1.0))
    assert d == e and np.array_equal(h, r)
    assert int(h.sum(dtype=np.int64)) + d == n_max
    del dst, dpp
    big = torch.zeros((2, n_max + 4096), dtype=torch.float32, device="cuda:0")
    bigp = torch.zeros((1, n_max + 4096), dtype=torch.float32, device="cuda:0")
    with pytest.raises(_ffi.FirefliesError) as ei:
        A.project_histogram_noalloc(sysobj, big, -1, 0, (-2.0, 4.0), (0.0, 1.0), 1024, 1024, pparams=bigp,
                                    pp_slot=[8])
    assert ei.value.status == _ffi.FF_E_NOMEM
