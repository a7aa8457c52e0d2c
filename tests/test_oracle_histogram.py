"""Pins of the oracle's 2D density projection.

The paper draws each particle as a point of light projected onto two chosen
axes and adds the contributions of overlapping points (Appendix A, "Render
Technique"; Appendix A.1, fragment shader with additive blending).  With unit
weight per particle this is a count per pixel: a 2D histogram over half-open
bins, with points outside the range or with NaN coordinates dropped.
"""
import numpy as np
import pytest


def brute(xs, ys, xr, yr, nx, ny):
    """Per-bin brute force: a point is in bin (ix, iy) iff it lies in
    [x_lo + ix dx, x_lo + (ix+1) dx) x [...]; on dyadic ranges these bounds are
    exact."""
    H = np.zeros((ny, nx), dtype=np.uint32)
    dropped = 0
    dx = (xr[1] - xr[0]) / nx
    dy = (yr[1] - yr[0]) / ny
    for x, y in zip(xs, ys):
        hit = False
        for iy in range(ny):
            if not (yr[0] + iy * dy <= y < yr[0] + (iy + 1) * dy):
                continue
            for ix in range(nx):
                if xr[0] + ix * dx <= x < xr[0] + (ix + 1) * dx:
                    H[iy, ix] += 1
                    hit = True
        dropped += 0 if hit else 1
    return H, dropped


def test_brute_force_tiny(ora):
    rng = np.random.default_rng(0)
    st = rng.uniform(-20, 20, size=(3, 300))
    st[2] = rng.uniform(-4, 36, 300)
    H, d = ora.histogram(st, 0, 2, (-16.0, 16.0), (0.0, 32.0), 8, 16)
    Hb, db = brute(st[0], st[2], (-16.0, 16.0), (0.0, 32.0), 8, 16)
    assert np.array_equal(H, Hb) and d == db
    assert int(H.sum()) + d == 300


def test_numpy_histogram2d_dyadic(ora):
    rng = np.random.default_rng(1)
    st = rng.normal(0, 6, size=(2, 200000))
    H, d = ora.histogram(st, 0, 1, (-16.0, 16.0), (-8.0, 8.0), 512, 256)
    # numpy counts x == hi in the last bin; values exactly at hi are absent here
    want, _, _ = np.histogram2d(st[1], st[0], bins=[256, 512], range=[[-8, 8], [-16, 16]])
    inside = (st[0] >= -16) & (st[0] < 16) & (st[1] >= -8) & (st[1] < 8)
    assert np.array_equal(H, want.astype(np.uint32))
    assert d == int((~inside).sum())


def test_edges_nan_inf(ora):
    st = np.array([[-16.0, 16.0, 16.0 - 2 ** -40, np.nan, np.inf, -np.inf, 0.0, 0.0,
                    np.nextafter(16.0, 0)],
                   [0.0, 0.0, 0.0, 0.0, 0.0, 0.0, np.nan, 8.0 - 2 ** -40, 0.0]])
    H, d = ora.histogram(st, 0, 1, (-16.0, 16.0), (0.0, 8.0), 32, 8)
    assert H[0, 0] == 1        # x = lo lands in bin 0
    assert H[0, 31] == 1       # just below hi lands in the last bin
    assert H[7, 16] == 1       # y just below hi
    assert H[0, 16] == 0
    # x = hi, NaN, +Inf, -Inf, NaN in y are dropped; so is the largest double
    # below hi, because (x - lo) * s rounds to exactly nx: the binning formula,
    # not the mathematical edge, decides
    assert d == 6
    assert int(H.sum()) + d == st.shape[1]


def test_all_in_one_bin_and_accumulate(ora):
    st = np.full((2, 100000), 0.3)
    H, d = ora.histogram(st, 0, 1, (0.0, 1.0), (0.0, 1.0), 1024, 1024)
    assert H[307, 307] == 100000 and d == 0 and H.sum() == 100000
    H2, d2 = ora.histogram(st[:, :10] + 5, 0, 1, (0.0, 1.0), (0.0, 1.0), 1024, 1024, hist=H, n_dropped=d)
    assert H2[307, 307] == 100000 and d2 == 10


def test_parameter_axis(ora):
    rng = np.random.default_rng(3)
    st = rng.uniform(0, 1, size=(2, 5000))
    pp = rng.uniform(-2, 4, size=(1, 5000))
    H, d = ora.histogram(st, -1, 0, (-2.0, 4.0), (0.0, 1.0), 96, 64, pparams=pp)
    want, _, _ = np.histogram2d(st[0], pp[0], bins=[64, 96], range=[[0, 1], [-2, 4]])
    # -2..4 over 96 bins is dyadic (bin width 1/16)
    assert np.array_equal(H, want.astype(np.uint32)) and d == 0


@pytest.mark.parametrize("bad", [dict(nx=0), dict(axis_x=3), dict(axis_y=-2)])
def test_invalid_arguments(ora, bad):
    args = dict(axis_x=0, axis_y=1, nx=4, ny=4)
    args.update(bad)
    with pytest.raises(ValueError):
        ora.histogram(np.zeros((3, 4)), args["axis_x"], args["axis_y"], (0.0, 1.0), (0.0, 1.0),
                      args["nx"], args["ny"])
