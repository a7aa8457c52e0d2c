"""GPU parity of ff_integrate_reset (the paper's reset rule, Section 2.1 and
Appendix A: trajectories that leave the region or exceed T_max restart from
new random initial conditions in the group's box) against the oracle."""
import numpy as np
import pytest

from helpers import api, mixed_error, quantiles, to_dev, to_host
from paper_1505_00344_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LORENZ_BOUNDS = [(-40.0, 40.0), (-60.0, 60.0), (-10.0, 80.0)]


@pytest.fixture(scope="module")
def A():
    return api()


def gpu_reset(A, sysname, dim, params, x, dt, nsteps, bounds, box, max_age=-1, seed=0, id_offset=0, prec="fp64",
              pp=None, pp_slot=(), tuning=None, splits=None):
    dtype = torch.float64 if prec == "fp64" else torch.float32
    st = to_dev(x, dtype)
    ppt = None if pp is None else to_dev(pp, dtype)
    comp = torch.zeros_like(st) if prec == "fp32_kahan" else None
    n = st.shape[1]
    age = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    nres = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    sysobj = A.System(sysname, dim, params)
    for k in (splits or [nsteps]):
        A.integrate_reset(sysobj, st, dt, k, bounds=bounds, box=box, age=age, n_resets=nres, max_age=max_age,
                          seed=seed, id_offset=id_offset, pparams=ppt, pp_slot=pp_slot, comp=comp, prec=prec,
                          tuning=tuning)
    torch.cuda.synchronize()
    return to_host(st), None if comp is None else to_host(comp), to_host(age), to_host(nres).view(np.uint32)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_kahan"])
def test_lorenz_4096_with_resets_matches_oracle_bitwise(A, ora, prec):
    w = I.lorenz_4096()
    e = I.generate(w)
    x = e.state if prec == "fp64" else e.state.astype(np.float32)
    outs = []
    for off, n, dt in zip(e.offsets, e.counts, e.dts):
        xs = x[:, off:off + n]
        got = gpu_reset(A, "lorenz", 3, w.params, xs, dt, w.nsteps, LORENZ_BOUNDS, I.LORENZ_BOX, max_age=600,
                        seed=2015, id_offset=off, prec=prec)
        ref = ora.rk4_reset(ora.LORENZ, w.params, xs, dt, w.nsteps, LORENZ_BOUNDS, I.LORENZ_BOX, max_age=600,
                            seed=2015, id_offset=off, prec=prec)
        assert np.array_equal(got[0], ref[0])
        if prec == "fp32_kahan":
            assert np.array_equal(got[1], ref[1])
        assert np.array_equal(got[2], ref[2]) and np.array_equal(got[3], ref[3])
        outs.append(got)
    # the backward group escapes and is recycled; age limits recycle the rest
    assert outs[1][3].sum() > e.counts[1]
    assert np.all(np.isfinite(outs[1][0]))


BOUND_CASES = [(60.000001, 80.5), (-1e-30, 1e-30), (-np.inf, 3.0), (-1e300, 1e300), (1.5, 1.5), (-np.inf, np.inf)]


def float_neighbours(b):
    f = np.float32(np.clip(b, -np.finfo(np.float32).max, np.finfo(np.float32).max))
    out = [f]
    with np.errstate(over="ignore"):  # stepping past the largest float gives inf
        for _ in range(2):
            out.append(np.nextafter(out[-1], np.float32(np.inf)))
        g = f
        for _ in range(2):
            g = np.nextafter(g, np.float32(-np.inf))
            out.append(g)
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp32_kahan", "fp64"])
def test_bounds_between_floats_decide_like_double(A, ora, prec):
    # x' = 0 x keeps a finite state exactly, so the bounds test sees the
    # initial values: bounds between two floats, at a float, infinite and
    # beyond the float range, with particles on the floats around each bound;
    # the single-precision kernels test against float thresholds, which must
    # decide exactly as the double comparison of the rule does
    vals = {np.float32(v) for v in (0.0, 1.0, -1.0, np.inf, -np.inf)}
    for lo, hi in BOUND_CASES:
        for b in (lo, hi):
            vals.update(float_neighbours(b))
    fin = np.array(sorted(v for v in vals if np.isfinite(v)), dtype=np.float32)
    x = np.concatenate([fin, np.array([np.inf, -np.inf, np.nan], dtype=np.float32)])[None, :]
    x = x.astype(np.float64) if prec == "fp64" else x
    for lo, hi in BOUND_CASES:
        got = gpu_reset(A, "linear", 1, [0.0], x, 0.01, 1, [(lo, hi)], [(0.25, 0.75)], seed=7, prec=prec)
        ref = ora.rk4_reset(ora.LINEAR, [0.0], x, 0.01, 1, [(lo, hi)], [(0.25, 0.75)], seed=7, prec=prec)
        assert np.array_equal(got[0], ref[0], equal_nan=True), (lo, hi)
        assert np.array_equal(got[3], ref[3]), (lo, hi)
        # the finite particles are reset exactly where the double comparison fails
        xf = x[0, :len(fin)].astype(np.float64)
        assert np.array_equal(got[3][:len(fin)] == 1, ~((xf >= lo) & (xf <= hi))), (lo, hi)


def test_wilson_cowan_backward_unit_square(A, ora):
    # the 2D model's setting of Section 2.1: ICs uniform on (0,1)^2, any
    # trajectory leaving the square is reset; backward particles leave it fast
    w = I.wilson_cowan_4m(n=6000)
    e = I.generate(w)
    nf = e.counts[0]
    x, pp = e.state[:, nf:], e.pparams[:, nf:]
    bounds = [(0.0, 1.0), (0.0, 1.0)]
    got = gpu_reset(A, "wilson_cowan", 2, w.params, x, -0.01, 400, bounds, I.WC_BOX, seed=5, prec="fp64", pp=pp,
                    pp_slot=w.pp_slot)
    ref = ora.rk4_reset(ora.WILSON_COWAN, w.params, x, -0.01, 400, bounds, I.WC_BOX, seed=5, pp_slot=w.pp_slot,
                        pparams=pp)
    assert np.array_equal(got[3], ref[3]) and np.array_equal(got[2], ref[2])
    err = mixed_error(got[0], ref[0])
    assert err.max() <= 1e-12, quantiles(err)
    assert got[3].sum() > x.shape[1]


def test_reset_launch_shape_and_call_splitting_invariance(A):
    w = I.lorenz_4096()
    e = I.generate(w)
    nf = e.counts[0]
    x = e.state[:, nf:].astype(np.float32)
    base = gpu_reset(A, "lorenz", 3, w.params, x, -0.005, 500, LORENZ_BOUNDS, I.LORENZ_BOX, max_age=77, seed=3,
                     prec="fp32_kahan")
    for tuning, splits in [((13, 2, 128), None), ((500, 1, 64), [123, 377]), ((1, 4, 256), [250, 250])]:
        got = gpu_reset(A, "lorenz", 3, w.params, x, -0.005, 500, LORENZ_BOUNDS, I.LORENZ_BOX, max_age=77, seed=3,
                        prec="fp32_kahan", tuning=tuning, splits=splits)
        for a, b in zip(got, base):
            assert np.array_equal(a, b)


def test_invalid_reset_arguments(A):
    sysobj = A.System("lorenz", 3, I.LORENZ_PARAMS)
    st = torch.zeros((3, 10), dtype=torch.float64, device="cuda:0")
    age = torch.zeros(10, dtype=torch.int32, device="cuda:0")
    nres = torch.zeros(10, dtype=torch.int32, device="cuda:0")
    for bounds, box in [([(1.0, 0.0)] * 3, I.LORENZ_BOX), (LORENZ_BOUNDS, [(0.0, 0.0)] * 3),
                        (LORENZ_BOUNDS, [(0.0, float("inf"))] * 3)]:
        with pytest.raises(A._ffi.FirefliesError, match="FF_E_INVALID"):
            A.integrate_reset(sysobj, st, 0.01, 5, bounds=bounds, box=box, age=age, n_resets=nres)
