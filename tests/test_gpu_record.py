"""GPU tests of ff_integrate_record (trajectory recording, the paper's
future-work item in Section 4: a subset of trajectories, or all of them at an
interval longer than the step) against the oracle: record k is the state after
(k+1)*every steps."""
import numpy as np
import pytest

from helpers import api, to_dev, to_host
from paper_1505_00344_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def A():
    return api()


@pytest.mark.parametrize("tuning", [None, (37, 2, 128)])
def test_lorenz_records_match_oracle_bitwise(A, ora, tuning):
    w = I.lorenz_4096()
    e = I.generate(w)
    nf = e.counts[0]
    x0 = e.state[:, :nf]
    sysobj = A.System("lorenz", 3, w.params)
    st = to_dev(x0, torch.float64)
    every, stride, nsteps = 100, 7, 1000
    out = A.integrate_record(sysobj, st, 0.005, nsteps, every, stride, tuning=tuning)
    torch.cuda.synchronize()
    rec = to_host(out)
    assert rec.shape == (10, 3, (nf + stride - 1) // stride)
    ref = x0.copy()
    for k in range(nsteps // every):
        ref = ora.rk4(ora.LORENZ, w.params, ref, 0.005, every)
        assert np.array_equal(rec[k], ref[:, ::stride]), k
    assert np.array_equal(to_host(st), ref)


def test_records_with_resets_match_oracle(A, ora):
    w = I.lorenz_4096()
    e = I.generate(w)
    nf = e.counts[0]
    x0 = e.state[:, nf:]
    n = x0.shape[1]
    bounds = [(-40.0, 40.0), (-60.0, 60.0), (-10.0, 80.0)]
    sysobj = A.System("lorenz", 3, w.params)
    st = to_dev(x0, torch.float64)
    age = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    nres = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    out = A.integrate_record(sysobj, st, -0.005, 450, 50, 1,
                             reset=dict(bounds=bounds, box=I.LORENZ_BOX, age=age, n_resets=nres, seed=11,
                                        max_age=120))
    torch.cuda.synchronize()
    rec = to_host(out)
    ref, a, r = x0.copy(), None, None
    for k in range(9):
        ref, _, a, r = ora.rk4_reset(ora.LORENZ, w.params, ref, -0.005, 50, bounds, I.LORENZ_BOX, max_age=120,
                                     seed=11, age=a, n_resets=r)
        assert np.array_equal(rec[k], ref), k
    assert np.array_equal(to_host(age), a) and np.array_equal(to_host(nres).view(np.uint32), r)


def test_kahan_records_equal_chunked_integration(A):
    w = I.wilson_cowan_4m(n=5000)
    e = I.generate(w)
    sysobj = A.System("wilson_cowan", 2, w.params)
    x = e.state.astype(np.float32)
    pp = to_dev(e.pparams.astype(np.float32), torch.float32)
    st = to_dev(x, torch.float32)
    comp = torch.zeros_like(st)
    out = A.integrate_record(sysobj, st, 0.01, 300, 60, 3, pparams=pp, pp_slot=w.pp_slot, comp=comp,
                             tuning=(25, 1, 256))
    st2 = to_dev(x, torch.float32)
    comp2 = torch.zeros_like(st2)
    for k in range(5):
        A.integrate(sysobj, st2, 0.01, 60, pparams=pp, pp_slot=w.pp_slot, comp=comp2)
        torch.cuda.synchronize()
        assert torch.equal(out[k], st2[:, ::3]), k
    assert torch.equal(st, st2) and torch.equal(comp, comp2)


def test_partial_interval_and_validation(A):
    sysobj = A.System("lorenz", 3, I.LORENZ_PARAMS)
    st = torch.ones((3, 100), dtype=torch.float64, device="cuda:0")
    out = A.integrate_record(sysobj, st, 0.001, 25, 10, 10)
    assert tuple(out.shape) == (2, 3, 10)
    with pytest.raises(A._ffi.FirefliesError, match="FF_E_INVALID"):
        A.integrate_record(sysobj, st, 0.001, 25, 0, 1)
