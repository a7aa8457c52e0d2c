"""Pins of the oracle's reset rule (Section 2.1: trajectories that leave the
region, or that have not been reset for more than T_max, restart from new
random initial conditions drawn from the group's box, Appendix A).

Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11),
pinned by the known-answer vectors published with the method's reference
implementation (Random123)."""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from paper_1505_00344_amd.inputs import LORENZ_BOX, LORENZ_PARAMS, WC_BOX, WC_PARAMS

from helpers import golden

# (counter, key, output) known-answer vectors of Philox4x32-10
KAT = [([int(w, 16) for w in v["counter"]], [int(w, 16) for w in v["key"]], [int(w, 16) for w in v["output"]])
       for v in golden("philox4x32_10_kat")["vectors"]]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ora, ctr, key, want):
    assert list(ora.philox4x32_10(ctr, key)) == want


def test_no_reset_is_plain_rk4(ora):
    # bounds never reached and no age limit: bitwise the plain map
    x = np.random.default_rng(0).uniform(0, 1, size=(2, 300))
    P = np.random.default_rng(1).uniform(-2, 4, size=(1, 300))
    got, _, age, nres = ora.rk4_reset(ora.WILSON_COWAN, WC_PARAMS, x, 0.01, 200, bounds=[(-1e9, 1e9)] * 2,
                                      box=WC_BOX, pp_slot=[8], pparams=P)
    assert np.array_equal(got, ora.rk4(ora.WILSON_COWAN, WC_PARAMS, x, 0.01, 200, pp_slot=[8], pparams=P))
    assert np.all(age == 200) and np.all(nres == 0)


def test_redraw_uses_documented_stream(ora):
    # max_age = 0: every step ends in a redraw, so the state after one step is
    # draw number 0 of each particle, computable from Philox directly
    seed, off = 0x1234_5678_9ABC_DEF0, 1000
    x = np.zeros((3, 5))
    got, _, age, nres = ora.rk4_reset(ora.LORENZ, LORENZ_PARAMS, x, 0.005, 1, bounds=[(-1e9, 1e9)] * 3,
                                      box=LORENZ_BOX, max_age=0, seed=seed, id_offset=off)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for i in range(5):
        g = off + i
        words = np.concatenate([ora.philox4x32_10([g & 0xFFFFFFFF, g >> 32, 0, j], key) for j in range(2)])
        for d, (lo, hi) in enumerate(LORENZ_BOX):
            a, b = int(words[2 * d]), int(words[2 * d + 1])
            u = ((a >> 5) * 67108864.0 + (b >> 6)) / 2.0 ** 53
            fused = float(Fraction(hi - lo) * Fraction(u) + Fraction(lo))  # one rounding = fma
            assert got[d, i] == fused
    assert np.all(age == 0) and np.all(nres == 1)


def test_escaped_particles_are_redrawn_in_the_box(ora):
    # backward Lorenz particles escape to infinity (Section 2.2 discusses why
    # backward particles are not useful there); with bounds they are recycled
    x = np.random.default_rng(2).uniform([[-20], [-30], [0]], [[20], [30], [50]], size=(3, 2000))
    bounds = [(-200.0, 200.0), (-300.0, 300.0), (-100.0, 400.0)]
    got, _, age, nres = ora.rk4_reset(ora.LORENZ, LORENZ_PARAMS, x, -0.005, 300, bounds=bounds, box=LORENZ_BOX,
                                      seed=7)
    assert nres.sum() > 1000            # most particles escaped at least once
    assert np.all(np.isfinite(got))
    for d, (lo, hi) in enumerate(bounds):
        assert np.all(got[d] >= lo) and np.all(got[d] <= hi)
    # a particle that was reset k steps ago is the k-step backward image of a
    # box draw; one step after a reset it lies within one step of the box
    fresh = age == 0
    for d, (lo, hi) in enumerate(LORENZ_BOX):
        assert np.all(got[d, fresh] >= lo) and np.all(got[d, fresh] < hi)


def test_age_limit(ora):
    # T_max: with max_age = 10 a particle that never leaves the bounds is
    # redrawn every 11 steps
    x = np.random.default_rng(3).uniform(0, 1, size=(2, 100))
    _, _, age, nres = ora.rk4_reset(ora.WILSON_COWAN, WC_PARAMS, x, 0.01, 55, bounds=[(-1e9, 1e9)] * 2,
                                    box=WC_BOX, max_age=10)
    assert np.all(nres == 5) and np.all(age == 0)
    _, _, age, nres = ora.rk4_reset(ora.WILSON_COWAN, WC_PARAMS, x, 0.01, 60, bounds=[(-1e9, 1e9)] * 2,
                                    box=WC_BOX, max_age=10)
    assert np.all(nres == 5) and np.all(age == 5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_redraws_are_uniform(ora, prec):
    # 20000 particles, max_age = 0, 5 steps: 100000 draws per component
    n = 20000
    x = np.zeros((2, n))
    vals = []
    a = r = None
    for _ in range(5):
        x, _, a, r = ora.rk4_reset(ora.WILSON_COWAN, WC_PARAMS, x, 0.01, 1, bounds=[(-1e9, 1e9)] * 2,
                                   box=[(-2.0, 4.0), (0.0, 1.0)], max_age=0, seed=99, age=a, n_resets=r,
                                   prec=prec)
        vals.append(np.array(x, dtype=np.float64))
    v = np.concatenate(vals, axis=1)
    assert stats.kstest((v[0] + 2.0) / 6.0, "uniform").pvalue > 1e-3
    assert stats.kstest(v[1], "uniform").pvalue > 1e-3
    assert abs(np.corrcoef(v[0], v[1])[0, 1]) < 0.01
    assert np.all(r == 5)
