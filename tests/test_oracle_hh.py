"""Pins of the oracle's Hodgkin-Huxley ring (Section 3, Eqs. hh_v, hh_h,
hh_m, hh_n, hh_isyn, hh_s).

The paper takes the squid-axon rates and constants from Hodgkin & Huxley
(1952).  Their paper writes the rates in its own convention (V = displacement
from rest, depolarisation negative); the oracle uses the modern convention
V_mod = -V_1952 - 65 mV.  The first test compares the oracle's rates with the
1952 forms evaluated through that change of variables, which catches a wrong
sign, shift or scale in any rate.  The paper's printed onset of repetitive
firing (I ~ 6.25) pins the assembled single-neuron model.
"""
import numpy as np
import pytest

from helpers import golden
from paper_1505_00344_amd.inputs import HH_PARAMS

NAMES = ["gNa", "gK", "gL", "ENa", "EK", "EL", "C", "Iext", "gsyn", "Esyn", "rr", "rd", "th", "sg"]


def params(**kw):
    p = list(HH_PARAMS)
    for k, v in kw.items():
        p[NAMES.index(k)] = v
    return p


# Hodgkin & Huxley (1952) rates, their convention (ms^-1, v in mV from rest,
# depolarisation negative)
def hh52(v):
    am = 0.1 * (v + 25) / (np.exp((v + 25) / 10) - 1)
    bm = 4 * np.exp(v / 18)
    ah = 0.07 * np.exp(v / 20)
    bh = 1 / (np.exp((v + 30) / 10) + 1)
    an = 0.01 * (v + 10) / (np.exp((v + 10) / 10) - 1)
    bn = 0.125 * np.exp(v / 80)
    return am, bm, ah, bh, an, bn


def oracle_rates(ora, V):
    """Read alpha, beta of each gate off the right-hand side: for a gate x,
    x' = alpha (1 - x) - beta x, so x' at x = 0 is alpha and at x = 1 is -beta."""
    p = params(gsyn=0.0)
    out = []
    for g in (1, 2, 3):  # m, h, n
        x0 = np.array([V, 0.5, 0.5, 0.5, 0.0])
        x1 = x0.copy()
        x0[g], x1[g] = 0.0, 1.0
        f0 = ora.rhs(ora.HH_RING, p, x0[None])[0, g]
        f1 = ora.rhs(ora.HH_RING, p, x1[None])[0, g]
        out += [f0, -f1]
    am, bm, ah, bh, an, bn = out
    return am, bm, ah, bh, an, bn


@pytest.mark.parametrize("V", [-90.0, -65.0, -52.5, -30.0, 0.0, 20.0, 38.0])
def test_rates_match_1952_forms(ora, V):
    got = oracle_rates(ora, V)
    want = hh52(-V - 65.0)
    assert np.allclose(got, want, rtol=1e-13, atol=0)


def test_resting_gates_and_potential(ora):
    # gate steady states at rest (1952 convention v = 0), printed to four
    # decimals by Hodgkin & Huxley (1952)
    g = golden("hh_resting_gates")
    tol = 0.5 * 10.0 ** -g["printed_decimals"]
    am, bm, ah, bh, an, bn = oracle_rates(ora, -65.0)
    assert abs(am / (am + bm) - g["m"]) < tol
    assert abs(ah / (ah + bh) - g["h"]) < tol
    assert abs(an / (an + bn) - g["n"]) < tol
    # with no drive the neuron settles at rest near -65 mV
    x = np.array([[-70.0], [0.05], [0.6], [0.32], [0.0]])
    got = ora.rk4(ora.HH_RING, params(Iext=0.0, gsyn=0.0), x, 0.01, 20000)
    assert abs(got[0, 0] + 65.0) < 0.05
    f = ora.rhs(ora.HH_RING, params(Iext=0.0, gsyn=0.0), got[:, 0][None])[0]
    assert np.abs(f).max() < 1e-6


def count_spikes(v):
    return int(np.sum((v[1:] > 0) & (v[:-1] <= 0)))


def run_traces(ora, x, I, nsteps, every=10):
    """Integrate single neurons with per-particle Iext; return V every `every`
    steps."""
    vs = []
    for _ in range(nsteps // every):
        x = ora.rk4(ora.HH_RING, params(gsyn=0.0), x, 0.01, every, pp_slot=[7], pparams=I[None])
        vs.append(x[0].copy())
    return x, np.array(vs)


def test_onset_of_repetitive_firing_near_6_25(ora):
    # Section 3: increasing I past ~6.25 gives a stable limit cycle (repetitive
    # firing).  Put neurons on the cycle with a strong drive, then lower it:
    # above the onset firing persists, below it the neuron falls silent.
    onset = golden("hh_repetitive_firing_onset")["I_onset"]
    n = 4
    x = np.tile(np.array([[-65.0], [0.05], [0.6], [0.32], [0.0]]), (1, n))
    x, _ = run_traces(ora, x, np.full(n, 12.0), 10000)
    I = np.array([5.0, 5.8, 6.8, 8.0])  # two below the printed onset, two above
    assert I[1] < onset < I[2]
    x, v = run_traces(ora, x, I, 40000)
    last = v[-1000:]  # the last 100 ms
    spikes = [count_spikes(last[:, i]) for i in range(n)]
    assert spikes[0] == 0 and spikes[1] == 0, spikes
    assert spikes[2] >= 4 and spikes[3] >= 4, spikes


def test_psi_select_at_removable_singularity(ora):
    # alpha_m has a removable singularity at V = -40 (alpha_n at V = -55); the
    # right-hand side there equals its limit
    p = params()
    for V in (-40.0, -55.0):
        x = np.array([V, 0.3, 0.4, 0.5, 0.2])
        f0 = ora.rhs(ora.HH_RING, p, x[None])[0]
        xs = np.array([x + np.array([d, 0, 0, 0, 0]) for d in (-1e-7, 1e-7)])
        fs = ora.rhs(ora.HH_RING, p, xs)
        assert np.all(np.isfinite(f0))
        assert np.allclose(f0, fs.mean(axis=0), rtol=1e-7, atol=1e-9)


def test_ring_wiring_and_synapse(ora):
    # neuron j receives the synapse of neuron (j - 1) mod 3: switching on s_0
    # changes only neuron 1's membrane equation, by gsyn (Esyn - V1) s_0 / C
    p = params()
    x = np.array([-60.0, 0.1, 0.5, 0.3, 0.0, -55.0, 0.1, 0.5, 0.3, 0.0, -50.0, 0.1, 0.5, 0.3, 0.0])
    f0 = ora.rhs(ora.HH_RING, p, x[None])[0]
    x1 = x.copy()
    x1[4] = 1.0
    f1 = ora.rhs(ora.HH_RING, p, x1[None])[0]
    d = f1 - f0
    assert d[0] == 0 and d[10] == 0
    assert abs(d[5] - 0.5 * (-80.0 + 55.0)) < 1e-12
    # at V = theta_syn the transmitter term is 1/2: s' = r_rise/2 (1 - s) - r_decay s
    x2 = x.copy()
    x2[0], x2[4] = -20.0, 0.25
    f2 = ora.rhs(ora.HH_RING, p, x2[None])[0]
    assert abs(f2[4] - (2.0 * 0.5 * 0.75 - 0.1 * 0.25)) < 1e-15


def test_fourth_order_convergence(ora):
    x0 = np.random.default_rng(1).uniform(0, 1, size=(15, 4))
    x0[0::5] = np.random.default_rng(2).uniform(-80, 40, size=(3, 4))
    ref = ora.rk4(ora.HH_RING, params(), x0, 1.0 / 51200, 51200)
    errs = [np.abs(ora.rk4(ora.HH_RING, params(), x0, 1.0 / n, n) - ref).max() for n in (800, 1600, 3200)]
    assert abs(errs[0] / errs[1] - 16) < 1.0 and abs(errs[1] / errs[2] - 16) < 1.0, errs
