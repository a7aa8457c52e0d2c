"""Seeded synthetic workloads (inputs only: no step of the method lives here).

The paper draws every initial condition uniformly from a per-group box
(Section 2.1 for the 2D model, the Lorenz figure captions of Section 2.2,
Appendix A "Particle Group"), and turns a parameter into a per-particle value
for dynamic bifurcation diagrams (Section 2.1, Section 2.2).  This module
builds such ensembles for the five workloads the library is measured on, with
one fixed recipe:

* generator ``numpy.random.default_rng(20150501 + k)`` for workload k;
* for each group in order: for each state component in order
  ``rng.uniform(lo, hi, n_group)``, then each per-particle parameter in slot
  order (uniform in its range, or a constant);
* forward groups come before backward groups in memory (the group list is
  written in that order).

Values are float64; single-precision runs round them with ``astype``.
Both the HIP path and the CPU oracle receive exactly these arrays.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 20150501

# System identifiers (same numbering as the C ABI's ff_rhs enum).
LINEAR, LORENZ, WILSON_COWAN, HH_RING = 0, 1, 2, 3

# Default parameter vectors.
#   Lorenz: [sigma, r, beta] (Section 2.2: sigma = 10, beta = 8/3).
LORENZ_PARAMS = [10.0, 28.0, 8.0 / 3.0]
#   Wilson-Cowan: [c1, c2, c3, c4, aE, thetaE, aI, thetaI, P, Q].
WC_PARAMS = [16.0, 12.0, 15.0, 3.0, 1.3, 4.0, 2.0, 3.7, 0.0, 0.0]
#   HH ring: [gNa, gK, gL, ENa, EK, EL, C, Iext, gsyn, Esyn, r_rise, r_decay,
#             theta_syn, sigma_syn].
HH_PARAMS = [120.0, 36.0, 0.3, 50.0, -77.0, -54.4, 1.0, 10.0, 0.5, -80.0, 2.0, 0.1, -20.0, 0.5]

LORENZ_BOX = [(-20.0, 20.0), (-30.0, 30.0), (0.0, 50.0)]
WC_BOX = [(0.0, 1.0), (0.0, 1.0)]
HH_NEURON_BOX = [(-80.0, 40.0), (0.0, 1.0), (0.0, 1.0), (0.0, 1.0), (0.0, 1.0)]


@dataclass
class Group:
    n: int
    dt: float
    box: Sequence[Tuple[float, float]]
    # one entry per per-particle parameter: (lo, hi) range or a float constant
    pp: Sequence = ()


@dataclass
class Workload:
    name: str
    seed_index: int
    system: int
    dim: int
    params: List[float]
    groups: List[Group]
    nsteps: int
    pp_slot: List[int] = field(default_factory=list)
    hist: Optional[dict] = None   # axis_x, axis_y, x_range, y_range, nx, ny
    prec: str = "fp64"
    adjoint: Optional[dict] = None  # nsteps, K

    @property
    def n(self) -> int:
        return sum(g.n for g in self.groups)


@dataclass
class Ensemble:
    workload: Workload
    state: np.ndarray           # (dim, n) float64
    pparams: Optional[np.ndarray]  # (n_pp, n) float64 or None
    offsets: List[int]          # start of each group
    counts: List[int]
    dts: List[float]


def _split(n_total: int, fractions: Sequence[float]) -> List[int]:
    sizes = [int(round(n_total * f)) for f in fractions]
    sizes[-1] = n_total - sum(sizes[:-1])
    return sizes


def lorenz_4096(n: int = 4096) -> Workload:
    """Lorenz, r = 28: 3/4 forward (h = +0.005), 1/4 backward (h = -0.005),
    1000 steps, FP64, (x, z) histogram 512 x 512."""
    nf, nb = _split(n, [0.75, 0.25])
    return Workload(
        "lorenz_4096_fp64", 0, LORENZ, 3, list(LORENZ_PARAMS),
        [Group(nf, 0.005, LORENZ_BOX), Group(nb, -0.005, LORENZ_BOX)], 1000,
        hist=dict(axis_x=0, axis_y=2, x_range=(-20.0, 20.0), y_range=(0.0, 50.0), nx=512, ny=512))


def wilson_cowan_4m(n: int = 4 * 1024 * 1024) -> Workload:
    """Wilson-Cowan dynamic bifurcation diagram: per-particle P ~ U[-2, 4],
    (E, I) ~ U[0, 1]^2, half forward / half backward (h = +-0.01), 1000 steps,
    (P, E) histogram 1024 x 1024."""
    nf, nb = _split(n, [0.5, 0.5])
    return Workload(
        "wilson_cowan_4m", 1, WILSON_COWAN, 2, list(WC_PARAMS),
        [Group(nf, 0.01, WC_BOX, [(-2.0, 4.0)]), Group(nb, -0.01, WC_BOX, [(-2.0, 4.0)])],
        1000, pp_slot=[8],
        hist=dict(axis_x=-1, axis_y=0, x_range=(-2.0, 4.0), y_range=(0.0, 1.0), nx=1024, ny=1024),
        prec="fp32_kahan")


def lorenz_8m(n: int = 8 * 1024 * 1024) -> Workload:
    """Lorenz bifurcation diagram: per-particle r ~ U[0, 50], initial states as
    the 4096-particle case, h = 0.005, 500 steps; adjoint of mean z(T) w.r.t.
    each particle's r over 200 steps with checkpoints every 50."""
    return Workload(
        "lorenz_8m", 2, LORENZ, 3, list(LORENZ_PARAMS),
        [Group(n, 0.005, LORENZ_BOX, [(0.0, 50.0)])], 500, pp_slot=[1],
        hist=dict(axis_x=-1, axis_y=1, x_range=(0.0, 50.0), y_range=(-30.0, 30.0), nx=1024, ny=1024),
        prec="fp32_kahan", adjoint=dict(nsteps=200, K=50))


def hh_ring_1m(n: int = 1024 * 1024) -> Workload:
    """Three-neuron Hodgkin-Huxley ring (15 state variables), V ~ U[-80, 40],
    gates and synapses ~ U[0, 1], per-particle (gsyn, Iext) = (0.5, 10),
    h = 0.01 ms, 2000 steps; adjoint of mean V1(T) w.r.t. (gsyn, Iext) with
    checkpoints every 100 steps."""
    return Workload(
        "hh_ring3_1m", 3, HH_RING, 15, list(HH_PARAMS),
        [Group(n, 0.01, HH_NEURON_BOX * 3, [0.5, 10.0])], 2000, pp_slot=[8, 7],
        hist=dict(axis_x=0, axis_y=5, x_range=(-90.0, 60.0), y_range=(-90.0, 60.0), nx=512, ny=512),
        prec="fp32_kahan", adjoint=dict(nsteps=2000, K=100))


WORKLOADS = {w.__name__: w for w in (lorenz_4096, wilson_cowan_4m, lorenz_8m, hh_ring_1m)}


def generate(w: Workload) -> Ensemble:
    """Draw the ensemble of workload ``w`` with the fixed recipe above."""
    rng = np.random.default_rng(SEED_BASE + w.seed_index)
    n = w.n
    state = np.empty((w.dim, n))
    npp = len(w.pp_slot)
    pp = np.empty((npp, n)) if npp else None
    offsets, counts, dts = [], [], []
    off = 0
    for g in w.groups:
        assert len(g.box) == w.dim and len(g.pp) == npp
        for d, (lo, hi) in enumerate(g.box):
            state[d, off:off + g.n] = rng.uniform(lo, hi, g.n)
        for k, spec in enumerate(g.pp):
            if isinstance(spec, tuple):
                pp[k, off:off + g.n] = rng.uniform(spec[0], spec[1], g.n)
            else:
                pp[k, off:off + g.n] = float(spec)
        offsets.append(off)
        counts.append(g.n)
        dts.append(g.dt)
        off += g.n
    return Ensemble(w, state, pp, offsets, counts, dts)


# ------------------------------------------------------------ mixed batch
def mixed_batch(scale: float = 1.0, seed_index: int = 4) -> List[Workload]:
    """The ragged mixed batch: 3M Wilson-Cowan (h = +-0.01, per-particle
    P ~ U[-2, 4]), 2M Lorenz (h = +-0.005, r = 28), 0.5M three-neuron HH
    (h = +0.01), each split into 8 groups whose sizes (a seeded uniform split,
    at least one 64-particle wavefront each) and directions (HH always
    forward) are drawn from ``default_rng(20150501 + 4)``.  Returns one
    Workload per system whose groups are those slices; 200 steps per frame."""
    rng = np.random.default_rng(SEED_BASE + seed_index)
    totals = [(WILSON_COWAN, int(3_000_000 * scale)), (LORENZ, int(2_000_000 * scale)),
              (HH_RING, int(500_000 * scale))]
    out = []
    for sysid, total in totals:
        ngroups = 8
        w = rng.uniform(0.0, 1.0, ngroups) + 0.25
        sizes = np.maximum(64, np.floor(total * w / w.sum()).astype(np.int64))
        sizes[-1] = max(64, total - int(sizes[:-1].sum()))
        signs = rng.choice([-1.0, 1.0], ngroups) if sysid != HH_RING else np.ones(ngroups)
        order = np.argsort(-signs, kind="stable")  # forward groups first
        if sysid == WILSON_COWAN:
            groups = [Group(int(sizes[i]), 0.01 * signs[i], WC_BOX, [(-2.0, 4.0)]) for i in order]
            out.append(Workload("mixed_wc", seed_index, WILSON_COWAN, 2, list(WC_PARAMS), groups,
                                200, pp_slot=[8], prec="fp32_kahan"))
        elif sysid == LORENZ:
            groups = [Group(int(sizes[i]), 0.005 * signs[i], LORENZ_BOX) for i in order]
            out.append(Workload("mixed_lorenz", seed_index, LORENZ, 3, list(LORENZ_PARAMS),
                                groups, 200, prec="fp32_kahan"))
        else:
            groups = [Group(int(sizes[i]), 0.01, HH_NEURON_BOX * 3, [0.5, 10.0]) for i in order]
            out.append(Workload("mixed_hh", seed_index, HH_RING, 15, list(HH_PARAMS), groups,
                                200, pp_slot=[8, 7], prec="fp32_kahan"))
    return out


def generate_mixed(ws: List[Workload], seed_index: int = 4) -> List[Ensemble]:
    """Draw the ensembles of the mixed batch from one generator, system by
    system, group by group, with the same per-group recipe as ``generate``."""
    rng = np.random.default_rng(SEED_BASE + 100 + seed_index)
    out = []
    for w in ws:
        n = w.n
        state = np.empty((w.dim, n))
        npp = len(w.pp_slot)
        pp = np.empty((npp, n)) if npp else None
        offsets, counts, dts = [], [], []
        off = 0
        for g in w.groups:
            for d, (lo, hi) in enumerate(g.box):
                state[d, off:off + g.n] = rng.uniform(lo, hi, g.n)
            for k, spec in enumerate(g.pp):
                pp[k, off:off + g.n] = (rng.uniform(spec[0], spec[1], g.n)
                                        if isinstance(spec, tuple) else float(spec))
            offsets.append(off)
            counts.append(g.n)
            dts.append(g.dt)
            off += g.n
        out.append(Ensemble(w, state, pp, offsets, counts, dts))
    return out


def random_state(seed: int, dim: int, n: int, box) -> np.ndarray:
    """Uniform points in a box, for small test cases."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(lo, hi, n) for lo, hi in box])
