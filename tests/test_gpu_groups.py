"""GPU tests of the ragged batch (several particle groups with different
systems, steps and directions in one persistent launch), the autotuner and a
captured frame loop (integrate all groups, then project), replayed."""
import numpy as np
import pytest

from helpers import api, to_dev, to_host
from paper_1505_00344_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def A():
    return api()


SYS = {I.WILSON_COWAN: ("wilson_cowan", 2), I.LORENZ: ("lorenz", 3), I.HH_RING: ("hh_ring", 15)}


def build(A, scale, dtype, kahan):
    ws = I.mixed_batch(scale)
    ens = I.generate_mixed(ws)
    out = []
    for w, e in zip(ws, ens):
        name, dim = SYS[w.system]
        sysobj = A.System(name, dim, w.params)
        st = to_dev(e.state, dtype)
        pp = None if e.pparams is None else to_dev(e.pparams, dtype)
        comp = torch.zeros_like(st) if kahan else None
        out.append(dict(w=w, e=e, sys=sysobj, st=st, pp=pp, comp=comp))
    return out


def specs(A, B, prec):
    sp = []
    for b in B:
        for off, n, dt in zip(b["e"].offsets, b["e"].counts, b["e"].dts):
            bt = A.make_batch(b["st"], n, b["pp"], b["w"].pp_slot, b["comp"], prec, off)
            sp.append((b["sys"], bt, dt))
    return sp


def snapshot(B):
    torch.cuda.synchronize()
    return [(to_host(b["st"]).copy(), None if b["comp"] is None else to_host(b["comp"]).copy()) for b in B]


@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32", "fp64"])
@pytest.mark.parametrize("tuning", [None, (37, 2, 128), (200, 4, 256), (10, 1, 64)])
def test_batch_equals_per_group_calls(A, prec, tuning):
    dtype = torch.float64 if prec == "fp64" else torch.float32
    kahan = prec == "fp32_kahan"
    B1 = build(A, 0.002, dtype, kahan)
    B2 = build(A, 0.002, dtype, kahan)
    sp = specs(A, B1, prec)
    assert len(sp) == 24
    groups = A.make_groups(sp)
    A.integrate_groups(groups, 200, tuning=tuning)
    for b in B2:
        for off, n, dt in zip(b["e"].offsets, b["e"].counts, b["e"].dts):
            A.integrate(b["sys"], b["st"], dt, 200, n=n, offset=off, pparams=b["pp"], pp_slot=b["w"].pp_slot,
                        comp=b["comp"], prec=prec)
    s1, s2 = snapshot(B1), snapshot(B2)
    for (a, ca), (b, cb) in zip(s1, s2):
        assert np.array_equal(a, b, equal_nan=True)
        if kahan:
            assert np.array_equal(ca, cb, equal_nan=True)


def test_batch_fp64_lorenz_groups_match_oracle(A, ora):
    B = build(A, 0.001, torch.float64, False)
    A.integrate_groups(A.make_groups(specs(A, B, "fp64")), 150)
    st = snapshot(B)
    for b, (got, _) in zip(B, st):
        if b["w"].system != I.LORENZ:
            continue
        e = b["e"]
        for off, n, dt in zip(e.offsets, e.counts, e.dts):
            ref = ora.rk4(ora.LORENZ, b["w"].params, e.state[:, off:off + n], dt, 150)
            g = got[:, off:off + n]
            fin = np.all(np.isfinite(ref), axis=0)
            assert np.array_equal(np.all(np.isfinite(g), axis=0), fin)
            assert np.array_equal(g[:, fin], ref[:, fin])


def test_autotune_picks_valid_shape_and_leaves_state(A, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FF_AUTOTUNE_CACHE", str(cache))
    B = build(A, 0.002, torch.float32, True)
    before = snapshot(B)
    groups = A.make_groups(specs(A, B, "fp32_kahan"))
    t = A.autotune(groups, 200)
    # the new choice is appended to the cache file
    line = cache.read_text().split("\n")[0].split()
    assert line[0].startswith("200|") and len(line[0].split("|")) == 25
    assert [int(v) for v in line[1:]] == [t.steps_per_launch, t.particles_per_thread, t.block]
    assert 10 <= t.steps_per_launch <= 200 and t.particles_per_thread in (1, 2, 4) and t.block in (128, 256)
    after = snapshot(B)
    for (a, ca), (b, cb) in zip(before, after):
        assert np.array_equal(a, b, equal_nan=True) and np.array_equal(ca, cb, equal_nan=True)
    t2 = A.autotune(groups, 200)  # cached
    assert (t2.steps_per_launch, t2.particles_per_thread, t2.block) == (t.steps_per_launch, t.particles_per_thread, t.block)
    # without a tuning the batch takes the cached choice; still bitwise per-group
    A.integrate_groups(groups, 200)
    B2 = build(A, 0.002, torch.float32, True)
    for b in B2:
        for off, n, dt in zip(b["e"].offsets, b["e"].counts, b["e"].dts):
            A.integrate(b["sys"], b["st"], dt, 200, n=n, offset=off, pparams=b["pp"], pp_slot=b["w"].pp_slot,
                        comp=b["comp"], prec="fp32_kahan")
    for (a, ca), (b, cb) in zip(snapshot(B), snapshot(B2)):
        assert np.array_equal(a, b, equal_nan=True) and np.array_equal(ca, cb, equal_nan=True)


def test_captured_frame_loop_replays_match_eager(A):
    """One frame = all groups advanced 50 steps (persistent launch) then the
    (E, I) density of the Wilson-Cowan particles; captured once, replayed;
    every replay is checked against the same frame run eagerly."""
    Bg = build(A, 0.002, torch.float32, True)
    Be = build(A, 0.002, torch.float32, True)
    wc_g = next(b for b in Bg if b["w"].system == I.WILSON_COWAN)
    wc_e = next(b for b in Be if b["w"].system == I.WILSON_COWAN)
    groups_g = A.make_groups(specs(A, Bg, "fp32_kahan"))
    groups_e = A.make_groups(specs(A, Be, "fp32_kahan"))
    n_wc = wc_g["st"].shape[1]
    gws = torch.empty(A.groups_workspace_size(len(groups_g)), dtype=torch.uint8, device="cuda:0")
    hws = torch.empty(max(A.histogram_workspace_size(n_wc, 256, 256), 1), dtype=torch.uint8, device="cuda:0")
    hist_g = torch.zeros((256, 256), dtype=torch.int32, device="cuda:0")
    drop_g = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    tuning = (25, 1, 256)

    def frame(groups, wc, hist, drop, ws_g, ws_h):
        A.integrate_groups(groups, 50, tuning=tuning, workspace=ws_g)
        A.project_histogram(wc["sys"], wc["st"], 0, 1, (0.0, 1.0), (0.0, 1.0), 256, 256, hist=hist, n_dropped=drop,
                            workspace=ws_h)

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        frame(groups_g, wc_g, hist_g, drop_g, gws, hws)
    torch.cuda.synchronize()
    # capturing does not execute: both ensembles still hold the initial state
    for rep in range(4):
        g.replay()
        A.integrate_groups(groups_e, 50, tuning=tuning)
        he, de = A.project_histogram(wc_e["sys"], wc_e["st"], 0, 1, (0.0, 1.0), (0.0, 1.0), 256, 256)
        torch.cuda.synchronize()
        for bg, be in zip(Bg, Be):
            assert np.array_equal(to_host(bg["st"]), to_host(be["st"]), equal_nan=True), rep
        assert torch.equal(hist_g, he) and int(drop_g.item()) == int(de.item()), rep
