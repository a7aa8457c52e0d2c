#!/usr/bin/env python3
"""Benchmark of the Fireflies hot path on one MI355X.

Workload (one "step" = one pass of the hot path over the ensemble):
  Wilson-Cowan dynamic bifurcation diagram, 4,194,304 particles (per-particle
  P ~ U[-2, 4], (E, I) ~ U[0, 1]^2), half integrated forward (h = +0.01) and
  half backward (h = -0.01), 1000 classical RK4 steps in the FP32
  Kahan-compensated precision, then the 1024 x 1024 (P, E) density grid.
  Inputs are resident in HBM before timing starts.

Prints one JSON line.  `value` is particle-RK4-steps/s of the whole step
(P * 1000 / step time).  `roofline` is for the dominant kernel (the fused
RK4 kernel): algorithmic FLOPs per launch / its average duration from HIP
events recorded on the stream it runs on.  `fp64` is the same workload in
double precision, `adjoint` the adjoint particle-steps/s of the Lorenz
bifurcation workload (8M particles, 200 steps, checkpoints every 50) with
the reverse sweep's fraction of the VALU peak, `workloads` the other
configurations of the metric (Lorenz 8M bifurcation in FP32, FP32-Kahan and
FP64; the HH ring 1M in FP32-Kahan and FP64 with its adjoint; the ragged mixed
batch, persistent against per-group launches, and its captured frame's
p50/p99) and of the rest of the path (the reset rule, recording, the render
technique, expression systems, the one-step-per-launch pattern, the paper's
Table 1 single-step times), and `cpu_baseline` times the CPU oracle (FP64,
all host threads) on a bounded sample of the ensemble.  --extended adds the
Lorenz 8M adjoint in every precision (with --only: one workload alone).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp64]
                  [--no-adjoint] [--no-workloads] [--extended [--only WORKLOAD]]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work per particle-step (counted from the canonical formulas;
# exp and a division each count as one operation, a fused multiply-add as 2):
#   Wilson-Cowan RHS per component: 2 fma + sub + mul + exp + add + div + sub
#   = 10 -> 20 per evaluation (16 FLOP + 2 exp + 2 div), 4 evaluations = 80;
#   stage points 3 x 2 fma = 12; combination per component add + fma + add +
#   fma = 6 -> 12.  Plain: 104.  Kahan update replaces the final fma (2) by
#   mul, sub, add, sub, sub (5): +3 per component -> 110.
#   Lorenz RHS: fx sub + mul (2), fy sub + fma (3), fz mul + fma (3) = 8,
#   x4 = 32; stages 9 fma = 18; combination 3 x 6 = 18.  Plain 68, Kahan 77.
#   Three-neuron HH ring, per neuron and evaluation: 67 (7 exp/expm1 and 4
#   divisions counted once each), plus 1 for 1/C: 202 per evaluation, x4 =
#   808; stages 15 fma = 90; combination 15 x 6 = 90.  Plain 988, Kahan 1033.
FLOP_PER_STEP = {"wilson_cowan": {"fp32": 104, "fp32_kahan": 110, "fp64": 104},
                 "lorenz": {"fp32": 68, "fp32_kahan": 77, "fp64": 68},
                 "hh_ring": {"fp32": 988, "fp32_kahan": 1033, "fp64": 988}}
PEAK_TFLOPS = {"fp32": 157.3, "fp32_kahan": 157.3, "fp64": 78.6}
HBM_PEAK_TBS = 8.0
# One Lorenz adjoint step with checkpoints (same counting): the forward step
# replayed from the checkpoint (68, or 77 compensated), the three stage points
# (3 right-hand sides + 9 fma = 42), four products J(y_s)^T abar_s (12 with
# sigma*a0 shared) with their parameter part (7) summed into g (3): 4 x 22 = 88,
# the stage weights abar_{s-1} = fma(w, g_s, w' lam) (3 x 9 = 27), a = h/6 lam
# (3) and lam += g (3): 68 + 163 = 231.  The kernel also replays every
# sub-block of its register tape (T states: 8 in single precision, 4 in
# double), keeping the stage points it computes there, so per segment of K
# steps it executes K - ceil(K/T) more forward steps and ceil(K/T) stage-point
# sets in place of the K stage-point sets counted above; the difference is
# counted apart (adj_replay_extra_flop).
ADJ_FLOP_PER_STEP = {"fp32": 231, "fp32_kahan": 240, "fp64": 231}
ADJ_TAPE = {"fp32": 8, "fp32_kahan": 8, "fp64": 4}
ADJ_STAGE_FLOP = 42


def adj_replay_extra_flop(prec, K):
    """Executed FLOP per adjoint step beyond ADJ_FLOP_PER_STEP (Lorenz)."""
    nsub = -(-K // ADJ_TAPE[prec])
    fwd = FLOP_PER_STEP["lorenz"][prec]
    return ((K - nsub) * fwd + nsub * ADJ_STAGE_FLOP) / K - ADJ_STAGE_FLOP
# Sources that define the dominant kernel and its launch shape (ff_api.hip
# holds the default tuning); the HBM traffic measured with rocprofv3 counters
# is reported only while their hash matches the one recorded next to the
# counters in profiles/.
KERNEL_SOURCES = ["paper_1505_00344_amd/csrc/ff_rhs.h", "paper_1505_00344_amd/csrc/ff_math.h",
                  "paper_1505_00344_amd/csrc/ff_kernel.h", "paper_1505_00344_amd/csrc/ff_rng.h",
                  "paper_1505_00344_amd/csrc/ff_rk4.h", "paper_1505_00344_amd/csrc/ff_internal.h",
                  "paper_1505_00344_amd/csrc/k_rk4_wc.hip", "paper_1505_00344_amd/csrc/ff_api.hip",
                  "paper_1505_00344_amd/build.py"]
COUNTERS_FILE = "profiles/wc4m_fp32kahan_hbm_counters.md"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """(bytes per launch, note) from the committed counter summary, or (None,
    reason) when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, COUNTERS_FILE)
    if not os.path.exists(path):
        return None, "no counter summary"
    vals = {}
    for line in open(path):
        if line.startswith("source_hash:") or line.startswith("traffic_bytes_per_launch:"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash():
        return None, "kernel changed since the counters were taken"
    return float(vals["traffic_bytes_per_launch"]), COUNTERS_FILE


METRIC = "particle-RK4-steps/s (FP32-comp vs FP64) + % VALU peak; adjoint steps/s"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--particles", type=int, default=4 * 1024 * 1024)
    ap.add_argument("--rk4-steps", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint measurement (lorenz_8m)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU work for the baseline (three timed runs of a third each)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the other configurations and parts of the path (the `workloads` object)")
    ap.add_argument("--extended", action="store_true",
                    help="also measure the Lorenz 8M adjoint in every precision, with the reset rule, recording, "
                         "render technique, expression systems, one step per launch and Table 1 again")
    ap.add_argument("--only", default=None,
                    help="with --extended: measure only this workload (lorenz_8m, hh_ring_1m, mixed_batch, "
                         "reset_record_render_expressions, one_step_per_launch, table1_single_step)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (for HBM counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}), flush=True)
        print("bench.py: only --gpus 1 is supported (the method shards trivially over particles; "
              "the multi-GPU design is documented but not built)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1505_00344_amd import api as A
    from paper_1505_00344_amd import inputs as I

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    w = I.wilson_cowan_4m(n=args.particles)
    w.nsteps = args.rk4_steps
    e = I.generate(w)
    hs = w.hist
    sysobj = A.System("wilson_cowan", 2, w.params)
    stream = torch.cuda.current_stream()

    def setup(prec, rounded=False):
        # rounded: the state, the per-particle parameters and the step rounded
        # to single precision first, so that an FP64 run starts from exactly
        # the values a single-precision run sees
        dt_ = torch.float64 if prec == "fp64" else torch.float32
        src_st, src_pp, dts = e.state, e.pparams, list(e.dts)
        if rounded:
            src_st = e.state.astype(np.float32).astype(np.float64)
            src_pp = e.pparams.astype(np.float32).astype(np.float64)
            dts = [float(np.float32(d)) for d in e.dts]
        st = torch.as_tensor(src_st, dtype=dt_, device=dev).contiguous()
        pp = torch.as_tensor(src_pp, dtype=dt_, device=dev).contiguous()
        comp = torch.zeros_like(st) if prec == "fp32_kahan" else None
        hist = torch.zeros((hs["ny"], hs["nx"]), dtype=torch.int32, device=dev)
        drop = torch.zeros(1, dtype=torch.int64, device=dev)
        ws = torch.empty(max(A.histogram_workspace_size(w.n, hs["nx"], hs["ny"]), 1), dtype=torch.uint8, device=dev)
        return dict(st=st, pp=pp, comp=comp, hist=hist, drop=drop, ws=ws, prec=prec, dts=dts)

    def one_step(B, ev=None):
        # forward group, backward group, then the density grid
        for k, (off, n, dt) in enumerate(zip(e.offsets, e.counts, B["dts"])):
            if ev is not None:
                ev[k][0].record(stream)
            A.integrate(sysobj, B["st"], dt, w.nsteps, n=n, offset=off, pparams=B["pp"], pp_slot=w.pp_slot,
                        comp=B["comp"], prec=B["prec"])
            if ev is not None:
                ev[k][1].record(stream)
        A.project_histogram(sysobj, B["st"], hs["axis_x"], hs["axis_y"], hs["x_range"], hs["y_range"], hs["nx"],
                            hs["ny"], hist=B["hist"], n_dropped=B["drop"], pparams=B["pp"], pp_slot=w.pp_slot,
                            prec="fp32" if B["prec"] != "fp64" else "fp64", workspace=B["ws"])

    def measure(prec, steps, warmup):
        B = setup(prec)
        for _ in range(warmup):
            one_step(B)
        torch.cuda.synchronize()
        evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in e.counts]
               for _ in range(steps)]
        t0 = time.perf_counter()
        for s in range(steps):
            one_step(B, evs[s])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kern_ms = [ev[0].elapsed_time(ev[1]) for step in evs for ev in step]
        return wall, kern_ms, B

    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    wall, kern_ms, B = measure("fp32_kahan", args.steps, args.warmup)
    ms_per_step = wall / args.steps * 1e3
    psteps = w.n * w.nsteps
    value = psteps / (wall / args.steps)
    avg_launch_ms = float(np.mean(kern_ms))
    particles_per_launch = float(np.mean(e.counts))
    flop_launch = particles_per_launch * w.nsteps * FLOP_PER_STEP["wilson_cowan"]["fp32_kahan"]
    achieved = flop_launch / (avg_launch_ms * 1e-3) / 1e12
    traffic, traffic_src = measured_traffic()
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["fp32_kahan"], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_TFLOPS["fp32_kahan"], 4), "traffic": traffic,
            "traffic_unit": "bytes per launch (HBM read + write, calibrated rocprofv3 FETCH_SIZE/WRITE_SIZE)",
            "traffic_source": traffic_src,
            "algorithmic_bytes_per_launch": particles_per_launch * 36,
            "kernel": "k_rk4<WilsonCowan<float>, float, Kahan, PPT 2>", "avg_launch_ms": round(avg_launch_ms, 4),
            "flop_per_particle_step": FLOP_PER_STEP["wilson_cowan"]["fp32_kahan"],
            "particles_per_launch": particles_per_launch, "steps_per_launch": w.nsteps}
    out = {
        "metric": METRIC, "value": value, "unit": "particle-RK4-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"wilson_cowan_4m: {w.n} particles (half h=+0.01, half h=-0.01), per-particle "
                               f"P~U[-2,4], {w.nsteps} RK4 steps FP32-Kahan + {hs['nx']}x{hs['ny']} (P,E) grid",
                   "precision": "fp32_kahan", "particles": w.n, "rk4_steps": w.nsteps},
        "roofline": roof,
    }
    # FP64 beside it (same workload), reported, not the headline value
    if not args.no_fp64:
        # same number of passes as the FP32 run, so both states are compared
        # after the same number of steps
        wall64, kern64, B64 = measure("fp64", args.steps, args.warmup)
        v64 = psteps / (wall64 / args.steps)
        a64 = particles_per_launch * w.nsteps * FLOP_PER_STEP["wilson_cowan"]["fp64"] / (np.mean(kern64) * 1e-3) / 1e12
        out["fp64"] = {"value": v64, "unit": "particle-RK4-steps/s", "avg_launch_ms": round(float(np.mean(kern64)), 4),
                       "achieved_tflops": round(a64, 3), "peak": PEAK_TFLOPS["fp64"],
                       "frac": round(a64 / PEAK_TFLOPS["fp64"], 4)}
        # accuracy: one pass (1000 RK4 steps) of FP32-comp against FP64, per
        # group, both from the single-precision inputs and step (the FP64 run
        # starts from exactly the values the FP32 run sees), so the figure is
        # the arithmetic's error alone; the effect of rounding the inputs is
        # reported apart (FP64 from the rounded vs the original inputs)
        del B64
        A32, A64, A64o = setup("fp32_kahan", rounded=True), setup("fp64", rounded=True), setup("fp64")
        one_step(A32)
        one_step(A64)
        one_step(A64o)
        torch.cuda.synchronize()

        def err_q(a, ref, idx):
            a = a[:, idx].double().cpu().numpy()
            r = ref[:, idx].cpu().numpy()
            err = np.linalg.norm(a - r, axis=0) / np.maximum(np.linalg.norm(r, axis=0), 1.0)
            fin = np.isfinite(err)
            return {"median": float(np.median(err[fin])), "p99": float(np.quantile(err[fin], 0.99)),
                    "max": float(err[fin].max()), "sample": int(len(idx)), "non_finite": int((~fin).sum())}

        acc, inp = {}, {}
        for name, off, n in zip(("forward", "backward"), e.offsets, e.counts):
            idx = np.arange(off, off + n, max(1, n // 32768))
            acc[name] = err_q(A32["st"], A64["st"], idx)
            inp[name] = err_q(A64["st"], A64o["st"], idx)
        acc["note"] = ("per particle ||x32 - x64|| / max(||x64||, 1) after %d RK4 steps; the FP64 run starts "
                       "from the FP32-rounded state, per-particle P and step" % w.nsteps)
        inp["note"] = "FP64 from the FP32-rounded inputs and step vs FP64 from the original ones, same metric"
        out["fp32_kahan_vs_fp64"] = acc
        out["fp64_input_rounding"] = inp
        del A32, A64, A64o
    del B
    torch.cuda.empty_cache()
    if not args.no_adjoint:
        out["adjoint"] = adjoint_line(A, I, torch)
    if not args.no_workloads:
        # the other configurations of the metric, measured in the same run
        out["workloads"] = extended(A, I, torch, np, names=DEFAULT_WORKLOADS, lorenz_adjoint_all=False)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(e, w, args.cpu_seconds)
    if args.extended:
        torch.cuda.empty_cache()
        names = EXTENDED_WORKLOADS if args.only is None else (args.only,)
        out["extended"] = extended(A, I, torch, np, names=names)
    print(json.dumps(out), flush=True)
    return 0


def _time_stream(torch, fn, reps=1):
    """Median over reps of fn()'s duration, HIP events on the current stream."""
    st = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def lorenz_adjoint(A, torch, w, sysobj, st0, pp, prec):
    """Adjoint of mean z(T) w.r.t. each particle's r on lorenz_8m (200 steps,
    checkpoints every 50): checkpointed forward pass, then the reverse sweep."""
    dev = st0.device
    adj = w.adjoint
    st = st0.clone()
    comp = torch.zeros_like(st) if prec == "fp32_kahan" else None
    nb = A.adjoint_workspace_size(sysobj, st, adj["nsteps"], adj["K"], pparams=pp, pp_slot=w.pp_slot, comp=comp,
                                  prec=prec)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    lam = torch.zeros_like(st)
    mu = torch.empty_like(pp)
    mug = torch.empty(3, dtype=torch.float64, device=dev)
    # median of three: the first call of a kernel in the process also loads it
    fwd = _time_stream(torch, lambda: A.integrate_checkpointed(sysobj, st, 0.005, adj["nsteps"], adj["K"], ws,
                                                                pparams=pp, pp_slot=w.pp_slot, comp=comp, prec=prec),
                       reps=3)

    def back():
        lam.zero_()
        lam[2].fill_(1.0 / w.n)
        A.adjoint(sysobj, st, 0.005, adj["nsteps"], adj["K"], ws, lam, mu=mu, mu_global=mug, pparams=pp,
                  pp_slot=w.pp_slot, prec=prec)
    back()
    bwd = _time_stream(torch, back, reps=3)
    rate = w.n * adj["nsteps"] / (bwd * 1e-3)
    tf = rate * ADJ_FLOP_PER_STEP[prec] / 1e12
    tf_exec = rate * (ADJ_FLOP_PER_STEP[prec] + adj_replay_extra_flop(prec, adj["K"])) / 1e12
    return {"reverse_ms": bwd, "forward_ckpt_ms": fwd,
            "adjoint_steps_per_s": rate,
            "adjoint_steps_per_s_incl_forward": w.n * adj["nsteps"] / ((bwd + fwd) * 1e-3),
            "flop_per_adjoint_step": ADJ_FLOP_PER_STEP[prec], "achieved_tflops": round(tf, 3),
            "peak": PEAK_TFLOPS[prec], "frac": round(tf / PEAK_TFLOPS[prec], 4),
            "frac_executed_incl_tape_replay": round(tf_exec / PEAK_TFLOPS[prec], 4)}


def adjoint_line(A, I, torch):
    """The metric's adjoint part on the workload that defines one (lorenz_8m:
    8,388,608 particles, d(mean z(T))/d r_i over 200 steps, K = 50), in FP64
    and FP32-Kahan."""
    w = I.lorenz_8m()
    e = I.generate(w)
    sysobj = A.System("lorenz", 3, w.params)
    out = {"workload": "lorenz_8m: 8388608 particles, per-particle r~U[0,50], d(mean z(T))/d r_i, "
                       "200 RK4 steps, checkpoints every 50", "unit": "adjoint particle-steps/s"}
    for prec in ("fp64", "fp32_kahan"):
        dt_ = torch.float64 if prec == "fp64" else torch.float32
        st0 = torch.as_tensor(e.state, dtype=dt_, device="cuda:0")
        pp = torch.as_tensor(e.pparams, dtype=dt_, device="cuda:0").contiguous()
        out[prec] = lorenz_adjoint(A, torch, w, sysobj, st0, pp, prec)
        del st0, pp
    torch.cuda.empty_cache()
    return out


DEFAULT_WORKLOADS = ("lorenz_8m", "hh_ring_1m", "mixed_batch", "reset_record_render_expressions",
                     "one_step_per_launch", "table1_single_step")
EXTENDED_WORKLOADS = ("lorenz_8m", "reset_record_render_expressions", "one_step_per_launch", "table1_single_step")


def extended(A, I, torch, np, names, lorenz_adjoint_all=True):
    """Throughput of the other workloads (each run after a warm-up).  The
    Lorenz 8M adjoint is measured per precision only with
    lorenz_adjoint_all (the headline line carries FP64 and FP32-Kahan)."""
    dev = torch.device("cuda:0")
    res = {}

    def lorenz8m():
        w = I.lorenz_8m()
        e = I.generate(w)
        sysobj = A.System("lorenz", 3, w.params)
        r = {}
        for prec in ("fp32", "fp32_kahan", "fp64"):
            dt_ = torch.float64 if prec == "fp64" else torch.float32
            st0 = torch.as_tensor(e.state, dtype=dt_, device=dev)
            pp = torch.as_tensor(e.pparams, dtype=dt_, device=dev).contiguous()
            st = st0.clone()
            comp = torch.zeros_like(st) if prec == "fp32_kahan" else None
            A.integrate(sysobj, st, 0.005, 20, pparams=pp, pp_slot=w.pp_slot, comp=comp, prec=prec)
            ms = _time_stream(torch, lambda: A.integrate(sysobj, st, 0.005, w.nsteps, pparams=pp, pp_slot=w.pp_slot,
                                                          comp=comp, prec=prec), reps=3)
            ps = w.n * w.nsteps / (ms * 1e-3)
            tf = ps * FLOP_PER_STEP["lorenz"][prec] / 1e12
            r[prec] = {"particle_steps_per_s": ps, "ms": ms, "tflops": tf, "frac_of_peak": tf / PEAK_TFLOPS[prec]}
            if lorenz_adjoint_all:
                r[prec]["adjoint"] = lorenz_adjoint(A, torch, w, sysobj, st0, pp, prec)
            del st, st0, pp, comp
        return r

    def hh1m():
        w = I.hh_ring_1m()
        e = I.generate(w)
        sysobj = A.System("hh_ring", 15, w.params)
        r = {}
        for prec in ("fp32_kahan", "fp64"):
            dt_ = torch.float64 if prec == "fp64" else torch.float32
            st0 = torch.as_tensor(e.state, dtype=dt_, device=dev)
            pp = torch.as_tensor(e.pparams, dtype=dt_, device=dev).contiguous()
            st = st0.clone()
            comp = torch.zeros_like(st) if prec == "fp32_kahan" else None
            A.integrate(sysobj, st, 0.01, 10, pparams=pp, pp_slot=w.pp_slot, comp=comp, prec=prec)
            ms = _time_stream(torch, lambda: A.integrate(sysobj, st, 0.01, w.nsteps, pparams=pp, pp_slot=w.pp_slot,
                                                          comp=comp, prec=prec))
            ps = w.n * w.nsteps / (ms * 1e-3)
            tf = ps * FLOP_PER_STEP["hh_ring"][prec] / 1e12
            r[prec] = {"particle_steps_per_s": ps, "ms": ms, "tflops": tf, "frac_of_peak": tf / PEAK_TFLOPS[prec]}
            adj = w.adjoint
            st = st0.clone()
            comp = torch.zeros_like(st) if prec == "fp32_kahan" else None
            nb = A.adjoint_workspace_size(sysobj, st, adj["nsteps"], adj["K"], pparams=pp, pp_slot=w.pp_slot, comp=comp,
                                          prec=prec)
            ws = torch.empty(nb, dtype=torch.uint8, device=dev)
            lam = torch.zeros_like(st)
            mu = torch.empty_like(pp)
            fwd = _time_stream(torch, lambda: A.integrate_checkpointed(sysobj, st, 0.01, adj["nsteps"], adj["K"], ws,
                                                                        pparams=pp, pp_slot=w.pp_slot, comp=comp,
                                                                        prec=prec))
            lam[0].fill_(1.0 / w.n)
            bwd = _time_stream(torch, lambda: A.adjoint(sysobj, st, 0.01, adj["nsteps"], adj["K"], ws, lam, mu=mu,
                                                        pparams=pp, pp_slot=w.pp_slot, prec=prec))
            r[prec]["adjoint"] = {"reverse_ms": bwd, "forward_ckpt_ms": fwd,
                                  "adjoint_steps_per_s": w.n * adj["nsteps"] / (bwd * 1e-3),
                                  "adjoint_steps_per_s_incl_forward": w.n * adj["nsteps"] / ((bwd + fwd) * 1e-3)}
            del st, st0, pp, comp, ws, lam, mu
        return r

    def mixed():
        ws_ = I.mixed_batch(1.0)
        ens = I.generate_mixed(ws_)
        names = {I.WILSON_COWAN: ("wilson_cowan", 2), I.LORENZ: ("lorenz", 3), I.HH_RING: ("hh_ring", 15)}
        objs, specs = [], []
        for w, e in zip(ws_, ens):
            nm, dim = names[w.system]
            sysobj = A.System(nm, dim, w.params)
            st = torch.as_tensor(e.state, dtype=torch.float32, device=dev).contiguous()
            pp = None if e.pparams is None else torch.as_tensor(e.pparams, dtype=torch.float32, device=dev).contiguous()
            comp = torch.zeros_like(st)
            objs.append((sysobj, st, pp, comp))
            for off, n, dt in zip(e.offsets, e.counts, e.dts):
                specs.append((sysobj, A.make_batch(st, n, pp, w.pp_slot, comp, "fp32_kahan", off), dt, w.pp_slot,
                              st, pp, comp, off, n))
        groups = A.make_groups([(s[0], s[1], s[2]) for s in specs])
        nsteps = 200
        t = A.autotune(groups, nsteps)
        tun = (t.steps_per_launch, t.particles_per_thread, t.block)
        gws = torch.empty(A.groups_workspace_size(len(groups)), dtype=torch.uint8, device=dev)
        A.integrate_groups(groups, nsteps, tuning=tun, workspace=gws)
        batched = _time_stream(torch, lambda: A.integrate_groups(groups, nsteps, tuning=tun, workspace=gws), reps=3)

        def separate():
            for s in specs:
                A.integrate(s[0], s[4], s[2], nsteps, n=s[8], offset=s[7], pparams=s[5], pp_slot=s[3], comp=s[6],
                            prec="fp32_kahan")
        separate()
        sep = _time_stream(torch, separate, reps=3)
        # frame loop: one captured graph per frame, replayed 100 times
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            A.integrate_groups(groups, nsteps, tuning=tun, workspace=gws)
        frames = []
        for _ in range(100):
            frames.append(_time_stream(torch, g.replay))
        ntot = sum(s[8] for s in specs)
        return {"particles": ntot, "groups": len(specs), "steps_per_frame": nsteps,
                "autotuned": {"steps_per_launch": tun[0], "particles_per_thread": tun[1], "block": tun[2]},
                "batched_ms": batched, "separate_ms": sep, "speedup_batched_vs_separate": sep / batched,
                "particle_steps_per_s_batched": ntot * nsteps / (batched * 1e-3),
                "frame_ms_p50": float(np.percentile(frames, 50)), "frame_ms_p99": float(np.percentile(frames, 99))}

    def reset_record_render_expressions():
        """Reset rule, trajectory recording, render technique and expression
        right-hand sides on the paper's large ensembles."""
        r = {}
        w = I.lorenz_8m()
        e = I.generate(w)
        n, steps = w.n, w.nsteps
        st0 = torch.as_tensor(e.state, dtype=torch.float32, device=dev)
        pp = torch.as_tensor(e.pparams, dtype=torch.float32, device=dev).contiguous()
        builtin = A.System("lorenz", 3, w.params)

        def rate(fn, reps=3):
            fn()
            ms = _time_stream(torch, fn, reps=reps)
            return {"ms": ms, "particle_steps_per_s": n * steps / (ms * 1e-3)}

        st, comp = st0.clone(), torch.zeros_like(st0)
        plain = rate(lambda: A.integrate(builtin, st, 0.005, steps, pparams=pp, pp_slot=w.pp_slot, comp=comp))
        r["lorenz_8m_fp32_kahan_plain"] = plain
        # the reset rule, backward in time (escaping particles redrawn in the initial-condition box)
        bounds = [(-60.0, 60.0), (-80.0, 80.0), (-30.0, 100.0)]
        age = torch.zeros(n, dtype=torch.int32, device=dev)
        nres = torch.zeros(n, dtype=torch.int32, device=dev)
        st, comp = st0.clone(), torch.zeros_like(st0)
        res = rate(lambda: A.integrate_reset(builtin, st, -0.005, steps, bounds=bounds, box=I.LORENZ_BOX, age=age,
                                             n_resets=nres, seed=1, max_age=400, pparams=pp, pp_slot=w.pp_slot,
                                             comp=comp))
        res["resets_per_particle_step"] = float(nres.double().sum().item()) / (4 * n * steps)
        r["reset_lorenz_8m_backward_fp32_kahan"] = res
        # trajectory recording: every 10th step of every 16th particle
        st, comp = st0.clone(), torch.zeros_like(st0)
        out = torch.empty((steps // 10, 3, (n + 15) // 16), dtype=torch.float32, device=dev)
        rec = rate(lambda: A.integrate_record(builtin, st, 0.005, steps, 10, 16, out=out, pparams=pp,
                                              pp_slot=w.pp_slot, comp=comp))
        rec["record_bytes"] = out.numel() * 4
        rec["slowdown_vs_plain"] = rec["ms"] / plain["ms"]
        r["record_lorenz_8m_every10_stride16"] = rec
        del out
        # the render technique: 8M particles drawn into a 1920 x 1080 frame, perspective camera
        f = 1.0 / np.tan(np.radians(60.0) / 2)
        aspect, near, far = 1920 / 1080, 1.0, 400.0
        proj = np.array([[f / aspect, 0, 0, 0], [0, f, 0, 0],
                         [0, 0, (far + near) / (near - far), 2 * far * near / (near - far)], [0, 0, -1, 0]])
        view = np.eye(4)
        view[:3, 3] = [0.0, -25.0, -120.0]
        view[:3, :3] = [[1, 0, 0], [0, 0, 1], [0, -1, 0]]  # look along +y with z up
        mvp = proj @ view
        img = torch.empty((1080, 1920, 3), dtype=torch.int32, device=dev)
        culled = torch.empty(1, dtype=torch.int64, device=dev)
        for radius in (0, 2):
            rws = torch.empty(max(A.render_workspace_size(n, 1920, 1080, radius), 1), dtype=torch.uint8, device=dev)

            def draw():
                A.render_image(builtin, st, (0, 1, 2), mvp, 1920, 1080, base=(0.2, 0.5, 1.0),
                               grad=[[0.01, 0, 0], [0, 0, 0], [0, 0, 0.01]], weight=0.05, radius=radius, img=img,
                               n_culled=culled, workspace=rws)
            draw()
            ms = _time_stream(torch, draw, reps=5)
            r[f"render_8m_1080p_radius{radius}"] = {"ms": ms, "particles_per_s": n / (ms * 1e-3),
                                                    "culled": int(culled.item()), "workspace_bytes": rws.numel()}
            del rws
        del img
        # the same systems given as expressions (compiled at run time)
        lorenz_expr = A.System.from_exprs(["p0*(x1-x0)", "fma(x0, p1-x2, -x1)", "fma(x0, x1, -(p2*x2))"], w.params)
        t0 = time.perf_counter()
        lorenz_expr.compile("fp32_kahan")
        compile_s = time.perf_counter() - t0
        st, comp = st0.clone(), torch.zeros_like(st0)
        ex = rate(lambda: A.integrate(lorenz_expr, st, 0.005, steps, pparams=pp, pp_slot=w.pp_slot, comp=comp))
        ex["vs_builtin"] = ex["particle_steps_per_s"] / plain["particle_steps_per_s"]
        ex["compile_s"] = compile_s
        r["expr_lorenz_8m_fp32_kahan"] = ex
        # adjoint of mean z(T) w.r.t. each r_i over 200 steps (K = 50), FP64: generated
        # vector-Jacobian products vs the built-in ones
        adj = {}
        x64 = torch.as_tensor(e.state, dtype=torch.float64, device=dev)
        p64 = torch.as_tensor(e.pparams, dtype=torch.float64, device=dev).contiguous()
        for name, sobj in (("builtin", builtin), ("expr", lorenz_expr)):
            xs = x64.clone()
            nb = A.adjoint_workspace_size(sobj, xs, 200, 50, pparams=p64, pp_slot=w.pp_slot)
            ws = torch.empty(nb, dtype=torch.uint8, device=dev)
            A.integrate_checkpointed(sobj, xs, 0.005, 200, 50, ws, pparams=p64, pp_slot=w.pp_slot)
            lam = torch.zeros_like(xs)
            mu = torch.empty_like(p64)

            def back():
                lam.zero_()
                lam[2].fill_(1.0 / n)
                A.adjoint(sobj, xs, 0.005, 200, 50, ws, lam, mu=mu, pparams=p64, pp_slot=w.pp_slot)
            back()
            ms = _time_stream(torch, back, reps=3)
            adj[name] = {"reverse_ms": ms, "adjoint_steps_per_s": n * 200 / (ms * 1e-3)}
            del ws, lam, mu, xs
        adj["expr_vs_builtin"] = adj["expr"]["adjoint_steps_per_s"] / adj["builtin"]["adjoint_steps_per_s"]
        r["expr_lorenz_8m_adjoint_fp64"] = adj
        del x64, p64
        del st, comp, st0, pp, age, nres
        wc = I.wilson_cowan_4m()
        ew = I.generate(wc)
        nf = ew.counts[0]
        wc_expr = A.System.from_exprs(["1/(1+exp(-(p4*(fma(p0, x0, fma(-p1, x1, p8)) - p5)))) - x0",
                                       "1/(1+exp(-(p6*(fma(p2, x0, fma(-p3, x1, p9)) - p7)))) - x1"], wc.params)
        wc_builtin = A.System("wilson_cowan", 2, wc.params)
        wc_fast = A.System.from_exprs(["1/(1+exp(-(p4*(fma(p0, x0, fma(-p1, x1, p8)) - p5)))) - x0",
                                       "1/(1+exp(-(p6*(fma(p2, x0, fma(-p3, x1, p9)) - p7)))) - x1"], wc.params,
                                      fast_f32=True)
        for prec in ("fp32_kahan", "fp64"):
            dt_ = torch.float64 if prec == "fp64" else torch.float32
            x = torch.as_tensor(ew.state[:, :nf], dtype=dt_, device=dev).contiguous()
            p_ = torch.as_tensor(ew.pparams[:, :nf], dtype=dt_, device=dev).contiguous()
            out_ = {}
            for name, sobj in (("builtin", wc_builtin), ("expr", wc_expr), ("expr_fast_f32", wc_fast)):
                if prec == "fp64" and name == "expr_fast_f32":
                    continue
                xs = x.clone()
                c_ = torch.zeros_like(xs) if prec == "fp32_kahan" else None

                def go():
                    A.integrate(sobj, xs, 0.01, wc.nsteps, pparams=p_, pp_slot=wc.pp_slot, comp=c_, prec=prec)
                go()
                ms = _time_stream(torch, go, reps=3)
                out_[name] = {"ms": ms, "particle_steps_per_s": nf * wc.nsteps / (ms * 1e-3)}
            out_["expr_vs_builtin"] = out_["expr"]["particle_steps_per_s"] / out_["builtin"]["particle_steps_per_s"]
            if "expr_fast_f32" in out_:
                out_["expr_fast_f32_vs_builtin"] = (out_["expr_fast_f32"]["particle_steps_per_s"] /
                                                    out_["builtin"]["particle_steps_per_s"])
            r[f"expr_wc_2m_forward_{prec}"] = out_
        return r

    def one_step_per_launch():
        """The paper's launch pattern (one RK4 step per kernel launch): each
        launch reads and writes the whole state, so it is bound by HBM.
        lorenz_8m in FP32: 3 state values read and written and r read, 28 B
        per particle-step, against the fused kernel on the same input."""
        w = I.lorenz_8m()
        e = I.generate(w)
        sysobj = A.System("lorenz", 3, w.params)
        st = torch.as_tensor(e.state, dtype=torch.float32, device=dev).contiguous()
        pp = torch.as_tensor(e.pparams, dtype=torch.float32, device=dev).contiguous()
        nl = 200
        r = {}
        for name, tun in (("one_step_per_launch", (1, 1, 256)), ("fused", None)):
            def go():
                A.integrate(sysobj, st, 0.005, nl, pparams=pp, pp_slot=w.pp_slot, tuning=tun, prec="fp32")
            go()
            ms = _time_stream(torch, go, reps=3)
            r[name] = {"ms_per_step": ms / nl, "particle_steps_per_s": w.n * nl / (ms * 1e-3)}
        bytes_per_launch = w.n * (2 * 3 * 4 + 4)
        tbs = bytes_per_launch / (r["one_step_per_launch"]["ms_per_step"] * 1e-3) / 1e12
        r["one_step_per_launch"].update({"bytes_per_launch": bytes_per_launch, "achieved_TB_per_s": tbs,
                                         "frac_of_hbm_peak": tbs / HBM_PEAK_TBS})
        r["fused_speedup"] = r["one_step_per_launch"]["ms_per_step"] / r["fused"]["ms_per_step"]
        return r

    def table1_single_step():
        """The paper's Table 1 timing on its own particle counts: the time to
        advance every particle by one RK4 step, averaged over 1000 steps, in
        single precision (the paper's).  The Wilson-Cowan pair stands in for
        the STN-GPe model (700k particles: half forward, half backward,
        per-particle P), Lorenz 3M (forward, per-particle r as in the
        bifurcation diagram), the three-neuron HH ring 500k.
        Each is timed launched once per step (the paper's pattern) and with
        the 1000 steps fused in one launch.  Context only: the paper's figures
        are for a GTX 460."""
        cases = [("wilson_cowan_700k", I.wilson_cowan_4m(n=700_000), "wilson_cowan", 2, 1.0),
                 ("lorenz_3m", I.lorenz_8m(n=3_000_000), "lorenz", 3, 3.0),
                 ("hh_ring3_500k", I.hh_ring_1m(n=500_000), "hh_ring", 15, 22.0)]
        out = {"precision": "fp32", "steps": 1000,
               "paper_gtx460_ms_per_step": {c[0]: c[4] for c in cases}}
        for name, w, nm, dim, _ in cases:
            e = I.generate(w)
            sysobj = A.System(nm, dim, w.params)
            st0 = torch.as_tensor(e.state, dtype=torch.float32, device=dev).contiguous()
            pp = None if e.pparams is None else torch.as_tensor(e.pparams, dtype=torch.float32,
                                                                 device=dev).contiguous()
            r = {"particles": w.n}
            for mode, tun in (("one_step_per_launch", (1, 1, 256)), ("fused", None)):
                st = st0.clone()

                def go():
                    for off, n, dt in zip(e.offsets, e.counts, e.dts):
                        A.integrate(sysobj, st, dt, 1000, n=n, offset=off, pparams=pp, pp_slot=w.pp_slot,
                                    tuning=tun, prec="fp32")
                go()
                st.copy_(st0)
                ms = _time_stream(torch, go, reps=3)
                r[mode] = {"ms_per_step": ms / 1000, "particle_steps_per_s": w.n * 1000 / (ms * 1e-3)}
                del st
            r["one_step_speedup_vs_paper"] = out["paper_gtx460_ms_per_step"][name] / r["one_step_per_launch"]["ms_per_step"]
            out[name] = r
            del st0, pp
        return out

    for name, fn in (("lorenz_8m", lorenz8m), ("hh_ring_1m", hh1m), ("mixed_batch", mixed),
                     ("reset_record_render_expressions", reset_record_render_expressions),
                     ("one_step_per_launch", one_step_per_launch), ("table1_single_step", table1_single_step)):
        if name not in names:
            continue
        try:
            res[name] = fn()
        except Exception as ex:  # report and continue with the next workload
            res[name] = {"error": repr(ex)}
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return res


def cpu_baseline(e, w, seconds):
    """Time the CPU oracle (FP64, OpenMP over particles, all host threads) on a
    bounded sample of the same ensemble: every k-th particle of each group."""
    import numpy as np

    import oracle

    oracle.lib()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)

    def run(m):
        t = 0.0
        for off, n, dt in zip(e.offsets, e.counts, e.dts):
            sel = np.arange(off, off + n)[:: max(1, n // m)][:m]
            x = e.state[:, sel]
            pp = e.pparams[:, sel]
            t0 = time.perf_counter()
            oracle.rk4(oracle.WILSON_COWAN, w.params, x, dt, w.nsteps, pp_slot=w.pp_slot, pparams=pp,
                       nthreads=threads)
            t += time.perf_counter() - t0
        return t

    # size the sample so that one timed run takes about seconds / 3, then
    # report the best of three runs of it
    m = 2048
    t = run(m)
    while t < seconds / 24 and m < min(e.counts):
        m = min(m * 4, min(e.counts))
        t = run(m)
    m_final = min(int(m * seconds / 3 / max(t, 1e-3)), min(e.counts))
    runs = [run(m_final) for _ in range(3)]
    t = min(runs)
    total = m_final * len(e.counts)
    # one thread, for comparison with the paper's single-core column (smaller
    # sample, also best of three)
    threads_all = threads
    threads = 1
    m1 = max(256, min(m_final, int(m_final * 0.5 / max(t * threads_all, 1e-3))))
    t1 = min(run(m1) for _ in range(3))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), model)
    except OSError:
        pass
    return {"value": total * w.nsteps / t, "unit": "particle-RK4-steps/s", "cores": threads_all, "kind": "oracle",
            "sample": f"{total} of {w.n} particles (every k-th of each group), {w.nsteps} steps, FP64; "
                      f"best of 3 runs: {t:.2f} s (runs {', '.join(f'{r:.2f}' for r in runs)} s)",
            "value_1_thread": m1 * len(e.counts) * w.nsteps / t1,
            "host": f"{model}; {os.cpu_count()} logical CPUs, {len(os.sched_getaffinity(0))} usable"}


if __name__ == "__main__":
    sys.exit(main())
