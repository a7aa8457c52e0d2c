"""Host checks of bench.py that need no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=300, cwd=ROOT)
    assert out.returncode == 2
    assert "one GPU" in json.loads(out.stdout.strip().splitlines()[-1])["error"]
    assert "--gpus 1" in out.stderr


def test_flop_counts_per_adjoint_step_add_up():
    sys.path.insert(0, ROOT)
    import bench
    # replayed forward step + 3 stage points (42) + 4 products (88) + weights (27) + 6
    for prec in ("fp32", "fp32_kahan", "fp64"):
        assert bench.ADJ_FLOP_PER_STEP[prec] == bench.FLOP_PER_STEP["lorenz"][prec] + 42 + 88 + 27 + 6


def test_adjoint_replay_accounting_matches_the_library_tape():
    """bench.adj_replay_extra_flop assumes the tape lengths of ADJ_TAPE; the
    library's workspace (one sub-checkpoint per tape) shows the ones it uses."""
    sys.path.insert(0, ROOT)
    import ctypes
    import bench
    from paper_1505_00344_amd import _ffi, api as A
    L = _ffi.lib()
    s = A.System("lorenz", 3, [10.0, 28.0, 8 / 3])

    def size(prec, K):
        b = _ffi.Batch()
        b.prec, b.state, b.n, b.ld = prec, 4096, 1024, 1024
        out = ctypes.c_size_t()
        assert L.ff_adjoint_workspace_size(s.handle, ctypes.byref(b), K, K, ctypes.byref(out)) == 0
        return out.value

    for name, prec in (("fp32", _ffi.FF_FP32), ("fp32_kahan", _ffi.FF_FP32_KAHAN), ("fp64", _ffi.FF_FP64)):
        T = bench.ADJ_TAPE[name]
        st = 3 * 1024 * (8 if prec == _ffi.FF_FP64 else 4) * (2 if prec == _ffi.FF_FP32_KAHAN else 1)
        # one segment of K steps: K = T needs one sub-checkpoint, K = T + 1 two
        assert size(prec, T + 1) - size(prec, T) == st, name
    # K = 50: 50 - ceil(50/T) more forward steps and ceil(50/T) stage-point sets per segment
    assert abs(bench.adj_replay_extra_flop("fp32", 50) - ((43 * 68 + 7 * 42) / 50 - 42)) < 1e-12
    assert abs(bench.adj_replay_extra_flop("fp32_kahan", 50) - ((43 * 77 + 7 * 42) / 50 - 42)) < 1e-12
    assert abs(bench.adj_replay_extra_flop("fp64", 50) - ((37 * 68 + 13 * 42) / 50 - 42)) < 1e-12


def test_traffic_is_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    # the committed counters belong to the committed kernel sources
    traffic, source = bench.measured_traffic()
    assert traffic is not None and 0.99 < traffic / (2097152 * 36) < 1.05, (traffic, source)
    # any change of those sources withdraws the figure
    f = tmp_path / "changed.h"
    f.write_text("// not the measured kernel\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", bench.KERNEL_SOURCES + [str(f)])
    assert bench.measured_traffic()[0] is None
