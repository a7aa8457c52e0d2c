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
