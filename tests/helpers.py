"""Helpers shared by the tests (no arithmetic of the method here)."""
import json
import os

import numpy as np

DEV = "cuda:0"


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    """A fixture of printed or published values from tests/golden/ (JSON with
    a `citation` field)."""
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


def record(name, **values):
    """Append measured error quantiles to the file named by FF_TEST_RECORD
    (if set), one JSON object per line."""
    path = os.environ.get("FF_TEST_RECORD")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps({"case": name, **values}) + "\n")


def api():
    from paper_1505_00344_amd import api as A
    A._ffi.lib()
    return A


def to_dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def to_host(t):
    return t.detach().cpu().numpy()


def mixed_error(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.linalg.norm(x - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1.0)


def quantiles(e):
    e = np.asarray(e)
    return dict(median=float(np.median(e)), p99=float(np.quantile(e, 0.99)), max=float(e.max()))


def f32_inputs(x):
    """Round an FP64 input array to FP32 and back (exact), so that FP32 and
    FP64 runs start from the same values."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def finite_cols(x):
    return np.all(np.isfinite(x), axis=0)
