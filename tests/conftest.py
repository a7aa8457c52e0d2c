"""Shared pytest configuration.

Tests marked ``gpu`` need an MI355X and the built HIP library; everything else
runs on the CPU (the oracle's pins, host-side logic, and the C-ABI export
check).
"""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def ora():
    import oracle
    oracle.lib()
    return oracle


def mixed_error(x, ref):
    """Per-particle error ||x - ref||_2 / max(||ref||_2, 1) over the state
    components (columns are particles)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.linalg.norm(x - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1.0)
