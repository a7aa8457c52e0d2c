"""MI355X-native hot path of "Fireflies" (arXiv:1505.00344): fused RK4 over
millions of independent particles, 2D density projection, discrete adjoint and
ragged batches, as HIP kernels for gfx950 behind the C ABI of
``include/fireflies.h`` (``libfireflies.so``).

The Python layer is marshalling only (see ``api``); ``inputs`` holds the
seeded synthetic workloads.  Importing the package does not load the library;
the first call does, and fails loudly if it has not been built.
"""
from . import inputs  # noqa: F401

__all__ = ["api", "inputs", "autograd"]


def __getattr__(name):
    if name in ("api", "autograd"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
