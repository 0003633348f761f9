"""MI355X-native Wilson twisted-mass Dirac operator and solvers (arXiv:1311.4462).

The compute path is libtm.so (HIP kernels for gfx950 behind the C ABI of
include/tm.h); ``api`` is its thin ctypes binding.  Import of ``api`` needs
torch; the library itself is loaded lazily and must have been built.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "api"]


def __getattr__(name):
    if name == "api":
        import importlib
        return importlib.import_module(".api", __name__)
    raise AttributeError(name)
