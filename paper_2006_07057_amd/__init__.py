"""MI355X-native linear-time Sinkhorn divergences with positive features.

The compute path is the HIP library ``libsinkhorn.so`` (C ABI in
``include/sinkhorn.h``); ``api`` is its PyTorch binding.  ``inputs`` holds
the seeded synthetic workload generators.  Importing the package does not
load the library; the first call does, and fails loudly if it is missing.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "api"]


def __getattr__(name):
    if name == "api":
        import importlib
        return importlib.import_module(".api", __name__)
    raise AttributeError(name)
