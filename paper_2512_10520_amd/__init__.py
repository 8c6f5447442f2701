"""MI355X-native histogram-sampling muon transport (HIP kernels for gfx950
behind a C ABI, with a thin torch binding).

Importing the package does not load the HIP library; the first call that
needs it does, and raises if ``libmt.so`` has not been built.
"""
import importlib

from . import workloads  # noqa: F401

__all__ = ["workloads", "api"]


def __getattr__(name):
    if name == "api":
        return importlib.import_module(__name__ + ".api")
    raise AttributeError(name)
