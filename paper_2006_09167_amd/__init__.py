"""Cluster-pair short-range nonbonded forces (Lennard-Jones + reaction field / Ewald real
space) with a dual pair list, native HIP on AMD MI355X (gfx950).

The compute path is the C-ABI library ``libnbmi.so`` (see include/nb.h); ``api`` holds the
thin torch binding.  ``systems`` builds seeded synthetic inputs.  Importing the package
does not load the library; ``api`` does, and fails loudly when it is not built.
"""
import importlib

__all__ = ["api", "systems", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(__name__ + "." + name)
    raise AttributeError(name)
