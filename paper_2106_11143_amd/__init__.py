"""MI355X-native all-pairs Coulomb forces and Paul-trap velocity-Verlet.

The compute path is the HIP library ``libcoulomb_mi355x.so`` (C ABI declared in
``include/coulomb.h``); ``paper_2106_11143_amd.api`` is its thin binding over
torch device tensors.  Submodules load lazily so that ``inputs`` (the seeded
generators) can be imported without the native library.
"""
import importlib

__all__ = ["api", "inputs", "autograd", "drivers", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
