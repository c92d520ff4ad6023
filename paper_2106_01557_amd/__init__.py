"""MI355X-native lattice Boltzmann update for the liquid-vapour phase transition.

The compute path is the HIP library built from csrc/ (liblbm.so) behind the C ABI
declared in include/lbm.h; `lbm` is its thin Python binding (ctypes argument
marshalling only).  `inputs` builds seeded initial fields.

Submodules are imported lazily so that `inputs` can be used without the built
library; `lbm` raises if the library is missing.
"""
import importlib

__all__ = ["lbm", "inputs"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
