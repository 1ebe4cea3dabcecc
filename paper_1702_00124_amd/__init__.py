"""MI355X-native two-flavour Wilson-fermion HMC hot path (gfx950 HIP + C ABI).

The compute path is libwilson_hmc.so (built by ``paper_1702_00124_amd.build``);
this package only marshals arguments to it.  Importing the binding classes
requires the built library: there is no CPU or PyTorch fallback.
"""
from ._lib import LIB_PATH, WilsonError, load  # noqa: F401


def __getattr__(name):
    if name in ("WilsonLattice", "Term", "CG", "CgResult"):
        from . import lattice
        return getattr(lattice, name)
    raise AttributeError(name)
