"""MI355X-native cascaded central-moment lattice Boltzmann step (D3Q27).

The step runs in hand-written HIP kernels (``libcmlbm.so``, built in-tree by
``paper_1202_6074_amd.build``) behind a C ABI; this package is a thin
binding over it. Importing the package does not load the library; the first
use does, and fails loudly if it has not been built.
"""
from . import _lib  # noqa: F401

__all__ = ["Lattice", "EnergyAdjoint", "energy_and_grad"]


def __getattr__(name):
    if name == "Lattice":
        from .lattice import Lattice
        return Lattice
    if name in ("EnergyAdjoint", "energy_and_grad"):
        from . import adjoint
        return getattr(adjoint, name)
    raise AttributeError(name)
