"""Two-component pseudopotential lattice Boltzmann (D3Q19) on MI355X.

The step runs in hand-written HIP kernels for gfx950 inside ``libmclbm.so``
(C ABI, ``include/mclbm.h``).  This package holds the thin ctypes binding
(``lattice``), the autograd wrapper (``autograd``) and seeded synthetic input
generators (``workloads``).  Importing the package does not load the library;
creating a :class:`Lattice` does, and fails loudly when it is missing.
"""

__all__ = ["Lattice", "LatticeParams", "Storage", "load_library"]


def __getattr__(name):
    if name in ("Lattice", "LatticeParams", "Storage", "load_library", "MclbmError"):
        from . import lattice
        return getattr(lattice, name)
    raise AttributeError(name)
