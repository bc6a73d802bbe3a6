"""MI355X-native stencil scaling for vector-valued P1 operators on
hierarchical hybrid grids (Drzisga, Ruede, Wohlmuth).

The compute path is the HIP library ``libhhg.so`` (C ABI in include/hhg.h);
this package only marshals arguments.  Importing it does not load the library;
the first handle does, and fails loudly if it is missing.
"""
from .hhg import Mesh, Multigrid  # noqa: F401

__all__ = ["Mesh", "Multigrid"]
