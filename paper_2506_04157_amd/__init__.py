"""MI355X-native matrix-free blended-shell Stokes solver (arXiv 2506.04157).

The compute path is the HIP/C++ library ``libstokes.so`` (C ABI in
``include/stokes.h``); this package only marshals arguments to it.  Importing
the package does not load the library; the first use does, and fails loudly
if it has not been built.
"""
from ._lib import (BC_DIRICHLET, BC_FREESLIP, MESH_CUBE, MESH_SHELL, STK_ENOCONV, StokesError,
                   load)

__all__ = ["load", "StokesError", "BC_DIRICHLET", "BC_FREESLIP", "MESH_CUBE", "MESH_SHELL",
           "STK_ENOCONV", "StokesContext", "default_params", "temp_params", "StokesSolve"]


def __getattr__(name):
    if name in ("StokesContext", "default_params", "temp_params"):
        from . import context
        return getattr(context, name)
    if name == "StokesSolve":
        from .autograd import StokesSolve
        return StokesSolve
    raise AttributeError(name)
