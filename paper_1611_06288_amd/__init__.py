"""MI355X (gfx950) FAS-multigrid solver for the second-order convex-splitting
scheme of the 3D phase field crystal equation (arXiv:1611.06288).

The compute path is the HIP library ``libpfc_hip.so`` (C ABI in
``include/pfc.h``); ``Solver`` marshals torch tensors into it.  Importing the
package loads nothing; the library is loaded on first use and its absence is
an error.
"""
from .inputs import RunParams  # noqa: F401

__all__ = ["Solver", "PFCError", "RunParams"]


def __getattr__(name):
    if name in ("Solver", "PFCError", "StepInfo"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
