"""MI355X (gfx950) band-limited FMM for radial basis functions.

The compute path is the HIP library ``lib/librbffmm.so`` (sources in ``csrc/``, C ABI in
``include/rbf_fmm.h``); this package only marshals arguments.  Importing it does not
load the library; the first plan does, and fails loudly if the library is missing.
"""
from ._lib import RbfError, load  # noqa: F401

__all__ = ["FmmPlan", "EvalPlan", "BatchPlan", "autotune", "RbfError", "load"]


def __getattr__(name):
    if name in ("FmmPlan", "EvalPlan", "BatchPlan", "autotune"):
        from . import fmm
        return getattr(fmm, name)
    raise AttributeError(name)
