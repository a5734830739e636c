"""MI355X CPR-FGMRES solver for 3x3-block black-oil Jacobians.

The solver is the HIP library ``libcpr_mi355x.so`` behind the C ABI declared in
``include/cpr.h`` (and ``include/cpr_inspect.h`` for single-step access).
This package only marshals arguments to it; there is no CPU fallback.
"""
from ._capi import CprError, lib  # noqa: F401
from .serve import Server  # noqa: F401
from .solver import (Params, Solver, host_galerkin, host_grouping,  # noqa: F401
                     host_interpolation, host_rs_split)
