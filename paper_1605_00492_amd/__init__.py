"""Tensor-product geometric multigrid for the anisotropic pressure equation
on MI355X (HIP, gfx950), after Mitchell & Mueller, arXiv:1605.00492.

The compute path is libtpmg.so (hand-written HIP kernels behind the C
interface in include/tpmg.h); this package only binds it.
"""
from .binding import (COLUMN_MAJOR, LEVEL_MAJOR, DG1Level, Hierarchy, TpmgError, bandwidth_probe, lib,
                      solve, workspace_bytes, make_desc)

__all__ = ["Hierarchy", "DG1Level", "TpmgError", "solve", "lib", "bandwidth_probe", "workspace_bytes",
           "make_desc", "LEVEL_MAJOR", "COLUMN_MAJOR"]
