"""MI355X-native leapfrog step of the 3D SBP-SAT FDTD method.

The compute path is the HIP library ``libsbpfdtd.so`` (C ABI declared in
``include/sbpfdtd.h``); ``binding`` marshals arguments to it.
"""
from .binding import Context, SbpError, build_problem, lib  # noqa: F401


def PermittivityObjective(*args, **kw):
    """See ``paper_2206_00638_amd.autograd.PermittivityObjective`` (imports torch)."""
    from .autograd import PermittivityObjective as _P
    return _P(*args, **kw)
