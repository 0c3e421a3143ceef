"""MI355X-native leapfrog step of the 3D SBP-SAT FDTD method.

The compute path is the HIP library ``libsbpfdtd.so`` (C ABI declared in
``include/sbpfdtd.h``); ``binding`` marshals arguments to it.
"""
from .binding import Context, SbpError, build_problem, lib  # noqa: F401
