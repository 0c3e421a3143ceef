"""Plain Yee FDTD reference (test infrastructure).

The classical staggered scheme the paper compares against: E on cell edges,
H on cell faces, PEC walls holding tangential E at zero, uniform medium.
Used only to pin the interior of the SBP-SAT update: inside the domain the
two methods sample the same nodes (Section II-A) with the same two-point
differences, so away from the faces they must agree to rounding.

Arrays are (Sz, Sy, Sx), x fastest; shapes
Ex (nz+1, ny+1, nx), Ey (nz+1, ny, nx+1), Ez (nz, ny+1, nx+1),
Hx (nz, ny, nx+1), Hy (nz, ny+1, nx), Hz (nz+1, ny, nx).
"""
import numpy as np


def shapes(n):
    nx, ny, nz = n
    return {"Ex": (nz + 1, ny + 1, nx), "Ey": (nz + 1, ny, nx + 1), "Ez": (nz, ny + 1, nx + 1),
            "Hx": (nz, ny, nx + 1), "Hy": (nz, ny + 1, nx), "Hz": (nz + 1, ny, nx)}


def step(f, h, dt, eps, mu):
    """One leapfrog step, in place: H^{n+1/2} from E^n, then E^{n+1}."""
    hx, hy, hz = h
    ex, ey, ez = f["Ex"], f["Ey"], f["Ez"]
    f["Hx"] += dt / mu * ((ey[1:, :, :] - ey[:-1, :, :]) / hz - (ez[:, 1:, :] - ez[:, :-1, :]) / hy)
    f["Hy"] += dt / mu * ((ez[:, :, 1:] - ez[:, :, :-1]) / hx - (ex[1:, :, :] - ex[:-1, :, :]) / hz)
    f["Hz"] += dt / mu * ((ex[:, 1:, :] - ex[:, :-1, :]) / hy - (ey[:, :, 1:] - ey[:, :, :-1]) / hx)
    Hx, Hy, Hz = f["Hx"], f["Hy"], f["Hz"]
    # interior (non-wall) E nodes only; tangential E on the walls stays zero
    ex[1:-1, 1:-1, :] += dt / eps * ((Hz[1:-1, 1:, :] - Hz[1:-1, :-1, :]) / hy
                                     - (Hy[1:, 1:-1, :] - Hy[:-1, 1:-1, :]) / hz)
    ey[1:-1, :, 1:-1] += dt / eps * ((Hx[1:, :, 1:-1] - Hx[:-1, :, 1:-1]) / hz
                                     - (Hz[1:-1, :, 1:] - Hz[1:-1, :, :-1]) / hx)
    ez[:, 1:-1, 1:-1] += dt / eps * ((Hy[:, 1:-1, 1:] - Hy[:, 1:-1, :-1]) / hx
                                     - (Hx[:, 1:, 1:-1] - Hx[:, :-1, 1:-1]) / hy)


def from_sbp(sbp_fields):
    """Yee arrays taken from the SBP arrays at the nodes the grids share.

    SBP "-" index j = 1..n is the Yee half-integer index j-1; "+" indices
    coincide.
    """
    s = sbp_fields
    return {"Ex": s["Ex"][:, :, 1:-1].copy(), "Ey": s["Ey"][:, 1:-1, :].copy(),
            "Ez": s["Ez"][1:-1, :, :].copy(), "Hx": s["Hx"][1:-1, 1:-1, :].copy(),
            "Hy": s["Hy"][1:-1, :, 1:-1].copy(), "Hz": s["Hz"][:, 1:-1, 1:-1].copy()}
