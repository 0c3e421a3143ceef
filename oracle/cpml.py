"""Convolutional perfectly matched layers on the SBP-SAT step (oracle, test
infrastructure; fp64 on the CPU).

The paper truncates its open problems with a 10-layer CPML (Section VI,
filter and head examples; the layer itself is the cited CFS-PML, not derived
in the paper).  Reading used here, written from the stretched-coordinate
formulation: inside a layer of d cells next to a face marked "cpml" every
difference along that face's normal, d_a u, is replaced by
    d_a u / kappa_a + psi_a,   psi_a <- b_a psi_a + c_a d_a u,
with, at depth rho in [0, 1] into the layer (rho = 1 on the face),
    sigma = sigma_max rho^m, kappa = 1 + (kappa_max - 1) rho^m,
    alpha = alpha_max (1 - rho),
    b = exp(-(sigma / kappa + alpha) dt / eps0),
    c = sigma (b - 1) / (sigma kappa + kappa^2 alpha),
evaluated at each node's own position along the axis (the "+" grid at i h,
the "-" grid at the Appendix nodes 0, (j - 1/2) h, n h).  sigma_max =
sigma_factor (m + 1) / (eta0 h).  The difference operators are the SBP ones
with their closure rows, and the face behind the layer is PEC (its SAT
belongs to the normal difference and is stretched with it).  The psi of the
H update are advanced with E^n, those of the E update with H^{n+1/2}.

With sigma = 0, kappa = 1, alpha = 0 the layer is the plain scheme (pinned
bitwise); its absorption is pinned by comparing with a domain large enough
that nothing returns in the time simulated.
"""
import math

import numpy as np

from . import operators as ops
from . import system as S

ETA0 = math.sqrt(S.MU0 / S.EPS0)


def node_positions(kind, n, h):
    """Node coordinates of the "+" (i h) or "-" (0, (j - 1/2) h, n h) grid."""
    if kind == "+":
        return np.arange(n + 1) * h
    x = (np.arange(n + 2) - 0.5) * h
    x[0], x[-1] = 0.0, n * h
    return x


def axis_profile(kind, n, h, lo_cells, hi_cells, p, dt):
    """(b, c, 1/kappa) per node of one grid along one axis; b = 1, c = 0,
    1/kappa = 1 outside the layers."""
    x = node_positions(kind, n, h)
    L = n * h
    rho = np.zeros_like(x)
    if lo_cells > 0:
        d = lo_cells * h
        rho = np.maximum(rho, np.clip((d - x) / d, 0.0, 1.0))
    if hi_cells > 0:
        d = hi_cells * h
        rho = np.maximum(rho, np.clip((x - (L - d)) / d, 0.0, 1.0))
    m = p["m"]
    smax = p["sigma_factor"] * (m + 1) / (ETA0 * h)
    sig = smax * rho ** m
    kap = 1.0 + (p["kappa_max"] - 1.0) * rho ** m
    alp = np.where(rho > 0, p["alpha_max"] * (1.0 - rho), 0.0)
    b = np.exp(-(sig / kap + alp) * dt / S.EPS0)
    den = sig * kap + kap * kap * alp
    c = np.where(sig > 0, sig * (b - 1.0) / np.where(den > 0, den, 1.0), 0.0)
    return b, c, 1.0 / kap


DEFAULT = {"cells": 10, "m": 3, "sigma_factor": 0.8, "kappa_max": 1.0, "alpha_max": 0.0}


def coefficients(sysm, problem, dt):
    """Per-axis (b, c, 1/kappa) vectors over all E nodes and all H nodes."""
    p = dict(DEFAULT)
    p.update(problem.get("cpml", {}))
    out = {}
    for field, comps, off, size in (("E", S.E_COMPS, sysm.e_off, sysm.ne), ("H", S.H_COMPS, sysm.h_off, sysm.nh)):
        bs = [np.ones(size) for _ in range(3)]
        cs = [np.zeros(size) for _ in range(3)]
        ks = [np.ones(size) for _ in range(3)]
        for bi, blk in enumerate(sysm.blocks):
            n, h = tuple(blk["n"]), tuple(blk["h"])
            for comp in comps:
                shape = S.comp_shape(comp, n)          # (sx, sy, sz)
                o = off[(bi, comp)]
                k = shape[0] * shape[1] * shape[2]
                for a in range(3):
                    lo = p["cells"] if blk["faces"][2 * a] == S.BC_CPML else 0
                    hi = p["cells"] if blk["faces"][2 * a + 1] == S.BC_CPML else 0
                    if lo == 0 and hi == 0:
                        continue
                    b1, c1, k1 = axis_profile(S.GRID[comp][a], n[a], h[a], lo, hi, p, dt)
                    # broadcast along the axis over the (sz, sy, sx) array
                    sl = [1, 1, 1]
                    sl[2 - a] = shape[a]
                    full = [shape[2], shape[1], shape[0]]
                    bs[a][o:o + k] = np.broadcast_to(b1.reshape(sl), full).reshape(-1)
                    cs[a][o:o + k] = np.broadcast_to(c1.reshape(sl), full).reshape(-1)
                    ks[a][o:o + k] = np.broadcast_to(k1.reshape(sl), full).reshape(-1)
        out[field] = (bs, cs, ks)
    return out


def run(problem, steps=None, dt=None, init=None):
    """Leapfrog time marching (Section V) with the CPML differences; returns
    the final fields, W^n per step and the probe series as system.run."""
    sysm = S.System(problem)
    steps = problem["steps"] if steps is None else steps
    if dt is None:
        dt = S.cfl_dt(problem["blocks"], problem["cfl"])
    ca, cb = sysm.coefficients(dt)
    co = coefficients(sysm, problem, dt)
    if init is None:
        e = np.zeros(sysm.ne)
        h = np.zeros(sysm.nh)
    else:
        e, h = sysm.join(init)
    psi_e = [np.zeros(sysm.ne) for _ in range(3)]
    psi_h = [np.zeros(sysm.nh) for _ in range(3)]
    srcs = [(sysm.node_index(s["block"], s["comp"], s["node"]), s) for s in problem.get("sources", [])]
    prb = [(p["comp"] in S.E_COMPS, sysm.node_index(p["block"], p["comp"], p["node"]))
           for p in problem.get("probes", [])]
    energy = np.zeros(steps)
    probes = np.zeros((len(prb), steps))
    bE, cE, kE = co["E"]
    bH, cH, kH = co["H"]
    for n in range(steps):
        rhs_h = np.zeros(sysm.nh)
        for a in range(3):
            d = sysm.K_he_ax[a] @ e
            psi_h[a] = bH[a] * psi_h[a] + cH[a] * d
            rhs_h += d * kH[a] + psi_h[a]
        h_new = h + dt / sysm.mu * rhs_h
        energy[n] = sysm.energy(e, h_new, h)
        h = h_new
        rhs = np.zeros(sysm.ne)
        for a in range(3):
            d = sysm.K_eh_ax[a] @ h
            psi_e[a] = bE[a] * psi_e[a] + cE[a] * d
            rhs += d * kE[a] + psi_e[a]
        t = (n + 0.5) * dt
        for (idx, s) in srcs:
            rhs[idx] += s["amp"] * S.waveform(s["waveform"], t, s["tw"], s["t0"], s.get("f0", 0.0))
        e = ca * e + cb * rhs
        for q, (is_e, idx) in enumerate(prb):
            probes[q, n] = e[idx] if is_e else h[idx]
    return {"fields": sysm.split(e, h), "energy": energy, "probes": probes, "dt": dt, "e": e, "h": h}
