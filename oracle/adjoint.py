"""Discrete adjoint of the leapfrog step (oracle, test infrastructure).

Objective (the region objective of the adjoint workload): the time-integrated
energy-like measure of the cell-centred field over a box of cells,

    J = dt * sum_{n=1..N} sum_{cells c in region} |Ebar_c^n|^2,

where Ebar_c is, per component, the mean of the four edges of cell c that
carry that component (Ex edges (i+1, j+dj, k+dk) on the (x-, y+, z+) grid of
Table T1, and likewise for Ey, Ez).

The time stepping is the Section V leapfrog of ``system.run``:

    H^{n+1/2} = H^{n-1/2} + Db * (K_he E^n),        Db = dt / mu
    E^{n+1}   = Ca * E^n + Cb * (K_eh H^{n+1/2} + s^{n+1/2})

with Ca, Cb from the node permittivity and conductivity (``coefficients``).
Its discrete adjoint (Lagrange multipliers lam_E^n, lam_H^{n+1/2}) runs
backwards in time with the transposed matrices:

    lam_E^N = dJ/dE^N,  lam_H^{N+1/2} = 0
    for n = N-1 .. 0:
        dJ/dCb += lam_E^{n+1} * (K_eh H^{n+1/2} + s^{n+1/2})
        dJ/dCa += lam_E^{n+1} * E^n
        lam_H^{n+1/2} = lam_H^{n+3/2} + K_eh^T (Cb * lam_E^{n+1})
        lam_E^n       = Ca * lam_E^{n+1} + K_he^T (Db * lam_H^{n+1/2}) + dJ/dE^n

and the gradient with respect to the per-cell relative permittivity follows
from Ca(eps), Cb(eps) and the node averaging of the per-cell values (the
material reading of ``system.node_material``).  Lossless and lossy blocks are
covered; absorbing faces are not (their damping depends on eps through the
wave impedance).
"""
import numpy as np
import scipy.sparse as sp

from . import operators as ops
from .system import (EPS0, E_COMPS, GRID, System, cfl_dt, comp_shape, waveform)

__all__ = ["region_operator", "node_material_matrix", "objective_and_gradient", "objective"]


def region_operator(sysm, block, region):
    """Sparse map E (global vector) -> cell-centred components over the
    region's cells, ordered (component, cell).  region = (i0, i1, j0, j1, k0,
    k1), a half-open box of cells of ``block``."""
    i0, i1, j0, j1, k0, k1 = region
    rows, cols = [], []
    r = 0
    for comp in E_COMPS:
        axis = "xyz".index(comp[1])
        for ck in range(k0, k1):
            for cj in range(j0, j1):
                for ci in range(i0, i1):
                    # the four edges of the cell along `axis`: the "-" index
                    # of the cell centre on that axis, both "+" neighbours on
                    # the other two
                    for d1 in (0, 1):
                        for d2 in (0, 1):
                            node = [ci, cj, ck]
                            node[axis] += 1
                            others = [a for a in range(3) if a != axis]
                            node[others[0]] += d1
                            node[others[1]] += d2
                            rows.append(r)
                            cols.append(sysm.node_index(block, comp, tuple(node)))
                    r += 1
    data = np.full(len(rows), 0.25)
    return sp.csr_matrix((data, (rows, cols)), shape=(r, sysm.ne))


def node_material_matrix(comp, n):
    """Sparse linear map from per-cell values (flattened (nz, ny, nx)) to the
    node values of ``comp``: the mean over the cells whose closed box contains
    the node (same rule as ``system.node_material``), as a matrix."""
    g = GRID[comp]
    per_axis = []
    for a in range(3):
        nn = n[a]
        lst = []
        for idx in range(ops.size(g[a], nn)):
            if g[a] == "+":
                lst.append([c for c in (idx - 1, idx) if 0 <= c < nn])
            else:
                lst.append([min(max(idx - 1, 0), nn - 1)])
        per_axis.append(lst)
    sx, sy, sz = comp_shape(comp, n)
    rows, cols, vals = [], [], []
    for k in range(sz):
        for j in range(sy):
            for i in range(sx):
                cells = [(ck, cj, ci) for ck in per_axis[2][k] for cj in per_axis[1][j] for ci in per_axis[0][i]]
                for (ck, cj, ci) in cells:
                    rows.append(i + sx * (j + sy * k))
                    cols.append(ci + n[0] * (cj + n[1] * ck))
                    vals.append(1.0 / len(cells))
    return sp.csr_matrix((vals, (rows, cols)), shape=(sx * sy * sz, n[0] * n[1] * n[2]))


def _forward(sysm, problem, steps, dt, A, e0=None, h0=None):
    ca, cb = sysm.coefficients(dt)
    inv_mu = 1.0 / sysm.mu
    e = np.zeros(sysm.ne) if e0 is None else e0.copy()
    h = np.zeros(sysm.nh) if h0 is None else h0.copy()
    srcs = [(sysm.node_index(s["block"], s["comp"], s["node"]), s) for s in problem.get("sources", [])]
    es, hs, rhss = [e.copy()], [], []
    J = 0.0
    for n in range(steps):
        h = h + dt * inv_mu * (sysm.K_he @ e)
        rhs = sysm.K_eh @ h
        t = (n + 0.5) * dt
        for (idx, s) in srcs:
            rhs[idx] += s["amp"] * waveform(s["waveform"], t, s["tw"], s["t0"], s.get("f0", 0.0))
        e = ca * e + cb * rhs
        ebar = A @ e
        J += dt * float(np.dot(ebar, ebar))
        es.append(e.copy())
        hs.append(h.copy())
        rhss.append(rhs)
    return J, es, hs, rhss, ca, cb


def objective(problem, steps, region, block=0, dt=None):
    """J of the forward run from rest (no adjoint)."""
    sysm = System(problem)
    if dt is None:
        dt = cfl_dt(problem["blocks"], problem["cfl"])
    A = region_operator(sysm, block, region)
    return _forward(sysm, problem, steps, dt, A)[0]


def objective_and_gradient(problem, steps, region, block=0, dt=None, _mistake=None):
    """J and dJ/d(eps_r) per cell of ``block`` (array (nz, ny, nx)), from rest.

    ``_mistake`` plants a named error (tests only): "K_he" uses K_he in place
    of K_eh^T in the adjoint H update."""
    for f in problem["blocks"][block]["faces"]:
        if f == "abc":
            raise ValueError("the oracle adjoint covers PEC/PMC faces and interfaces only")
    sysm = System(problem)
    if dt is None:
        dt = cfl_dt(problem["blocks"], problem["cfl"])
    A = region_operator(sysm, block, region)
    J, es, hs, rhss, ca, cb = _forward(sysm, problem, steps, dt, A)
    db = dt / sysm.mu
    K_ehT = sysm.K_he if _mistake == "K_he" else sysm.K_eh.T.tocsr()
    K_heT = sysm.K_he.T.tocsr()
    AtA = (A.T @ A).tocsr()

    def dJdE(n):
        return 2.0 * dt * (AtA @ es[n]) if n >= 1 else np.zeros(sysm.ne)

    lam_e = dJdE(steps)
    lam_h = np.zeros(sysm.nh)
    g_cb = np.zeros(sysm.ne)
    g_ca = np.zeros(sysm.ne)
    for n in range(steps - 1, -1, -1):
        g_cb += lam_e * rhss[n]
        g_ca += lam_e * es[n]
        lam_h = lam_h + K_ehT @ (cb * lam_e)
        lam_e = ca * lam_e + K_heT @ (db * lam_h) + dJdE(n)
    # Ca = (1-b)/(1+b), Cb = (dt/eps)/(1+b), b = dt sigma / (2 eps)
    eps = sysm.eps
    beta = dt * sysm.sig / (2.0 * eps)
    dca = 2.0 * beta / (eps * (1.0 + beta) ** 2)
    dcb = -dt / (eps ** 2 * (1.0 + beta) ** 2)
    g_eps_node = g_cb * dcb + g_ca * dca
    n = tuple(problem["blocks"][block]["n"])
    grad = np.zeros(n[0] * n[1] * n[2])
    for comp in E_COMPS:
        o = sysm.e_off[(block, comp)]
        M = node_material_matrix(comp, n)
        grad += EPS0 * (M.T @ g_eps_node[o:o + M.shape[0]])
    return J, grad.reshape(n[2], n[1], n[0])
