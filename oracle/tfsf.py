"""Total-field / scattered-field (TF/SF) plane-wave injection (oracle, test
infrastructure; fp64 on the CPU).

The paper brings the incident wave of its filter and head examples in
through a TF/SF boundary (Section VI; the technique is cited, not derived).
Reading used here, written from its definition: a box of cells splits the
block into a total-field region T (the nodes on or inside the box) and a
scattered-field region S.  Every difference of the step that couples a node
of one region to a node of the other takes the neighbour's value in the
first node's own convention, so with an incident field (e_inc, h_inc):
    H update:  + K_he[T, S] e_inc(S)  - K_he[S, T] e_inc(T)
    E update:  + K_eh[T, S] h_inc(S)  - K_eh[S, T] h_inc(T)
(the E correction enters inside the Cb bracket like a current).  The box
lies at least 4 cells inside the block, so these differences are the
interior two-point ones.

The incident field is a plane wave along +axis with E along `pol`, taken
from a one-dimensional line stepped with the same dt, h, eps0 and mu0 (the
interior difference along the axis; PEC ends; a soft current source near
its low end, with the waveforms of Section VI).  In vacuum around the box
the 3D step restricted to such a wave is that line's step, so with no
scatterer the S region stays zero and T carries the incident wave exactly;
both are pinned.
"""
import numpy as np

from . import system as S


def _pair(axis, pol):
    """(E component, H component, sign of d_axis in the H equation, sign in the E equation)."""
    ep = S.E_COMPS[pol]
    for hq in S.H_COMPS:
        for (src, ax, sh) in S.CURL[hq]:
            if src == ep and ax == axis:
                for (src2, ax2, se) in S.CURL[ep]:
                    if src2 == hq and ax2 == axis:
                        return ep, hq, sh, se
    raise ValueError("polarisation must be transverse to the axis")


def _inside_1d(kind, n, lo, hi):
    """Membership of the nodes of a grid along one axis in [lo h, hi h]."""
    if kind == "+":
        idx = np.arange(n + 1)
        return (idx >= lo) & (idx <= hi)
    idx = np.arange(n + 2)          # "-" node j at (j - 1/2) h, face nodes outside
    return (idx >= lo + 1) & (idx <= hi)


def masks(sysm, block, box):
    """Boolean vectors over all E and all H nodes: True in T."""
    mt_e = np.zeros(sysm.ne, bool)
    mt_h = np.zeros(sysm.nh, bool)
    blk = sysm.blocks[block]
    n = tuple(blk["n"])
    for comps, off, mt in ((S.E_COMPS, sysm.e_off, mt_e), (S.H_COMPS, sysm.h_off, mt_h)):
        for c in comps:
            g = S.GRID[c]
            m = [_inside_1d(g[a], n[a], box[2 * a], box[2 * a + 1]) for a in range(3)]
            inside = m[2][:, None, None] & m[1][None, :, None] & m[0][None, None, :]
            o = off[(block, c)]
            mt[o:o + inside.size] = inside.reshape(-1)
    return mt_e, mt_h


class Line:
    """The incident wave: one-dimensional leapfrog along the axis over 3D
    "+" node indices -margin .. n + margin (E at i h, H at (i + 1/2) h)."""

    def __init__(self, n, h, dt, sh, se, margin, src):
        self.n, self.h, self.dt, self.sh, self.se, self.m = n, h, dt, sh, se, margin
        self.e = np.zeros(n + 2 * margin + 1)
        self.hh = np.zeros(n + 2 * margin)
        self.src = src

    def e_at(self, i):                 # E at 3D "+" index i
        return self.e[i + self.m]

    def h_at(self, i):                 # H at (i + 1/2) h
        return self.hh[i + self.m]

    def step_h(self):
        self.hh += self.dt / S.MU0 * self.sh * (self.e[1:] - self.e[:-1]) / self.h

    def step_e(self, t):
        d = self.se * (self.hh[1:] - self.hh[:-1]) / self.h
        self.e[1:-1] += self.dt / S.EPS0 * d
        s = self.src
        self.e[s["cell"] + self.m] += self.dt / S.EPS0 * s["amp"] * S.waveform(s["waveform"], t, s["tw"], s["t0"],
                                                                             s.get("f0", 0.0))


def incident_vectors(sysm, block, axis, ep, hq, line):
    """Full E and H vectors holding the incident components of the line."""
    e_inc = np.zeros(sysm.ne)
    h_inc = np.zeros(sysm.nh)
    n = tuple(sysm.blocks[block]["n"])
    sx, sy, sz = S.comp_shape(ep, n)
    arr = np.zeros((sz, sy, sx))
    vals = np.array([line.e_at(i) for i in range(n[axis] + 1)])
    shp = [1, 1, 1]
    shp[2 - axis] = n[axis] + 1
    arr[...] = vals.reshape(shp)
    o = sysm.e_off[(block, ep)]
    e_inc[o:o + arr.size] = arr.reshape(-1)
    sx, sy, sz = S.comp_shape(hq, n)
    arr = np.zeros((sz, sy, sx))
    vals = np.zeros(n[axis] + 2)
    vals[1:n[axis] + 1] = [line.h_at(j - 1) for j in range(1, n[axis] + 1)]
    shp = [1, 1, 1]
    shp[2 - axis] = n[axis] + 2
    arr[...] = vals.reshape(shp)
    o = sysm.h_off[(block, hq)]
    h_inc[o:o + arr.size] = arr.reshape(-1)
    return e_inc, h_inc


def run(problem, steps=None, dt=None, init=None, record=None, _flip=1.0):
    """Leapfrog (Section V) with the TF/SF corrections of problem["tfsf"]:
    {block, box (6 cell indices lo/hi per axis), axis, pol, margin, source
    {cell, waveform, tw, t0, f0, amp}}.  Returns fields, W^n, probes, and the
    incident vectors of the last step (e_inc at n, h_inc at n + 1/2)."""
    sysm = S.System(problem)
    tf = problem["tfsf"]
    b, box, axis = tf["block"], tuple(tf["box"]), tf["axis"]
    n = tuple(sysm.blocks[b]["n"])
    for a in range(3):
        if box[2 * a] < 4 or box[2 * a + 1] > n[a] - 4 or box[2 * a] >= box[2 * a + 1]:
            raise ValueError("the TF/SF box must lie at least 4 cells inside the block")
    steps = problem["steps"] if steps is None else steps
    if dt is None:
        dt = S.cfl_dt(problem["blocks"], problem["cfl"])
    ca, cb = sysm.coefficients(dt)
    ep, hq, sh, se = _pair(axis, tf["pol"])
    line = Line(n[axis], sysm.blocks[b]["h"][axis], dt, sh, se, tf.get("margin", 16), tf["source"])
    mt_e, mt_h = masks(sysm, b, box)
    ms_e = ~mt_e
    ms_h = ~mt_h
    # only the block's own nodes take part
    in_blk_e = np.zeros(sysm.ne, bool)
    in_blk_h = np.zeros(sysm.nh, bool)
    for c in S.E_COMPS:
        o = sysm.e_off[(b, c)]
        in_blk_e[o:o + S.comp_size(c, n)] = True
    for c in S.H_COMPS:
        o = sysm.h_off[(b, c)]
        in_blk_h[o:o + S.comp_size(c, n)] = True
    ms_e &= in_blk_e
    ms_h &= in_blk_h
    mt_e &= in_blk_e
    mt_h &= in_blk_h
    if init is None:
        e = np.zeros(sysm.ne)
        h = np.zeros(sysm.nh)
    else:
        e, h = sysm.join(init)
    srcs = [(sysm.node_index(s["block"], s["comp"], s["node"]), s) for s in problem.get("sources", [])]
    prb = [(p["comp"] in S.E_COMPS, sysm.node_index(p["block"], p["comp"], p["node"]))
           for p in problem.get("probes", [])]
    energy = np.zeros(steps)
    probes = np.zeros((len(prb), steps))
    e_inc = h_inc = None
    for step in range(steps):
        e_inc, _ = incident_vectors(sysm, b, axis, ep, hq, line)
        corr_h = mt_h * (sysm.K_he @ (ms_e * e_inc)) - ms_h * (sysm.K_he @ (mt_e * e_inc))
        h_new = h + dt / sysm.mu * (sysm.K_he @ e + _flip * corr_h)
        energy[step] = sysm.energy(e, h_new, h)
        h = h_new
        line.step_h()
        _, h_inc = incident_vectors(sysm, b, axis, ep, hq, line)
        corr_e = mt_e * (sysm.K_eh @ (ms_h * h_inc)) - ms_e * (sysm.K_eh @ (mt_h * h_inc))
        rhs = sysm.K_eh @ h + corr_e
        t = (step + 0.5) * dt
        for (idx, s) in srcs:
            rhs[idx] += s["amp"] * S.waveform(s["waveform"], t, s["tw"], s["t0"], s.get("f0", 0.0))
        e = ca * e + cb * rhs
        line.step_e(t)
        for q, (is_e, idx) in enumerate(prb):
            probes[q, step] = e[idx] if is_e else h[idx]
    e_inc, _ = incident_vectors(sysm, b, axis, ep, hq, line)
    return {"fields": sysm.split(e, h), "energy": energy, "probes": probes, "dt": dt, "e": e, "h": h,
            "e_inc": e_inc, "h_inc": h_inc, "mask_t": (mt_e, mt_h), "mask_s": (ms_e, ms_h), "system": sysm}
