"""Matrix form of the 3D SBP-SAT FDTD method (oracle, test infrastructure).

Follows the paper section by section:

* Table T1: the grid type of each field component per axis.
* E7-E12 with ED_1-ED_3: the semi-discrete curl as Kronecker products
  (x fastest).
* E13-E15 (PEC) and E19-E21 (PMC): penalties sigma (P''')^-1 R^T P'' E_face
  on the H equations and chi (P''')^-1 R^T P'' H_face on the E equations, with
  the values of E18 and E23.  Reading of the face letters: the labels on the
  sigma of E13-E15 are swapped relative to E17; the energy rate E17 fixes
  which face each sigma belongs to (b/f = -x/+x, l/r = -y/+y, d/t = -z/+z), and
  that assignment is used with the values of E18.
* EPBC1-EPBC6 with sigma = chi = +-1/2 (EPBCP): periodic faces.  The two
  faces of an axis of one block are penalised with each other's values, the
  high face's neighbour value being e^{-j alpha} times the low face's and the
  low face's e^{+j alpha} times the high face's (alpha = k0_axis times the
  block length along the axis); with alpha != 0 the fields are complex.
* The same pattern with alpha = 0 couples two blocks across a shared face.
  Blocks of
  different mesh sizes (1:2) use the same pattern with the neighbour's face
  values interpolated (see ``operators.interp_c2f``); the paper defers that
  construction, so it is a reading.
* First-order absorbing face (not in the paper, which truncates with CPML):
  the PMC penalty with H_face replaced by H_face - chi E_face / eta, i.e. a
  penalty on the incoming characteristic.  Reading.
* Section V: leapfrog in time, E at integer and H at half-integer steps; loss
  (conductivity and the absorbing self term) is time-averaged over the step
  (semi-implicit), the source enters as a current density.
* E16: the discrete energy, with the leapfrog pairing
  W^n = 1/2 E^n' (eps P''') E^n + 1/2 H^{n+1/2}' (mu P''') H^{n-1/2},
  which the scheme conserves exactly in lossless media.

Material reading (paper silent): the permittivity, permeability and
conductivity of a node are the arithmetic mean of the per-cell values over
the cells whose closed box contains the node, within the node's own block.
The weight matrices P'' and P''' are geometric (the 1D norms with h); the
material enters as a separate diagonal.

Field vectors are numpy arrays of shape (Sz, Sy, Sx) per component (x fastest
when flattened), for every block.
"""
import math

import numpy as np
import scipy.sparse as sp

from . import operators as ops

MU0 = 4e-7 * math.pi
C0 = 299792458.0
EPS0 = 1.0 / (MU0 * C0 * C0)

E_COMPS = ("Ex", "Ey", "Ez")
H_COMPS = ("Hx", "Hy", "Hz")
COMPS = E_COMPS + H_COMPS

# Table T1: grid type along (x, y, z)
GRID = {"Ex": "-++", "Ey": "+-+", "Ez": "++-",
        "Hx": "+--", "Hy": "-+-", "Hz": "--+"}

# E7-E12: d(target)/dt = sum sign * D^axis (source)
CURL = {"Ex": (("Hz", 1, +1), ("Hy", 2, -1)),
        "Ey": (("Hx", 2, +1), ("Hz", 0, -1)),
        "Ez": (("Hy", 0, +1), ("Hx", 1, -1)),
        "Hx": (("Ey", 2, +1), ("Ez", 1, -1)),
        "Hy": (("Ez", 0, +1), ("Ex", 2, -1)),
        "Hz": (("Ex", 1, +1), ("Ey", 0, -1))}

# face index -> paper letter; axis = face // 2, high side = face % 2
FACE_LETTER = ("b", "f", "l", "r", "d", "t")

# E18 values, placed on faces as E17 assigns them
SIGMA_PEC = {("Hx", "d"): +1, ("Hx", "t"): -1, ("Hx", "l"): -1, ("Hx", "r"): +1,
             ("Hy", "b"): +1, ("Hy", "f"): -1, ("Hy", "d"): -1, ("Hy", "t"): +1,
             ("Hz", "b"): -1, ("Hz", "f"): +1, ("Hz", "l"): +1, ("Hz", "r"): -1}
# E23 values, placed on faces as E22 assigns them
CHI_PMC = {("Ex", "t"): +1, ("Ex", "d"): -1, ("Ex", "r"): -1, ("Ex", "l"): +1,
           ("Ey", "b"): -1, ("Ey", "f"): +1, ("Ey", "t"): -1, ("Ey", "d"): +1,
           ("Ez", "b"): +1, ("Ez", "f"): -1, ("Ez", "r"): +1, ("Ez", "l"): -1}

BC_PEC, BC_PMC, BC_ABC, BC_IFACE, BC_CPML = "pec", "pmc", "abc", "iface", "cpml"


def cfl_dt(blocks, cfl, c=C0):
    """Largest Yee time step over the blocks times cfl (Section VI cavity)."""
    return cfl * min(1.0 / (c * math.sqrt(sum(1.0 / hh ** 2 for hh in b["h"])))
                     for b in blocks)


def comp_shape(comp, n):
    """(Sx, Sy, Sz) node counts of a component for a block of n cells."""
    return tuple(ops.size(g, nn) for g, nn in zip(GRID[comp], n))


def comp_size(comp, n):
    s = comp_shape(comp, n)
    return s[0] * s[1] * s[2]


def _kron3(mz, my, mx):
    return sp.kron(mz, sp.kron(my, mx, format="csr"), format="csr")


def _eye(k):
    return sp.identity(k, format="csr")


def axis_operator(target, source, axis, n, h):
    """ED_1-ED_3: I (x) D (x) I along ``axis`` from source grid to target grid."""
    gt, gs = GRID[target], GRID[source]
    mats = []
    for a in range(3):
        if a == axis:
            assert gt[a] != gs[a]
            d = ops.d_plus(n[a], h[a]) if gt[a] == "+" else ops.d_minus(n[a], h[a])
            mats.append(sp.csr_matrix(d))
        else:
            assert gt[a] == gs[a]
            mats.append(_eye(ops.size(gt[a], n[a])))
    return _kron3(mats[2], mats[1], mats[0])


def norm_diag(comp, n, h):
    """Diagonal of P''' (EP_1) for a component: w_z (x) w_y (x) w_x, geometric."""
    g = GRID[comp]
    w = [ops.weights(g[a], n[a], h[a]) for a in range(3)]
    return np.kron(w[2], np.kron(w[1], w[0]))


def _tangential_axes(axis):
    return [a for a in range(3) if a != axis]


def face_select(comp, n, face):
    """R^T of Section III: selects the nodes of ``comp`` on ``face``."""
    axis, hi = divmod(face, 2)
    g = GRID[comp]
    mats = []
    for a in range(3):
        k = ops.size(g[a], n[a])
        if a == axis:
            e = np.zeros((1, k))
            e[0, k - 1 if hi else 0] = 1.0
            mats.append(sp.csr_matrix(e))
        else:
            mats.append(_eye(k))
    return _kron3(mats[2], mats[1], mats[0])


def face_norm(comp, n, h, face):
    """Diagonal of P'' (EP_2) on ``face`` for ``comp``'s tangential grids."""
    axis = face // 2
    g = GRID[comp]
    t = _tangential_axes(axis)
    w0 = ops.weights(g[t[0]], n[t[0]], h[t[0]])
    w1 = ops.weights(g[t[1]], n[t[1]], h[t[1]])
    return np.kron(w1, w0)


def node_material(cell_values, comp, n):
    """Per-node mean of per-cell values over the cells containing the node.

    ``cell_values`` has shape (nz, ny, nx).  For each axis, a "+" node i lies
    on the cell boundary shared by cells i-1 and i (those that exist); a "-"
    node j lies inside cell j-1 (j = 1..n), or on the block face (j = 0 ->
    cell 0, j = n+1 -> cell n-1).
    """
    g = GRID[comp]
    cells_per_axis = []
    for a in range(3):
        nn = n[a]
        lst = []
        for idx in range(ops.size(g[a], nn)):
            if g[a] == "+":
                lst.append([c for c in (idx - 1, idx) if 0 <= c < nn])
            else:
                lst.append([0] if idx == 0 else [nn - 1] if idx == nn + 1 else [idx - 1])
        cells_per_axis.append(lst)
    sx, sy, sz = comp_shape(comp, n)
    out = np.zeros((sz, sy, sx))
    # mean over the product set, written out axis by axis
    for k in range(sz):
        for j in range(sy):
            for i in range(sx):
                acc, cnt = 0.0, 0
                for ck in cells_per_axis[2][k]:
                    for cj in cells_per_axis[1][j]:
                        for ci in cells_per_axis[0][i]:
                            acc += cell_values[ck, cj, ci]
                            cnt += 1
                out[k, j, i] = acc / cnt
    return out


class System:
    """The assembled semi-discrete system of a set of coupled blocks.

    problem: dict with
      blocks: list of {n: (nx,ny,nz), h: (hx,hy,hz), eps_r, mu_r, sigma
              (per-cell arrays (nz,ny,nx) or None), faces: 6 bc names}
      interfaces: list of (block_a, face_a, block_b, face_b, ratio), ratio =
              cells of b per cell of a (1 or 2)
      periodic: list of (block, axis, alpha): both faces of the axis are
              periodic with the phase shift e^{-j alpha} (EPBC1-EPBC6)
    """

    def __init__(self, problem):
        self.blocks = problem["blocks"]
        self.interfaces = list(problem.get("interfaces", []))
        self.periodic = [(int(b), int(a), float(al)) for (b, a, al) in problem.get("periodic", [])]
        self.complex = any(al != 0.0 for (_, _, al) in self.periodic)
        self._index()
        self._materials()
        self._assemble()

    # ------------------------------------------------------------ layout
    def _index(self):
        self.e_off, self.h_off = {}, {}
        ne = nh = 0
        for b, blk in enumerate(self.blocks):
            n = tuple(blk["n"])
            for c in E_COMPS:
                self.e_off[(b, c)] = ne
                ne += comp_size(c, n)
            for c in H_COMPS:
                self.h_off[(b, c)] = nh
                nh += comp_size(c, n)
        self.ne, self.nh = ne, nh
        # which faces are interfaces, and with whom
        self.face_link = {}
        self.face_phase = {}  # factor on the neighbour's face values (periodic faces)
        for (b, axis, alpha) in self.periodic:
            lo, hi = 2 * axis, 2 * axis + 1
            if (b, lo) in self.face_link or (b, hi) in self.face_link:
                raise ValueError("face already coupled")
            self.face_link[(b, hi)] = (b, lo, "same")
            self.face_link[(b, lo)] = (b, hi, "same")
            if alpha == 0.0:
                self.face_phase[(b, hi)] = self.face_phase[(b, lo)] = 1.0
            else:
                self.face_phase[(b, hi)] = complex(math.cos(alpha), -math.sin(alpha))
                self.face_phase[(b, lo)] = complex(math.cos(alpha), math.sin(alpha))
        for (ba, fa, bb, fb, ratio) in self.interfaces:
            if ratio not in (1, 2):
                raise ValueError("interface ratio must be 1 or 2")
            if fa // 2 != fb // 2 or fa % 2 == fb % 2:
                raise ValueError("interface faces must be opposite faces of one axis")
            self.face_link[(ba, fa)] = (bb, fb, "coarse" if ratio == 2 else "same")
            self.face_link[(bb, fb)] = (ba, fa, "fine" if ratio == 2 else "same")
            na, nb = self.blocks[ba]["n"], self.blocks[bb]["n"]
            for a in _tangential_axes(fa // 2):
                if nb[a] != ratio * na[a]:
                    raise ValueError("interface faces do not match")

    def _bc(self, b, face):
        if (b, face) in self.face_link:
            return BC_IFACE
        bc = self.blocks[b]["faces"][face]
        if bc not in (BC_PEC, BC_PMC, BC_ABC, BC_IFACE, BC_CPML):
            raise ValueError(f"unknown face condition {bc!r}")
        return bc

    def _materials(self):
        self.eps = np.zeros(self.ne)
        self.mu_e = np.zeros(self.ne)
        self.sig = np.zeros(self.ne)
        self.mu = np.zeros(self.nh)
        for b, blk in enumerate(self.blocks):
            n = tuple(blk["n"])
            shape = (n[2], n[1], n[0])
            er = blk.get("eps_r")
            mr = blk.get("mu_r")
            sg = blk.get("sigma")
            er = np.ones(shape) if er is None else np.asarray(er, np.float64)
            mr = np.ones(shape) if mr is None else np.asarray(mr, np.float64)
            sg = np.zeros(shape) if sg is None else np.asarray(sg, np.float64)
            for c in E_COMPS:
                o, k = self.e_off[(b, c)], comp_size(c, n)
                self.eps[o:o + k] = EPS0 * node_material(er, c, n).reshape(-1)
                self.mu_e[o:o + k] = MU0 * node_material(mr, c, n).reshape(-1)
                self.sig[o:o + k] = node_material(sg, c, n).reshape(-1)
            for c in H_COMPS:
                o, k = self.h_off[(b, c)], comp_size(c, n)
                self.mu[o:o + k] = MU0 * node_material(mr, c, n).reshape(-1)
        self.w_e = np.zeros(self.ne)
        self.w_h = np.zeros(self.nh)
        for b, blk in enumerate(self.blocks):
            n, h = tuple(blk["n"]), tuple(blk["h"])
            for c in E_COMPS:
                o = self.e_off[(b, c)]
                d = norm_diag(c, n, h)
                self.w_e[o:o + len(d)] = d
            for c in H_COMPS:
                o = self.h_off[(b, c)]
                d = norm_diag(c, n, h)
                self.w_h[o:o + len(d)] = d

    # ---------------------------------------------------------- assembly
    def _face_interp(self, b, face, comp):
        """Map from the neighbour's face vector of ``comp`` to ours."""
        nb, fnb, role = self.face_link[(b, face)]
        n_own = self.blocks[b]["n"]
        t = _tangential_axes(face // 2)
        g = GRID[comp]
        if role == "same":
            k = 1
            for a in t:
                k *= ops.size(g[a], n_own[a])
            return _eye(k)
        mats = []
        for a in t:
            if role == "fine":      # we are fine, neighbour coarse
                mats.append(sp.csr_matrix(ops.interp_c2f(g[a], n_own[a] // 2)))
            else:                   # we are coarse, neighbour fine
                mats.append(sp.csr_matrix(ops.interp_f2c(g[a], n_own[a])))
        return sp.kron(mats[1], mats[0], format="csr")

    def _assemble(self):
        abc_diag = np.zeros(self.ne)
        # terms kept per axis of their difference (the face normal for the
        # penalties): K = K_0 + K_1 + K_2, used by the stretched-coordinate
        # absorbing layers (oracle.cpml)
        per_eh, per_he = ([], [], []), ([], [], [])

        def place(rows_off, cols_off, m, nrows, ncols, store):
            coo = m.tocoo()
            store.append((coo.data, coo.row + rows_off, coo.col + cols_off))

        def build(store, shape):
            data = np.concatenate([np.asarray(s[0], complex if self.complex else float) for s in store])
            rows = np.concatenate([s[1] for s in store])
            cols = np.concatenate([s[2] for s in store])
            return sp.csr_matrix((data, (rows, cols)), shape=shape)  # duplicates summed

        for b, blk in enumerate(self.blocks):
            n, h = tuple(blk["n"]), tuple(blk["h"])
            # interior operators with the boundary closures (E7-E12)
            for tgt in COMPS:
                for (src, axis, sgn) in CURL[tgt]:
                    m = sgn * axis_operator(tgt, src, axis, n, h)
                    if tgt in E_COMPS:
                        place(self.e_off[(b, tgt)], self.h_off[(b, src)], m,
                              self.ne, self.nh, per_eh[axis])
                    else:
                        place(self.h_off[(b, tgt)], self.e_off[(b, src)], m,
                              self.nh, self.ne, per_he[axis])
            # penalties, face by face
            for face in range(6):
                axis = face // 2
                blocks_eh, blocks_he = per_eh[axis], per_he[axis]
                bc = self._bc(b, face)
                if bc == BC_CPML:   # a PEC face behind the absorbing layer
                    bc = BC_PEC
                letter = FACE_LETTER[face]
                # H equations: tangential E on the face (E13-E15 / EPBC1-3)
                for hc in H_COMPS:
                    for (ec, ax, _s) in CURL[hc]:
                        if ax != axis:
                            continue
                        sigma = SIGMA_PEC[(hc, letter)]
                        sat = (sp.diags(1.0 / norm_diag(hc, n, h))
                               @ face_select(hc, n, face).T
                               @ sp.diags(face_norm(ec, n, h, face)))
                        if bc == BC_PEC:
                            place(self.h_off[(b, hc)], self.e_off[(b, ec)],
                                  sigma * sat @ face_select(ec, n, face),
                                  self.nh, self.ne, blocks_he)
                        elif bc == BC_IFACE:
                            nb, fnb, _ = self.face_link[(b, face)]
                            nn = tuple(self.blocks[nb]["n"])
                            place(self.h_off[(b, hc)], self.e_off[(b, ec)],
                                  0.5 * sigma * sat @ face_select(ec, n, face),
                                  self.nh, self.ne, blocks_he)
                            place(self.h_off[(b, hc)], self.e_off[(nb, ec)],
                                  -0.5 * sigma * self.face_phase.get((b, face), 1.0) * sat
                                  @ self._face_interp(b, face, ec) @ face_select(ec, nn, fnb),
                                  self.nh, self.ne, blocks_he)
                # E equations: tangential H on the face (E19-E21 / EPBC4-6)
                for ec in E_COMPS:
                    for (hc, ax, _s) in CURL[ec]:
                        if ax != axis:
                            continue
                        chi = CHI_PMC[(ec, letter)]
                        sat = (sp.diags(1.0 / norm_diag(ec, n, h))
                               @ face_select(ec, n, face).T
                               @ sp.diags(face_norm(ec, n, h, face)))
                        if bc in (BC_PMC, BC_ABC):
                            place(self.e_off[(b, ec)], self.h_off[(b, hc)],
                                  chi * sat @ face_select(hc, n, face),
                                  self.ne, self.nh, blocks_eh)
                        if bc == BC_ABC:
                            # -chi * chi / eta * E_face, carried as damping
                            o = self.e_off[(b, ec)]
                            k = comp_size(ec, n)
                            eta = np.sqrt(self.mu_e[o:o + k] / self.eps[o:o + k])
                            d = (sat @ face_select(ec, n, face)).diagonal()
                            abc_diag[o:o + k] += d / eta
                        elif bc == BC_IFACE:
                            nb, fnb, _ = self.face_link[(b, face)]
                            nn = tuple(self.blocks[nb]["n"])
                            place(self.e_off[(b, ec)], self.h_off[(b, hc)],
                                  0.5 * chi * sat @ face_select(hc, n, face),
                                  self.ne, self.nh, blocks_eh)
                            place(self.e_off[(b, ec)], self.h_off[(nb, hc)],
                                  -0.5 * chi * self.face_phase.get((b, face), 1.0) * sat
                                  @ self._face_interp(b, face, hc) @ face_select(hc, nn, fnb),
                                  self.ne, self.nh, blocks_eh)
        empty = [(np.zeros(0), np.zeros(0, int), np.zeros(0, int))]
        self.K_eh_ax = [build(per_eh[a] + empty, (self.ne, self.nh)) for a in range(3)]
        self.K_he_ax = [build(per_he[a] + empty, (self.nh, self.ne)) for a in range(3)]
        self.K_eh = self.K_eh_ax[0] + self.K_eh_ax[1] + self.K_eh_ax[2]
        self.K_he = self.K_he_ax[0] + self.K_he_ax[1] + self.K_he_ax[2]
        for m in self.K_eh_ax + self.K_he_ax + [self.K_eh, self.K_he]:
            m.eliminate_zeros()
        self.abc = abc_diag  # geometric damping rate coefficient (x 1/eps -> 1/s)

    # ----------------------------------------------------- vectors <-> fields
    def split(self, e, h):
        """Global vectors -> {(block, comp): array (Sz, Sy, Sx)}."""
        out = {}
        for b, blk in enumerate(self.blocks):
            n = tuple(blk["n"])
            for c in COMPS:
                sx, sy, sz = comp_shape(c, n)
                if c in E_COMPS:
                    o = self.e_off[(b, c)]
                    out[(b, c)] = e[o:o + sx * sy * sz].reshape(sz, sy, sx)
                else:
                    o = self.h_off[(b, c)]
                    out[(b, c)] = h[o:o + sx * sy * sz].reshape(sz, sy, sx)
        return out

    def join(self, fields):
        cplx = self.complex or any(np.iscomplexobj(a) for a in fields.values())
        dtype = np.complex128 if cplx else np.float64
        e = np.zeros(self.ne, dtype)
        h = np.zeros(self.nh, dtype)
        for (b, c), arr in fields.items():
            arr = np.asarray(arr, dtype).reshape(-1)
            if c in E_COMPS:
                o = self.e_off[(b, c)]
                e[o:o + arr.size] = arr
            else:
                o = self.h_off[(b, c)]
                h[o:o + arr.size] = arr
        return e, h

    def node_index(self, b, comp, node):
        i, j, k = node
        sx, sy, sz = comp_shape(comp, tuple(self.blocks[b]["n"]))
        if not (0 <= i < sx and 0 <= j < sy and 0 <= k < sz):
            raise ValueError("node outside component grid")
        base = self.e_off[(b, comp)] if comp in E_COMPS else self.h_off[(b, comp)]
        return base + i + sx * (j + sy * k)

    # ------------------------------------------------------------ energy
    def energy(self, e, h_new, h_old):
        """W^n of E16 with the leapfrog pairing of H (for complex fields the
        real part of the Hermitian form: the sum over real and imaginary
        parts)."""
        return float(np.real(0.5 * np.vdot(e, self.eps * self.w_e * e) +
                             0.5 * np.vdot(h_old, self.mu * self.w_h * h_new)))

    def energy_instant(self, e, h):
        """E16 with E and H taken at the same time level (oscillates under leapfrog)."""
        return float(np.real(0.5 * np.vdot(e, self.eps * self.w_e * e) +
                             0.5 * np.vdot(h, self.mu * self.w_h * h)))

    # --------------------------------------------------------- time step
    def coefficients(self, dt):
        beta = dt * (self.sig + self.abc) / (2.0 * self.eps)
        ca = (1.0 - beta) / (1.0 + beta)
        cb = (dt / self.eps) / (1.0 + beta)
        return ca, cb


def waveform(kind, t, tw, t0, f0):
    """Source time functions: Gaussian pulse (DR example) and modulated
    Gaussian (filter example) of Section VI."""
    g = math.exp(-4.0 * math.pi * (t - t0) ** 2 / (tw * tw))
    if kind == "gauss":
        return g
    if kind == "modgauss":
        return math.sin(2.0 * math.pi * f0 * t) * g
    raise ValueError(kind)


def run(problem, steps=None, dt=None, init=None, record_fields_every=0):
    """Leapfrog time marching (Section V) of ``problem``.

    Returns dict with final fields, per-step energy W^n (n = 0..steps-1),
    probe series (sample n = node value of E^{n+1}, or of H^{n+1/2} for an H
    component) and dt.
    """
    sysm = System(problem)
    steps = problem["steps"] if steps is None else steps
    if dt is None:
        dt = cfl_dt(problem["blocks"], problem["cfl"])
    ca, cb = sysm.coefficients(dt)
    inv_mu = 1.0 / sysm.mu
    if init is None:
        dtype = np.complex128 if sysm.complex else np.float64
        e = np.zeros(sysm.ne, dtype)
        h = np.zeros(sysm.nh, dtype)
    else:
        e, h = sysm.join(init)
    srcs = [(sysm.node_index(s["block"], s["comp"], s["node"]), s) for s in problem.get("sources", [])]
    prb = [(p["comp"] in E_COMPS, sysm.node_index(p["block"], p["comp"], p["node"]))
           for p in problem.get("probes", [])]
    energy = np.zeros(steps)
    probes = np.zeros((len(prb), steps), e.dtype)
    snaps = []
    for n in range(steps):
        h_new = h + dt * inv_mu * (sysm.K_he @ e)
        energy[n] = sysm.energy(e, h_new, h)
        h = h_new
        rhs = sysm.K_eh @ h
        t = (n + 0.5) * dt
        for (idx, s) in srcs:
            rhs[idx] += s["amp"] * waveform(s["waveform"], t, s["tw"], s["t0"], s.get("f0", 0.0))
        e = ca * e + cb * rhs
        for p, (is_e, idx) in enumerate(prb):
            probes[p, n] = e[idx] if is_e else h[idx]
        if record_fields_every and (n + 1) % record_fields_every == 0:
            snaps.append((n + 1, sysm.split(e.copy(), h.copy())))
    return {"fields": sysm.split(e, h), "energy": energy, "probes": probes, "dt": dt,
            "system": sysm, "e": e, "h": h, "snapshots": snaps}
