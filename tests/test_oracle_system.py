"""Pins of the assembled oracle against what the paper and mathematics fix (CPU)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from oracle import system as S
from oracle import yee as Y

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def blk(n, h=(1.0, 1.0, 1.0), faces=("pec",) * 6, **kw):
    d = {"n": n, "h": h, "eps_r": None, "mu_r": None, "sigma": None, "faces": list(faces)}
    d.update(kw)
    return d


def weighted_ops(sysm):
    """G = W_E K_eh and F = W_H K_he: the energy-weighted operators."""
    return sp.diags(sysm.w_e) @ sysm.K_eh, sp.diags(sysm.w_h) @ sysm.K_he


def skew_residual(problem):
    s = S.System(problem)
    g, f = weighted_ops(s)
    return abs(g + f.T).max() / abs(g).max()


def rand_fields(sysm, rng):
    return rng.standard_normal(sysm.ne), rng.standard_normal(sysm.nh)


# ------------------------------------------------------------ skewness E17
FACE_SETS = [["pec"] * 6, ["pmc"] * 6, ["pec", "pmc", "pmc", "pec", "pec", "pmc"],
             ["pmc", "pec", "pec", "pmc", "pmc", "pec"]]


@pytest.mark.parametrize("faces", FACE_SETS)
def test_pec_pmc_energy_rate_zero(faces):
    # E17/E18 and E22/E23: dE/dt = 0 -> P A + (P A)^T = 0
    assert skew_residual({"blocks": [blk((5, 6, 7), (1.0, 1.3, 0.8), faces)]}) < 1e-15


def test_interfaces_energy_rate_zero():
    a = blk((5, 6, 7))
    b = blk((4, 6, 7))
    assert skew_residual({"blocks": [a, b], "interfaces": [(0, 1, 1, 0, 1)]}) < 1e-15
    c = blk((6, 7, 5), faces=["pmc"] * 6)
    f = blk((12, 14, 9), (0.5, 0.5, 0.5))
    assert skew_residual({"blocks": [f, c], "interfaces": [(1, 4, 0, 5, 2)]}) < 1e-14
    assert skew_residual({"blocks": [c, f], "interfaces": [(0, 5, 1, 4, 2)]}) < 1e-14


def test_planted_literal_E13_labels_break_energy(monkeypatch):
    # Planted mistake: read the sigma labels of E13-E15 literally with E18's
    # values.  The x- and y-face penalties then carry the wrong sign and the
    # energy identity fails -- the skewness pin detects it.
    literal = dict(S.SIGMA_PEC)
    for key in [("Hx", "r"), ("Hx", "l"), ("Hy", "b"), ("Hy", "f"),
                ("Hz", "r"), ("Hz", "l"), ("Hz", "b"), ("Hz", "f")]:
        literal[key] = -literal[key]
    monkeypatch.setattr(S, "SIGMA_PEC", literal)
    assert skew_residual({"blocks": [blk((5, 6, 7))]}) > 0.1


def test_planted_dropped_closure_breaks_energy(monkeypatch):
    # Planted mistake: replace the D- boundary closure by the interior row.
    from oracle import operators as ops
    orig = ops.d_minus

    def bad(n, h=1.0):
        d = orig(n, h)
        d[2, :] = 0.0
        d[2, 1], d[2, 2] = -1.0 / h, 1.0 / h
        return d
    monkeypatch.setattr(ops, "d_minus", bad)
    assert skew_residual({"blocks": [blk((5, 6, 7))]}) > 0.01


def test_absorbing_faces_dissipative():
    s = S.System({"blocks": [blk((5, 6, 5), faces=["abc"] * 6)]})
    g, f = weighted_ops(s)
    # the conservative part stays skew; the absorbing self term is a
    # non-negative damping on the face E nodes only
    assert abs(g + f.T).max() / abs(g).max() < 1e-15
    assert (s.abc >= 0).all() and s.abc.max() > 0
    on_face = s.abc > 0
    assert on_face.sum() < s.ne


# ------------------------------------------------------- leapfrog energy
def _lossless_energy(problem, steps=60, dt_frac=0.9, seed=0):
    sysm = S.System(problem)
    rng = np.random.default_rng(seed)
    e, h = rand_fields(sysm, rng)
    dt = S.cfl_dt(problem["blocks"], dt_frac)
    inv_mu = 1.0 / sysm.mu
    ca, cb = sysm.coefficients(dt)
    w = []
    for _ in range(steps):
        hn = h + dt * inv_mu * (sysm.K_he @ e)
        w.append(sysm.energy(e, hn, h))
        h = hn
        e = ca * e + cb * (sysm.K_eh @ h)
    return np.array(w)


@pytest.mark.parametrize("faces", FACE_SETS[:3])
def test_leapfrog_energy_conserved(faces):
    w = _lossless_energy({"blocks": [blk((6, 5, 7), (1e-3, 1e-3, 1e-3), faces)]})
    assert np.abs(w / w[0] - 1).max() < 1e-12


def test_leapfrog_energy_conserved_subgrid():
    c = blk((6, 7, 6), (1e-3,) * 3)
    f = blk((12, 14, 12), (5e-4,) * 3)
    w = _lossless_energy({"blocks": [c, f], "interfaces": [(0, 1, 1, 0, 2)]}, steps=80)
    assert np.abs(w / w[0] - 1).max() < 1e-12


def test_leapfrog_energy_nonincreasing_lossy():
    rng = np.random.default_rng(3)
    b = blk((6, 6, 6), (1e-3,) * 3, faces=["abc", "pec", "abc", "pmc", "abc", "abc"],
            sigma=rng.uniform(0, 0.5, (6, 6, 6)), eps_r=rng.uniform(1, 4, (6, 6, 6)))
    w = _lossless_energy({"blocks": [b]}, steps=80)
    assert (np.diff(w) <= 1e-13 * w[0]).all()
    assert w[-1] < 0.99 * w[0]


def test_planted_wrong_damping_sign_breaks_monotone(monkeypatch):
    # Planted mistake: loss with the wrong sign gains energy -> the monotonicity pin fails.
    orig = S.System.coefficients

    def bad(self, dt):
        self.sig = -np.abs(self.sig)
        return orig(self, dt)
    monkeypatch.setattr(S.System, "coefficients", bad)
    b = blk((5, 5, 5), (1e-3,) * 3, sigma=np.full((5, 5, 5), 0.3))
    w = _lossless_energy({"blocks": [b]}, steps=20)
    assert (np.diff(w) > 0).any()


# ------------------------------------------------------------------- CFL
def test_cfl_matches_paper_cavity_time_step():
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as fh:
        g = json.load(fh)
    h = g["cavity_mesh_m"]
    dt = S.cfl_dt([{"h": (h, h, h)}], 1.0, c=g["cavity_c_used"])
    assert dt * 1e12 == pytest.approx(g["cavity_dt_ps"], abs=0.005)


def _omega_max(problem):
    s = S.System(problem)
    g, _ = weighted_ops(s)
    me = np.sqrt(s.eps * s.w_e)
    mh = np.sqrt(s.mu * s.w_h)
    c = sp.diags(1 / me) @ g @ sp.diags(1 / mh)
    return math.sqrt(spl.eigsh(c @ c.T, k=1, which="LA", return_eigenvectors=False)[0])


@pytest.mark.parametrize("n", [5, 8, 12])
def test_sbp_time_step_limit_not_below_yee(n):
    h = 1e-3
    om = _omega_max({"blocks": [blk((n, n, n), (h, h, h))]})
    dt_max = 2.0 / om                      # leapfrog limit for the 2nd-order form
    dt_yee = S.cfl_dt([{"h": (h, h, h)}], 1.0)
    assert dt_max >= dt_yee * (1 - 1e-9)
    assert dt_max <= dt_yee * 1.2


# ------------------------------------------------------- cavity modes
def _closest_mode(n, target):
    L = 1.0
    h = L / n
    s = S.System({"blocks": [blk((n, n, n), (h, h, h))]})
    g, _ = weighted_ops(s)
    c = sp.diags(1 / np.sqrt(s.eps * s.w_e)) @ g @ sp.diags(1 / np.sqrt(s.mu * s.w_h))
    m = (c @ c.T).tocsc()
    vals = spl.eigsh(m, k=4, sigma=target ** 2, which="LM", return_eigenvectors=False)
    return np.sqrt(vals[np.argmin(np.abs(vals - target ** 2))])


def test_cavity_mode_converges_second_order():
    # TE/TM 110 mode of the 1 m PEC cube (Section VI-A: 200-400 MHz band)
    w_exact = S.C0 * math.pi * math.sqrt(2.0)
    assert w_exact / (2 * math.pi) / 1e6 == pytest.approx(211.985, abs=1e-3)
    errs = []
    for n in (12, 16):
        w = _closest_mode(n, w_exact)
        errs.append(abs(w - w_exact) / w_exact)
        # the semi-discrete Yee frequency of the same mode, closed form
        h = 1.0 / n
        w_yee = S.C0 * math.sqrt(2 * (2 / h * math.sin(math.pi * h / 2)) ** 2)
        assert abs(w - w_exact) <= 1.25 * abs(w_yee - w_exact)
    order = math.log(errs[0] / errs[1]) / math.log(16 / 12)
    assert 1.8 < order < 2.7   # pre-asymptotic at these sizes; 2.10 between 16 and 24


# --------------------------------------------------- interior equals Yee
def test_interior_equals_yee():
    rng = np.random.default_rng(7)
    n = (22, 21, 23)
    h = (1e-3, 1.1e-3, 0.9e-3)
    b = blk(n, h)
    prob = {"blocks": [b], "cfl": 0.9, "steps": 4}
    sysm = S.System(prob)
    init = {}
    for c in S.COMPS:
        sx, sy, sz = S.comp_shape(c, n)
        init[(0, c)] = rng.standard_normal((sz, sy, sx))
    yf = Y.from_sbp({c: init[(0, c)] for c in S.COMPS})
    r = S.run(prob, init=init)
    dt = r["dt"]
    for _ in range(4):
        Y.step(yf, h, dt, S.EPS0, S.MU0)
    ys = Y.from_sbp({c: r["fields"][(0, c)] for c in S.COMPS})
    m = 3 + 4
    for c in S.COMPS:
        a = ys[c][m:-m, m:-m, m:-m]
        b_ = yf[c][m:-m, m:-m, m:-m]
        assert a.size > 0
        assert np.abs(a - b_).max() <= 1e-15 * np.abs(b_).max()


# ----------------------------------------------- two oracle forms agree
def test_matrix_and_loop_forms_agree(oracle_lib):
    rng = np.random.default_rng(1)
    n = (5, 6, 7)
    b = blk(n, (1e-3, 1.2e-3, 0.9e-3), ["pec", "pmc", "abc", "pec", "abc", "pmc"],
            eps_r=rng.uniform(1, 4, (7, 6, 5)), mu_r=rng.uniform(1, 2, (7, 6, 5)),
            sigma=rng.uniform(0, 0.1, (7, 6, 5)))
    prob = {"blocks": [b], "cfl": 0.9, "steps": 25,
            "sources": [{"block": 0, "comp": "Ez", "node": (2, 3, 3), "waveform": "modgauss",
                         "tw": 2e-11, "t0": 2e-11, "f0": 1e10, "amp": 1.0}],
            "probes": [{"block": 0, "comp": "Ez", "node": (1, 2, 3)},
                       {"block": 0, "comp": "Hx", "node": (1, 2, 3)}]}
    init = {}
    for c in S.COMPS:
        sx, sy, sz = S.comp_shape(c, n)
        init[c] = rng.standard_normal((sz, sy, sx))
    rm = S.run(prob, init={(0, c): v for c, v in init.items()})
    rl = oracle_lib.run_block(prob, init=init)
    for c in S.COMPS:
        a, b_ = rm["fields"][(0, c)], rl["fields"][c]
        assert np.abs(a - b_).max() <= 1e-13 * np.abs(a).max()
    assert np.abs(rm["energy"] - rl["energy"]).max() <= 1e-13 * rm["energy"].max()
    assert np.abs(rm["probes"] - rl["probes"]).max() <= 1e-13 * np.abs(rm["probes"]).max()


# --------------------------------------------------------- materials
def test_node_material_brute_force():
    n = (4, 5, 6)
    rng = np.random.default_rng(0)
    cells = rng.standard_normal((6, 5, 4))
    for comp in S.COMPS:
        out = S.node_material(cells, comp, n)
        g = S.GRID[comp]
        sx, sy, sz = S.comp_shape(comp, n)
        # brute force from coordinates: cells whose closed box contains the node
        from oracle import operators as ops
        xs = [ops.grid(g[a], n[a], 1.0) for a in range(3)]
        for k in range(sz):
            for j in range(sy):
                for i in range(sx):
                    p = (xs[0][i], xs[1][j], xs[2][k])
                    vals = [cells[c, b, a] for c in range(n[2]) for b in range(n[1]) for a in range(n[0])
                            if a <= p[0] <= a + 1 and b <= p[1] <= b + 1 and c <= p[2] <= c + 1]
                    assert out[k, j, i] == pytest.approx(np.mean(vals), rel=1e-14, abs=1e-14)


def test_node_material_reproduces_linear_profile_inside():
    n = (6, 6, 6)
    zc, yc, xc = np.meshgrid(*(np.arange(6) + 0.5,) * 3, indexing="ij")
    cells = 1.0 + 0.3 * xc - 0.2 * yc + 0.1 * zc
    for comp in S.COMPS:
        out = S.node_material(cells, comp, n)
        from oracle import operators as ops
        g = S.GRID[comp]
        xs = [ops.grid(g[a], n[a], 1.0) for a in range(3)]
        Z, Yy, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
        ref = 1.0 + 0.3 * X - 0.2 * Yy + 0.1 * Z
        sl = (slice(1, -1),) * 3
        assert np.abs(out[sl] - ref[sl]).max() < 1e-13


# ------------------------------------------------------ absorbing face
def test_absorbing_face_absorbs_normal_plane_wave():
    # TEM pulse (Ey, Hz) travelling along x between PEC y-walls and PMC z-walls:
    # exactly one-dimensional; the characteristic penalty must let it out.
    nx, ny, nz = 80, 4, 4
    h = 1e-3
    b = blk((nx, ny, nz), (h, h, h), ["abc", "abc", "pec", "pec", "pmc", "pmc"])
    sysm = S.System({"blocks": [b]})
    dt = S.cfl_dt([b], 0.5)
    x = np.arange(nx + 1) * h
    prof = np.exp(-((x - 40 * h) / (5 * h)) ** 2)
    fields = {}
    for c in S.COMPS:
        sx, sy, sz = S.comp_shape(c, (nx, ny, nz))
        fields[(0, c)] = np.zeros((sz, sy, sx))
    fields[(0, "Ey")][:] = prof[None, None, :]
    e, hh = sysm.join(fields)
    ca, cb = sysm.coefficients(dt)
    inv_mu = 1 / sysm.mu
    w = []
    for _ in range(int(3 * nx * h / (S.C0 * dt))):
        hn = hh + dt * inv_mu * (sysm.K_he @ e)
        w.append(sysm.energy(e, hn, hh))
        hh = hn
        e = ca * e + cb * (sysm.K_eh @ hh)
    w = np.array(w)
    assert (np.diff(w) <= 1e-13 * w[0]).all()
    assert w[-1] < 1e-6 * w[0]


def test_waveforms():
    assert S.waveform("gauss", 1.0, 0.5, 1.0, 0.0) == 1.0
    assert S.waveform("gauss", 1.5, 1.0, 1.0, 0.0) == pytest.approx(math.exp(-math.pi))
    assert S.waveform("modgauss", 0.25, 1.0, 0.25, 1.0) == pytest.approx(1.0)


def test_memory_overhead_counts():
    # Section V: node counts of the SBP arrays against Yee's
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as fh:
        nx, ny, nz = json.load(fh)["memory_case_n"]
    n = (nx, ny, nz)
    assert S.comp_size("Ex", n) == (nx + 2) * (ny + 1) * (nz + 1)
    assert S.comp_size("Hx", n) == (nx + 1) * (ny + 2) * (nz + 2)
    ys = Y.shapes(n)
    assert S.comp_size("Hx", n) - np.prod(ys["Hx"]) == 2 * (nx + 1) * (ny + nz + 2)
    assert S.comp_size("Ex", n) - np.prod(ys["Ex"]) == 2 * (ny + 1) * (nz + 1)
