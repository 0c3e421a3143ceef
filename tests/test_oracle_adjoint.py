"""Pins of the oracle's discrete adjoint (oracle/adjoint.py).

The adjoint gradient is checked against central finite differences of the
oracle's own forward objective (an independent route: the forward run is
pinned by the energy, closed-form and Yee tests), a planted transpose mistake
must fail that check, and the region average and the node-averaging matrix
are checked against their definitions written out by hand.
"""
import numpy as np

from oracle import adjoint
from oracle.system import node_material, run


def _problem(seed, n=(6, 5, 7), lossy=True, faces=("pec", "pmc", "pec", "pec", "pmc", "pec")):
    rng = np.random.default_rng(seed)
    shape = (n[2], n[1], n[0])
    return {"blocks": [{"n": n, "h": (1e-3, 1.1e-3, 0.9e-3), "origin": (0.0, 0.0, 0.0),
                        "eps_r": rng.uniform(1.0, 4.0, shape), "mu_r": rng.uniform(1.0, 1.5, shape),
                        "sigma": rng.uniform(0.0, 0.3, shape) if lossy else None, "faces": list(faces)}],
            "interfaces": [], "cfl": 0.9,
            "sources": [{"block": 0, "comp": "Ez", "node": (2, 2, 3), "waveform": "modgauss",
                         "tw": 2e-11, "t0": 2e-11, "f0": 3e10, "amp": 1.0},
                        {"block": 0, "comp": "Ex", "node": (4, 1, 5), "waveform": "gauss",
                         "tw": 1.5e-11, "t0": 1.5e-11, "f0": 0.0, "amp": 0.7}],
            "probes": []}


def _fd(problem, steps, region, cells, rel=1e-5):
    from oracle.system import cfl_dt
    dt = cfl_dt(problem["blocks"], problem["cfl"])
    out = []
    for (k, j, i) in cells:
        eps = problem["blocks"][0]["eps_r"]
        d = rel * eps[k, j, i]
        vals = []
        for s in (1.0, -1.0):
            p = dict(problem)
            b = dict(problem["blocks"][0])
            e2 = eps.copy()
            e2[k, j, i] += s * d
            b["eps_r"] = e2
            p["blocks"] = [b]
            vals.append(adjoint.objective(p, steps, region, dt=dt))
        out.append((vals[0] - vals[1]) / (2 * d))
    return np.array(out)


CELLS = [(0, 0, 0), (3, 2, 2), (2, 2, 1), (6, 4, 5), (4, 1, 3), (3, 3, 4)]
REGION = (1, 3, 1, 3, 2, 4)


def test_adjoint_matches_central_differences_lossy():
    prob = _problem(1)
    J, g = adjoint.objective_and_gradient(prob, 30, REGION)
    assert J > 0
    fd = _fd(prob, 30, REGION, CELLS)
    ad = np.array([g[c] for c in CELLS])
    scale = np.max(np.abs(g))
    assert np.max(np.abs(ad - fd)) <= 1e-6 * scale, (ad, fd)


def test_adjoint_matches_central_differences_lossless():
    prob = _problem(2, lossy=False, faces=("pec",) * 6)
    J, g = adjoint.objective_and_gradient(prob, 40, REGION)
    fd = _fd(prob, 40, REGION, CELLS)
    ad = np.array([g[c] for c in CELLS])
    assert np.max(np.abs(ad - fd)) <= 1e-6 * np.max(np.abs(g)), (ad, fd)


def test_planted_transpose_mistake_fails_fd():
    prob = _problem(1)
    _, g = adjoint.objective_and_gradient(prob, 30, REGION, _mistake="K_he")
    fd = _fd(prob, 30, REGION, CELLS)
    ad = np.array([g[c] for c in CELLS])
    assert np.max(np.abs(ad - fd)) > 1e-2 * np.max(np.abs(fd))


def test_objective_is_the_region_average_written_out():
    """J from the adjoint module equals dt * sum_n sum_cells |Ebar|^2 with the
    cell averages taken by direct indexing of the recorded fields."""
    prob = _problem(3)
    steps = 12
    ref = run(prob, steps=steps, record_fields_every=1)
    dt = ref["dt"]
    i0, i1, j0, j1, k0, k1 = REGION
    J = 0.0
    for _, f in ref["snapshots"]:
        ex, ey, ez = f[(0, "Ex")], f[(0, "Ey")], f[(0, "Ez")]   # arrays (z, y, x)
        for ck in range(k0, k1):
            for cj in range(j0, j1):
                for ci in range(i0, i1):
                    bx = 0.25 * (ex[ck, cj, ci + 1] + ex[ck, cj + 1, ci + 1] + ex[ck + 1, cj, ci + 1] + ex[ck + 1, cj + 1, ci + 1])
                    by = 0.25 * (ey[ck, cj + 1, ci] + ey[ck, cj + 1, ci + 1] + ey[ck + 1, cj + 1, ci] + ey[ck + 1, cj + 1, ci + 1])
                    bz = 0.25 * (ez[ck + 1, cj, ci] + ez[ck + 1, cj, ci + 1] + ez[ck + 1, cj + 1, ci] + ez[ck + 1, cj + 1, ci + 1])
                    J += dt * (bx * bx + by * by + bz * bz)
    assert abs(adjoint.objective(prob, steps, REGION) - J) <= 1e-13 * J


def test_node_material_matrix_matches_rule():
    rng = np.random.default_rng(4)
    n = (5, 4, 6)
    cells = rng.uniform(1, 4, (n[2], n[1], n[0]))
    for comp in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"):
        m = adjoint.node_material_matrix(comp, n) @ cells.reshape(-1)
        assert np.allclose(m, node_material(cells, comp, n).reshape(-1), rtol=1e-15, atol=0)
