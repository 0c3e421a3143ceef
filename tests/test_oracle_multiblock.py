"""Pins of the multi-block loop form of the oracle (``oracle/multiblock.c``)
against the matrix form and against what the method itself fixes (CPU).

- The two forms are written independently: rows and face rules in C, the
  penalties of E13-E15 / E19-E21 / EPBC1-EPBC6 as assembled matrices in
  ``oracle.system``.  They agree to rounding on every face kind, on 1:1 and
  1:2 interfaces along each axis and on the 27-block subgrid workload.
- Lossless coupled blocks conserve the leapfrog energy W^n (E16 with the
  leapfrog pairing) exactly, which pins the interface rows and the
  norm-compatible 1:2 maps; a restriction that is not the norm-compatible
  transpose of the interpolation (a planted mistake) breaks it.
- The energy of a lossless PEC cavity stays constant over 10^6 steps: the
  paper runs its cavity about 1.3 million steps at the largest stable time
  step without divergence (Section VI-A).
"""
import numpy as np
import pytest

from oracle import loops
from oracle import system as S


def blk(n, h=(1e-3, 1e-3, 1e-3), faces=("pec",) * 6, **kw):
    d = {"n": tuple(n), "h": tuple(h), "eps_r": None, "mu_r": None, "sigma": None, "faces": list(faces)}
    d.update(kw)
    return d


def rand_init(problem, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    out = {}
    for b, B in enumerate(problem["blocks"]):
        for c in S.COMPS:
            sx, sy, sz = S.comp_shape(c, tuple(B["n"]))
            out[(b, c)] = scale * rng.standard_normal((sz, sy, sx))
    return out


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def pair(kind, seed):
    """Two coupled blocks with mixed faces, materials, loss and a source."""
    rng = np.random.default_rng(seed)
    if kind == "1:1x":
        a = blk((7, 8, 6), faces=("pec", "pec", "pmc", "abc", "pec", "pmc"),
                eps_r=rng.uniform(1, 3, (6, 8, 7)), mu_r=rng.uniform(1, 2, (6, 8, 7)))
        b = blk((9, 8, 6), faces=("pec", "abc", "pmc", "pec", "pec", "pmc"), sigma=rng.uniform(0, 0.3, (6, 8, 9)))
        ifc = [(0, 1, 1, 0, 1)]
    elif kind == "1:2y":
        a = blk((6, 5, 7), faces=("pec", "pmc", "pec", "pec", "abc", "pec"), sigma=rng.uniform(0, 0.3, (7, 5, 6)))
        b = blk((12, 10, 14), (5e-4,) * 3, faces=("pec", "pec", "pec", "pmc", "pec", "abc"),
                eps_r=rng.uniform(1, 2, (14, 10, 12)))
        ifc = [(0, 3, 1, 2, 2)]
    elif kind == "1:2x":
        a = blk((6, 7, 6), faces=("pmc", "pec", "abc", "pec", "pec", "pec"))
        b = blk((10, 14, 12), (5e-4,) * 3, faces=("pec", "pmc", "pec", "pec", "abc", "pec"),
                mu_r=rng.uniform(1, 2, (12, 14, 10)))
        ifc = [(0, 1, 1, 0, 2)]
    else:  # "1:2z": fine below coarse
        a = blk((6, 7, 5), faces=("pmc", "pec", "pec", "pec", "pec", "abc"), eps_r=rng.uniform(1, 4, (5, 7, 6)))
        b = blk((12, 14, 9), (5e-4,) * 3, faces=("pec", "abc", "pec", "pec", "pec", "pec"))
        ifc = [(0, 4, 1, 5, 2)]
    return {"blocks": [a, b], "interfaces": ifc, "cfl": 0.9,
            "sources": [{"block": 1, "comp": "Ez", "node": (4, 3, 3), "waveform": "modgauss",
                         "tw": 2e-11, "t0": 2e-11, "f0": 2e10, "amp": 1.0},
                        {"block": 0, "comp": "Ex", "node": (2, 1, 2), "waveform": "gauss",
                         "tw": 2e-11, "t0": 2e-11, "f0": 0.0, "amp": 0.5}],
            "probes": [{"block": 0, "comp": "Ey", "node": (3, 2, 2)},
                       {"block": 1, "comp": "Hx", "node": (2, 3, 4)},
                       {"block": 1, "comp": "Ez", "node": (5, 5, 5)}]}


@pytest.mark.parametrize("kind", ["1:1x", "1:2x", "1:2y", "1:2z"])
def test_loop_form_matches_matrix_form_coupled(kind, oracle_lib):
    prob = pair(kind, 3)
    init = rand_init(prob, 9)
    steps = 30
    r1 = S.run(prob, steps=steps, init=init)
    r2 = loops.run_blocks(prob, steps=steps, init=init)
    for k in r1["fields"]:
        assert rel(r2["fields"][k], r1["fields"][k]) < 1e-13, k
    assert rel(r2["energy"], r1["energy"]) < 1e-13
    assert rel(r2["probes"], r1["probes"]) < 1e-13


def test_loop_form_matches_matrix_form_subgrid_workload(oracle_lib):
    """The 27-block 1:2 workload (coarse 1 mm region around a fine 0.5 mm
    block, absorbing outer faces, lossy box) at 1/8 of its size."""
    from sbp_inputs import make_config
    prob = make_config(3, scale=8)
    init = rand_init(prob, 4, scale=1e-3)
    steps = 40
    r1 = S.run(prob, steps=steps, init=init)
    m = loops.MultiBlock(prob, init=init)
    e1, p1 = m.advance(15)      # in two pieces: the state carries over
    e2, p2 = m.advance(steps - 15)
    for k in r1["fields"]:
        assert rel(m.fields[k], r1["fields"][k]) < 1e-13, k
    assert rel(np.concatenate([e1, e2]), r1["energy"]) < 1e-13
    assert rel(np.concatenate([p1, p2], axis=1), r1["probes"]) < 1e-13


def _ring(faces=("pec",) * 6):
    """A coarse block with a fine block on its low x side at 1:2 and a 1:1
    neighbour above it in z: lossless, mixed PEC / PMC outer faces."""
    a = blk((6, 6, 6), faces=faces)
    f = blk((8, 12, 12), (5e-4,) * 3, faces=("pec", "pmc", "pmc", "pec", "pec", "pmc"))
    g = blk((6, 6, 5), faces=("pmc", "pec", "pec", "pmc", "pec", "pec"))
    f["origin"] = (-4e-3, 0.0, 0.0)
    return {"blocks": [a, f, g], "interfaces": [(0, 0, 1, 1, 2), (0, 5, 2, 4, 1)], "cfl": 0.95,
            "sources": [], "probes": []}


def test_coupled_lossless_energy_conserved(oracle_lib):
    prob = _ring()
    m = loops.MultiBlock(prob, init=rand_init(prob, 2))
    e, _ = m.advance(3000)
    assert np.abs(e / e[0] - 1.0).max() < 1e-12


def test_planted_plain_restriction_breaks_energy(oracle_lib, monkeypatch):
    """Planted mistake: the coarse side takes the plain transpose of the
    interpolation (rows rescaled to sum to one) instead of the
    norm-compatible restriction W_c^-1 I_c2f^T W_f; the discrete energy is
    then no longer conserved."""
    from oracle import operators as ops
    good = ops.interp_f2c

    def plain(kind, nc):
        m = ops.interp_c2f(kind, nc).T.copy()
        return m / m.sum(axis=1, keepdims=True)

    prob = _ring()
    init = rand_init(prob, 2)
    monkeypatch.setattr(ops, "interp_f2c", plain)
    m = loops.MultiBlock(prob, init=init)
    e, _ = m.advance(3000)
    monkeypatch.setattr(ops, "interp_f2c", good)
    assert np.abs(e / e[0] - 1.0).max() > 1e-8


def test_energy_constant_over_a_million_steps(oracle_lib):
    """8^3 lossless PEC cavity from seeded random fields at 0.99 of the Yee
    limit: W^n constant to 1e-10 over 10^6 steps (Section VI-A reports no
    divergence over about 1.3 million steps)."""
    prob = {"blocks": [blk((8, 8, 8))], "interfaces": [], "cfl": 0.99, "sources": [], "probes": []}
    m = loops.MultiBlock(prob, init=rand_init(prob, 1), threads=1)
    w0 = None
    worst = 0.0
    for _ in range(10):
        e, _p = m.advance(100_000)
        w0 = e[0] if w0 is None else w0
        worst = max(worst, float(np.abs(e / w0 - 1.0).max()))
    assert m.steps_done == 1_000_000
    assert worst < 1e-10, worst
