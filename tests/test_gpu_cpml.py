"""GPU parity of the convolutional PML faces against the fp64 oracle
(oracle.cpml): fields, W^n and probes, fp64 1e-12 / fp32 1e-5 relative; and
the layer's recursion variables travel with the saved state."""
import numpy as np
import pytest

from gpu_util import COMPS, TOL, check_fields, random_fields, rel_l2, write_fields

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def sbp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_00638_amd as p
    p.lib()
    return p


def _problem(seed, n=(14, 12, 16), faces=("cpml", "pec", "pmc", "cpml", "cpml", "cpml"), cells=4, **cp):
    rng = np.random.default_rng(seed)
    shape = (n[2], n[1], n[0])
    b = {"n": tuple(n), "h": (1e-3, 1.2e-3, 0.9e-3), "faces": list(faces),
         "eps_r": rng.uniform(1.0, 3.0, shape), "mu_r": None, "sigma": None}
    params = {"cells": cells, "m": 3, "sigma_factor": 0.8, "kappa_max": 1.0, "alpha_max": 0.0}
    params.update(cp)
    return {"blocks": [b], "cfl": 0.9, "cpml": params,
            "sources": [{"block": 0, "comp": "Ez", "node": (7, 6, 8), "waveform": "modgauss",
                         "tw": 3e-11, "t0": 3e-11, "f0": 2e10, "amp": 1.0}],
            "probes": [{"block": 0, "comp": "Ez", "node": (2, 6, 8)},
                       {"block": 0, "comp": "Hy", "node": (0, 3, 2)}]}


def _gpu(sbp, prob, prec, steps, init):
    ctx = sbp.build_problem(prob, prec=prec, history=steps + 8)
    write_fields(ctx, init)
    ctx.step(steps)
    out = {"fields": {(0, c): ctx.read_field(0, c) for c in COMPS}, "energy": ctx.read_energy(0, steps),
           "probes": np.array([ctx.read_probe(p, 0, steps) for p in range(len(prob["probes"]))])}
    ctx.close()
    return out


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("params", [{}, {"kappa_max": 4.0, "alpha_max": 0.05}])
def test_cpml_matches_oracle(sbp, prec, params):
    from oracle import cpml as C
    prob = _problem(2, **params)
    init = random_fields(prob, 8)
    steps = 50
    g = _gpu(sbp, prob, prec, steps, init)
    r = C.run(prob, steps=steps, init=init)
    check_fields(g["fields"], r["fields"], prec, f"cpml {sorted(params.items())}")
    assert rel_l2(g["energy"], r["energy"]) < TOL[prec]
    assert rel_l2(g["probes"], r["probes"]) < TOL[prec]


def test_cpml_absorbs_like_the_oracle(sbp):
    """A modulated pulse leaving a 24^3 box through 8-cell layers on every
    face (fp64): the GPU probe series equals the oracle's, and the energy
    left in the box after the pulse has gone is small."""
    from oracle import cpml as C
    n = 24
    c = n // 2
    b = {"n": (n, n, n), "h": (1e-3,) * 3, "faces": ["cpml"] * 6, "eps_r": None, "mu_r": None, "sigma": None}
    prob = {"blocks": [b], "cfl": 0.9, "cpml": {"cells": 8},
            # t0 f0 = 1.5: the pulse carries no net charge (no static field stays behind)
            "sources": [{"block": 0, "comp": "Ez", "node": (c, c, c + 1), "waveform": "modgauss",
                         "tw": 6e-11, "t0": 5e-11, "f0": 3e10, "amp": 1.0}],
            "probes": [{"block": 0, "comp": "Ez", "node": (c + 2, c, c + 1)}]}
    steps = 400
    ctx = sbp.build_problem(prob, prec="f64", history=steps + 8)
    ctx.step(steps)
    gp = ctx.read_probe(0, 0, steps)
    ge = ctx.read_energy(0, steps)
    ctx.close()
    r = C.run(prob, steps=steps)
    assert rel_l2(gp, r["probes"][0]) < 1e-12
    assert rel_l2(ge, r["energy"]) < 1e-12
    assert ge[-1] < 1e-6 * ge.max()


def test_cpml_state_save_load_bitwise(sbp):
    import torch
    prob = _problem(3)
    init = random_fields(prob, 5)
    a = sbp.build_problem(prob, prec="f32", history=64)
    write_fields(a, init)
    a.step(30)
    ref = {c: a.read_field(0, c) for c in COMPS}
    a.close()
    b = sbp.build_problem(prob, prec="f32", history=64)
    write_fields(b, init)
    b.step(12)
    nb = b.state_bytes()
    buf = torch.empty(nb, dtype=torch.uint8, device="cuda")
    b.save_state(buf.data_ptr(), nb)
    b.step(7)                         # diverge, then restore and finish
    b.load_state(buf.data_ptr(), nb)
    b.step(18)
    for c in COMPS:
        assert np.array_equal(b.read_field(0, c), ref[c])
    b.close()
