"""GPU parity of periodic faces (EPBC1-EPBC6 with EPBCP) against the fp64
oracle: real fields with zero phase, and complex fields with a Bloch phase
(the HIP path holds the real and imaginary parts in two blocks whose
periodic faces mix them by cos / sin alpha).

The bar is the one of the other parity tests (``gpu_util.check_fields``):
relative L2 against the fp64 oracle, fp64 1e-12 per component array and per
field, fp32 1e-5 per field, and the probe and energy series likewise."""
import math

import numpy as np
import pytest

from gpu_util import COMPS, TOL, check_fields, rel_l2, write_fields

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def sbp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_00638_amd as p
    p.lib()
    return p


def _problem(seed, n, periodic, faces=("pec", "pec", "pmc", "pmc", "pec", "pec")):
    rng = np.random.default_rng(seed)
    shape = (n[2], n[1], n[0])
    b = {"n": tuple(n), "h": (1e-3, 1.1e-3, 0.9e-3), "faces": list(faces),
         "eps_r": rng.uniform(1.0, 3.0, shape), "mu_r": None, "sigma": None}
    return {"blocks": [b], "periodic": periodic, "cfl": 0.9,
            "sources": [{"block": 0, "comp": "Ez", "node": (2, 3, 3), "waveform": "modgauss",
                         "tw": 3e-11, "t0": 3e-11, "f0": 1e10, "amp": 1.0}],
            "probes": [{"block": 0, "comp": "Ez", "node": (1, 2, 2)},
                       {"block": 0, "comp": "Hx", "node": (0, 1, 1)}]}


def _complex_init(problem, seed):
    from oracle.system import comp_shape
    rng = np.random.default_rng(seed)
    n = tuple(problem["blocks"][0]["n"])
    out = {}
    for c in COMPS:
        sx, sy, sz = comp_shape(c, n)
        out[(0, c)] = rng.standard_normal((sz, sy, sx)) + 1j * rng.standard_normal((sz, sy, sx))
    return out


def _run(sbp, problem, prec, steps, init):
    ctx = sbp.build_problem(problem, prec=prec, history=steps + 8)
    im = ctx.imag_part.get(0)
    write_fields(ctx, {k: np.real(v) for k, v in init.items()})
    if im is not None:
        write_fields(ctx, {(im, c): np.imag(v) for (b, c), v in init.items()})
    ctx.step(steps)
    f = {(0, c): ctx.read_field(0, c) + (1j * ctx.read_field(im, c) if im is not None else 0.0) for c in COMPS}
    out = {"fields": f, "energy": ctx.read_energy(0, steps),
           "probes": np.array([ctx.read_probe(p, 0, steps) for p in range(len(problem["probes"]))])}
    ctx.close()
    return out


def _check(g, r, prec, complex_probes, label):
    check_fields(g["fields"], r["fields"], prec, label)
    assert rel_l2(g["energy"], r["energy"]) < TOL[prec]
    # probes sample the block of the real part
    assert rel_l2(g["probes"], np.real(r["probes"]) if complex_probes else r["probes"]) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_periodic_zero_phase(sbp, prec):
    from oracle import system as S
    prob = _problem(3, (11, 9, 13), [(0, 0, 0.0), (0, 2, 0.0)])
    init = {k: np.real(v) for k, v in _complex_init(prob, 5).items()}
    steps = 40
    g = _run(sbp, prob, prec, steps, init)
    r = S.run(prob, steps=steps, init=init)
    _check(g, r, prec, False, "periodic x, z zero phase")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("periodic", [[(0, 2, 1.3)], [(0, 0, 0.9), (0, 1, 0.0), (0, 2, -2.1)]])
def test_bloch_phase_complex_fields(sbp, prec, periodic):
    from oracle import system as S
    faces = ("pec", "pec", "pmc", "pmc", "pec", "pec")
    prob = _problem(4, (12, 10, 9), periodic, faces)
    init = _complex_init(prob, 6)
    steps = 40
    g = _run(sbp, prob, prec, steps, init)
    r = S.run(prob, steps=steps, init=init)
    assert np.iscomplexobj(r["e"])
    _check(g, r, prec, True, f"Bloch {periodic}")


def test_bloch_energy_conserved_and_graph(sbp):
    """All faces periodic with a Bloch phase, fp64: after the source has ended
    W^n stays constant (EPBCE with EPBCP), and graph replays give the eager
    result bit for bit."""
    prob = _problem(5, (16, 12, 20), [(0, 0, 0.4), (0, 1, -1.2), (0, 2, 2.5)])
    prob["sources"][0]["tw"] = 1.5e-11
    prob["sources"][0]["t0"] = 1.5e-11
    steps = 400
    eager = sbp.build_problem(prob, prec="f64", history=steps + 8)
    eager.step(steps)
    w = eager.read_energy(0, steps)
    assert w[150] > 0
    assert np.abs(w[150:] / w[150] - 1.0).max() < 1e-12
    import torch
    stream = torch.cuda.Stream()
    graph = sbp.build_problem(prob, prec="f64", history=steps + 8, stream=stream)
    graph.use_graph(100)
    graph.step(steps)
    stream.synchronize()
    for b in (0, graph.imag_part[0]):
        for c in COMPS:
            assert np.array_equal(graph.read_field(b, c), eager.read_field(b, c))
    assert np.array_equal(graph.read_energy(0, steps), w)
    eager.close()
    graph.close()


def test_set_periodic_errors(sbp):
    ctx = sbp.Context("f64")
    a = ctx.add_block((6, 6, 6), (1e-3,) * 3)
    b = ctx.add_block((6, 6, 7), (1e-3,) * 3)
    with pytest.raises(sbp.SbpError):
        ctx.set_periodic(a, 0, 0.5)           # a phase needs the imaginary part
    with pytest.raises(sbp.SbpError):
        ctx.set_periodic(a, 3, 0.0)           # bad axis
    with pytest.raises(sbp.SbpError):
        ctx.set_periodic(a, 1, 0.5, b)        # parts of different sizes
    ctx.set_periodic(a, 2, 0.0)
    with pytest.raises(sbp.SbpError):
        ctx.set_periodic(a, 2, 0.0)           # faces already coupled
    c = ctx.add_block((6, 6, 6), (1e-3,) * 3)
    d = ctx.add_block((6, 6, 6), (1e-3,) * 3)
    e = ctx.add_block((6, 6, 6), (1e-3,) * 3)
    ctx.set_periodic(c, 0, 0.3, d)
    with pytest.raises(sbp.SbpError):
        ctx.set_periodic(c, 1, 0.3, e)        # a second partner
    with pytest.raises(sbp.SbpError):
        ctx.set_periodic(d, 1, 0.3, c)        # the imaginary part as a real part
    with pytest.raises(sbp.SbpError):
        ctx.set_periodic(c, 1, 0.0)           # a complex block without its imaginary part
    with pytest.raises(sbp.SbpError):
        ctx.connect(c, 5, e, 4, 1)            # interfaces on a complex block
    ctx.set_periodic(c, 1, 0.0, d)            # zero phase on another axis of the pair
    ctx.close()


def test_bloch_eigenmode_rotates_by_its_eigenvalue(sbp):
    """Section IV on the GPU: the eigenvector of the one-step amplification
    matrix (oracle, dense eigen-decomposition) whose numerical wavenumber is
    nearest k0, stepped by the HIP path in fp64, is multiplied by its
    eigenvalue at every step; the wavenumber read back from the run
    (E_NUMWN) equals the eigen-analysis one."""
    import cmath
    from oracle import dispersion as D
    from oracle import system as S
    h = (1e-3, 1e-3, 1e-3)
    n = (4, 4, 4)
    k0 = 2.0 * math.pi * 0.08 / h[0]
    kv = (0.3 * k0, 0.0, math.sqrt(1 - 0.09) * k0)
    alphas = [kv[a] * n[a] * h[a] for a in range(3)]
    dt = 0.99 / (S.C0 * math.sqrt(3.0) / h[0])
    box = D.sbp_box(n, h, alphas)
    lam = D.amplification_matrix(box.K_eh, box.K_he, box.eps, box.mu, dt)
    ev, vec = np.linalg.eig(lam)
    kts = D.numerical_wavenumbers(ev, dt)
    m = int(np.argmin(np.abs(kts - k0)))
    u = vec[:, m] / np.abs(vec[:, m]).max()
    fields = box.split(u[:box.ne].copy(), u[box.ne:].copy())
    blk = {"n": n, "h": h, "faces": ["pec"] * 6, "eps_r": None, "mu_r": None, "sigma": None}
    prob = {"blocks": [blk], "periodic": [(0, a, alphas[a]) for a in range(3)], "sources": [], "probes": []}
    ctx = sbp.build_problem(prob, prec="f64", cfl=0.99)
    assert abs(ctx.dt - dt) < 1e-12 * dt
    im = ctx.imag_part[0]
    for (b, c), v in fields.items():
        ctx.write_field(0, c, np.real(v))
        ctx.write_field(im, c, np.imag(v))
    steps = 60
    ctx.step(steps)
    got = np.concatenate([(ctx.read_field(0, c) + 1j * ctx.read_field(im, c)).reshape(-1) for c in COMPS])
    ctx.close()
    want = np.concatenate([(ev[m] ** steps * fields[(0, c)]).reshape(-1) for c in COMPS])
    assert np.abs(got - want).max() < 1e-11
    # the wavenumber measured from the run: the mean rotation per step
    ratio = np.vdot(np.concatenate([fields[(0, c)].reshape(-1) for c in COMPS]), got) / \
        np.vdot(np.concatenate([fields[(0, c)].reshape(-1) for c in COMPS]),
                np.concatenate([fields[(0, c)].reshape(-1) for c in COMPS]))
    k_run = cmath.log(ratio) / (1j * S.C0 * dt * steps)
    # the principal log of lambda^steps wraps: compare modulo 2 pi / (c dt steps)
    wrap = 2.0 * math.pi / (S.C0 * dt * steps)
    d = (k_run - kts[m]).real
    assert abs(d - wrap * round(d / wrap)) < 1e-9 * abs(kts[m])
    assert abs(k_run.imag) < 1e-9 * abs(kts[m])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_bloch_box_workload_reduced(sbp, prec):
    """The benchmark's Bloch-periodic box recipe at 16^3 cells against the
    oracle (complex fields), 80 steps from rest with its source."""
    from oracle import system as S
    from sbp_inputs import bloch_box
    prob = bloch_box(scale=12)
    steps = 80
    ctx = sbp.build_problem(prob, prec=prec, history=steps + 8)
    ctx.step(steps)
    im = ctx.imag_part[0]
    g = {(0, c): ctx.read_field(0, c) + 1j * ctx.read_field(im, c) for c in COMPS}
    ge = ctx.read_energy(0, steps)
    gp = ctx.read_probe(0, 0, steps)
    ctx.close()
    r = S.run(prob, steps=steps)
    check_fields(g, r["fields"], prec, "Bloch box 16^3")
    assert rel_l2(ge, r["energy"]) < TOL[prec]
    assert rel_l2(gp, np.real(r["probes"][0])) < TOL[prec]
