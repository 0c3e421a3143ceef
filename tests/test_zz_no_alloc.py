"""The allocation-free step (sbp_step_static, through the C ABI) against
sbp_step: bitwise equal fields, probes and energies on two calls in a row,
the second on a smaller problem (fewer partial sums and face values than
the first left in the fixed scratch array), and a clear refusal of a launch
shape that needs more partial sums than the array holds."""
import numpy as np
import pytest

from gpu_util import COMPS, block, random_fields, write_fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_00638_amd as p
    p.lib()
    return p


def _run(sbp, prob, prec, init, steps, static):
    ctx = sbp.build_problem(prob, prec=prec, history=steps + 8)
    write_fields(ctx, init)
    if static:
        ctx.step_static(steps)
    else:
        ctx.step(steps)
    nb = len(prob["blocks"])
    out = ({(b, c): ctx.read_field(b, c) for b in range(nb) for c in COMPS}, ctx.read_energy(0, steps),
           np.array([ctx.read_probe(k, 0, steps) for k in range(len(prob.get("probes", [])))]))
    assert ctx.steps_done() == steps
    ctx.close()
    return out


def _small_pair():
    """A coarse block below a fine one in y at 1:2, with loss and an
    absorbing face: far fewer tiles and face values than the first case."""
    rng = np.random.default_rng(5)
    a = block((6, 5, 7), faces=("pec", "pmc", "pec", "pec", "abc", "pec"), sigma=rng.uniform(0, 0.3, (7, 5, 6)))
    b = block((12, 10, 14), (5e-4, 5e-4, 5e-4), faces=("pec", "pec", "pec", "pmc", "pec", "pec"))
    b["origin"] = (0.0, 5e-3, 0.0)
    return {"blocks": [a, b], "interfaces": [(0, 3, 1, 2, 2)], "cfl": 0.9,
            "sources": [{"block": 1, "comp": "Ez", "node": (4, 3, 3), "waveform": "gauss",
                         "tw": 2e-11, "t0": 2e-11, "f0": 0.0, "amp": 1.0}],
            "probes": [{"block": 0, "comp": "Ey", "node": (3, 2, 2)},
                       {"block": 1, "comp": "Hx", "node": (2, 3, 4)}]}


def test_step_static_equals_step_on_two_calls(sbp):
    from sbp_inputs import make_config
    cases = [(make_config(3, scale=2), "f32", 40), (_small_pair(), "f64", 35)]
    for q, (prob, prec, steps) in enumerate(cases):
        init = random_fields(prob, 17 + q, scale=1e-3)
        ref = _run(sbp, prob, prec, init, steps, static=False)
        got = _run(sbp, prob, prec, init, steps, static=True)
        for k in ref[0]:
            assert np.array_equal(got[0][k], ref[0][k]), (q, k)
        assert np.array_equal(got[1], ref[1]), q
        assert np.array_equal(got[2], ref[2]), q


def test_step_static_refuses_oversized_launch(sbp):
    from paper_2206_00638_amd.binding import SBP_EINVAL, SbpError
    prob = {"blocks": [block((256, 256, 256))], "interfaces": [], "cfl": 0.9, "sources": [], "probes": []}
    # 64-node tiles of one plane: 1041 * 258 = 269 K tiles, a workgroup
    # each, two partial sums per workgroup (H and E launches)
    ctx = sbp.build_problem(prob, prec="f32", launch=(64, 1, 1, 0))
    with pytest.raises(SbpError) as e:
        ctx.step_static(1)
    assert e.value.status == SBP_EINVAL
    assert "partial sums" in str(e.value)
    assert ctx.steps_done() == 0
    ctx.step(1)  # the allocating step still serves it
    assert ctx.steps_done() == 1
    ctx.close()
