"""Pins of the oracle's local time stepping (oracle.lts, CPU): one substep
and no refined block are the global leapfrog; beyond the fine block's CFL
limit, where the global leapfrog blows up, the scheme conserves its energy
and stays bounded; its energy operator is symmetric with the stability
bound dt^2 L_p < 4 holding there; second-order convergence to the global
solution."""
import numpy as np
import pytest

from oracle import lts as T
from oracle import system as S

COMPS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")


def _problem(nA=(8, 6, 6)):
    """A 2 mm block with a 1 mm block (1:2) on its +x face."""
    A = {"n": nA, "h": (2e-3,) * 3, "origin": (0.0, 0.0, 0.0), "eps_r": None, "mu_r": None, "sigma": None,
         "faces": ["pec", "iface", "pec", "pmc", "pec", "pec"]}
    nB = (8, 2 * nA[1], 2 * nA[2])
    B = {"n": nB, "h": (1e-3,) * 3, "origin": (nA[0] * 2e-3, 0.0, 0.0), "eps_r": None, "mu_r": None,
         "sigma": None, "faces": ["iface", "pec", "pmc", "pec", "pec", "pec"]}
    return {"blocks": [A, B], "interfaces": [(0, 1, 1, 0, 2)], "cfl": 0.9}


def _positions(kind, n, h, x0):
    if kind == "+":
        return x0 + np.arange(n + 1) * h
    return x0 + np.clip(np.arange(n + 2) - 0.5, 0, n) * h


def _smooth_init(prob, scale_h=1.0 / 377.0):
    """E = 0 and a Gaussian bump of Hz centred in the coarse block."""
    out = {}
    c = np.array([8e-3, 6e-3, 6e-3])
    for b, blk in enumerate(prob["blocks"]):
        n, h, x0 = blk["n"], blk["h"], blk["origin"]
        for comp in COMPS:
            sx, sy, sz = S.comp_shape(comp, tuple(n))
            if comp != "Hz":
                out[(b, comp)] = np.zeros((sz, sy, sx))
                continue
            g = S.GRID[comp]
            xs = [_positions(g[a], n[a], h[a], x0[a]) for a in range(3)]
            r2 = ((xs[2][:, None, None] - c[2]) ** 2 + (xs[1][None, :, None] - c[1]) ** 2 +
                  (xs[0][None, None, :] - c[0]) ** 2)
            out[(b, comp)] = scale_h * np.exp(-r2 / (3e-3) ** 2)
    return out


def _random_init(prob, seed):
    rng = np.random.default_rng(seed)
    out = {}
    for b, blk in enumerate(prob["blocks"]):
        for comp in COMPS:
            sx, sy, sz = S.comp_shape(comp, tuple(blk["n"]))
            v = rng.standard_normal((sz, sy, sx))
            out[(b, comp)] = v / 377.0 if comp[0] == "H" else v
    return out


def _leapfrog_e(prob, init, steps, dt):
    r = S.run(dict(prob, steps=steps), steps=steps, dt=dt, init=init)
    e, _ = S.System(prob).join(r["fields"])
    return e


@pytest.mark.parametrize("fine,p", [([1], 1), ([], 2), ([], 3)])
def test_reduces_to_the_leapfrog(fine, p):
    prob = _problem()
    init = _random_init(prob, 1)
    dt = S.cfl_dt(prob["blocks"], 0.9)
    r = T.run(prob, fine, p, 30, dt, init)
    ref = _leapfrog_e(prob, init, 30, dt)
    assert np.abs(r["e"][-1] - ref).max() < 1e-12 * np.abs(ref).max()


def test_energy_conserved_beyond_the_fine_cfl():
    prob = _problem()
    init = _random_init(prob, 2)
    dt = 1.5 * S.cfl_dt(prob["blocks"], 0.9)  # 1.35x the fine block's Yee limit
    r = T.run(prob, [1], 2, 300, dt, init)
    w = r["energy"]
    assert w[0] > 0
    assert np.abs(w / w[0] - 1).max() < 1e-11
    big = np.abs(r["e"][0]).max()
    assert max(np.abs(e).max() for e in r["e"]) < 30 * big
    # the global leapfrog at the same step blows up
    with np.errstate(all="ignore"):
        g = T.run(prob, [1], 1, 300, dt, init)
        last = np.abs(g["e"][-1]).max()
    assert not np.isfinite(last) or last > 1e6 * big


def test_energy_operator_symmetric_and_within_the_stability_bound():
    prob = _problem((4, 6, 6))
    dt = 1.5 * S.cfl_dt(prob["blocks"], 0.9)
    lts = T.Lts(prob, [1], 2)
    ne = lts.sys.ne
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(ne), rng.standard_normal(ne)
    a = np.dot(lts.M * lts.Lp(x, dt), y)
    b = np.dot(x, lts.M * lts.Lp(y, dt))
    assert abs(a - b) < 1e-12 * abs(a)
    # largest eigenvalue of the symmetric form by power iteration: dt^2 L_p < 4
    s = np.sqrt(lts.M)
    v = rng.standard_normal(ne)
    lam = 0.0
    for _ in range(400):
        u = s * lts.Lp(v / s, dt)
        lam = float(np.dot(v, u) / np.dot(v, v))
        v = u / np.linalg.norm(u)
    assert 0.0 < dt * dt * lam < 4.0


def test_second_order_convergence():
    prob = _problem()
    init = _smooth_init(prob)
    dt0 = 1.2 * S.cfl_dt(prob["blocks"], 0.9)
    steps = 40
    ref = _leapfrog_e(prob, init, 8 * steps, dt0 / 8)
    errs = []
    for q in (1, 2):
        r = T.run(prob, [1], 2, q * steps, dt0 / q, init)
        errs.append(np.linalg.norm(r["e"][-1] - ref) / np.linalg.norm(ref))
    assert errs[0] < 0.2
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


def _node_distance(prob, fine):
    """Chebyshev distance, in the block's own cells, of every E node from the
    box of the refined block (0 inside)."""
    sysm = S.System(prob)
    F = prob["blocks"][fine]
    lo = np.array(F["origin"])
    hi = lo + np.array(F["n"]) * np.array(F["h"])
    dist = np.zeros(sysm.ne)
    for b, blk in enumerate(prob["blocks"]):
        n, h, x0 = blk["n"], blk["h"], blk["origin"]
        for c in ("Ex", "Ey", "Ez"):
            xs = [_positions(S.GRID[c][a], n[a], h[a], x0[a]) for a in range(3)]
            d = [np.maximum(np.maximum(lo[a] - xs[a], xs[a] - hi[a]), 0.0) / h[a] for a in range(3)]
            D = np.maximum(np.maximum(d[2][:, None, None], d[1][None, :, None]), d[0][None, None, :])
            o = sysm.e_off[(b, c)]
            dist[o:o + D.size] = D.reshape(-1)
    return dist


def test_refined_coupling_reaches_one_cell():
    """The 27-block 1:2 subgrid geometry (reduced, absorbing faces made PEC):
    L P x vanishes on every E node more than one of its block's cells from
    the refined block, and the refined rows of L E read no E beyond one
    cell.  A correction that only touches the refined block's neighbourhood
    (a few cells wide) therefore carries the whole difference between the
    local and the global step."""
    from sbp_inputs import lossless_subgrid
    prob, fine = lossless_subgrid(8)
    lts = T.Lts(prob, [fine], 2)
    dist = _node_distance(prob, fine)
    rng = np.random.default_rng(5)
    y = lts.L(lts.P * rng.standard_normal(lts.sys.ne))
    reach = dist[np.abs(y) > 0].max()
    assert 0.5 < reach <= 1.0 + 1e-9, reach
    e = rng.standard_normal(lts.sys.ne)
    ref = lts.P * lts.L(e)
    got = lts.P * lts.L(e * (dist <= 1.0 + 1e-9))
    assert np.array_equal(got, ref)
    # and the reach is real: cutting at half a cell changes the refined rows
    cut = lts.P * lts.L(e * (dist <= 0.4))
    assert np.abs(cut - ref).max() > 1e-3 * np.abs(ref).max()


def test_float32_run_follows_the_fp64_run():
    """The float32 mode (which sizes the fp32 tolerance of the GPU path) is
    the same recursion: close to the fp64 run, not equal to it, and its
    energy constant to fp32 rounding."""
    prob = _problem()
    init = _random_init(prob, 2)
    dt = 1.5 * S.cfl_dt(prob["blocks"], 0.9)
    r64 = T.run(prob, [1], 2, 40, dt, init)
    r32 = T.run(prob, [1], 2, 40, dt, init, dtype=np.float32)
    assert r32["e"][-1].dtype == np.float32
    err = np.linalg.norm(r32["e"][-1] - r64["e"][-1]) / np.linalg.norm(r64["e"][-1])
    assert 1e-8 < err < 1e-4, err
    w = r32["energy"]
    assert np.abs(w / w[0] - 1).max() < 1e-4
