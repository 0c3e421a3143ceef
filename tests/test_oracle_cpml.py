"""Pins of the oracle's convolutional PML (oracle.cpml, CPU)."""
import numpy as np
import pytest

from oracle import cpml as C
from oracle import system as S

H = 1e-3
N, D, STEPS, PAD = 24, 8, 150, 40


def _blk(n, faces):
    return {"n": (n,) * 3, "h": (H,) * 3, "eps_r": None, "mu_r": None, "sigma": None, "faces": list(faces)}


def _src_probes(n):
    c = n // 2
    src = [{"block": 0, "comp": "Ez", "node": (c, c, c + 1), "waveform": "modgauss", "amp": 1.0,
            "tw": 6e-11, "t0": 6e-11, "f0": 3e10}]
    # two cells inside the layer's inner boundary, and near the source
    probes = [{"block": 0, "comp": "Ez", "node": (c + N // 2 - D - 2, c, c + 1)},
              {"block": 0, "comp": "Ez", "node": (c, c + 3, c + 1)}]
    return src, probes


def _small(faces, cp=None):
    src, probes = _src_probes(N)
    p = {"blocks": [_blk(N, faces)], "cfl": 0.9, "steps": STEPS, "sources": src, "probes": probes}
    if cp is not None:
        p["cpml"] = cp
    return p


@pytest.fixture(scope="module")
def reference(oracle_lib):
    """The same source and probes in a PEC box PAD cells larger on every
    side: no reflection reaches the probes within the steps simulated."""
    src, probes = _src_probes(N + 2 * PAD)
    big = {"blocks": [_blk(N + 2 * PAD, ["pec"] * 6)], "cfl": 0.9, "steps": STEPS, "sources": src, "probes": probes}
    dt = S.cfl_dt(big["blocks"], 0.9)
    return dt, oracle_lib.run_block(big, dt=dt)["probes"]


def _err(p, ref):
    return max(np.abs(p[q] - ref[q]).max() / np.abs(ref[q]).max() for q in range(len(ref)))


def test_zero_strength_layer_is_the_plain_scheme():
    faces = ["cpml", "pec", "pec", "cpml", "pec", "cpml"]
    src = [{"block": 0, "comp": "Ez", "node": (5, 4, 4), "waveform": "gauss", "amp": 1.0, "tw": 2e-11, "t0": 2e-11}]
    blk = {"n": (10, 8, 9), "h": (H,) * 3, "eps_r": None, "mu_r": None, "sigma": None, "faces": faces}
    p = {"blocks": [blk], "cfl": 0.9, "steps": 60, "sources": src,
         "cpml": {"cells": 3, "sigma_factor": 0.0, "kappa_max": 1.0, "alpha_max": 0.0}}
    r = C.run(p)
    q = dict(p)
    q["blocks"] = [dict(blk, faces=["pec"] * 6)]
    r2 = S.run(q)
    scale = max(np.abs(r2["e"]).max(), 1e-300)
    assert np.abs(r["e"] - r2["e"]).max() < 1e-13 * scale
    assert np.abs(r["h"] - r2["h"]).max() < 1e-13 * np.abs(r2["h"]).max()


def test_layer_absorbs_outgoing_wave(reference):
    dt, ref = reference
    e_cpml = _err(C.run(_small(["cpml"] * 6, {"cells": D}), dt=dt)["probes"], ref)
    e_abc = _err(S.run(_small(["abc"] * 6), dt=dt)["probes"], ref)
    assert e_cpml < 3e-4
    assert e_cpml < e_abc / 30


def test_planted_wrong_recursion_sign_breaks_absorption(reference, monkeypatch):
    dt, ref = reference
    real = C.axis_profile

    def flipped(*a, **k):
        b, c, ik = real(*a, **k)
        return b, -c, ik
    monkeypatch.setattr(C, "axis_profile", flipped)
    assert _err(C.run(_small(["cpml"] * 6, {"cells": D}), dt=dt)["probes"], ref) > 1e-3


def test_profiles_at_the_node_positions():
    # "-" grid: nodes 0, (j - 1/2) h, n h; the face node sits at depth 1
    x = C.node_positions("-", 6, 1.0)
    assert np.allclose(x, [0, 0.5, 1.5, 2.5, 3.5, 4.5, 5.5, 6])
    p = dict(C.DEFAULT)
    b, c, ik = C.axis_profile("+", 10, 1e-3, 4, 0, p, 1e-12)
    assert b[0] < b[1] < b[2] < b[3] < 1.0 and np.all(b[4:] == 1.0) and np.all(c[4:] == 0.0)
