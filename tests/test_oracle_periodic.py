"""Pins of the oracle's periodic faces (EPBC1-EPBC6, EPBCP) and of the
dispersion procedure of Section IV (CPU)."""
import cmath
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dispersion as D
from oracle import system as S

H = (1e-3, 1e-3, 1e-3)


def blk(n, h=H, faces=("pec",) * 6):
    return {"n": tuple(n), "h": tuple(h), "eps_r": None, "mu_r": None, "sigma": None, "faces": list(faces)}


def hermitian_skew_residual(sysm):
    g = sp.diags(sysm.w_e) @ sysm.K_eh
    f = sp.diags(sysm.w_h) @ sysm.K_he
    return abs(g + f.conj().T).max() / abs(g).max()


def march(sysm, dt, e, h, steps):
    ca, cb = sysm.coefficients(dt)
    for _ in range(steps):
        h = h + dt / sysm.mu * (sysm.K_he @ e)
        e = ca * e + cb * (sysm.K_eh @ h)
    return e, h


@pytest.mark.parametrize("alphas", [(0.0, None, 0.0), (0.7, None, None), (None, 1.9, -0.4), (0.3, 2.2, math.pi)])
def test_periodic_energy_rate_zero(alphas):
    # EPBCE with EPBCP: dE/dt = 0 for any phase -> W_E K_eh + (W_H K_he)^H = 0
    per = [(0, a, al) for a, al in enumerate(alphas) if al is not None]
    s = S.System({"blocks": [blk((4, 5, 6), (1e-3, 1.3e-3, 0.8e-3), ("pec", "pec", "pmc", "pmc", "pec", "pmc"))],
                  "periodic": per})
    assert s.complex == any(al != 0.0 for (_, _, al) in per)
    assert hermitian_skew_residual(s) < 1e-15


def test_zero_phase_is_real_and_two_pi_equals_zero():
    a = S.System({"blocks": [blk((4, 4, 5))], "periodic": [(0, 2, 0.0)]})
    b = S.System({"blocks": [blk((4, 4, 5))], "periodic": [(0, 2, 2.0 * math.pi)]})
    assert not a.complex and b.complex
    assert abs(a.K_eh - b.K_eh).max() < 1e-12 * abs(a.K_eh).max()
    assert abs(a.K_he - b.K_he).max() < 1e-12 * abs(a.K_he).max()


def _ring_vs_bloch(M, m, steps=25, conj_phase=False):
    """A Bloch-periodic block with alpha = 2 pi m / M along z against M copies
    of it joined in a ring by conforming interfaces: copy q must carry
    e^{-j alpha q} times the Bloch solution (u(z + L) = e^{-j alpha} u(z))."""
    n = (4, 5, 4)
    alpha = 2.0 * math.pi * m / M
    faces = ("pec", "pec", "pmc", "pmc", "pec", "pec")
    bloch = S.System({"blocks": [blk(n, faces=faces)], "periodic": [(0, 2, alpha)]})
    if conj_phase:  # planted mistake: the opposite sign convention
        bloch.face_phase = {k: v.conjugate() for k, v in bloch.face_phase.items()}
        bloch._assemble()
    ring = S.System({"blocks": [blk(n, faces=faces) for _ in range(M)],
                     "interfaces": [(q, 5, (q + 1) % M, 4, 1) for q in range(M)]})
    rng = np.random.default_rng(7)
    e0 = rng.standard_normal(bloch.ne) + 1j * rng.standard_normal(bloch.ne)
    h0 = rng.standard_normal(bloch.nh) + 1j * rng.standard_normal(bloch.nh)
    dt = 0.9 * S.cfl_dt([blk(n)], 1.0)
    ph = [cmath.exp(-1j * alpha * q) for q in range(M)]
    er = np.concatenate([p * e0 for p in ph])
    hr = np.concatenate([p * h0 for p in ph])
    eb, hb = march(bloch, dt, e0, h0, steps)
    er, hr = march(ring, dt, er.astype(complex), hr.astype(complex), steps)
    err = 0.0
    for q in range(M):
        err = max(err, np.abs(er[q * bloch.ne:(q + 1) * bloch.ne] - ph[q] * eb).max() / np.abs(eb).max(),
                  np.abs(hr[q * bloch.nh:(q + 1) * bloch.nh] - ph[q] * hb).max() / np.abs(hb).max())
    return err


@pytest.mark.parametrize("M,m", [(4, 1), (4, 3), (3, 1), (2, 1)])
def test_bloch_block_equals_ring_of_blocks(M, m):
    assert _ring_vs_bloch(M, m) < 1e-12


def test_planted_conjugate_phase_breaks_ring():
    assert _ring_vs_bloch(4, 1, conj_phase=True) > 1e-3


def test_bloch_leapfrog_energy_conserved():
    prob = {"blocks": [blk((5, 4, 6))], "periodic": [(0, 0, 0.9), (0, 2, -2.1)], "cfl": 0.95, "steps": 300,
            "sources": [{"block": 0, "comp": "Ez", "node": (2, 2, 3), "waveform": "gauss", "amp": 1.0,
                         "tw": 30 * 1.8e-12, "t0": 30 * 1.8e-12}]}
    r = S.run(prob)
    w = r["energy"][200:]
    assert np.iscomplexobj(r["e"])
    assert np.abs(w - w[0]).max() < 1e-13 * w[0]


# ------------------------------------------------------------ Section IV
def _dt(h, frac=0.99):
    return frac / (S.C0 * math.sqrt(sum(1.0 / x ** 2 for x in h)))


@pytest.mark.parametrize("frac", [0.05, 0.1, 0.2])
@pytest.mark.parametrize("angles", [(0.0, 0.0), (0.6, 0.3), (1.1, 2.0)])
def test_eigen_procedure_reproduces_yee_dispersion_relation(frac, angles):
    # the procedure applied to the Yee scheme must give the textbook relation
    th, ph = angles
    k0 = 2.0 * math.pi * frac / H[0]
    kv = (k0 * math.sin(th) * math.cos(ph), k0 * math.sin(th) * math.sin(ph), k0 * math.cos(th))
    n = (4, 4, 4)
    dt = _dt(H)
    kt = D.yee_wavenumber(n, H, kv, dt)
    ref = D.yee_textbook_wavenumber(H, kv, dt)
    assert abs(kt - ref) < 1e-12 * ref


@pytest.mark.parametrize("frac", [0.05, 0.1])
def test_sbp_dispersion_no_dissipation_and_not_below_yee(frac):
    # Section IV: negligible dissipation, dispersion error at least the Yee scheme's
    k0 = 2.0 * math.pi * frac / H[0]
    kv = (0.0, 0.0, k0)
    dt = _dt(H)
    ks, ev = D.sbp_wavenumber((4, 4, 4), H, kv, dt)
    ky = D.yee_wavenumber((4, 4, 4), H, kv, dt)
    assert np.abs(np.abs(ev) - 1.0).max() < 1e-12
    ds, dis, gs = D.errors(k0, ks)
    dy, _, gy = D.errors(k0, ky)
    assert dis < 1e-10
    assert ds >= dy and gs >= gy
