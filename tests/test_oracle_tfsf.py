"""Pins of the oracle's total-field / scattered-field injection (oracle.tfsf, CPU)."""
import numpy as np
import pytest

from oracle import tfsf as T

N = (20, 12, 14)


def _problem(axis=0, pol=2, eps_box=None, faces=("pec",) * 6):
    eps = None
    if eps_box is not None:
        eps = np.ones((N[2], N[1], N[0]))
        eps[6:9, 5:7, 8:11] = eps_box
    blk = {"n": N, "h": (1e-3, 1.1e-3, 0.9e-3), "eps_r": eps, "mu_r": None, "sigma": None, "faces": list(faces)}
    box = [4, N[0] - 4, 4, N[1] - 4, 4, N[2] - 4]
    box[2 * axis] = 5
    tf = {"block": 0, "box": tuple(box), "axis": axis, "pol": pol, "margin": 16,
          "source": {"cell": -12, "waveform": "modgauss", "tw": 4e-11, "t0": 5e-11, "f0": 3e10, "amp": 1.0}}
    return {"blocks": [blk], "cfl": 0.9, "tfsf": tf}


@pytest.mark.parametrize("axis,pol", [(0, 2), (0, 1), (1, 0), (2, 1)])
def test_vacuum_scattered_region_stays_zero_and_total_is_incident(axis, pol):
    r = T.run(_problem(axis, pol), steps=110)
    mt_e, mt_h = r["mask_t"]
    ms_e, ms_h = r["mask_s"]
    e, h = r["e"], r["h"]
    big = np.abs(e[mt_e]).max()
    assert big > 1e-4
    assert np.abs(e[ms_e]).max() < 1e-12 * big
    assert np.abs(h[ms_h]).max() < 1e-12 * np.abs(h[mt_h]).max()
    assert np.abs(e[mt_e] - r["e_inc"][mt_e]).max() < 1e-12 * big
    assert np.abs(h[mt_h] - r["h_inc"][mt_h]).max() < 1e-12 * np.abs(h[mt_h]).max()


def test_planted_correction_sign_leaks():
    r = T.run(_problem(), steps=110, _flip=-1.0)
    mt_e, _ = r["mask_t"]
    ms_e, _ = r["mask_s"]
    assert np.abs(r["e"][ms_e]).max() > 1e-2 * np.abs(r["e"][mt_e]).max()


def test_scatterer_radiates_into_the_scattered_region():
    r = T.run(_problem(eps_box=4.0), steps=110)
    mt_e, _ = r["mask_t"]
    ms_e, _ = r["mask_s"]
    assert np.abs(r["e"][ms_e]).max() > 1e-3 * np.abs(r["e"][mt_e]).max()


def test_box_must_stay_inside_the_interior():
    p = _problem()
    p["tfsf"]["box"] = (3, 15, 4, 8, 4, 10)
    with pytest.raises(ValueError):
        T.run(p, steps=2)
