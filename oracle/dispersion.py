"""Numerical dispersion of the leapfrog step on a periodic box (Section IV).

Test infrastructure (the oracle), fp64 / complex128 on the CPU.

The procedure of Section IV: the state U^n = [E^n, H^{n-1/2}] of a box whose
faces are all periodic with the Bloch phase of a wave vector k0 (alpha_i =
k0_i times the box length, EPBC1-EPBC6) is advanced by one leapfrog step,
U^{n+1} = Lambda U^n (EDISPLAMBDA).  Each eigenvalue lambda_m of Lambda gives
a numerical wavenumber k_m = ln(lambda_m) / (j c dt) (E_NUMWN); the one
nearest the analytic k0 is compared with it through the dispersion,
dissipation and global errors (E_DISPER, E_DISSIP, E_GLOB) over one
wavelength lambda = 2 pi / k0.

Reading: the dissipation error is taken as |1 - e^{Im(k) lambda}|, the
amplitude change of e^{-j k lambda} over one wavelength (the printed form
puts j in the exponent, which would measure a phase).

``yee_periodic_operators`` is the classical Yee scheme on the same periodic
box (no closures), for which the procedure must reproduce the textbook
dispersion relation (sin(w dt/2)/(c dt))^2 = sum_i (sin(k_i h_i/2)/h_i)^2;
that pins the procedure itself.  The SBP-SAT numbers have no printed values
to compare with (parity unpinned); their qualitative properties are pinned:
no dissipation (|lambda| = 1, from the conserved energy E16 with EPBCP) and
a dispersion error not below the Yee scheme's.
"""
import cmath
import math

import numpy as np
import scipy.sparse as sp

from . import system as S


def amplification_matrix(k_eh, k_he, eps, mu, dt):
    """Lambda of EDISPLAMBDA for the lossless leapfrog step of Section V:
    H^{n+1/2} = H^{n-1/2} + dt/mu K_he E^n, E^{n+1} = E^n + dt/eps K_eh H^{n+1/2}."""
    a = sp.diags(dt / np.asarray(mu, float)) @ k_he     # H <- E
    b = sp.diags(dt / np.asarray(eps, float)) @ k_eh    # E <- H
    a = a.toarray()
    b = b.toarray()
    ne, nh = b.shape
    lam = np.zeros((ne + nh, ne + nh), dtype=complex)
    lam[:ne, :ne] = np.eye(ne) + b @ a
    lam[:ne, ne:] = b
    lam[ne:, :ne] = a
    lam[ne:, ne:] = np.eye(nh)
    return lam


def numerical_wavenumbers(eigenvalues, dt, c=S.C0):
    """E_NUMWN: k_m = ln(lambda_m) / (j c dt) (principal logarithm)."""
    return np.array([cmath.log(z) / (1j * c * dt) for z in eigenvalues])


def nearest(kts, k0):
    """The numerical wavenumber nearest the analytic one."""
    return kts[np.argmin(np.abs(kts - k0))]


def errors(k0, kt):
    """(dispersion, dissipation, global) errors of E_DISPER, E_DISSIP, E_GLOB."""
    lam = 2.0 * math.pi / k0
    disp = abs(cmath.exp(-1j * k0 * lam) - cmath.exp(-1j * kt.real * lam))
    diss = abs(1.0 - math.exp(kt.imag * lam))
    glob = abs(cmath.exp(-1j * k0 * lam) - cmath.exp(-1j * kt * lam))
    return disp, diss, glob


def sbp_box(n, h, alphas):
    """The SBP-SAT system of one vacuum block with all faces periodic."""
    blk = {"n": tuple(n), "h": tuple(h), "eps_r": None, "mu_r": None, "sigma": None,
           "faces": ["pec"] * 6}
    return S.System({"blocks": [blk], "periodic": [(0, a, alphas[a]) for a in range(3)]})


def sbp_wavenumber(n, h, k0_vec, dt):
    """Numerical wavenumber of the SBP-SAT scheme for the wave vector k0_vec on
    an n-cell periodic box (alpha_i = k0_i n_i h_i)."""
    alphas = [k0_vec[a] * n[a] * h[a] for a in range(3)]
    s = sbp_box(n, h, alphas)
    lam = amplification_matrix(s.K_eh, s.K_he, s.eps, s.mu, dt)
    k0 = float(np.linalg.norm(k0_vec))
    return nearest(numerical_wavenumbers(np.linalg.eigvals(lam), dt), k0), np.linalg.eigvals(lam)


def _diff_forward(m, h, alpha):
    """(u_{i+1} - u_i)/h on a periodic lattice of m nodes, u_m = e^{-j alpha} u_0."""
    d = np.zeros((m, m), dtype=complex)
    for i in range(m):
        d[i, i] -= 1.0 / h
        if i + 1 < m:
            d[i, i + 1] += 1.0 / h
        else:
            d[i, 0] += cmath.exp(-1j * alpha) / h
    return d


def _diff_backward(m, h, alpha):
    """(v_i - v_{i-1})/h on a periodic lattice of m nodes, v_{-1} = e^{+j alpha} v_{m-1}."""
    d = np.zeros((m, m), dtype=complex)
    for i in range(m):
        d[i, i] += 1.0 / h
        if i >= 1:
            d[i, i - 1] -= 1.0 / h
        else:
            d[i, m - 1] -= cmath.exp(1j * alpha) / h
    return d


def yee_periodic_operators(n, h, alphas):
    """K_eh, K_he of the Yee scheme on a periodic box of n cells per axis.

    Every component has n_x n_y n_z nodes (x fastest).  E <- H takes backward
    differences along the axes where H sits half a cell ahead; H <- E forward
    ones (E7-E12 without closures), with the Bloch phases at the wrap."""
    eye = [np.eye(n[a]) for a in range(3)]
    fwd = [_diff_forward(n[a], h[a], alphas[a]) for a in range(3)]
    bwd = [_diff_backward(n[a], h[a], alphas[a]) for a in range(3)]

    def along(mats, axis):
        m = [eye[0], eye[1], eye[2]]
        m[axis] = mats[axis]
        return np.kron(m[2], np.kron(m[1], m[0]))

    N = n[0] * n[1] * n[2]
    z = np.zeros((N, N))
    e_idx = {"Ex": 0, "Ey": 1, "Ez": 2}
    h_idx = {"Hx": 0, "Hy": 1, "Hz": 2}
    k_eh = [[z] * 3 for _ in range(3)]
    k_he = [[z] * 3 for _ in range(3)]
    for tgt, terms in S.CURL.items():
        for (src, axis, sgn) in terms:
            if tgt in e_idx:
                k_eh[e_idx[tgt]][h_idx[src]] = k_eh[e_idx[tgt]][h_idx[src]] + sgn * along(bwd, axis)
            else:
                k_he[h_idx[tgt]][e_idx[src]] = k_he[h_idx[tgt]][e_idx[src]] + sgn * along(fwd, axis)
    return np.block(k_eh), np.block(k_he)


def yee_wavenumber(n, h, k0_vec, dt):
    """Numerical wavenumber of the Yee scheme by the same eigen-procedure."""
    alphas = [k0_vec[a] * n[a] * h[a] for a in range(3)]
    k_eh, k_he = yee_periodic_operators(n, h, alphas)
    N = 3 * n[0] * n[1] * n[2]
    lam = amplification_matrix(sp.csr_matrix(k_eh), sp.csr_matrix(k_he), np.full(N, S.EPS0), np.full(N, S.MU0), dt)
    k0 = float(np.linalg.norm(k0_vec))
    return nearest(numerical_wavenumbers(np.linalg.eigvals(lam), dt), k0)


def yee_textbook_wavenumber(h, k_vec, dt, c=S.C0):
    """Closed form: the Yee dispersion relation solved for w, returned as w/c."""
    s = sum((math.sin(k_vec[a] * h[a] / 2.0) / h[a]) ** 2 for a in range(3))
    w = 2.0 / dt * math.asin(c * dt * math.sqrt(s))
    return w / c
