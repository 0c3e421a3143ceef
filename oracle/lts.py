"""Local time stepping at 1:p for refined blocks (oracle, test
infrastructure; fp64 on the CPU).

The paper defers multi-block coupling to later work, so it gives no local
time stepping; this is the reading used here, written from the explicit,
energy-conserving local time stepping for second-order wave equations of
Diaz and Grote (SIAM J. Sci. Comput. 31, 2009), applied to the lossless
SBP-SAT system.  Eliminating H from the leapfrog of Section V,
    H^{n+1/2} = H^{n-1/2} + dt B E^n,   E^{n+1} = E^n + dt A H^{n+1/2}
(B = mu^-1 K_he, A = eps^-1 K_eh), gives
    E^{n+1} - 2 E^n + E^{n-1} = -dt^2 L E^n,   L = -A B,
and M L is symmetric positive semidefinite in the energy weights M =
diag(eps w_E), because the SAT operator is skew in the E16 norm.  With P
the diagonal projector onto the E nodes of the refined blocks, one coarse
step of length dt advances the refined part with p substeps:
    w = L (I - P) E^n,
    q_0 = E^n,  q_1 = q_0 - (dt/p)^2 / 2 (w + L P q_0),
    q_{m+1} = 2 q_m - q_{m-1} - (dt/p)^2 (w + L P q_m),   m = 1 .. p-1,
    E^{n+1} = -E^{n-1} + 2 q_p.
This is E^{n+1} - 2 E^n + E^{n-1} = -dt^2 L_p E^n with L_p = (2/dt^2)(I - Q)
(Q: E^n -> q_p), M L_p symmetric, so
    W^{n+1/2} = 1/2 |E^{n+1} - E^n|_M^2 / dt^2 + 1/2 <E^{n+1}, M L_p E^n>
is conserved (the leapfrog energy of the scheme).  p = 1, or no refined
block, gives the global leapfrog exactly.  Each coarse step applies L once
to the whole state and p times to the refined part (with the coarse nodes it
couples to), so the coarse blocks advance at dt while only the refined
blocks (and their interface neighbours) pay the fine step.  Lossless blocks
only (PEC / PMC faces, interfaces); sources are not part of this reading.
`band` > 0 adds the coarse E nodes within that many cells of a face shared
with a refined block to the substepped part.
"""
import numpy as np

from . import system as S


class Lts:
    """The operators of the scheme for a problem whose blocks listed in
    `fine` are stepped with p substeps."""

    def __init__(self, problem, fine, p, band=0):
        for blk in problem["blocks"]:
            if blk.get("sigma") is not None or any(f == S.BC_ABC for f in blk["faces"]):
                raise ValueError("local time stepping covers lossless blocks")
        self.sys = S.System(problem)
        self.p = int(p)
        if self.p < 1:
            raise ValueError("p must be >= 1")
        sysm = self.sys
        self.P = np.zeros(sysm.ne)
        for b in fine:
            for c in S.E_COMPS:
                o = sysm.e_off[(b, c)]
                self.P[o:o + S.comp_size(c, tuple(sysm.blocks[b]["n"]))] = 1.0
        # the E nodes of a coarse block within `band` cells of a face it shares
        # with a refined block join the substepped part
        for (ba, fa, bb, fb, _r) in problem.get("interfaces", []):
            for (cb, cf, other) in ((ba, fa, bb), (bb, fb, ba)):
                if cb in fine or other not in fine or band <= 0:
                    continue
                n = tuple(sysm.blocks[cb]["n"])
                ax, hi = cf // 2, cf % 2
                for c in S.E_COMPS:
                    kind = S.GRID[c][ax]
                    m = n[ax] + 1 if kind == "+" else n[ax] + 2
                    pos = np.arange(m, dtype=float) if kind == "+" else np.clip(np.arange(m) - 0.5, 0, n[ax])
                    sel = pos >= n[ax] - band if hi else pos <= band
                    sx, sy, sz = S.comp_shape(c, n)
                    mask = np.zeros((sz, sy, sx), bool)
                    idx = [slice(None)] * 3
                    idx[2 - ax] = sel
                    mask[tuple(idx)] = True
                    o = sysm.e_off[(cb, c)]
                    self.P[o:o + mask.size] = np.maximum(self.P[o:o + mask.size], mask.reshape(-1))
        self.M = sysm.eps * sysm.w_e
        self.inv_mu = 1.0 / sysm.mu
        self.inv_eps = 1.0 / sysm.eps

    def L(self, v):
        """L v = -A B v."""
        sysm = self.sys
        return -self.inv_eps * (sysm.K_eh @ (self.inv_mu * (sysm.K_he @ v)))

    def Q(self, e, dt):
        """q_p of the substep recursion started from E^n = e."""
        p = self.p
        tau2 = (dt / p) ** 2
        w = self.L((1.0 - self.P) * e)
        q_prev = e
        q = e - 0.5 * tau2 * (w + self.L(self.P * e))
        for _ in range(1, p):
            q, q_prev = 2.0 * q - q_prev - tau2 * (w + self.L(self.P * q)), q
        return q

    def step(self, e_prev, e, dt):
        """E^{n+1} from E^{n-1}, E^n."""
        return -e_prev + 2.0 * self.Q(e, dt)

    def Lp(self, e, dt):
        """L_p e = (2/dt^2)(e - Q e)."""
        return (2.0 / dt ** 2) * (e - self.Q(e, dt))

    def energy(self, e_new, e, dt):
        """W^{n+1/2} of the scheme."""
        d = e_new - e
        return float(0.5 * np.dot(d, self.M * d) / dt ** 2 + 0.5 * np.dot(e_new, self.M * self.Lp(e, dt)))


def start(lts, e0, h_half, dt):
    """E^{-1} consistent with the leapfrog from E^0 and H^{-1/2}."""
    sysm = lts.sys
    return e0 - dt * lts.inv_eps * (sysm.K_eh @ h_half)


def run(problem, fine, p, steps, dt, init=None, band=0, dtype=np.float64):
    """E^0 .. E^steps of the scheme from init (E^0, H^{-1/2}); returns the
    E vectors at every step and W^{n+1/2} for n = 0 .. steps-1.

    dtype=np.float32 runs the same recursion with the operators, vectors and
    arithmetic in float32 (the energy still in fp64).  It is not a
    reference: its distance from the fp64 run measures the rounding the
    scheme itself incurs in that precision, which sizes the tolerance of an
    fp32 implementation."""
    lts = Lts(problem, fine, p, band)
    sysm = lts.sys
    if init is None:
        e = np.zeros(sysm.ne)
        h = np.zeros(sysm.nh)
    else:
        e, h = sysm.join(init)
    if dtype is np.float64:
        e_prev = start(lts, e, h, dt)
        step = lts.step
    else:
        A = sysm.K_eh.multiply(lts.inv_eps[:, None]).tocsr().astype(dtype)
        B = sysm.K_he.multiply(lts.inv_mu[:, None]).tocsr().astype(dtype)
        P = lts.P.astype(dtype)
        e, h = e.astype(dtype), h.astype(dtype)
        e_prev = (e - dtype(dt) * (A @ h)).astype(dtype)
        tau2 = dtype(dt / lts.p) ** 2

        def L(v):
            return -(A @ (B @ v))

        def step(ep, en, _dt):
            w = L((1 - P) * en)
            q_prev, q = en, en - dtype(0.5) * tau2 * (w + L(P * en))
            for _ in range(1, lts.p):
                q, q_prev = dtype(2) * q - q_prev - tau2 * (w + L(P * q)), q
            return -ep + dtype(2) * q
    hist = [e.copy()]
    energy = np.zeros(steps)
    for n in range(steps):
        e_new = step(e_prev, e, dt)
        energy[n] = lts.energy(e_new.astype(np.float64), e.astype(np.float64), dt)
        e_prev, e = e, e_new
        hist.append(e.copy())
    return {"e": hist, "energy": energy, "lts": lts}
