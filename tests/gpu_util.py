"""Shared helpers of the GPU tests (no method arithmetic here)."""
import math

import numpy as np

COMPS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")


def rel_l2(a, b):
    """||a - b||_2 / ||b||_2 (the relative error measure of the parity bar)."""
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


def random_fields(problem, seed, scale=1.0):
    """Seeded random initial E^0 / H^{-1/2} per block and component."""
    from oracle.system import comp_shape
    rng = np.random.default_rng(seed)
    out = {}
    for b, blk in enumerate(problem["blocks"]):
        n = tuple(blk["n"])
        for c in COMPS:
            sx, sy, sz = comp_shape(c, n)
            out[(b, c)] = scale * rng.standard_normal((sz, sy, sx))
    return out


def gpu_fields(ctx, problem):
    return {(b, c): ctx.read_field(b, c) for b in range(len(problem["blocks"])) for c in COMPS}


def write_fields(ctx, fields):
    for (b, c), v in fields.items():
        ctx.write_field(b, c, v)


def field_errors(gpu, ref, floor=1e-6):
    """Relative L2 error per component array.

    A component whose reference norm is below ``floor`` times the largest
    component of the same field (E or H) is measured against that largest
    norm instead.  Its own relative error would measure the rounding of the
    larger components, not its own accuracy: e.g. Hz driven by an Ez point
    source in vacuum is zero up to fp64 rounding, and in a dielectric it is a
    few percent of Hx while carrying Hx-sized fp32 rounding.  The tests use
    floor 1e-6 for fp64 and 1e-1 for fp32, and also bound the per-field
    errors (all components of E, or of H, together: ``per_field_errors``)."""
    out = {}
    for k in ref:
        kind = k[-1][0] if isinstance(k, tuple) else k[0]
        big = max(float(np.linalg.norm(ref[q])) for q in ref
                  if (q[-1][0] if isinstance(q, tuple) else q[0]) == kind)
        own = float(np.linalg.norm(ref[k]))
        den = own if own >= floor * big else big
        out[k] = float(np.linalg.norm(gpu[k] - ref[k])) / (den if den > 0 else 1.0)
    return out


def per_field_errors(gpu, ref):
    """Relative L2 error of all E components together and of all H components together."""
    out = {}
    for kind in "EH":
        keys = [k for k in ref if (k[-1][0] if isinstance(k, tuple) else k[0]) == kind]
        num = math.sqrt(sum(float(np.linalg.norm(gpu[k] - ref[k])) ** 2 for k in keys))
        den = math.sqrt(sum(float(np.linalg.norm(ref[k])) ** 2 for k in keys))
        out[kind] = num / (den if den > 0 else 1.0)
    return out


FLOOR = {"f64": 1e-6, "f32": 1e-1}

EPS0 = 1.0 / (4e-7 * math.pi * 299792458.0 ** 2)
MU0 = 4e-7 * math.pi


def energy_norm_error(gpu, ref):
    """Relative error of (E, H) together in the vacuum energy norm,
    sqrt(sum eps0 dE^2 + mu0 dH^2) / sqrt(sum eps0 E^2 + mu0 H^2): the scale
    the method itself conserves.  Unlike the per-field errors it stays
    meaningful when one field decays, e.g. H after a Gaussian (non-zero mean)
    current pulse has ended and left a static E field."""
    num = den = 0.0
    for k in ref:
        w = EPS0 if (k[-1][0] if isinstance(k, tuple) else k[0]) == "E" else MU0
        num += w * float(np.sum((gpu[k] - ref[k]) ** 2))
        den += w * float(np.sum(ref[k] ** 2))
    return math.sqrt(num / den) if den > 0 else math.sqrt(num)


def block(n, h=(1e-3, 1e-3, 1e-3), faces=("pec",) * 6, **kw):
    d = {"n": tuple(n), "h": tuple(h), "origin": (0.0, 0.0, 0.0), "eps_r": None, "mu_r": None,
         "sigma": None, "faces": list(faces)}
    d.update(kw)
    return d
