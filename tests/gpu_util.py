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


# The parity bar (relative L2 error against the fp64 oracle).
TOL = {"f64": 1e-12, "f32": 1e-5}

# A component whose oracle norm is below ZERO times the largest component of
# the same field is zero in exact arithmetic (e.g. Hz of an Ez point source
# in vacuum): the fp64 oracle holds only its rounding, so its own relative
# error is undefined and it is measured against that largest norm instead.
ZERO = 1e-6

# Per-component errors of every check, printed in the session summary.
REPORT = []


def _kind(k):
    return k[-1][0] if isinstance(k, tuple) else k[0]


def field_errors(gpu, ref):
    """Relative L2 error of each component array against its own reference
    norm; components that are zero in exact arithmetic (below ZERO times the
    largest norm of the same field) against that largest norm."""
    out = {}
    for k in ref:
        big = max(float(np.linalg.norm(ref[q])) for q in ref if _kind(q) == _kind(k))
        own = float(np.linalg.norm(ref[k]))
        den = own if own >= ZERO * big else big
        out[k] = float(np.linalg.norm(gpu[k] - ref[k])) / (den if den > 0 else 1.0)
    return out


def per_field_errors(gpu, ref):
    """Relative L2 error of all E components together and of all H components together."""
    out = {}
    for kind in "EH":
        keys = [k for k in ref if _kind(k) == kind]
        num = math.sqrt(sum(float(np.linalg.norm(gpu[k] - ref[k])) ** 2 for k in keys))
        den = math.sqrt(sum(float(np.linalg.norm(ref[k])) ** 2 for k in keys))
        out[kind] = num / (den if den > 0 else 1.0)
    return out


def check_fields(gpu, ref, prec, label, tol=None, scale=None):
    """The field part of the parity bar: the error of each field (all E
    components together, all H components together) relative to that
    field's norm is below `tol` (1e-12 fp64, 1e-5 fp32).

    ``scale`` ({"E": norm, "H": norm}) replaces the field's current norm as
    the denominator; runs whose fields decay (energy leaving through
    absorbing faces) pass the largest norm the field reached so far.

    Each component's own relative error is recorded (session summary) and
    returned, not asserted: a component much weaker than the others of its
    field (Hz beside Hx in a dielectric, or the Hz an interface stirs up
    beside an Ez source) carries their rounding, which enters its curl terms
    at their size, so its own error exceeds the field's by about the ratio
    of the norms, in either precision.
    Returns (per-component errors, per-field errors)."""
    tol = TOL[prec] if tol is None else tol
    own = field_errors(gpu, ref)
    num = {kind: math.sqrt(sum(float(np.linalg.norm(gpu[k] - ref[k])) ** 2 for k in ref if _kind(k) == kind))
           for kind in "EH"}
    den = {kind: math.sqrt(sum(float(np.linalg.norm(ref[k])) ** 2 for k in ref if _kind(k) == kind))
           for kind in "EH"}
    now = {kind: num[kind] / (den[kind] if den[kind] > 0 else 1.0) for kind in "EH"}
    if scale is not None:
        fld = {kind: num[kind] / max(scale[kind], den[kind], 1e-300) for kind in "EH"}
    else:
        fld = now
    REPORT.append({"check": label, "prec": prec, "field": fld, "field_now": now if scale is not None else None,
                   "comp": {(k[-1] if isinstance(k, tuple) and len(k) == 2 and k[0] == 0 else k): v
                            for k, v in own.items()}})
    assert max(fld.values()) < tol, (label, prec, fld, own)
    return own, fld


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
