"""The five synthetic workloads, seeded.

Each ``make_config(k, scale=1)`` returns a problem dict:

  blocks:     list of {n: (nx, ny, nz) cells, h: (hx, hy, hz) metres,
                       origin: (x0, y0, z0), eps_r / mu_r / sigma: per-cell
                       arrays of shape (nz, ny, nx) (x fastest) or None,
                       faces: 6 names from "pec", "pmc", "abc" (-x,+x,-y,+y,-z,+z)}
  interfaces: list of (block_a, face_a, block_b, face_b, ratio)
  sources:    list of {block, comp, node (i,j,k), waveform, tw, t0, f0, amp}
  probes:     list of {block, comp, node}
  steps, cfl, prec ("f64" | "f32"), name
  (config 5 also: region (6 ints, cell box lo/hi), fd_cells, ckpt_every)

A probe or source placed "at cell (i, j, k)" uses the Ez node (i, j, k+1),
i.e. the node at (x_i, y_j, z_{k+1/2}).  Random numbers come from
numpy.random.default_rng([2206, k]) drawn in the order written below.
``scale`` divides every cell count (and the step count of the long runs) so
that the same recipe yields small parity cases.

These stand in for the paper's own workloads (a PEC cavity, a dielectric
resonator, an iris filter, a head model), whose geometry data and
measurement references are not available here.
"""
import math

import numpy as np

C0 = 299792458.0
CONFIG_NAMES = {
    1: "pec-cavity-16^3-fp64",
    2: "dielectric-boxes-256^3-fp32",
    3: "subgrid-1:2-27-blocks-fp32",
    4: "batched-64-cavities-fp32",
    5: "adjoint-96^3-fp32",
}


def nominal_dt(h, cfl):
    """Time unit of the source recipes: cfl * h / (c0 sqrt(3)) for a cubic mesh h."""
    return cfl * h / (C0 * math.sqrt(3.0))


def _ez_cell(block, cell, **kw):
    i, j, k = (int(v) for v in cell)
    d = {"block": block, "comp": "Ez", "node": (i, j, k + 1)}
    d.update(kw)
    return d


def _paint_boxes(rng, n, nbox, size_lo, size_hi, eps_lo=1.0, eps_hi=4.0):
    eps = np.ones((n[2], n[1], n[0]))
    for _ in range(nbox):
        lo = [int(rng.integers(0, n[a] - size_lo + 1)) for a in range(3)]
        sz = [int(rng.integers(size_lo, size_hi + 1)) for a in range(3)]
        val = float(rng.uniform(eps_lo, eps_hi))
        hi = [min(lo[a] + sz[a], n[a]) for a in range(3)]
        eps[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = val
    return eps


def config1(scale=1):
    rng = np.random.default_rng([2206, 1])
    n = 16
    h = 1e-3
    cfl = 0.9
    dt = nominal_dt(h, cfl)
    src = rng.integers(4, 12, size=3)
    probes = [rng.integers(2, 14, size=3) for _ in range(3)]
    return {
        "name": CONFIG_NAMES[1], "prec": "f64", "cfl": cfl, "steps": 200,
        "blocks": [{"n": (n, n, n), "h": (h, h, h), "origin": (0.0, 0.0, 0.0),
                    "eps_r": None, "mu_r": None, "sigma": None, "faces": ["pec"] * 6}],
        "interfaces": [],
        "sources": [_ez_cell(0, src, waveform="gauss", tw=40 * dt, t0=40 * dt, f0=0.0, amp=1.0)],
        "probes": [_ez_cell(0, p) for p in probes],
    }


def config2(scale=1):
    rng = np.random.default_rng([2206, 2])
    n = 256 // scale
    h = 1e-3
    cfl = 0.9
    eps = np.ones((n, n, n))
    for _ in range(32):
        lo = [int(rng.integers(0, 256 - 8 + 1)) for a in range(3)]
        sz = [int(rng.integers(8, 64 + 1)) for a in range(3)]
        val = float(rng.uniform(1.0, 4.0))
        lo = [v // scale for v in lo]
        hi = [min(lo[a] + max(sz[a] // scale, 1), n) for a in range(3)]
        eps[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = val
    src = [int(v) // scale for v in rng.integers(64, 192, size=3)]
    probes = [[int(v) // scale for v in rng.integers(16, 256 - 16, size=3)] for _ in range(3)]
    return {
        "name": CONFIG_NAMES[2], "prec": "f32", "cfl": cfl, "steps": 1000 // scale,
        "blocks": [{"n": (n, n, n), "h": (h, h, h), "origin": (0.0, 0.0, 0.0),
                    "eps_r": eps, "mu_r": None, "sigma": None, "faces": ["pec"] * 6}],
        "interfaces": [],
        "sources": [_ez_cell(0, src, waveform="modgauss", tw=0.2e-9, t0=0.2e-9, f0=10e9, amp=1.0)],
        "probes": [_ez_cell(0, p) for p in probes],
    }


def config3(scale=1):
    """Coarse 192^3 region (1 mm) with an embedded fine 96^3 block (0.5 mm)
    over coarse cells [72, 120)^3: 26 coarse blocks split 72+48+72 per axis
    around the fine block, all interfaces full-face."""
    rng = np.random.default_rng([2206, 3])
    hc = 1e-3
    hf = hc / 2
    cfl = 0.9
    split = [72 // scale, 48 // scale, 72 // scale]
    starts = [0, split[0], split[0] + split[1]]
    blocks, index = [], {}
    lossy_lo = [int(rng.integers(0, 9)) // scale for _ in range(3)]
    lossy_n = 64 // scale
    for c in range(3):
        for b in range(3):
            for a in range(3):
                fine = (a, b, c) == (1, 1, 1)
                pos = (a, b, c)
                n = tuple((2 * split[pos[t]] if fine else split[pos[t]]) for t in range(3))
                hh = hf if fine else hc
                origin = (starts[a] * hc, starts[b] * hc, starts[c] * hc)
                faces = []
                for t, idx in enumerate((a, b, c)):
                    faces.append("abc" if idx == 0 else "iface")
                    faces.append("abc" if idx == 2 else "iface")
                blk = {"n": n, "h": (hh, hh, hh), "origin": origin, "eps_r": None,
                       "mu_r": None, "sigma": None, "faces": faces}
                if (a, b, c) == (0, 0, 0):
                    sig = np.zeros((n[2], n[1], n[0]))
                    sig[lossy_lo[2]:lossy_lo[2] + lossy_n, lossy_lo[1]:lossy_lo[1] + lossy_n,
                        lossy_lo[0]:lossy_lo[0] + lossy_n] = rng.uniform(0.0, 0.1, (lossy_n,) * 3)
                    blk["sigma"] = sig
                index[(a, b, c)] = len(blocks)
                blocks.append(blk)
    interfaces = []
    for (a, b, c), ib in index.items():
        for t in range(3):
            nb = [a, b, c]
            nb[t] += 1
            if nb[t] > 2:
                continue
            jb = index[tuple(nb)]
            fine_a = (a, b, c) == (1, 1, 1)
            fine_b = tuple(nb) == (1, 1, 1)
            if fine_a:      # a fine, b coarse: ratio is cells of b per cell of a
                interfaces.append((jb, 2 * t, ib, 2 * t + 1, 2))
            elif fine_b:
                interfaces.append((ib, 2 * t + 1, jb, 2 * t, 2))
            else:
                interfaces.append((ib, 2 * t + 1, jb, 2 * t, 1))
    for blk in blocks:   # interface faces are described by the interface list
        blk["faces"] = [f if f != "iface" else "pec" for f in blk["faces"]]
    fine_id = index[(1, 1, 1)]
    nf = blocks[fine_id]["n"][0]
    src = [int(v) * nf // 96 for v in rng.integers(16, 80, size=3)]
    coarse_probes = []
    for _ in range(3):
        cell = rng.integers(0, 192, size=3) // scale
        # locate the coarse block holding the cell (skip the fine region)
        ab = [0 if v < starts[1] else (1 if v < starts[2] else 2) for v in cell]
        if tuple(ab) == (1, 1, 1):
            ab[0] = 0
            cell[0] = cell[0] % max(split[0], 1)
        blk = index[tuple(ab)]
        local = [int(cell[t] - starts[ab[t]]) for t in range(3)]
        coarse_probes.append(_ez_cell(blk, local))
    fine_probes = [_ez_cell(fine_id, [int(v) * nf // 96 for v in rng.integers(8, 88, size=3)])
                   for _ in range(3)]
    return {
        "name": CONFIG_NAMES[3], "prec": "f32", "cfl": cfl, "steps": 4000 // scale,
        "blocks": blocks, "interfaces": interfaces,
        "sources": [_ez_cell(fine_id, src, waveform="modgauss", tw=0.2e-9, t0=0.2e-9,
                             f0=10e9, amp=1.0)],
        "probes": coarse_probes + fine_probes,
        "fine_block": fine_id,
    }


def config4(scale=1, ncav=64):
    rng = np.random.default_rng([2206, 4])
    h = 1e-3
    cfl = 0.9
    dt = nominal_dt(h, cfl)
    blocks, sources, probes = [], [], []
    for c in range(ncav):
        n = tuple(max(int(rng.integers(32, 129)) // scale, 8) for _ in range(3))
        eps = np.ones((n[2], n[1], n[0]))
        for _ in range(4):
            lo = [int(rng.integers(0, n[a] - 4 + 1)) for a in range(3)]
            sz = [int(rng.integers(4, max(n[a] // 2, 4) + 1)) for a in range(3)]
            val = float(rng.uniform(1.0, 4.0))
            hi = [min(lo[a] + sz[a], n[a]) for a in range(3)]
            eps[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = val
        blocks.append({"n": n, "h": (h, h, h), "origin": (0.0, 0.0, 0.0), "eps_r": eps,
                       "mu_r": None, "sigma": None, "faces": ["pec"] * 6})
        s = [int(rng.integers(n[a] // 4, 3 * n[a] // 4)) for a in range(3)]
        sources.append(_ez_cell(c, s, waveform="gauss", tw=40 * dt, t0=40 * dt, f0=0.0, amp=1.0))
        p = [int(rng.integers(2, n[a] - 2)) for a in range(3)]
        probes.append(_ez_cell(c, p))
    return {"name": CONFIG_NAMES[4], "prec": "f32", "cfl": cfl, "steps": 100,
            "blocks": blocks, "interfaces": [], "sources": sources, "probes": probes}


def config5(scale=1):
    rng = np.random.default_rng([2206, 5])
    n = 96 // scale
    h = 1e-3
    cfl = 0.9
    L = n * h
    x = (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    g = np.zeros((n, n, n))
    for _ in range(8):
        while True:
            k = rng.integers(0, 4, size=3)
            if k.any():
                break
        a = rng.standard_normal()
        phi = rng.uniform(0.0, 2 * math.pi)
        g += a * np.cos(2 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z) / L + phi)
    eps = 2.5 + 1.5 * g / np.abs(g).max()
    lo = [int(v) * n // 96 for v in rng.integers(8, 85, size=3)]
    rsz = max(4 // scale, 2)
    region = (lo[0], lo[0] + rsz, lo[1], lo[1] + rsz, lo[2], lo[2] + rsz)
    while True:
        s = rng.integers(2, n - 2, size=3)
        d = max(max(lo[a] - s[a], s[a] - (lo[a] + rsz - 1), 0) for a in range(3))
        if d >= max(16 // scale, 3):
            break
    fd_cells = [tuple(int(v) for v in rng.integers(0, n, size=3)) for _ in range(20)]
    return {"name": CONFIG_NAMES[5], "prec": "f32", "cfl": cfl, "steps": 2000 // scale,
            "blocks": [{"n": (n, n, n), "h": (h, h, h), "origin": (0.0, 0.0, 0.0), "eps_r": eps,
                        "mu_r": None, "sigma": None, "faces": ["pec"] * 6}],
            "interfaces": [],
            "sources": [_ez_cell(0, s, waveform="modgauss", tw=0.2e-9, t0=0.2e-9, f0=10e9, amp=1.0)],
            "probes": [], "region": region, "fd_cells": fd_cells,
            "ckpt_every": max(45 // scale, 2)}


def bloch_box(n=192, frac=0.05, theta=0.6, phi=0.3, scale=1):
    """A vacuum box of n^3 cells at h = 1 mm with every face periodic, with
    the Bloch phases of an oblique plane wave (the setting of Section IV's
    oblique-incidence study: mesh lambda/20, i.e. k0 h / 2 pi = frac = 0.05,
    dt = 0.99 of the Yee limit); alpha_i = k0_i n h.  Fields are complex.  A
    modulated Gaussian Ez source at the centre (real part) excites it."""
    n = max(n // scale, 4)
    h = 1e-3
    k0 = 2.0 * math.pi * frac / h
    kv = (k0 * math.sin(theta) * math.cos(phi), k0 * math.sin(theta) * math.sin(phi), k0 * math.cos(theta))
    cfl = 0.99
    return {"name": f"bloch-periodic-{n}^3-complex-fp32", "prec": "f32", "cfl": cfl, "steps": 1000,
            "blocks": [{"n": (n, n, n), "h": (h, h, h), "origin": (0.0, 0.0, 0.0), "eps_r": None,
                        "mu_r": None, "sigma": None, "faces": ["pec"] * 6}],
            "interfaces": [], "periodic": [(0, a, kv[a] * n * h) for a in range(3)],
            "sources": [_ez_cell(0, (n // 2, n // 2, n // 2), waveform="modgauss", tw=0.2e-9, t0=0.2e-9,
                                 f0=10e9, amp=1.0)],
            "probes": [_ez_cell(0, (n // 4, n // 2, n // 2))], "wave_vector": kv}


def lossless_subgrid(scale=1):
    """The 1:2 subgrid geometry of config3 with its absorbing faces made PEC,
    no conductivity and no source or probe: the case local time stepping
    covers.  Returns (problem, index of the refined block)."""
    prob = config3(scale)
    blocks = []
    for b in prob["blocks"]:
        b = dict(b)
        b["faces"] = ["pec" if f == "abc" else f for f in b["faces"]]
        b["sigma"] = None
        blocks.append(b)
    return ({"name": prob["name"] + "-lossless", "prec": prob["prec"], "cfl": prob["cfl"], "steps": prob["steps"],
             "blocks": blocks, "interfaces": prob["interfaces"], "sources": [], "probes": []},
            prob["fine_block"])


def embedded_refinement(side=384, fine=24, h=1e-3):
    """A lossless coarse cube of `side` cells (PEC outer faces) with a cube of
    `fine` coarse cells at its centre refined 1:2: 27 blocks split
    (side - fine)/2 + fine + (side - fine)/2 per axis, the refined block
    holding 2 * fine cells per axis; no source or probe.  The shape of a
    small subgridded region in a large domain (where local time stepping
    pays).  Returns (problem, index of the refined block)."""
    a = (side - fine) // 2
    split = [a, fine, side - fine - a]
    starts = [0, split[0], split[0] + split[1]]
    blocks, index = [], {}
    for c in range(3):
        for b in range(3):
            for a3 in range(3):
                pos = (a3, b, c)
                refined = pos == (1, 1, 1)
                n = tuple((2 * split[pos[t]] if refined else split[pos[t]]) for t in range(3))
                hh = h / 2 if refined else h
                index[pos] = len(blocks)
                blocks.append({"n": n, "h": (hh, hh, hh), "origin": tuple(starts[pos[t]] * h for t in range(3)),
                               "eps_r": None, "mu_r": None, "sigma": None, "faces": ["pec"] * 6})
    interfaces = []
    for pos, ib in index.items():
        for t in range(3):
            nb = list(pos)
            nb[t] += 1
            if nb[t] > 2:
                continue
            jb = index[tuple(nb)]
            if pos == (1, 1, 1):
                interfaces.append((jb, 2 * t, ib, 2 * t + 1, 2))
            elif tuple(nb) == (1, 1, 1):
                interfaces.append((ib, 2 * t + 1, jb, 2 * t, 2))
            else:
                interfaces.append((ib, 2 * t + 1, jb, 2 * t, 1))
    return ({"name": f"embedded-refinement-{side}^3-{fine}^3-1:2-fp32", "prec": "f32", "cfl": 0.9, "steps": 100,
             "blocks": blocks, "interfaces": interfaces, "sources": [], "probes": []}, index[(1, 1, 1)])


def make_config(k, scale=1):
    return {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}[k](scale)
