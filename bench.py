"""Benchmark of the SBP-SAT FDTD leapfrog step on one MI355X.

One "step" is one leapfrog step (H half step, E step, energy W^n, source and
probe samples) of the dielectric-boxes workload: one 256^3-cell block, 32
seeded dielectric boxes (eps_r in [1, 4]), PEC faces, modulated-Gaussian Ez
source, fp32 fields with fp64 energy accumulation.  Inputs are resident in
HBM before timing.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1]

Extra keys: the fp64 path on the same workload, the field error of both
paths against the fp64 oracle on a reduced case of the same recipe (per
field and per component), the roofline of the dominant kernel (algorithmic
bytes / mean launch time from HIP events on the kernel's stream), the other
workloads (batched cavities, 1:2 subgrid, CPML, TF/SF, Bloch box, adjoint;
fp64 beside fp32 for the batched and adjoint legs), same-harness bandwidth
references, the paper's own figures with its hardware, and the oracle timed
on the host cores (all cores and one) on a bounded sample of the workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def node_counts(n):
    nx, ny, nz = n
    e = (nx + 2) * (ny + 1) * (nz + 1) + (nx + 1) * (ny + 2) * (nz + 1) + (nx + 1) * (ny + 1) * (nz + 2)
    h = (nx + 1) * (ny + 2) * (nz + 2) + (nx + 2) * (ny + 1) * (nz + 2) + (nx + 2) * (ny + 2) * (nz + 1)
    return e, h


def plain(block):
    """Blocks the one-pass step takes: PEC / PMC faces only, no conductivity,
    no per-cell permeability (interfaces are listed separately)."""
    return (block.get("sigma") is None and block.get("mu_r") is None
            and all(f in ("pec", "pmc") for f in block["faces"]))


_TABLED = {}


def tabled(block, elem):
    """Whether the library holds the block's permittivity as byte indices
    into a table: at most 64 distinct values in the field precision."""
    eps = block.get("eps_r")
    if eps is None:
        return False
    key = (id(eps), elem)
    if key not in _TABLED:
        import numpy as np
        dt = np.float32 if elem == 4 else np.float64
        _TABLED[key] = (eps, np.unique(np.asarray(eps, dtype=dt)).size <= 64)
    return _TABLED[key][1]


def algorithmic_bytes(problem, elem, fused=False):
    """Bytes each launch group must move per step: every node read once and
    written once per update, the other field read once (two passes) or both
    fields read and written once (one pass), per-cell materials read once
    (the permittivity of a plain block with at most 64 distinct values as one
    byte per cell: its table index).  Returns (H pass, E pass, one pass)."""
    eb = hb = fb = 0
    iface = {a for (a, _, b, _, _) in problem.get("interfaces", [])} | \
        {b for (_, _, b, _, _) in problem.get("interfaces", [])}
    for q, b in enumerate(problem["blocks"]):
        ne, nh = node_counts(b["n"])
        cells = b["n"][0] * b["n"][1] * b["n"][2]
        e_mats = sum(1 for k in ("eps_r", "sigma") if b.get(k) is not None)
        h_mats = 1 if b.get("mu_r") is not None else 0
        if fused and plain(b) and q not in iface:
            fb += elem * (2 * ne + 2 * nh + e_mats * cells)
        else:
            tf = (problem.get("tfsf") or {}).get("block")
            lean = plain(b) and q not in iface and tf != q and tabled(b, elem)
            eb += elem * (2 * ne + nh + e_mats * cells) - ((elem - 1) * cells if lean else 0)
            hb += elem * (2 * nh + ne + h_mats * cells)
    return hb, eb, fb


def traffic_entry(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_2206_00638_amd", "csrc", "step.hip")
    try:
        with open(path) as fh:
            t = json.load(fh)
        with open(src, "rb") as fh:
            h = hashlib.sha256(fh.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if t.get("step_hip_sha256") != h:
        return None
    return t.get("kernels", {}).get(kernel)


def run_gpu(problem, prec, steps, warmup, profile_kernels, fused=False):
    import torch
    from paper_2206_00638_amd import build_problem
    stream = torch.cuda.Stream()
    ctx = build_problem(problem, prec=prec, stream=stream, history=max(steps + warmup + 8, 64))
    if fused:
        ctx.set_fused(True, 8)
    ctx.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ctx.last_step_ms()
    kern = None
    if profile_kernels:
        ctx.profile(True)
        ctx.step(min(steps, 50))
        torch.cuda.synchronize()
        kern = ctx.kernel_ms()
        ctx.profile(False)
    launch = ctx.get_launch()
    n = ctx.steps_done()
    energy = ctx.read_energy(n - 1, 1)[0]
    ctx.close()
    return {"wall_s": wall, "event_ms": ev_ms, "kernel_ms": kern, "launch": launch, "last_energy": energy}


def batched(steps, warmup, prec="f32", tune=True):
    """The batched workload: 64 uneven cavities (sides 32..128, 32.8 M cells)
    in one tile list, launch shape from the autotuner, steps replayed from
    HIP graphs of min(steps, 100) steps: the timed steps are a whole number
    of replays."""
    import numpy as np
    import torch
    from paper_2206_00638_amd import build_problem
    from sbp_inputs import make_config
    prob = make_config(4)
    cells = int(sum(np.prod(b["n"]) for b in prob["blocks"]))
    gsteps = max(1, min(steps, 100))
    replays = -(-steps // gsteps)
    timed = replays * gsteps
    stream = torch.cuda.Stream()
    ctx = build_problem(prob, prec=prec, stream=stream, history=max(timed + warmup + 8, 64))
    tune_ms = ctx.autotune(5) if tune else None
    launch = ctx.get_launch()
    ctx.use_graph(gsteps)
    ctx.step(-(-warmup // gsteps) * gsteps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(timed)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    elem = 4 if prec == "f32" else 8
    hb, eb, fb = algorithmic_bytes(prob, elem)
    ms = wall * 1e3 / timed
    return {"workload": prob["name"] if prec == "f32" else prob["name"].replace("fp32", "fp64"),
            "cells": cells, "blocks": len(prob["blocks"]), "steps": timed,
            "graph_steps": gsteps, "graph_replays": replays, "launch": list(launch), "autotune_ms_per_step": tune_ms,
            "value": cells * timed / wall / 1e6, "unit": "Mcell-updates/s", "ms_per_step": ms,
            "step_hbm_gbs_algorithmic": (hb + eb + fb) / (ms * 1e-3) / 1e9}


def batched_accuracy(steps=100, sample=3):
    """fp32 and fp64 error of the batched run against the fp64 loop oracle
    on its smallest cavities (each stepped alone by the oracle, with the
    batched problem's time step), per field and per component."""
    import numpy as np
    from oracle import loops
    from oracle.system import cfl_dt
    from paper_2206_00638_amd import build_problem
    from sbp_inputs import make_config
    prob = make_config(4)
    sizes = [int(np.prod(b["n"])) for b in prob["blocks"]]
    pick = sorted(range(len(sizes)), key=lambda b: sizes[b])[:sample]
    dt = cfl_dt(prob["blocks"], prob["cfl"])
    refs = {}
    for b in pick:
        one = {"blocks": [prob["blocks"][b]], "interfaces": [], "cfl": prob["cfl"],
               "sources": [dict(q, block=0) for q in prob["sources"] if q["block"] == b], "probes": []}
        refs[b] = loops.run_block(one, steps=steps, dt=dt)["fields"]
    out = {"workload": f"batched cavities {pick} (the smallest), {steps} steps"}
    for prec in ("f32", "f64"):
        ctx = build_problem(prob, prec=prec)
        ctx.step(steps)
        got = {b: {c: ctx.read_field(b, c) for c in COMPS} for b in pick}
        ctx.close()
        out[prec] = field_error_report({(b, c): got[b][c] for b in pick for c in COMPS},
                                       {(b, c): refs[b][c] for b in pick for c in COMPS})
    return out


def bloch(steps, warmup):
    """Periodic faces with a Bloch phase: a 192^3 vacuum box, complex fields
    (two 192^3 blocks holding the real and imaginary parts), fp32, phases of
    an oblique wave at lambda/20; launch shape from the autotuner."""
    import numpy as np
    import torch
    from paper_2206_00638_amd import build_problem
    from sbp_inputs import bloch_box
    prob = bloch_box()
    cells = int(np.prod(prob["blocks"][0]["n"]))
    stream = torch.cuda.Stream()
    ctx = build_problem(prob, prec="f32", stream=stream, history=max(steps + warmup + 8, 64))
    ctx.autotune(5)
    launch = ctx.get_launch()
    ctx.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile(True)
    ctx.step(20)
    torch.cuda.synchronize()
    kern = ctx.kernel_ms()
    ctx.close()
    hb, eb, fb = algorithmic_bytes(prob, 4)
    ms = wall * 1e3 / steps
    return {"workload": prob["name"], "complex_cells": cells, "real_blocks": 2, "steps": steps,
            "launch": list(launch),
            "value": cells * steps / wall / 1e6, "unit": "Mcell-updates/s (complex cells)",
            "ms_per_step": ms, "kernels_ms": list(kern),
            "step_hbm_gbs_algorithmic": 2 * (hb + eb + fb) / (ms * 1e-3) / 1e9}


def cpml_problem(tfsf=False):
    """The dielectric-boxes 256^3 recipe behind 10-cell CPML layers, with a
    TF/SF plane wave if `tfsf`; (problem, workload name)."""
    from sbp_inputs import make_config
    prob = make_config(2)
    prob["blocks"][0]["faces"] = ["cpml"] * 6
    prob["cpml"] = {"cells": 10}
    name = "dielectric-boxes-256^3-fp32-cpml10"
    if tfsf:
        n = prob["blocks"][0]["n"]
        prob["tfsf"] = {"block": 0, "box": (16, n[0] - 16, 16, n[1] - 16, 16, n[2] - 16), "axis": 2, "pol": 0,
                        "margin": 16, "source": {"cell": -12, "waveform": "modgauss", "tw": 2e-10, "t0": 2.5e-10,
                                                 "f0": 1e10, "amp": 1.0}}
        name += "-tfsf16"
    return prob, name


def cpml_leg(steps, warmup, tfsf=False):
    """The dielectric-boxes 256^3 fp32 workload with every face a PEC face
    behind a 10-cell convolutional PML (the truncation of the paper's open
    examples) instead of a PEC cavity wall; with `tfsf`, the boxes also
    scatter a plane wave (along +z, E along x) brought in through a
    total-field / scattered-field box 16 cells inside the faces."""
    import numpy as np
    import torch
    from paper_2206_00638_amd import build_problem
    prob, name = cpml_problem(tfsf)
    cells = int(np.prod(prob["blocks"][0]["n"]))
    stream = torch.cuda.Stream()
    ctx = build_problem(prob, prec="f32", stream=stream, history=max(steps + warmup + 8, 64))
    ctx.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile(True)
    ctx.step(20)
    torch.cuda.synchronize()
    kern = ctx.kernel_ms()
    ctx.close()
    ms = wall * 1e3 / steps
    return {"workload": name, "cells": cells, "steps": steps,
            "value": cells * steps / wall / 1e6, "unit": "Mcell-updates/s", "ms_per_step": ms,
            "kernels_ms": list(kern)}


def subgrid(steps, warmup, prec="f32"):
    """The 1:2 subgrid workload: 27 blocks (coarse 192^3 region at 1 mm around
    a fine 96^3 block at 0.5 mm), absorbing outer faces, a lossy box."""
    import numpy as np
    import torch
    from paper_2206_00638_amd import build_problem
    from sbp_inputs import make_config
    prob = make_config(3)
    cells = int(sum(np.prod(b["n"]) for b in prob["blocks"]))
    stream = torch.cuda.Stream()
    ctx = build_problem(prob, prec=prec, stream=stream, history=max(steps + warmup + 8, 64))
    ctx.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile(True)
    ctx.step(20)
    torch.cuda.synchronize()
    kern = ctx.kernel_ms()
    ctx.close()
    hb, eb, fb = algorithmic_bytes(prob, 4 if prec == "f32" else 8)
    ms = wall * 1e3 / steps
    return {"workload": prob["name"] if prec == "f32" else prob["name"].replace("fp32", "fp64"), "cells": cells,
            "blocks": len(prob["blocks"]), "interfaces": len(prob["interfaces"]), "steps": steps,
            "value": cells * steps / wall / 1e6, "unit": "Mcell-updates/s", "ms_per_step": ms,
            "kernels_ms": list(kern), "step_hbm_gbs_algorithmic": (hb + eb + fb) / (ms * 1e-3) / 1e9}


def fp32_vs_fp64(prob, steps=240):
    """The fp32 fields of `prob` against its fp64 run after `steps` steps
    (every block, the imaginary-part blocks of complex fields included).  The
    fp64 run is the reference: the GPU tests pin the fp64 path to the oracle
    on these recipes (at full size for the subgrid workload, reduced for the
    periodic, CPML and TF/SF ones)."""
    import torch
    from paper_2206_00638_amd import build_problem
    runs = {}
    for prec in ("f32", "f64"):
        ctx = build_problem(prob, prec=prec, stream=torch.cuda.Stream(), history=steps + 8)
        ctx.step(steps)
        nb = len(prob["blocks"]) + len(ctx.imag_part)
        runs[prec] = {(b, c): ctx.read_field(b, c) for b in range(nb)
                      for c in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")}
        ctx.close()
    return dict(field_accuracy(runs["f32"], runs["f64"]), steps=steps)


def subgrid_accuracy(steps=240):
    """The subgrid workload's fp32 fields against its fp64 run after `steps`
    steps (240: the source's peak, while the pulse is inside the domain;
    later most of it has left through the absorbing faces and a relative
    error would be taken against what remains)."""
    from sbp_inputs import make_config
    return fp32_vs_fp64(make_config(3), steps)


def field_accuracy(got, ref):
    """Relative L2 error per field (E, H over all blocks) and per component,
    against the reference run; a component below 1e-6 of its field's norm in
    the reference (zero in exact arithmetic) is measured against the field's
    norm instead."""
    import numpy as np
    out = {}
    for group, comps in (("E", ("Ex", "Ey", "Ez")), ("H", ("Hx", "Hy", "Hz"))):
        num = sum(float(np.sum((got[k] - ref[k]) ** 2)) for k in ref if k[1] in comps)
        den = sum(float(np.sum(ref[k] ** 2)) for k in ref if k[1] in comps)
        out[f"{group}_rel_l2"] = (num / den) ** 0.5
    comp, frac, zero = {}, {}, []
    for c in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"):
        num = sum(float(np.sum((got[k] - ref[k]) ** 2)) for k in ref if k[1] == c)
        den = sum(float(np.sum(ref[k] ** 2)) for k in ref if k[1] == c)
        tot = sum(float(np.sum(ref[k] ** 2)) for k in ref if k[1][0] == c[0])
        frac[c] = (den / tot) ** 0.5
        if frac[c] < 1e-6:  # zero in exact arithmetic: its error against the field's norm
            comp[c] = (num / tot) ** 0.5
            zero.append(c)
        else:
            comp[c] = (num / den) ** 0.5
    out["components_rel_l2"] = comp
    out["components_norm_over_field_norm"] = frac  # a weak component's relative error is large
    out["components_zero_in_exact_arithmetic"] = zero
    return out


def _lts_case(prob, fine, coarse_steps, warmup, init_blocks):
    """Global leapfrog against local time stepping (refined block substepped
    twice per coarse step of twice the global step) on one problem, from the
    same seeded fields in `init_blocks` (zero elsewhere); energy not formed."""
    import numpy as np
    import torch
    from paper_2206_00638_amd import build_problem
    cells = int(sum(np.prod(b["n"]) for b in prob["blocks"]))

    def fresh():
        rng = np.random.default_rng(7)
        ctx = build_problem(prob, prec="f32", stream=torch.cuda.Stream(), history=2 * (coarse_steps + warmup) + 64)
        for b in init_blocks:
            for c in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"):
                shp = ctx.field_shape(b, c)
                ctx.write_field(b, c, rng.standard_normal(shp[::-1]) * (1.0 if c[0] == "E" else 1.0 / 377.0))
        return ctx

    def timed(fn, n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(n)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n

    g = fresh()
    dt = g.dt
    g.step(2 * warmup)
    ms_global = timed(g.step, 2 * coarse_steps)
    g.close()
    c = fresh()
    c.lts_start([fine], 2, 2.0 * dt, 0)
    c.lts_step(warmup)
    ms = timed(c.lts_step, coarse_steps)
    info = c.lts_info()
    c.close()
    return {"workload": prob["name"], "cells": cells, "refined_block": fine,
            "refined_cells_frac": float(np.prod(prob["blocks"][fine]["n"])) / cells, "substeps": 2,
            "dt_coarse_over_global": 2.0, "global_ms_per_step": ms_global, "lts_ms_per_coarse_step": ms,
            "near": info, "speedup_same_physical_time": 2.0 * ms_global / ms,
            "value": cells * 2.0 / (ms * 1e-3) / 1e6,
            "unit": "Mcell-updates/s of the global leapfrog covering the same physical time"}


def lts_leg(coarse_steps, warmup):
    """Local time stepping (lossless problems, fp32; the refined block takes 2
    substeps per coarse step of twice the global step), timed beside the
    global leapfrog over the same physical time: the subgrid geometry of
    config 3 made lossless (the refined block 11% of the cells; seeded random
    fields everywhere), with the cost of forming W^{n+1/2} every 100 steps
    and its drift over a run that forms it every step; and a 384^3 coarse
    region with a 24-cell refined cube at its centre (0.2% of the cells;
    seeded random fields in the refined block)."""
    import numpy as np
    import torch
    from paper_2206_00638_amd import build_problem
    from sbp_inputs import embedded_refinement, lossless_subgrid
    prob, fine = lossless_subgrid(1)
    rec = _lts_case(prob, fine, coarse_steps, warmup, range(len(prob["blocks"])))
    # the energy: every 100 steps (cost) and every step (drift)
    rng = np.random.default_rng(7)
    for every in (100, 1):
        c = build_problem(prob, prec="f32", stream=torch.cuda.Stream(), history=2 * (coarse_steps + warmup) + 64)
        for b in range(len(prob["blocks"])):
            for comp in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"):
                shp = c.field_shape(b, comp)
                c.write_field(b, comp, rng.standard_normal(shp[::-1]) * (1.0 if comp[0] == "E" else 1.0 / 377.0))
        c.lts_start([fine], 2, 2.0 * c.dt, every)
        if every == 100:
            c.lts_step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.lts_step(coarse_steps)
            torch.cuda.synchronize()
            rec["lts_ms_per_coarse_step_energy_every_100"] = (time.perf_counter() - t0) * 1e3 / coarse_steps
        else:
            n = min(coarse_steps, 200)
            c.lts_step(n)
            w = c.read_energy(0, n)
            rec["energy_drift_fp32"] = float(np.abs(w / w[0] - 1.0).max())
            rec["energy_steps"] = n
        c.close()
    prob2, fine2 = embedded_refinement(384, 24)
    rec["embedded_refinement"] = _lts_case(prob2, fine2, min(coarse_steps, 100), warmup, [fine2])
    return rec


def adjoint_leg(prec="f32"):
    """The adjoint workload: 96^3, J over 2000 steps, checkpoints every 45
    steps; one sbp_adjoint call (forward run, segment replays, reverse
    sweep) timed, next to the forward run alone.  Returns the record and
    the gradient (host array)."""
    import numpy as np
    import torch
    from paper_2206_00638_amd import build_problem
    from sbp_inputs import make_config
    prob = make_config(5)
    n = prob["blocks"][0]["n"]
    cells = int(np.prod(n))
    steps = prob["steps"]
    stream = torch.cuda.Stream()
    ctx = build_problem(prob, prec=prec, stream=stream, history=steps + 8)
    nb = ctx.state_bytes()
    snap = torch.empty(nb, dtype=torch.uint8, device="cuda")
    ctx.save_state(snap.data_ptr(), nb)
    grad = torch.zeros((n[2], n[1], n[0]), dtype=torch.float64, device="cuda")
    ctx.adjoint(0, steps, prob["region"], grad.data_ptr(), prob["ckpt_every"])  # warm-up
    ctx.load_state(snap.data_ptr(), nb)
    grad.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = ctx.adjoint(0, steps, prob["region"], grad.data_ptr(), prob["ckpt_every"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.load_state(snap.data_ptr(), nb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    ctx.close()
    rec = {"workload": prob["name"] if prec == "f32" else prob["name"].replace("fp32", "fp64"),
           "cells": cells, "steps": steps, "ckpt_every": prob["ckpt_every"],
           "J": J, "gradient_s": wall, "forward_s": fwd, "gradient_over_forward": wall / fwd,
           "value": cells * steps / wall / 1e6,
           "unit": "Mcell-updates/s (forward-step equivalents per second of the gradient)"}
    return rec, grad.cpu().numpy()


COMPS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")


def field_error_report(got, ref):
    """Relative L2 errors against the oracle: per field (all E, all H
    components together), of both fields together in the vacuum energy norm
    (eps0 |dE|^2 + mu0 |dH|^2: meaningful when one field has decayed, as H
    has after a Gaussian current pulse that left a static E field) and each
    component on its own."""
    import numpy as np
    num = {"E": 0.0, "H": 0.0}
    den = {"E": 0.0, "H": 0.0}
    comp = {}
    for k, r in ref.items():
        c = k[-1] if isinstance(k, tuple) else k
        d = float(np.sum((got[k] - r) ** 2))
        q = float(np.sum(r * r))
        num[c[0]] += d
        den[c[0]] += q
        key = c if not isinstance(k, tuple) else f"{k[0]}/{c}"
        comp[key] = math.sqrt(d / q) if q > 0 else math.sqrt(d)
    eps0, mu0 = 8.8541878128e-12, 1.25663706212e-6
    energy = math.sqrt((eps0 * num["E"] + mu0 * num["H"]) / (eps0 * den["E"] + mu0 * den["H"]))
    return {"E_rel_l2": math.sqrt(num["E"] / den["E"]), "H_rel_l2": math.sqrt(num["H"] / den["H"]),
            "energy_norm_rel": energy, "components_rel_l2": comp}


def accuracy(scale):
    """Field/probe/energy error of the fp32 and fp64 paths against the fp64
    loop oracle on the same recipe at 256/scale cells per axis."""
    import numpy as np
    from oracle import loops
    from paper_2206_00638_amd import build_problem
    from sbp_inputs import make_config
    prob = make_config(2, scale=scale)
    steps = prob["steps"]
    ref = loops.run_block(prob)
    out = {"workload": f"same recipe at {prob['blocks'][0]['n'][0]}^3, {steps} steps"}
    for prec in ("f32", "f64"):
        ctx = build_problem(prob, prec=prec)
        ctx.step(steps)
        got = {c: ctx.read_field(0, c) for c in COMPS}
        pr = np.array([ctx.read_probe(p, 0, steps) for p in range(len(prob["probes"]))])
        en = ctx.read_energy(0, steps)
        ctx.close()
        out[prec] = field_error_report(got, ref["fields"])
        out[prec]["probe_rel_l2"] = float(np.linalg.norm(pr - ref["probes"]) / np.linalg.norm(ref["probes"]))
        out[prec]["energy_rel"] = float(np.linalg.norm(en - ref["energy"]) / np.linalg.norm(ref["energy"]))
    return out


def copy_ceiling():
    """Same-harness references for HBM bandwidth on 1 GiB fp32 arrays (far
    above the 256 MB Infinity Cache): a device-to-device copy (one read and
    one write per element) and torch's vectorised elementwise add c = a + b
    (two reads, one write); bytes moved over the best of 5 runs, timed with
    torch.cuda events on the current stream."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.ones(n, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)

    def best(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        t = None
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            t = ms if t is None else min(t, ms)
        return t

    t_copy = best(lambda: c.copy_(a))
    t_add = best(lambda: torch.add(a, b, out=c))
    del a, b, c
    gb = (1 << 30) / 1e9
    return {"copy_gbs": 2 * gb / (t_copy * 1e-3), "add_gbs": 3 * gb / (t_add * 1e-3),
            "note": "1 GiB fp32 arrays: device-to-device copy (1 read + 1 write) and c = a + b (2 reads + 1 write)"}


def pattern_ceiling(h_ms, e_ms):
    """The update kernels' own access patterns on the 256^3 node box (the
    probe library: same loads, stores, tiles and tile walk, no closure rows,
    energy or probes), timed in this process; the algorithmic bytes of the H
    and E launches over the probe times give the pattern's attainable rate,
    and the kernels' times over the probe times the cost of everything else.
    The stream probe keeps the E launch's bytes (six components and the
    cells' permittivity table indices read, three components written in
    place) without the neighbour reads: the rate that mix of streams reaches
    on its own."""
    import ctypes
    import os
    from sbp_inputs import make_config
    lib = ctypes.CDLL(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2206_00638_amd",
                                   "libsbppattern.so"))
    out = (ctypes.c_double * 3)()
    rc = lib.sbp_pattern_time(256, 128, 8, 50, out)
    if rc != 0:
        raise RuntimeError(f"pattern probe failed: HIP error {rc}")
    hb, eb, _ = algorithmic_bytes(make_config(2), 4)
    return {"h_pattern_ms": out[0], "e_pattern_ms": out[1], "e_streams_ms": out[2],
            "h_pattern_gbs": hb / (out[0] * 1e-3) / 1e9, "e_pattern_gbs": eb / (out[1] * 1e-3) / 1e9,
            "e_streams_gbs": eb / (out[2] * 1e-3) / 1e9,
            "h_kernel_over_pattern": h_ms / out[0], "e_kernel_over_pattern": e_ms / out[1],
            "e_kernel_over_streams": e_ms / out[2],
            "note": "128 threads x 8 planes, grouped tile walk; algorithmic bytes of the 256^3 H and E launches"}


def host_cpu():
    """CPU model and the number of cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count()
    return model, ncpu


_ALL_THREADS = []


def all_threads():
    """The oracle's thread count before any one-thread run (a one-thread run
    leaves OpenMP at one thread, and thread count 0 keeps that setting), so
    every all-core run passes it explicitly."""
    if not _ALL_THREADS:
        from oracle import loops
        _ALL_THREADS.append(loops.max_threads())
    return _ALL_THREADS[0]


def progress(msg):
    """A line on stderr per finished measurement (the JSON line stays alone on
    stdout)."""
    print(msg, file=sys.stderr, flush=True)


def grow_rate(timed, cells, target_s):
    """Cell-updates per second from `timed(steps)` (wall seconds of one call,
    its set-up included): a call of 1 step, then calls of k + 1 steps with k
    growing until the k steps beyond the first call take about target_s (the
    set-up cancels in the difference)."""
    t1 = timed(1)
    k = 2
    while True:
        dt = timed(k + 1) - t1
        progress(f"  cpu: {k} steps of {cells} cells in {dt:.2f} s")
        if dt >= 0.8 * target_s or k >= 2000:
            return k * cells / max(dt, 1e-9), k
        k = int(min(2000, 8 * k, max(2 * k, k * target_s / max(dt, 1e-3))))


def cpu_rate(problem, threads, target_s):
    """Cell-updates per second of the loop oracle on `threads` host threads,
    its one-off set-up (node coefficients) excluded (grow_rate)."""
    from oracle import loops
    n = problem["blocks"][0]["n"]

    def timed(steps):
        t0 = time.perf_counter()
        loops.run_block(problem, steps=steps, threads=threads)
        return time.perf_counter() - t0
    return grow_rate(timed, n[0] * n[1] * n[2], target_s)


def cpu_baseline(problem):
    """The loop oracle (plain C, fp64, OpenMP over z planes) on the host
    cores, on a bounded sample of the workload (the full block for a few
    steps): on all the cores this process may use, and on one core."""
    model, ncpu = host_cpu()
    threads = all_threads()
    rate_all, k_all = cpu_rate(problem, threads, 12.0)
    rate_one, k_one = cpu_rate(problem, 1, 8.0)
    n = problem["blocks"][0]["n"]
    return {"value": rate_all / 1e6, "unit": "Mcell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"full {n[0]}^3 block, {k_all} steps on {threads} threads and {k_one} steps on 1 "
                      f"(set-up excluded), fp64 loop form",
            "one_core": {"value": rate_one / 1e6, "unit": "Mcell-updates/s", "cores": 1},
            "cpu_model": model, "nproc": ncpu}


def cpu_configs(targets=((1, 3.0), (3, 10.0), (4, 10.0), (5, 6.0))):
    """The loop oracle on the other workloads, on all the host threads this
    process may use and on one, fp64, cell-updates per second with each
    call's set-up excluded (grow_rate).  Single blocks (configs 1 and 5, the latter's forward
    run) take the one-block loop form; config 4's cavities are independent,
    so a sample of its first 8 cavities takes it cavity by cavity; config 3's
    27 coupled blocks take the multi-block form in full."""
    import numpy as np
    from oracle import loops
    from sbp_inputs import make_config

    def single(prob, b):
        blk = dict(prob["blocks"][b])
        pick = lambda items: [dict(x, block=0) for x in items if x["block"] == b]
        return {"blocks": [blk], "interfaces": [], "cfl": prob["cfl"], "steps": prob.get("steps", 1),
                "sources": pick(prob.get("sources", [])), "probes": pick(prob.get("probes", []))}

    def multi_rate(prob, threads, target):
        m = loops.MultiBlock(prob, threads=threads)

        def timed(steps):
            t0 = time.perf_counter()
            m.advance(steps)
            return time.perf_counter() - t0
        return grow_rate(timed, int(sum(np.prod(b["n"]) for b in prob["blocks"])), target)

    out = {}
    for cfg, target in targets:
        prob = make_config(cfg)
        rec = {"workload": prob["name"], "cells": int(sum(np.prod(b["n"]) for b in prob["blocks"])),
               "blocks": len(prob["blocks"])}
        for threads, label in ((all_threads(), "all_cores"), (1, "one_core")):
            if cfg == 3:
                rate, k = multi_rate(prob, threads, target)
                sample = f"all 27 blocks, {k} steps, multi-block loop form"
            elif cfg == 4:
                work = secs = 0.0
                for b in range(8):
                    one = single(prob, b)
                    r, k = cpu_rate(one, threads, target / 8)
                    cells = int(np.prod(one["blocks"][0]["n"]))
                    work += k * cells
                    secs += k * cells / r
                rate = work / secs
                sample = "cavities 0-7 of 64 (one-block loop form, cavity by cavity)"
            else:
                rate, k = cpu_rate(prob, threads, target)
                sample = f"the full block, {k} steps, one-block loop form"
            rec[label] = {"value": rate / 1e6, "unit": "Mcell-updates/s", "sample": sample}
            progress(f"cpu config {cfg} {label}: {rate / 1e6:.1f} Mcell-updates/s")
        out[f"config{cfg}"] = rec
    return out


def paper_context(problem):
    """The paper's own figures with the hardware it states (Section VI-D,
    Table T3), beside this layout's field storage against the Yee grid's."""
    def yee_nodes(n):
        nx, ny, nz = n
        return (nx * (ny + 1) * (nz + 1) + (nx + 1) * ny * (nz + 1) + (nx + 1) * (ny + 1) * nz +
                (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1))

    def sbp_nodes(n):
        e, h = node_counts(n)
        return e + h

    def layout_nodes(n):
        nx, ny, nz = n
        sxy = -(-((nx + 2) * (ny + 2)) // 64) * 64
        return 6 * sxy * (nz + 2)

    out = {"throughput_mcells": 21.15e6 * 5196 / 36187.0 / 1e6,
           "throughput_note": "SBP-SAT head-model run: 300x300x235 = 21.15 M cells, 10 ns, 36,187 s "
                              "(Table T3); 5196 steps assumes dt = 1 mm / (c sqrt 3), which the paper "
                              "does not state",
           "hardware": "Intel i7-7700 @ 3.6 GHz, one thread, 256 GB RAM; precision not stated",
           "runtime_overhead_vs_fdtd_pct": 100.0 * (36187.0 / 36138.0 - 1.0),
           "memory_overhead_vs_fdtd_pct": 100.0 * (984.1 / 973.5 - 1.0),
           "overhead_note": "whole solvers with CPML and TF/SF (Table T3); the abstract rounds the memory "
                            "overhead to 1.2 %"}
    for name, n in (("head_grid_300x300x235", (300, 300, 235)), ("workload", tuple(problem["blocks"][0]["n"]))):
        y = yee_nodes(n)
        out[f"field_nodes_vs_yee_pct_{name}"] = {
            "method": 100.0 * (sbp_nodes(n) / y - 1.0),
            "this_layout": 100.0 * (layout_nodes(n) / y - 1.0)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="also time the loop oracle on configs 1, 3, 4 and 5 (about two minutes of CPU)")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-subgrid", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-lts", action="store_true")
    ap.add_argument("--no-bloch", action="store_true")
    ap.add_argument("--no-cpml", action="store_true")
    ap.add_argument("--no-tfsf", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device-to-device copy first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (one block "
              "set per GPU with halo exchange between them is a design only); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from sbp_inputs import make_config
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    prob = make_config(2)
    n = prob["blocks"][0]["n"]
    cells = n[0] * n[1] * n[2]
    f32 = run_gpu(prob, "f32", args.steps, args.warmup, profile_kernels=True)
    ms_per_step = f32["wall_s"] * 1e3 / args.steps
    value = cells * args.steps / f32["wall_s"] / 1e6
    hb, eb, fb = algorithmic_bytes(prob, 4)
    h_ms, e_ms, f_ms = f32["kernel_ms"]
    dom, dom_ms, dom_bytes = max([("h_update", h_ms, hb), ("e_update", e_ms, eb), ("step_fused", f_ms, fb)],
                                 key=lambda x: x[1])
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    tr = traffic_entry(dom)
    out = {
        "metric": "Mcell-updates/s and HBM GB/s (% peak), FP32 vs FP64 step at stated field error",
        "value": value, "unit": "Mcell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": prob["name"], "cells": cells, "block": list(n), "dx_m": 1e-3,
                   "faces": "pec", "source": "modulated gaussian Ez 10 GHz", "launch": list(f32["launch"])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if tr is None else tr["bytes_per_launch"],
                     "kernel": dom, "algorithmic_bytes_per_launch": dom_bytes, "launch_ms": dom_ms,
                     "bytes_note": "per node: the updated field read and written, the other field read (elem "
                                   "bytes each); per cell: the permittivity, one byte (its table index) when the "
                                   "block has at most 64 values, else elem bytes"},
        "kernels_ms": {"h_update": h_ms, "e_update": e_ms, "step_fused": f_ms},
        "step_hbm_gbs_algorithmic": (hb + eb + fb) / (ms_per_step * 1e-3) / 1e9,
        "event_ms_per_step": f32["event_ms"] / args.steps,
    }
    if not args.no_fp64:
        f64 = run_gpu(prob, "f64", args.steps, args.warmup, profile_kernels=True)
        hb8, eb8, fb8 = algorithmic_bytes(prob, 8)
        out["fp64"] = {"value": cells * args.steps / f64["wall_s"] / 1e6, "unit": "Mcell-updates/s",
                       "ms_per_step": f64["wall_s"] * 1e3 / args.steps, "kernels_ms": list(f64["kernel_ms"]),
                       "step_hbm_gbs_algorithmic": (hb8 + eb8 + fb8) / (f64["wall_s"] / args.steps) / 1e9}
    if not args.no_fp64:
        one = run_gpu(prob, "f32", args.steps, args.warmup, profile_kernels=True, fused=True)
        fb1 = algorithmic_bytes(prob, 4, fused=True)[2]
        out["one_pass"] = {"value": cells * args.steps / one["wall_s"] / 1e6, "unit": "Mcell-updates/s",
                           "ms_per_step": one["wall_s"] * 1e3 / args.steps, "kernel_ms": one["kernel_ms"][2],
                           "algorithmic_bytes_per_launch": fb1,
                           "achieved_gbs": fb1 / (one["kernel_ms"][2] * 1e-3) / 1e9}
    if not args.no_batched:
        out["batched"] = batched(args.steps, max(args.warmup, 100))
        if not args.no_fp64:
            out["batched"]["fp64"] = batched(args.steps, max(args.warmup, 100), prec="f64")
        if not args.no_accuracy:
            out["batched"]["accuracy"] = batched_accuracy()
    if not args.no_subgrid:
        out["subgrid"] = subgrid(min(args.steps, 1000), max(args.warmup, 20))
        if not args.no_fp64:
            out["subgrid"]["fp64"] = subgrid(min(args.steps, 1000), max(args.warmup, 20), prec="f64")
            out["subgrid"]["accuracy_vs_fp64"] = subgrid_accuracy()
    if not args.no_lts:
        out["lts"] = lts_leg(min(args.steps, 500), max(args.warmup, 10))
    out["copy_ceiling"] = copy_ceiling()
    out["pattern_ceiling"] = pattern_ceiling(h_ms, e_ms)
    if not args.no_cpml:
        out["cpml"] = cpml_leg(min(args.steps, 1000), max(args.warmup, 20))
        if not args.no_accuracy:
            out["cpml"]["accuracy_vs_fp64"] = fp32_vs_fp64(cpml_problem()[0])
    if not args.no_tfsf:
        out["cpml_tfsf"] = cpml_leg(min(args.steps, 1000), max(args.warmup, 20), tfsf=True)
        if not args.no_accuracy:
            out["cpml_tfsf"]["accuracy_vs_fp64"] = fp32_vs_fp64(cpml_problem(True)[0])
    if not args.no_bloch:
        out["bloch"] = bloch(min(args.steps, 1000), max(args.warmup, 20))
        if not args.no_accuracy:
            from sbp_inputs import bloch_box
            out["bloch"]["accuracy_vs_fp64"] = fp32_vs_fp64(bloch_box())
    if not args.no_adjoint:
        import numpy as np
        out["adjoint"], g32 = adjoint_leg("f32")
        if not args.no_fp64:
            rec64, g64 = adjoint_leg("f64")
            out["adjoint"]["fp64"] = rec64
            # the fp64 gradient is the reference here: the GPU tests pin it to
            # the oracle's adjoint and to central differences
            out["adjoint"]["accuracy_vs_fp64"] = {
                "J_rel": abs(out["adjoint"]["J"] - rec64["J"]) / abs(rec64["J"]),
                "grad_rel_l2": float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))}
    if not args.no_accuracy:
        out["accuracy"] = accuracy(4)
    out["paper"] = paper_context(prob)
    pc = out["pattern_ceiling"]
    out["paper"]["this_closure_rows_and_energy_overhead_pct"] = 100.0 * (
        (h_ms + e_ms) / (pc["h_pattern_ms"] + pc["e_pattern_ms"]) - 1.0)
    out["paper"]["this_overhead_note"] = (
        "the 256^3 step's H and E launches against the same access pattern without the closure / SAT rows, "
        "the energy sums and probes (pattern_ceiling); the paper's figure compares whole solvers")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    if args.cpu_configs:
        model, ncpu = host_cpu()
        out["cpu_configs"] = {"cpu_model": model, "nproc": ncpu, "threads": all_threads(), **cpu_configs()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
