"""Thin Python binding of the sbpfdtd C ABI (argument marshalling only).

Every step of the method runs in the HIP library ``libsbpfdtd.so``; this
module loads it with ctypes, passes torch's caching allocator and current
stream to it, and converts numpy arrays to pointers.  There is no fallback:
if the library is missing, ``lib()`` raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsbpfdtd.so")

SBP_OK, SBP_EINVAL, SBP_ENOMEM, SBP_EHIP, SBP_ESTATE, SBP_EUNSTABLE, SBP_ERANGE = 0, -1, -2, -3, -4, -5, -6
SBP_FP64, SBP_FP32 = 0, 1
BC = {"pec": 0, "pmc": 1, "abc": 2, "cpml": 3}
COMPS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")
WAVE = {"gauss": 0, "modgauss": 1}
STATUS_NAMES = {0: "SBP_OK", -1: "SBP_EINVAL", -2: "SBP_ENOMEM", -3: "SBP_EHIP", -4: "SBP_ESTATE",
                -5: "SBP_EUNSTABLE", -6: "SBP_ERANGE"}

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_P = ctypes.c_void_p
_I = ctypes.c_int
_L = ctypes.c_long
_D = ctypes.c_double
_S = ctypes.c_size_t
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)

# name -> argtypes (all return sbp_status unless noted)
SIGNATURES = {
    "sbp_create": [ctypes.POINTER(_P), _I, _P, ALLOC_FN, FREE_FN, _P],
    "sbp_add_block": [_P, _I, _I, _I, _D, _D, _D, _D, _D, _D, _P, _P, _P, _IP],
    "sbp_set_face_bc": [_P, _I, _I, _I],
    "sbp_connect": [_P, _I, _I, _I, _I, _I],
    "sbp_set_periodic": [_P, _I, _I, _I, _D],
    "sbp_set_cpml": [_P, _I, _I, _D, _D, _D],
    "sbp_set_tfsf": [_P, _I, _IP, _I, _I, _I, _I, _I, _DP, _D],
    "sbp_add_source": [_P, _I, _I, _I, _I, _I, _I, _DP, _D, _IP],
    "sbp_add_probe": [_P, _I, _I, _I, _I, _I, _IP],
    "sbp_finalize": [_P, _D, _I, _L, _DP],
    "sbp_set_materials": [_P, _I, _P, _P, _P],
    "sbp_step": [_P, _L],
    "sbp_step_static": [_P, _L],
    "sbp_lts_start": [_P, _IP, _I, _I, ctypes.c_double, _L],
    "sbp_lts_step": [_P, _L],
    "sbp_lts_info": [_P, ctypes.POINTER(ctypes.c_long)],
    "sbp_steps_done": [_P, ctypes.POINTER(_L)],
    "sbp_field_shape": [_P, _I, _I, _IP],
    "sbp_read_field": [_P, _I, _I, _P, _S],
    "sbp_write_field": [_P, _I, _I, _P, _S],
    "sbp_read_energy": [_P, _L, _L, _P],
    "sbp_read_probe": [_P, _I, _L, _L, _P],
    "sbp_state_bytes": [_P, ctypes.POINTER(_S)],
    "sbp_save_state": [_P, _P, _S],
    "sbp_load_state": [_P, _P, _S],
    "sbp_adjoint": [_P, _I, _L, _IP, _L, _DP, _P],
    "sbp_set_launch": [_P, _I, _I, _I, _I],
    "sbp_set_fused": [_P, _I, _I],
    "sbp_set_cell_tables": [_P, _I],
    "sbp_get_launch": [_P, _IP],
    "sbp_autotune": [_P, _I, _DP],
    "sbp_use_graph": [_P, _I],
    "sbp_last_step_ms": [_P, _DP],
    "sbp_profile": [_P, _I],
    "sbp_kernel_ms": [_P, _DP],
    "sbp_last_error": [_P],
    "sbp_destroy": [_P],
}

_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        h = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(h, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        h.sbp_last_error.restype = ctypes.c_char_p
        h.sbp_destroy.restype = None
        _lib = h
    return _lib


class SbpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _f64(a):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=np.float64)


class _TorchMemory:
    """Allocator callbacks backed by torch's caching allocator on a stream."""

    def __init__(self, device, stream):
        import torch
        self.torch = torch
        self.device = device
        self.stream = stream

        def _alloc(nbytes, _user):
            return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)

        def _free(p, _user):
            try:
                self.torch.cuda.caching_allocator_delete(p)
            except (AttributeError, TypeError):
                # a context destroyed during interpreter shutdown, after torch
                # has been torn down: the device memory goes with the process
                pass

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)


class Context:
    """One sbp_ctx.  Methods map 1:1 onto the C ABI calls (same names without
    the ``sbp_`` prefix); errors raise SbpError with the library's message."""

    def __init__(self, prec="f64", device=None, stream=None, use_torch_memory=True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to torch")
        self._lib = lib()
        self.imag_part = {}  # block -> block holding its imaginary part (Bloch-periodic faces)
        dev = torch.cuda.current_device() if device is None else device
        torch.cuda.set_device(dev)
        st = torch.cuda.current_stream(dev) if stream is None else stream
        self.stream = st
        self._mem = _TorchMemory(dev, st) if use_torch_memory else None
        h = ctypes.c_void_p()
        prec_id = SBP_FP64 if prec in ("f64", SBP_FP64) else SBP_FP32
        alloc = self._mem.alloc if self._mem else ALLOC_FN()
        free = self._mem.free if self._mem else FREE_FN()
        rc = self._lib.sbp_create(ctypes.byref(h), prec_id, ctypes.c_void_p(st.cuda_stream), alloc, free, None)
        if rc != SBP_OK:
            raise SbpError(rc, "sbp_create failed")
        self.h = h
        self.prec = "f64" if prec_id == SBP_FP64 else "f32"

    def _chk(self, rc):
        if rc != SBP_OK:
            raise SbpError(rc, self._lib.sbp_last_error(self.h).decode())

    def add_block(self, n, h, origin=(0.0, 0.0, 0.0), eps_r=None, mu_r=None, sigma=None):
        bid = ctypes.c_int()
        e, m, s = _f64(eps_r), _f64(mu_r), _f64(sigma)
        for a in (e, m, s):
            if a is not None and a.size != n[0] * n[1] * n[2]:
                raise ValueError("per-cell array has the wrong size")
        self._chk(self._lib.sbp_add_block(self.h, n[0], n[1], n[2], h[0], h[1], h[2], origin[0], origin[1],
                                          origin[2], _ptr(e), _ptr(m), _ptr(s), ctypes.byref(bid)))
        return bid.value

    def set_face_bc(self, block, face, bc):
        self._chk(self._lib.sbp_set_face_bc(self.h, block, face, BC[bc] if isinstance(bc, str) else bc))

    def connect(self, a, fa, b, fb, ratio):
        self._chk(self._lib.sbp_connect(self.h, a, fa, b, fb, ratio))

    def set_periodic(self, block, axis, alpha=0.0, block_im=-1):
        """Both faces of `axis` periodic with the Bloch phase e^{-j alpha};
        alpha != 0 needs `block_im`, the block holding the imaginary part."""
        self._chk(self._lib.sbp_set_periodic(self.h, int(block), int(block_im), int(axis), float(alpha)))
        if block_im >= 0:
            self.imag_part[int(block)] = int(block_im)

    def set_cpml(self, cells=10, m=3, sigma_factor=0.8, kappa_max=1.0, alpha_max=0.0):
        """Parameters of the convolutional PML behind faces set to "cpml"."""
        self._chk(self._lib.sbp_set_cpml(self.h, int(cells), int(m), float(sigma_factor), float(kappa_max),
                                         float(alpha_max)))

    def set_tfsf(self, block, box, axis, pol, cell, waveform, tw, t0, f0=0.0, amp=1.0, margin=16):
        """Total-field / scattered-field box (cells lo/hi per axis) with a
        plane wave along +axis, E along component `pol` (0-2), from a line
        source on line node `cell`."""
        b = (ctypes.c_int * 6)(*[int(v) for v in box])
        p = (ctypes.c_double * 3)(tw, t0, f0)
        self._chk(self._lib.sbp_set_tfsf(self.h, int(block), b, int(axis), int(pol), int(margin), int(cell),
                                         WAVE[waveform], p, float(amp)))

    def add_source(self, block, comp, node, waveform, tw, t0, f0=0.0, amp=1.0):
        p = (ctypes.c_double * 3)(tw, t0, f0)
        sid = ctypes.c_int()
        self._chk(self._lib.sbp_add_source(self.h, block, COMPS.index(comp), node[0], node[1], node[2],
                                           WAVE[waveform], p, amp, ctypes.byref(sid)))
        return sid.value

    def add_probe(self, block, comp, node):
        pid = ctypes.c_int()
        self._chk(self._lib.sbp_add_probe(self.h, block, COMPS.index(comp), node[0], node[1], node[2],
                                          ctypes.byref(pid)))
        return pid.value

    def finalize(self, cfl, force=False, history=1 << 16):
        dt = ctypes.c_double()
        self._chk(self._lib.sbp_finalize(self.h, cfl, int(bool(force)), history, ctypes.byref(dt)))
        self.dt = dt.value
        return self.dt

    def set_materials(self, block, eps_r=None, mu_r=None, sigma=None):
        e, m, s = _f64(eps_r), _f64(mu_r), _f64(sigma)
        self._chk(self._lib.sbp_set_materials(self.h, block, _ptr(e), _ptr(m), _ptr(s)))

    def step(self, nsteps):
        self._chk(self._lib.sbp_step(self.h, int(nsteps)))

    def step_static(self, nsteps):
        self._chk(self._lib.sbp_step_static(self.h, int(nsteps)))

    def lts_start(self, refined, substeps, dt_coarse, energy_every=1):
        """Local time stepping of the blocks in ``refined`` with ``substeps``
        substeps per coarse step ``dt_coarse``; W^{n+1/2} every
        ``energy_every`` coarse steps (0: none); see sbp_lts_start."""
        r = (ctypes.c_int * max(len(refined), 1))(*[int(b) for b in refined])
        self._chk(self._lib.sbp_lts_start(self.h, r, len(refined), int(substeps), float(dt_coarse),
                                          int(energy_every)))

    def lts_step(self, nsteps):
        self._chk(self._lib.sbp_lts_step(self.h, int(nsteps)))

    def lts_info(self):
        """{near_tiles, tiles, near_nodes, nodes}: the extent of the local
        time stepping's correction; see sbp_lts_info."""
        out = (ctypes.c_long * 4)()
        self._chk(self._lib.sbp_lts_info(self.h, out))
        return dict(zip(("near_tiles", "tiles", "near_nodes", "nodes"), [int(v) for v in out]))

    def steps_done(self):
        n = ctypes.c_long()
        self._chk(self._lib.sbp_steps_done(self.h, ctypes.byref(n)))
        return n.value

    def field_shape(self, block, comp):
        s = (ctypes.c_int * 3)()
        self._chk(self._lib.sbp_field_shape(self.h, block, COMPS.index(comp), s))
        return tuple(s)

    def read_field(self, block, comp):
        sx, sy, sz = self.field_shape(block, comp)
        out = np.empty((sz, sy, sx), dtype=np.float64)
        self._chk(self._lib.sbp_read_field(self.h, block, COMPS.index(comp), _ptr(out), out.size))
        return out

    def write_field(self, block, comp, values):
        sx, sy, sz = self.field_shape(block, comp)
        v = _f64(values).reshape(sz, sy, sx)
        self._chk(self._lib.sbp_write_field(self.h, block, COMPS.index(comp), _ptr(v), v.size))

    def read_energy(self, first, count):
        out = np.empty(count, dtype=np.float64)
        self._chk(self._lib.sbp_read_energy(self.h, first, count, _ptr(out)))
        return out

    def read_probe(self, pid, first, count):
        out = np.empty(count, dtype=np.float64)
        self._chk(self._lib.sbp_read_probe(self.h, pid, first, count, _ptr(out)))
        return out

    def state_bytes(self):
        b = ctypes.c_size_t()
        self._chk(self._lib.sbp_state_bytes(self.h, ctypes.byref(b)))
        return b.value

    def save_state(self, dev_ptr, nbytes):
        self._chk(self._lib.sbp_save_state(self.h, ctypes.c_void_p(dev_ptr), nbytes))

    def load_state(self, dev_ptr, nbytes):
        self._chk(self._lib.sbp_load_state(self.h, ctypes.c_void_p(dev_ptr), nbytes))

    def adjoint(self, block, nsteps, region, grad_ptr, ckpt_every=0):
        """J and dJ/d eps_r of ``block`` (written to the device doubles at
        ``grad_ptr``; 0 or None: J alone); see sbp_adjoint."""
        r = (ctypes.c_int * 6)(*[int(v) for v in region])
        J = ctypes.c_double()
        self._chk(self._lib.sbp_adjoint(self.h, int(block), int(nsteps), r, int(ckpt_every), ctypes.byref(J),
                                        ctypes.c_void_p(grad_ptr or None)))
        return J.value

    def set_launch(self, tx, ty, cz, workgroups=0):
        self._chk(self._lib.sbp_set_launch(self.h, tx, ty, cz, workgroups))

    def set_cell_tables(self, enable):
        self._chk(self._lib.sbp_set_cell_tables(self.h, int(bool(enable))))

    def set_fused(self, enable, planes=32):
        self._chk(self._lib.sbp_set_fused(self.h, int(bool(enable)), int(planes)))

    def get_launch(self):
        o = (ctypes.c_int * 4)()
        self._chk(self._lib.sbp_get_launch(self.h, o))
        return tuple(o)

    def autotune(self, steps_per_trial=5):
        ms = ctypes.c_double()
        self._chk(self._lib.sbp_autotune(self.h, steps_per_trial, ctypes.byref(ms)))
        return ms.value

    def use_graph(self, steps):
        self._chk(self._lib.sbp_use_graph(self.h, steps))

    def last_step_ms(self):
        ms = ctypes.c_double()
        self._chk(self._lib.sbp_last_step_ms(self.h, ctypes.byref(ms)))
        return ms.value

    def profile(self, enable):
        self._chk(self._lib.sbp_profile(self.h, int(bool(enable))))

    def kernel_ms(self):
        o = (ctypes.c_double * 3)()
        self._chk(self._lib.sbp_kernel_ms(self.h, o))
        return tuple(o)

    def close(self):
        if getattr(self, "h", None):
            self._lib.sbp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_problem(problem, prec=None, cfl=None, history=1 << 16, launch=None, force=False, stream=None,
                  cell_tables=None):
    """Creates and finalizes a Context from a problem dict (see sbp_inputs);
    launch and cell_tables (sbp_set_cell_tables) are applied before finalize."""
    ctx = Context(prec or problem.get("prec", "f64"), stream=stream)
    for b in problem["blocks"]:
        bid = ctx.add_block(b["n"], b["h"], b.get("origin", (0.0, 0.0, 0.0)), b.get("eps_r"),
                            b.get("mu_r"), b.get("sigma"))
        for f, bc in enumerate(b["faces"]):
            if bc == "iface":  # coupled by the interface list below
                continue
            if bc not in BC:
                raise ValueError(f"unknown face condition {bc!r}")
            ctx.set_face_bc(bid, f, bc)
    for (a, fa, b, fb, r) in problem.get("interfaces", []):
        ctx.connect(a, fa, b, fb, r)
    if "cpml" in problem:
        ctx.set_cpml(**problem["cpml"])
    # periodic axes (block, axis, alpha); a block with a nonzero phase on any
    # axis has complex fields: a twin block, appended after the problem's
    # blocks, holds the imaginary part (ctx.imag_part[block])
    periodic = [(int(b), int(a), float(al)) for (b, a, al) in problem.get("periodic", [])]
    for b in sorted({b for (b, _, al) in periodic if al != 0.0}):
        src = problem["blocks"][b]
        tw = ctx.add_block(src["n"], src["h"], src.get("origin", (0.0, 0.0, 0.0)), src.get("eps_r"),
                           src.get("mu_r"), src.get("sigma"))
        for f, bc in enumerate(src["faces"]):
            if bc in BC:
                ctx.set_face_bc(tw, f, bc)
        ctx.imag_part[b] = tw
    for (b, a, al) in periodic:
        ctx.set_periodic(b, a, al, ctx.imag_part.get(b, -1))
    if "tfsf" in problem:
        tf = problem["tfsf"]
        src = tf["source"]
        ctx.set_tfsf(tf["block"], tf["box"], tf["axis"], tf["pol"], src["cell"], src["waveform"], src["tw"],
                     src["t0"], src.get("f0", 0.0), src.get("amp", 1.0), tf.get("margin", 16))
    for s in problem.get("sources", []):
        ctx.add_source(s["block"], s["comp"], s["node"], s["waveform"], s["tw"], s["t0"], s.get("f0", 0.0),
                       s.get("amp", 1.0))
    for p in problem.get("probes", []):
        ctx.add_probe(p["block"], p["comp"], p["node"])
    if launch is not None:
        ctx.set_launch(*launch)
    if cell_tables is not None:
        ctx.set_cell_tables(cell_tables)
    ctx.finalize(problem.get("cfl", 0.9) if cfl is None else cfl, force=force, history=history)
    return ctx
