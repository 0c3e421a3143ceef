"""ctypes wrappers of the loop-form oracle (test infrastructure): ``loops.c``
(one block) and ``multiblock.c`` (coupled blocks, interfaces at 1:1 and 1:2).

``build()`` compiles both with gcc into ``liboracle.so`` next to them (plain
C, -O2, OpenMP over z planes).
"""
import ctypes
import os
import subprocess

import numpy as np

from .system import COMPS, comp_shape, cfl_dt

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "loops.c"), os.path.join(_HERE, "multiblock.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_FACE = {"pec": 0, "pmc": 1, "abc": 2}
_WAVE = {"gauss": 0, "modgauss": 1}
_lib = None


def build(force=True):
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("h", ctypes.c_double * 3),
                ("eps_r", ctypes.c_void_p), ("mu_r", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
                ("faces", ctypes.c_int * 6), ("dt", ctypes.c_double),
                ("nsrc", ctypes.c_int), ("src_comp", ctypes.c_void_p), ("src_node", ctypes.c_void_p),
                ("src_wave", ctypes.c_void_p), ("src_par", ctypes.c_void_p),
                ("nprobe", ctypes.c_int), ("probe_comp", ctypes.c_void_p), ("probe_node", ctypes.c_void_p),
                ("step0", ctypes.c_long)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        _lib.oracle_run.restype = ctypes.c_int
        _lib.oracle_run.argtypes = [ctypes.POINTER(_Cfg)] + [ctypes.c_void_p] * 6 + \
            [ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        _lib.oracle_threads.restype = ctypes.c_int
        _lib.mb_run.restype = ctypes.c_int
        _lib.mb_run.argtypes = [ctypes.POINTER(_MbCfg), ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    return _lib


def max_threads():
    return _load().oracle_threads()


def _ptr(a):
    return None if a is None else a.ctypes.data


def run_block(problem, steps=None, dt=None, init=None, threads=0, step0=0):
    """Run the single block of ``problem`` with the loop oracle.

    ``init``: optional {comp: array (Sz,Sy,Sx)} initial E^0 / H^{-1/2}.
    Returns {"fields": {comp: array}, "energy": (steps,), "probes": (np, steps), "dt"}.
    """
    blocks = problem["blocks"]
    if len(blocks) != 1 or problem.get("interfaces"):
        raise ValueError("the loop oracle handles one block without interfaces")
    blk = blocks[0]
    steps = problem["steps"] if steps is None else steps
    if dt is None:
        dt = cfl_dt(blocks, problem["cfl"])
    n = tuple(int(v) for v in blk["n"])
    keep = []

    def arr(a, dtype=np.float64):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dtype)
        keep.append(a)
        return a

    cfg = _Cfg()
    cfg.n[:] = n
    cfg.h[:] = [float(v) for v in blk["h"]]
    cfg.eps_r = _ptr(arr(blk.get("eps_r")))
    cfg.mu_r = _ptr(arr(blk.get("mu_r")))
    cfg.sigma = _ptr(arr(blk.get("sigma")))
    cfg.faces[:] = [_FACE[f] for f in blk["faces"]]
    cfg.dt = dt
    srcs = problem.get("sources", [])
    cfg.nsrc = len(srcs)
    if srcs:
        cfg.src_comp = _ptr(arr([COMPS.index(s["comp"]) for s in srcs], np.int32))
        cfg.src_node = _ptr(arr([list(s["node"]) for s in srcs], np.int32))
        cfg.src_wave = _ptr(arr([_WAVE[s["waveform"]] for s in srcs], np.int32))
        cfg.src_par = _ptr(arr([[s["tw"], s["t0"], s.get("f0", 0.0), s["amp"]] for s in srcs]))
    prbs = problem.get("probes", [])
    cfg.nprobe = len(prbs)
    if prbs:
        cfg.probe_comp = _ptr(arr([COMPS.index(p["comp"]) for p in prbs], np.int32))
        cfg.probe_node = _ptr(arr([list(p["node"]) for p in prbs], np.int32))
    cfg.step0 = step0
    fields = {}
    for c in COMPS:
        sx, sy, sz = comp_shape(c, n)
        if init is not None and c in init:
            fields[c] = np.ascontiguousarray(init[c], dtype=np.float64).reshape(sz, sy, sx).copy()
        else:
            fields[c] = np.zeros((sz, sy, sx))
    energy = np.zeros(steps)
    probes = np.zeros((len(prbs), steps))
    rc = _load().oracle_run(ctypes.byref(cfg), *[fields[c].ctypes.data for c in COMPS],
                            steps, energy.ctypes.data, probes.ctypes.data, int(threads))
    if rc != 0:
        raise ValueError("oracle_run failed (block needs >= 4 cells per axis)")
    return {"fields": fields, "energy": energy, "probes": probes, "dt": dt}


# ------------------------------------------------------------ several blocks
class _MbBlock(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("h", ctypes.c_double * 3),
                ("eps_r", ctypes.c_void_p), ("mu_r", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
                ("faces", ctypes.c_int * 6), ("f", ctypes.c_void_p * 6)]


class _MbMap(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _MbLink(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("face", ctypes.c_int), ("nb", ctypes.c_int), ("nb_face", ctypes.c_int),
                ("map", (_MbMap * 2) * 2)]


class _MbCfg(ctypes.Structure):
    _fields_ = [("nblocks", ctypes.c_int), ("blocks", ctypes.c_void_p), ("nlinks", ctypes.c_int),
                ("links", ctypes.c_void_p), ("dt", ctypes.c_double), ("nsrc", ctypes.c_int),
                ("src", ctypes.c_void_p), ("src_par", ctypes.c_void_p), ("nprobe", ctypes.c_int),
                ("probe", ctypes.c_void_p), ("step0", ctypes.c_long)]


_MB_FACE = {"pec": 0, "pmc": 1, "abc": 2}


class MultiBlock:
    """Coupled blocks stepped by ``multiblock.c``; the state stays here
    between ``advance`` calls (so a long run can be taken in pieces).

    ``problem`` as for ``system.run``: blocks (n, h, eps_r, mu_r, sigma,
    faces), interfaces (block_a, face_a, block_b, face_b, ratio), sources,
    probes, cfl.  The 1:2 maps along each tangential axis are the
    interpolation of ``operators.interp_c2f`` (fine side) and its
    norm-compatible restriction ``operators.interp_f2c`` (coarse side)."""

    def __init__(self, problem, dt=None, init=None, threads=0):
        from scipy import sparse
        from . import operators as ops
        if problem.get("periodic"):
            raise ValueError("periodic faces: use the matrix form")
        self.problem = problem
        self.threads = int(threads)
        blocks = problem["blocks"]
        self.dt = cfl_dt(blocks, problem["cfl"]) if dt is None else dt
        self._keep = []
        nb = len(blocks)
        self.fields = {}
        links = []
        linked = {}
        for (ba, fa, bb, fb, ratio) in problem.get("interfaces", []):
            if ratio not in (1, 2) or fa // 2 != fb // 2 or fa % 2 == fb % 2:
                raise ValueError("bad interface")
            linked[(ba, fa)] = (bb, fb, "same" if ratio == 1 else "coarse")
            linked[(bb, fb)] = (ba, fa, "same" if ratio == 1 else "fine")
        self._blocks = (_MbBlock * nb)()
        for b, blk in enumerate(blocks):
            n = tuple(int(v) for v in blk["n"])
            B = self._blocks[b]
            B.n[:] = n
            B.h[:] = [float(v) for v in blk["h"]]
            B.eps_r = _ptr(self._arr(blk.get("eps_r")))
            B.mu_r = _ptr(self._arr(blk.get("mu_r")))
            B.sigma = _ptr(self._arr(blk.get("sigma")))
            B.faces[:] = [3 if (b, f) in linked else _MB_FACE[blk["faces"][f]] for f in range(6)]
            for ci, c in enumerate(COMPS):
                sx, sy, sz = comp_shape(c, n)
                a = np.zeros((sz, sy, sx))
                if init is not None and (b, c) in init:
                    a[...] = np.asarray(init[(b, c)], np.float64).reshape(sz, sy, sx)
                self.fields[(b, c)] = a
                B.f[ci] = a.ctypes.data
        for (b, f), (nbk, nf, role) in linked.items():
            L = _MbLink()
            L.block, L.face, L.nb, L.nb_face = b, f, nbk, nf
            tang = [a for a in range(3) if a != f // 2]
            n_own = blocks[b]["n"]
            for t, ax in enumerate(tang):
                for g, kind in ((1, "+"), (0, "-")):
                    if role == "same":
                        L.map[t][g].ptr = None
                        continue
                    m = ops.interp_f2c(kind, n_own[ax]) if role == "coarse" else ops.interp_c2f(kind, n_own[ax] // 2)
                    csr = sparse.csr_matrix(m)
                    L.map[t][g].ptr = _ptr(self._arr(csr.indptr, np.int32))
                    L.map[t][g].col = _ptr(self._arr(csr.indices, np.int32))
                    L.map[t][g].val = _ptr(self._arr(csr.data))
            links.append(L)
        self._links = (_MbLink * max(len(links), 1))(*links)
        self._nlinks = len(links)
        srcs = problem.get("sources", [])
        self._src = self._arr([[s["block"], COMPS.index(s["comp"])] + list(s["node"]) + [_WAVE[s["waveform"]]]
                               for s in srcs] or np.zeros((0, 6)), np.int32)
        self._src_par = self._arr([[s["tw"], s["t0"], s.get("f0", 0.0), s["amp"]] for s in srcs] or np.zeros((0, 4)))
        self._nsrc = len(srcs)
        prbs = problem.get("probes", [])
        self._prb = self._arr([[p["block"], COMPS.index(p["comp"])] + list(p["node"]) for p in prbs]
                              or np.zeros((0, 5)), np.int32)
        self._nprb = len(prbs)
        self.steps_done = 0

    def _arr(self, a, dtype=np.float64):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dtype)
        self._keep.append(a)
        return a

    def advance(self, steps):
        """Runs ``steps`` steps; returns (W^n of each step, probe series)."""
        cfg = _MbCfg()
        cfg.nblocks = len(self._blocks)
        cfg.blocks = ctypes.addressof(self._blocks)
        cfg.nlinks = self._nlinks
        cfg.links = ctypes.addressof(self._links)
        cfg.dt = self.dt
        cfg.nsrc = self._nsrc
        cfg.src = self._src.ctypes.data
        cfg.src_par = self._src_par.ctypes.data
        cfg.nprobe = self._nprb
        cfg.probe = self._prb.ctypes.data
        cfg.step0 = self.steps_done
        energy = np.zeros(steps)
        probes = np.zeros((self._nprb, steps))
        rc = _load().mb_run(ctypes.byref(cfg), steps, energy.ctypes.data, probes.ctypes.data, self.threads)
        if rc != 0:
            raise ValueError(f"mb_run failed ({rc})")
        self.steps_done += steps
        return energy, probes


def run_blocks(problem, steps=None, dt=None, init=None, threads=0):
    """The coupled blocks of ``problem`` through ``multiblock.c``; returns
    {"fields": {(block, comp): array}, "energy", "probes", "dt"}."""
    steps = problem["steps"] if steps is None else steps
    m = MultiBlock(problem, dt=dt, init=init, threads=threads)
    e, p = m.advance(steps)
    return {"fields": m.fields, "energy": e, "probes": p, "dt": m.dt}
