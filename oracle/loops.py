"""ctypes wrapper of the loop-form oracle ``loops.c`` (test infrastructure).

``build()`` compiles ``loops.c`` with gcc into ``liboracle.so`` next to it
(plain C, -O2, OpenMP over z planes).
"""
import ctypes
import os
import subprocess

import numpy as np

from .system import COMPS, comp_shape, cfl_dt

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "loops.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_FACE = {"pec": 0, "pmc": 1, "abc": 2}
_WAVE = {"gauss": 0, "modgauss": 1}
_lib = None


def build(force=True):
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
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
