"""Builds the HIP library libsbpfdtd.so in-tree for gfx950 (hipcc), and the
access-pattern probe libsbppattern.so that the benchmark uses as a bandwidth
reference (not loaded by the library)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsbpfdtd.so")
SOURCES = ["api.hip", "step.hip", "adjoint.hip", "lts.hip"]
PATTERN_LIB = os.path.join(HERE, "libsbppattern.so")
PATTERN_SOURCES = ["pattern.hip"]
ARCH = os.environ.get("SBP_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # no packed fp32 instructions (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _link(sources, lib, verbose):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = lib + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + [os.path.join(CSRC, s) for s in sources] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)


def build(verbose=False):
    _link(SOURCES, LIB, verbose)
    _link(PATTERN_SOURCES, PATTERN_LIB, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
