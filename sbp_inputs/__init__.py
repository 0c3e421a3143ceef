"""Seeded synthetic workloads (shared by the oracle tests, the GPU tests and
the benchmark).  Holds none of the method's arithmetic: only problem
geometry, materials, sources and probes drawn from a seeded generator."""
from .configs import make_config, bloch_box, lossless_subgrid, embedded_refinement, CONFIG_NAMES  # noqa: F401
