"""FP64 CPU oracle for the 3D SBP-SAT FDTD leapfrog step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything in this
package; only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
and ``accuracy`` legs of ``bench.py`` use it.  It shares no code, headers, tables or constant
generators with the HIP path.

Two independent forms of the same method:

* ``operators`` / ``system``: the matrix form.  The 1D SBP operators of the
  paper's Appendix, the 3D operators as Kronecker products (ED_1-ED_3), the
  SAT penalties written as sigma (P''')^-1 R^T P'' (...) exactly as in
  E13-E15, E19-E21 and EPBC1-EPBC6, leapfrog time marching (Section V) and
  the discrete energy (E16).  scipy.sparse matrices, fp64.
* ``loops``: plain C loops applying the same step row by row (Appendix
  rows, E24): ``loops.c`` for one block, ``multiblock.c`` for coupled blocks
  (interfaces at 1:1 and 1:2, written separately from the matrix form and
  pinned against it); fast enough to time on the host and to run the
  workloads at full size and length.

``yee`` is a plain Yee FDTD reference, used only to pin the interior.

``dispersion``: the eigen-procedure of Section IV on a periodic box (the
amplification matrix of one leapfrog step, numerical wavenumbers, the
dispersion / dissipation / global errors), for the SBP-SAT scheme with
periodic faces (EPBC1-EPBC6) and, to pin the procedure, for the classical
Yee scheme against its closed-form dispersion relation.

``cpml``: convolutional perfectly matched layers on the SBP-SAT differences
(the truncation the paper's open examples use), pinned by the plain scheme
at zero strength and by absorption against a larger domain.

``tfsf``: total-field / scattered-field plane-wave injection from a
one-dimensional incident line, pinned by an empty scattered region (to
rounding) in vacuum.

``lts``: local time stepping at 1:p for refined blocks (an energy-conserving
two-level scheme on the E-only form of the lossless leapfrog), pinned by its
reduction to the leapfrog, energy conservation beyond the fine CFL limit and
second-order convergence.

``adjoint``: the discrete adjoint of the leapfrog step in the matrix form
(explicit transposes), giving the gradient of a region objective with
respect to the per-cell permittivity; pinned by central finite differences
of the forward objective.

Parity pins live in ``tests/test_oracle_*.py``.  Functions whose results no
pin covers say "parity unpinned" in their docstring.
"""
