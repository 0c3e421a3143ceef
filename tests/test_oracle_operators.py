"""Pins of the 1D SBP operators and the 1:2 interpolation (oracle, CPU)."""
import json
import os
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import operators as ops

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden():
    mats, name, rows = {}, None, []
    with open(os.path.join(GOLDEN, "appendix_n6.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0].isalpha() or parts[0][0].isalpha():
                if name:
                    mats[name] = rows
                name, rows = parts[0], []
            else:
                rows.append([F(v) for v in parts])
    mats[name] = rows
    return mats


def _mm(a, b):
    return [[sum(a[i][k] * b[k][j] for k in range(len(b))) for j in range(len(b[0]))] for i in range(len(a))]


def _tr(a):
    return [list(r) for r in zip(*a)]


def test_appendix_matches_printed_matrices():
    g = _read_golden()
    n = 6
    assert ops.d_plus_exact(n) == g["Dplus"]
    assert ops.d_minus_exact(n) == g["Dminus"]
    assert ops.q_plus_exact(n) == g["Qplus"]
    assert ops.q_minus_exact(n) == g["Qminus"]
    assert ops.p_plus_exact(n) == g["Pplus"][0]
    assert ops.p_minus_exact(n) == g["Pminus"][0]


@pytest.mark.parametrize("n", list(range(4, 41)))
def test_factorisation_E3(n):
    # D = P^-1 Q, exactly, for the printed D, P and Q
    for d, p, q in ((ops.d_plus_exact(n), ops.p_plus_exact(n), ops.q_plus_exact(n)),
                    (ops.d_minus_exact(n), ops.p_minus_exact(n), ops.q_minus_exact(n))):
        assert [[p[i] * d[i][j] for j in range(len(d[0]))] for i in range(len(d))] == q


@pytest.mark.parametrize("n", list(range(4, 65)))
def test_sbp_property_EQB(n):
    qp, qm = ops.q_plus_exact(n), ops.q_minus_exact(n)
    s = [[qp[i][j] + _tr(qm)[i][j] for j in range(n + 2)] for i in range(n + 1)]
    assert s == ops.b_exact(n)


@pytest.mark.parametrize("n", [4, 5, 6, 9, 17, 32])
def test_accuracy_E2_exact(n):
    xp = [F(i) for i in range(n + 1)]
    xm = [F(0)] + [F(2 * j - 1, 2) for j in range(1, n + 1)] + [F(n)]
    dp, dm = ops.d_plus_exact(n), ops.d_minus_exact(n)
    # k = 0: D applied to constants vanishes; k = 1: D applied to x is 1
    assert _mm(dp, [[F(1)] for _ in xm]) == [[F(0)] for _ in xp]
    assert _mm(dm, [[F(1)] for _ in xp]) == [[F(0)] for _ in xm]
    assert _mm(dp, [[v] for v in xm]) == [[F(1)] for _ in xp]
    assert _mm(dm, [[v] for v in xp]) == [[F(1)] for _ in xm]
    # second derivative is not reproduced at the boundary (order 2 closure, not higher)
    assert _mm(dp, [[v * v] for v in xm]) != [[2 * v] for v in xp]


@pytest.mark.parametrize("n", [4, 7, 12])
def test_boundary_identity_E6(n):
    rng = np.random.default_rng(n)
    xp = rng.standard_normal(n + 1)
    xm = rng.standard_normal(n + 2)
    b = np.array([[float(v) for v in r] for r in ops.b_exact(n)])
    assert xp @ b @ xm == pytest.approx(xp[n] * xm[n + 1] - xp[0] * xm[0], abs=1e-14)


@pytest.mark.parametrize("n", [4, 8, 13])
def test_norms_integrate_linears(n):
    for kind in "+-":
        w = ops.weights(kind, n, 0.7)
        x = ops.grid(kind, n, 0.7)
        assert w.sum() == pytest.approx(n * 0.7, rel=1e-15)
        assert (w * x).sum() == pytest.approx((n * 0.7) ** 2 / 2, rel=1e-14)


def test_skew_adjoint_pair_1d():
    # w+ D+ + (w- D-)^T = B: the discrete integration by parts of E6
    n, h = 9, 0.3
    lhs = np.diag(ops.weights_plus(n, h)) @ ops.d_plus(n, h) + (np.diag(ops.weights_minus(n, h)) @ ops.d_minus(n, h)).T
    b = np.array([[float(v) for v in r] for r in ops.b_exact(n)])
    assert np.abs(lhs - b).max() < 1e-14


def test_min_cells():
    with pytest.raises(ValueError):
        ops.d_plus_exact(3)


# ---------------------------------------------------- 1:2 interpolation
@pytest.mark.parametrize("kind", ["+", "-"])
@pytest.mark.parametrize("nc", [6, 7, 10, 24])
def test_interp_norm_compatible(kind, nc):
    ic2f = ops.interp_c2f(kind, nc)
    if2c = ops.interp_f2c(kind, nc)
    wc = ops.weights(kind, nc, 1.0)
    wf = ops.weights(kind, 2 * nc, 0.5)
    assert ic2f.shape == (ops.size(kind, 2 * nc), ops.size(kind, nc))
    # Wc I_f2c = (Wf I_c2f)^T
    assert np.abs(wc[:, None] * if2c - (wf[:, None] * ic2f).T).max() < 1e-14
    # constants preserved both ways
    assert np.abs(ic2f.sum(1) - 1).max() < 1e-14
    assert np.abs(if2c.sum(1) - 1).max() < 1e-14


@pytest.mark.parametrize("nc", [6, 11])
def test_interp_accuracy(nc):
    # "+" grid: linear interpolation, exact for linears everywhere
    xc, xf = ops.grid_plus(nc, 1.0), ops.grid_plus(2 * nc, 0.5)
    assert np.abs(ops.interp_c2f("+", nc) @ xc - xf).max() < 1e-13
    # "-" grid: exact for linears away from the 4 boundary rows of each end
    xc, xf = ops.grid_minus(nc, 1.0), ops.grid_minus(2 * nc, 0.5)
    err = ops.interp_c2f("-", nc) @ xc - xf
    assert np.abs(err[4:-4]).max() < 1e-13
    assert np.abs(err).max() < 0.12  # first-order boundary rows, error <= 5/46 h_c


def test_interp_minus_no_linear_exact_solution():
    # the reason the "-" boundary rows are only constant-exact: with linear
    # rows elsewhere, the Wf-weighted first moment of any linear-exact
    # interpolation misses the coarse one by 1/8 (h_c = 1) per end.
    nc = 10
    xc, xf = ops.grid_minus(nc, 1.0), ops.grid_minus(2 * nc, 0.5)
    wc, wf = ops.weights_minus(nc, 1.0), ops.weights_minus(2 * nc, 0.5)
    lin = ops._linear_interp_matrix(xf, xc)
    cols = 6  # coarse columns 0..5; fine rows fully inside them
    lhs = sum(wf[r] * sum(lin[r, s] * xc[s] for s in range(cols)) for r in range(len(xf)))
    rhs = sum(wc[s] * xc[s] for s in range(cols))
    assert lhs - rhs == pytest.approx(-1.0 / 8.0, abs=1e-12)


def test_head_model_memory_overhead_matches_table_t3():
    """The oracle's grids (Table T1 shapes: a "-" axis of n cells holds n + 2
    nodes) against the Yee grid's on the head model's 300 x 300 x 235 cells:
    the extra field nodes come to the memory overhead Table T3 measures
    (984.1 MB against 973.5 MB, 1.089 %) within 0.01 percentage points; a
    transposed component shape or a dropped face node moves it by more."""
    from oracle.system import COMPS, comp_size
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as fh:
        d = json.load(fh)
    n = tuple(d["head_grid"])
    nx, ny, nz = n
    yee = (nx * (ny + 1) * (nz + 1) + (nx + 1) * ny * (nz + 1) + (nx + 1) * (ny + 1) * nz +
           (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1))
    sbp = sum(comp_size(c, n) for c in COMPS)
    measured = 100.0 * (d["head_memory_mb_sbp"] / d["head_memory_mb_fdtd"] - 1.0)
    assert abs(100.0 * (sbp / yee - 1.0) - measured) < 0.01
    # a shape mistake (Ex with n+1 instead of n+2 nodes along x) misses it
    wrong = sbp - (ny + 1) * (nz + 1)
    assert abs(100.0 * (wrong / yee - 1.0) - measured) > 0.01
