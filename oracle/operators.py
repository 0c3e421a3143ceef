"""1D SBP operators and 1:2 interface interpolation (oracle, test infrastructure).

Grids (Section II-A): for an axis of n cells of width h the "+" grid holds the
n+1 nodes x_i = i h and the "-" grid the n+2 nodes 0, h/2, 3h/2, ..., nh - h/2,
nh.  D+ maps data on the "-" grid to the "+" grid (size N+ x N-), D- maps "+"
data to the "-" grid (N- x N+), E2.

The matrices below are the printed rows of the paper's Appendix (D+, D-,
P+, P-, Q+, Q-).  Reading of the Appendix: the printed P carries the material
(epsilon or mu) where the geometric cell width h belongs, and D carries
1/epsilon or 1/mu where 1/h belongs; the material is applied separately here
(as a diagonal per node) and P, D carry h.  So P+ = h diag(1/2, 1, ..., 1, 1/2),
P- = h diag(1/2, 1/4, 5/4, 1, ..., 1, 5/4, 1/4, 1/2), D+- = P+-^-1 Q+-, and
Q+ + Q-^T = B (E_QB, E4).

Exact rational versions (``*_exact``) use ``fractions.Fraction`` so the SBP
identities can be checked without rounding.
"""
from fractions import Fraction as F

import numpy as np

MIN_CELLS = 4  # the boundary closures of the Appendix need n >= 4


def _check_n(n):
    if n < MIN_CELLS:
        raise ValueError(f"SBP closures need at least {MIN_CELLS} cells, got {n}")


# ---------------------------------------------------------------- node grids
def grid_plus(n, h=1.0):
    """Node coordinates of the "+" grid (Section II-A): x_i = i h, i = 0..n."""
    return np.arange(n + 1, dtype=np.float64) * h


def grid_minus(n, h=1.0):
    """Node coordinates of the "-" grid (Section II-A): 0, (j - 1/2) h, n h."""
    return np.concatenate([[0.0], (np.arange(1, n + 1) - 0.5) * h, [n * h]])


# ------------------------------------------------------ Appendix, exact form
def _dense(rows, ncols):
    m = [[F(0)] * ncols for _ in rows]
    for r, entries in enumerate(rows):
        for c, v in entries:
            m[r][c] = F(v)
    return m


def q_plus_exact(n):
    """Q+ of the Appendix, (n+1) x (n+2), h-free rationals."""
    _check_n(n)
    rows = [[(0, F(-1, 2)), (1, F(1, 4)), (2, F(1, 4))],
            [(0, F(-1, 2)), (1, F(-1, 4)), (2, F(3, 4))]]
    for i in range(2, n - 1):
        rows.append([(i, -1), (i + 1, 1)])
    rows.append([(n - 1, F(-3, 4)), (n, F(1, 4)), (n + 1, F(1, 2))])
    rows.append([(n - 1, F(-1, 4)), (n, F(-1, 4)), (n + 1, F(1, 2))])
    return _dense(rows, n + 2)


def q_minus_exact(n):
    """Q- of the Appendix, (n+2) x (n+1), h-free rationals."""
    _check_n(n)
    rows = [[(0, F(-1, 2)), (1, F(1, 2))],
            [(0, F(-1, 4)), (1, F(1, 4))],
            [(0, F(-1, 4)), (1, F(-3, 4)), (2, 1)]]
    for j in range(3, n - 1):
        rows.append([(j - 1, -1), (j, 1)])
    rows.append([(n - 2, -1), (n - 1, F(3, 4)), (n, F(1, 4))])
    rows.append([(n - 1, F(-1, 4)), (n, F(1, 4))])
    rows.append([(n - 1, F(-1, 2)), (n, F(1, 2))])
    return _dense(rows, n + 1)


def d_plus_exact(n):
    """D+ of the Appendix times h, (n+1) x (n+2), as printed (rows of E24)."""
    _check_n(n)
    rows = [[(0, -1), (1, F(1, 2)), (2, F(1, 2))],
            [(0, F(-1, 2)), (1, F(-1, 4)), (2, F(3, 4))]]
    for i in range(2, n - 1):
        rows.append([(i, -1), (i + 1, 1)])
    rows.append([(n - 1, F(-3, 4)), (n, F(1, 4)), (n + 1, F(1, 2))])
    rows.append([(n - 1, F(-1, 2)), (n, F(-1, 2)), (n + 1, 1)])
    return _dense(rows, n + 2)


def d_minus_exact(n):
    """D- of the Appendix times h, (n+2) x (n+1), as printed."""
    _check_n(n)
    rows = [[(0, -1), (1, 1)],
            [(0, -1), (1, 1)],
            [(0, F(-1, 5)), (1, F(-3, 5)), (2, F(4, 5))]]
    for j in range(3, n - 1):
        rows.append([(j - 1, -1), (j, 1)])
    rows.append([(n - 2, F(-4, 5)), (n - 1, F(3, 5)), (n, F(1, 5))])
    rows.append([(n - 1, -1), (n, 1)])
    rows.append([(n - 1, -1), (n, 1)])
    return _dense(rows, n + 1)


def p_plus_exact(n):
    """Diagonal of P+ / h: [1/2, 1, ..., 1, 1/2] (n+1 entries)."""
    _check_n(n)
    return [F(1, 2)] + [F(1)] * (n - 1) + [F(1, 2)]


def p_minus_exact(n):
    """Diagonal of P- / h: [1/2, 1/4, 5/4, 1, ..., 1, 5/4, 1/4, 1/2] (n+2)."""
    _check_n(n)
    return [F(1, 2), F(1, 4), F(5, 4)] + [F(1)] * (n - 4) + [F(5, 4), F(1, 4), F(1, 2)]


def b_exact(n):
    """B of E4: (n+1) x (n+2), -1 at (0, 0), +1 at (n, n+1), zero elsewhere."""
    m = [[F(0)] * (n + 2) for _ in range(n + 1)]
    m[0][0] = F(-1)
    m[n][n + 1] = F(1)
    return m


# ------------------------------------------------------ fp64 working form
def _to_np(m):
    return np.array([[float(v) for v in row] for row in m], dtype=np.float64)


def weights_plus(n, h=1.0):
    """Geometric norm weights of the "+" grid, diag(P+) with h."""
    return np.array([float(v) for v in p_plus_exact(n)]) * h


def weights_minus(n, h=1.0):
    """Geometric norm weights of the "-" grid, diag(P-) with h."""
    return np.array([float(v) for v in p_minus_exact(n)]) * h


def d_plus(n, h=1.0):
    """D+ = P+^-1 Q+ (E3), fp64, including 1/h."""
    return _to_np(d_plus_exact(n)) / h


def d_minus(n, h=1.0):
    """D- = P-^-1 Q- (E3), fp64, including 1/h."""
    return _to_np(d_minus_exact(n)) / h


def weights(kind, n, h=1.0):
    return weights_plus(n, h) if kind == "+" else weights_minus(n, h)


def grid(kind, n, h=1.0):
    return grid_plus(n, h) if kind == "+" else grid_minus(n, h)


def size(kind, n):
    return n + 1 if kind == "+" else n + 2


# ------------------------------------------- 1:2 interface interpolation
# The paper defers blocks of different mesh sizes to a follow-up article.
# Reading used here: the coupling of a coarse face (n cells of h) and a fine
# face (2n cells of h/2) uses an interpolation I_c2f (fine values from
# coarse ones) and I_f2c = Wc^-1 I_c2f^T Wf, which makes the penalties of
# E13-E15/E19-E21 (with sigma = chi = +-1/2 as in EPBCP) cancel in the
# energy rate for any I_c2f.  I_f2c must reproduce constants, i.e. the
# Wf-weighted column sums of I_c2f must equal the coarse weights Wc.
#
# "+" grid: fine nodes 2i coincide with coarse node i and fine node 2i+1 is
#   the midpoint; plain linear interpolation already satisfies the column
#   sum condition.
# "-" grid: plain linear interpolation violates it in the first three coarse
#   columns at each end.  No interpolation exact for linear functions in its
#   boundary rows can satisfy it (the first moments differ by h_c^2/8 per
#   end), so the boundary rows are constant-exact only: rows 0..3 of each end
#   (fine nodes 0, h_c/4, 3h_c/4, 5h_c/4) over coarse columns 0..2 are the
#   rows closest, in the Frobenius norm, to plain linear interpolation that
#   satisfy: every row sums to 1 and the Wf-weighted sums of coarse columns
#   0..3 equal Wc.  Solved below as an equality-constrained least-squares
#   problem (KKT system), independently of any other implementation.

def _linear_interp_matrix(xf, xc):
    m = np.zeros((len(xf), len(xc)))
    for r, p in enumerate(xf):
        i = np.searchsorted(xc, p, side="right") - 1
        i = min(max(i, 0), len(xc) - 2)
        t = (p - xc[i]) / (xc[i + 1] - xc[i])
        m[r, i] = 1.0 - t
        m[r, i + 1] = t
    return m


def _minus_boundary_block(nc):
    """Rows 0..3 / columns 0..2 of I_c2f on the "-" grid (lower end), h-free."""
    xc = grid_minus(nc, 1.0)
    xf = grid_minus(2 * nc, 0.5)
    wc = weights_minus(nc, 1.0)
    wf = weights_minus(2 * nc, 0.5)
    lin = _linear_interp_matrix(xf, xc)
    nr, ns = 4, 3
    # unknowns: block entries a[r, s], r < nr, s < ns; all other entries of
    # rows < nr are zero, rows >= nr stay linear.
    nu = nr * ns
    rows, rhs = [], []
    for r in range(nr):                       # row sums = 1
        a = np.zeros(nu)
        a[r * ns:(r + 1) * ns] = 1.0
        rows.append(a)
        rhs.append(1.0)
    fixed = lin.copy()
    fixed[:nr, :] = 0.0
    for s in range(ns + 1):                   # weighted column sums = Wc
        a = np.zeros(nu)
        if s < ns:
            for r in range(nr):
                a[r * ns + s] = wf[r]
        rows.append(a)
        rhs.append(wc[s] - wf @ fixed[:, s])
    c = np.array(rows)
    d = np.array(rhs)
    target = lin[:nr, :ns].reshape(-1)
    # minimise |a - target|^2 subject to c a = d  (KKT)
    m = len(d)
    kkt = np.zeros((nu + m, nu + m))
    kkt[:nu, :nu] = 2.0 * np.eye(nu)
    kkt[:nu, nu:] = c.T
    kkt[nu:, :nu] = c
    sol = np.linalg.lstsq(kkt, np.concatenate([2.0 * target, d]), rcond=None)[0]
    return sol[:nu].reshape(nr, ns)


def interp_c2f(kind, nc):
    """I_c2f for one tangential axis: (size(kind, 2nc) x size(kind, nc))."""
    xc = grid(kind, nc, 1.0)
    xf = grid(kind, 2 * nc, 0.5)
    m = _linear_interp_matrix(xf, xc)
    if kind == "-":
        if nc < 6:
            raise ValueError("1:2 interpolation on the '-' grid needs >= 6 coarse cells")
        blk = _minus_boundary_block(nc)
        nfr, ncl = m.shape
        m[:4, :] = 0.0
        m[:4, :3] = blk
        # mirror image at the upper end (x -> L - x reverses both grids)
        m[nfr - 4:, :] = 0.0
        m[nfr - 4:, ncl - 3:] = blk[::-1, ::-1]
    return m


def interp_f2c(kind, nc):
    """I_f2c = Wc^-1 I_c2f^T Wf (norm-compatible restriction), one axis."""
    wc = weights(kind, nc, 1.0)
    wf = weights(kind, 2 * nc, 0.5)
    return (interp_c2f(kind, nc).T * wf[None, :]) / wc[:, None]
