"""Grid-transfer (prolongation) matrices in 1D.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``paper_prolongator``: P = T_m(1+cos theta) K_m^T with the cutting matrix K
  that keeps the even-indexed unknowns (Sec. 6.1), i.e. the stencil
  (1/2)[1 2 1]^T with stride 2.  The paper states it for odd m (m_c = (m-1)/2);
  for even m this module takes m_c = m/2 and truncates the last column at row m.
* ``knot_insertion_prolongator``: exact embedding of the Dirichlet spline
  space on n/2 uniform intervals into the one on n intervals, obtained by
  inserting the new knots (2i+1)/n one at a time with Boehm's algorithm.
  The coarse operators are then the Galerkin products P^T X P (Sec. 6.1).
"""
import numpy as np

from .bspline import knots


def paper_prolongator(m):
    mc = m // 2
    P = np.zeros((m, mc))
    for j in range(1, mc + 1):  # one-based coarse index; fine rows 2j-1, 2j, 2j+1
        for i, v in ((2 * j - 1, 0.5), (2 * j, 1.0), (2 * j + 1, 0.5)):
            if 1 <= i <= m:
                P[i - 1, j - 1] = v
    return P


def _boehm_insert(xi, p, C, t):
    """Insert knot t once into knot vector xi (degree p).  C holds B-spline
    coefficients in its rows (one column per represented function).  Returns
    the new knot vector and coefficient matrix."""
    # interval index k (zero-based) with xi[k] <= t < xi[k+1]
    k = np.searchsorted(xi, t, side="right") - 1
    nfun = C.shape[0]
    Cn = np.zeros((nfun + 1, C.shape[1]))
    for i in range(nfun + 1):
        if i <= k - p:
            a = 1.0
        elif i >= k + 1:
            a = 0.0
        else:
            a = (t - xi[i]) / (xi[i + p] - xi[i])
        left = C[i - 1] if i >= 1 else 0.0
        right = C[i] if i < nfun else 0.0
        Cn[i] = (1.0 - a) * left + a * right
    return np.insert(xi, k + 1, t), Cn


def knot_insertion_prolongator(n_fine, p, full=False):
    """Matrix P with N^{coarse}_j = sum_i P_ij N^{fine}_i for the uniform open
    knots with n_fine/2 (coarse) and n_fine (fine) intervals.  By default the
    rows/columns of the two boundary functions are dropped (Dirichlet space,
    Sec. 3.1), giving a (n_fine+p-2) x (n_fine/2+p-2) matrix."""
    if n_fine % 2:
        raise ValueError("knot insertion halving needs an even number of intervals")
    nc = n_fine // 2
    xi = knots(nc, p)
    C = np.eye(nc + p)
    for i in range(nc):
        xi, C = _boehm_insert(xi, p, C, (2 * i + 1) / n_fine)
    if full:
        return C
    return C[1:-1, 1:-1]
