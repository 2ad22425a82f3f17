"""Univariate B-splines and cardinal B-splines (Sec. 3.1 of the paper).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Index conventions: the paper numbers knots xi_1..xi_{n+2p+1} and B-splines
N_1..N_{n+p} from one; the arrays here are zero-based, so ``xi[k]`` is
xi_{k+1} and column ``i`` of a basis matrix is N_{i+1}.
"""
import math

import numpy as np


def knots(n, p):
    """Open uniform knot sequence of Sec. 3.1: p+1 zeros, the breakpoints
    i/n for i=0..n (xi_{i+p+1} = i/n), p+1 ones; length n+2p+1."""
    if n < 1 or p < 0:
        raise ValueError("need n >= 1 and p >= 0")
    xi = np.empty(n + 2 * p + 1)
    xi[: p + 1] = 0.0
    xi[p : p + n + 1] = np.arange(n + 1) / n
    xi[p + n :] = 1.0
    return xi


def _cox_de_boor(xi, p, x):
    """All B-splines N_i^p(x) on knot vector ``xi`` by the recursion of
    the B-spline definition of Sec. 3.1 (degree 0: indicator of [xi_i, xi_{i+1}); degree k: the two
    divided-difference weights; a fraction with zero denominator counts as 0).
    Returns an array of shape (len(x), len(xi)-1-p)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    nfun = len(xi) - 1
    N = np.zeros((x.size, nfun))
    for i in range(nfun):
        N[:, i] = (xi[i] <= x) & (x < xi[i + 1])
    for k in range(1, p + 1):
        Nk = np.zeros((x.size, nfun - k))
        for i in range(nfun - k):
            d1 = xi[i + k] - xi[i]
            d2 = xi[i + k + 1] - xi[i + 1]
            if d1 > 0:
                Nk[:, i] += (x - xi[i]) / d1 * N[:, i]
            if d2 > 0:
                Nk[:, i] += (xi[i + k + 1] - x) / d2 * N[:, i + 1]
        N = Nk
    return N


def basis(n, p, x):
    """Matrix [N_j^p(x_k)], j = 1..n+p (columns), on the uniform open knots."""
    return _cox_de_boor(knots(n, p), p, x)


def basis_deriv(n, p, x):
    """Matrix [(N_j^p)'(x_k)] from the differentiation rule of Sec. 3.1:
    (N_i^p)' = p (N_i^{p-1}/(xi_{i+p}-xi_i) - N_{i+1}^{p-1}/(xi_{i+p+1}-xi_{i+1}))."""
    if p == 0:
        return np.zeros((np.atleast_1d(x).size, n))
    xi = knots(n, p)
    Nm = _cox_de_boor(xi, p - 1, x)  # n+p+1 functions of degree p-1 on the same knots
    out = np.zeros((Nm.shape[0], n + p))
    for i in range(n + p):
        d1 = xi[i + p] - xi[i]
        d2 = xi[i + p + 1] - xi[i + 1]
        if d1 > 0:
            out[:, i] += p * Nm[:, i] / d1
        if d2 > 0:
            out[:, i] -= p * Nm[:, i + 1] / d2
    return out


def cardinal(p, t):
    """Cardinal B-spline phi_p by the recursion of Sec. 3.1:
    phi_0 = indicator of [0,1); phi_p(t) = t/p phi_{p-1}(t) + (p+1-t)/p phi_{p-1}(t-1).
    The recursion is evaluated bottom-up over the shifts t, t-1, ..., t-p so
    that each phi_k(t-s) is computed once."""
    t = np.asarray(t, dtype=np.float64)
    vals = [((t - s >= 0) & (t - s < 1)).astype(np.float64) for s in range(p + 1)]
    for k in range(1, p + 1):
        vals = [(t - s) / k * vals[s] + (k + 1 - (t - s)) / k * vals[s + 1] for s in range(p + 1 - k)]
    return vals[0]


def cardinal_deriv(p, t, r=1):
    """r-th derivative of phi_p: the rule phi_p' = phi_{p-1}(t) - phi_{p-1}(t-1)
    of Sec. 3.1 applied r times, i.e. sum_j (-1)^j C(r,j) phi_{p-r}(t-j)."""
    if r == 0:
        return cardinal(p, t)
    if p < r:
        raise ValueError("derivative order exceeds degree")
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros(np.broadcast(t).shape)
    for j in range(r + 1):
        out = out + (-1) ** j * math.comb(r, j) * cardinal(p - r, t - j)
    return out
