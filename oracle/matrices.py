"""1D IgA matrices and the Toeplitz preconditioner factor.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* M^p_n, A^p_n, S^p_n (Sec. 3.2): Gram matrices of the Dirichlet B-splines
  N_2..N_{n+p-1} (value/value, value/derivative, derivative/derivative),
  size m = n+p-2.  Integrals are computed element by element with (p+1)-point
  Gauss-Legendre quadrature, which is exact for the degree-2p integrands.
* Central Toeplitz entries of the same matrices in terms of phi_{2p+1}
  (Sec. 3.2).
* T_m(m_{p-1}), the banded Toeplitz factor of the post-smoother's
  preconditioner (Sec. 6.1): entries phi_{2p-1}(p-i+j) for |i-j| < p.
"""
import numpy as np

from .bspline import basis, basis_deriv, cardinal, cardinal_deriv


def gauss_points(n, q):
    """q-point Gauss-Legendre nodes and weights on each of the n uniform
    elements [i/n, (i+1)/n] of [0, 1]."""
    t, w = np.polynomial.legendre.leggauss(q)
    left = np.arange(n)[:, None] / n
    x = left + (t[None, :] + 1.0) / (2.0 * n)
    wx = np.broadcast_to(w[None, :] / (2.0 * n), x.shape)
    return x.ravel(), wx.ravel().copy()


def dirichlet_size(n, p):
    """Number of Dirichlet B-splines per direction, m = n+p-2 (Sec. 4.1)."""
    return n + p - 2


def mass_adv_stiff(n, p):
    """Return (M, A, S) of Sec. 3.2 as dense m x m float64 arrays:
    M_ij = int N_{i+1} N_{j+1},  A_ij = int N_{i+1} N'_{j+1},
    S_ij = int N'_{i+1} N'_{j+1},  i, j = 1..m."""
    m = dirichlet_size(n, p)
    if m < 1:
        raise ValueError("n+p-2 must be >= 1")
    x, w = gauss_points(n, p + 1)
    B = basis(n, p, x)[:, 1 : n + p - 1]
    D = basis_deriv(n, p, x)[:, 1 : n + p - 1]
    M = B.T @ (w[:, None] * B)
    A = B.T @ (w[:, None] * D)
    S = D.T @ (w[:, None] * D)
    return M, A, S


def central_entries(n, p, k):
    """Central Toeplitz entries at offset k = i-j (Sec. 3.2):
    M = phi_{2p+1}(p+1-k)/n,  A = -phi'_{2p+1}(p+1-k),  S = -n phi''_{2p+1}(p+1-k)."""
    t = p + 1 - np.asarray(k, dtype=np.float64)
    return (
        cardinal(2 * p + 1, t) / n,
        -cardinal_deriv(2 * p + 1, t, 1),
        -n * cardinal_deriv(2 * p + 1, t, 2),
    )


def toeplitz_T(m, p):
    """T_m(m_{p-1}): (T)_ij = phi_{2p-1}(p-i+j) if |i-j| < p, else 0 (Sec. 6.1)."""
    T = np.zeros((m, m))
    for i in range(m):
        for j in range(max(0, i - p + 1), min(m, i + p)):
            T[i, j] = cardinal(2 * p - 1, p - i + j)
    return T
