"""Spectral symbols (Sec. 3.2, Sec. 5, Sec. 6.1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* m_p, a_p, s_p: symbols of {n M}, {-i A}, {S/n} (theorem of Sec. 3.2).
* f^{p,alpha,beta}: the d x d matrix-valued symbol of {n^{d-2} A^{p,alpha,beta}}
  (Sec. 5.1 for d = 2, Sec. 5.2 for d = 3), here for nu = (1,...,1) unless
  given.
* Laplacian symbol (Sec. 5.1, 5.2) and g_p = prod_i m_{p-1}(theta_i) (Sec. 6.1).
"""
import numpy as np

from .bspline import cardinal, cardinal_deriv


def m_sym(p, theta):
    th = np.asarray(theta, dtype=np.float64)
    out = cardinal(2 * p + 1, p + 1) * np.ones_like(th)
    for k in range(1, p + 1):
        out = out + 2 * cardinal(2 * p + 1, p + 1 - k) * np.cos(k * th)
    return out


def a_sym(p, theta):
    th = np.asarray(theta, dtype=np.float64)
    out = np.zeros_like(th)
    for k in range(1, p + 1):
        out = out - 2 * cardinal_deriv(2 * p + 1, p + 1 - k, 1) * np.sin(k * th)
    return out


def s_sym(p, theta):
    th = np.asarray(theta, dtype=np.float64)
    out = -cardinal_deriv(2 * p + 1, p + 1, 2) * np.ones_like(th)
    for k in range(1, p + 1):
        out = out - 2 * cardinal_deriv(2 * p + 1, p + 1 - k, 2) * np.cos(k * th)
    return out


def curl_div_symbol(p, alpha, beta, thetas, nu=None):
    """f^{p,alpha,beta}(theta) for d = len(thetas); each theta_i is an array of
    the same shape.  Returns an array of shape (..., d, d)."""
    d = len(thetas)
    nu = np.ones(d) if nu is None else np.asarray(nu, dtype=np.float64)
    mm = [m_sym(p, t) for t in thetas]
    aa = [a_sym(p, t) for t in thetas]
    ss = [s_sym(p, t) for t in thetas]
    shape = np.broadcast(*thetas).shape
    f = np.zeros(shape + (d, d))
    if d == 2:
        r21, r12 = nu[1] / nu[0], nu[0] / nu[1]
        f[..., 0, 0] = alpha * r21 * mm[0] * ss[1] + beta * r12 * ss[0] * mm[1]
        f[..., 1, 1] = alpha * r12 * ss[0] * mm[1] + beta * r21 * mm[0] * ss[1]
        f[..., 0, 1] = f[..., 1, 0] = -(alpha - beta) * aa[0] * aa[1]
    elif d == 3:
        prod = nu.prod()
        gam = nu**2 / prod
        dl = 1.0 / nu
        lap_terms = [
            gam[0] * ss[0] * mm[1] * mm[2],
            gam[1] * mm[0] * ss[1] * mm[2],
            gam[2] * mm[0] * mm[1] * ss[2],
        ]
        for c in range(3):
            f[..., c, c] = sum((beta if e == c else alpha) * lap_terms[e] for e in range(3))
        f[..., 0, 1] = f[..., 1, 0] = -(alpha - beta) * dl[2] * aa[0] * aa[1] * mm[2]
        f[..., 0, 2] = f[..., 2, 0] = -(alpha - beta) * dl[1] * aa[0] * mm[1] * aa[2]
        f[..., 1, 2] = f[..., 2, 1] = -(alpha - beta) * dl[0] * mm[0] * aa[1] * aa[2]
    else:
        raise ValueError("d must be 2 or 3")
    return f


def laplacian_symbol(p, thetas, nu=None):
    """Symbol of the tensor B-spline Laplacian (Sec. 5.1 for d=2, 5.2 for d=3)."""
    d = len(thetas)
    nu = np.ones(d) if nu is None else np.asarray(nu, dtype=np.float64)
    mm = [m_sym(p, t) for t in thetas]
    ss = [s_sym(p, t) for t in thetas]
    if d == 2:
        return nu[1] / nu[0] * mm[0] * ss[1] + nu[0] / nu[1] * ss[0] * mm[1]
    gam = nu**2 / nu.prod()
    return (gam[0] * ss[0] * mm[1] * mm[2] + gam[1] * mm[0] * ss[1] * mm[2]
            + gam[2] * mm[0] * mm[1] * ss[2])


def g_sym(p, thetas):
    """g_p(theta) = prod_i m_{p-1}(theta_i), the symbol of T (Sec. 6.1)."""
    out = 1.0
    for t in thetas:
        out = out * m_sym(p - 1, t)
    return out


def grid_gamma(m, d):
    """The uniform grid Gamma = {k pi / m : k = 1..m}^d of Sec. 5.3."""
    t = np.arange(1, m + 1) * np.pi / m
    return np.meshgrid(*([t] * d), indexing="ij")


def central_symbol(K, d, ms, thetas):
    """Symbol of the Toeplitz part of an assembled level operator K (sparse,
    d components of prod(ms) points each, component-major, last axis fastest):
    F_ce(theta) = sum_k K[(c, x0), (e, x0 + k)] exp(i k . theta), read off the
    rows of the central grid point x0 (Sec. 5: for the finest level this is
    n^{2-d} f^{p,alpha,beta}).  thetas: d arrays of one shape.  Returns an
    array of shape (..., d, d)."""
    ms = tuple(int(m) for m in ms)
    G = int(np.prod(ms))
    x0 = tuple(m // 2 for m in ms)
    lin0 = int(np.ravel_multi_index(x0, ms))
    K = K.tocsr()
    shape = np.broadcast(*thetas).shape
    F = np.zeros(shape + (d, d), dtype=np.complex128)
    for c in range(d):
        row = K.getrow(c * G + lin0)
        for col, val in zip(row.indices, row.data):
            e, rest = divmod(int(col), G)
            idx = np.unravel_index(rest, ms)
            phase = sum((int(idx[l]) - x0[l]) * thetas[l] for l in range(d))
            F[..., c, e] += val * np.exp(1j * phase)
    return F


def symbol_bound(K, d, ms, samples):
    """max over theta in [0, pi]^d (samples points per axis) of the largest
    eigenvalue of Dh^{-1/2} F(theta) Dh^{-1/2}, F = central_symbol(K) and Dh
    its constant diagonal: the symbol's value of lambda_max(diag(K)^{-1} K)
    away from the boundary."""
    t = np.linspace(0.0, np.pi, samples)
    th = np.meshgrid(*([t] * d), indexing="ij")
    F = central_symbol(K, d, ms, th)
    G = int(np.prod(ms))
    x0 = tuple(int(m) // 2 for m in ms)
    lin0 = int(np.ravel_multi_index(x0, tuple(int(m) for m in ms)))
    dh = np.array([K[c * G + lin0, c * G + lin0] for c in range(d)])
    s = 1.0 / np.sqrt(dh)
    H = F * s[:, None] * s[None, :]
    return float(np.linalg.eigvalsh(H).max())
