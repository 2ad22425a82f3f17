"""Reference solves of A^{p,alpha,beta} u = b.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``solve_direct``: sparse LU of the explicitly assembled matrix (library
  routine, SuperLU).
* ``cg``: unpreconditioned conjugate gradients with zero initial guess and
  the stopping rule ||r_k||_2 / ||r_0||_2 < tol of Sec. 6.2.
* ``fast_diag_solve``: for alpha = beta the system decouples into d copies of
  alpha times the scalar IgA Laplacian sum_e D_e (Sec. 5.1 and 5.2, case
  alpha = beta); each copy is solved exactly with the generalized
  eigendecomposition S V = M V Lambda, V^T M V = I.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .matrices import mass_adv_stiff


def solve_direct(K, b):
    return spla.spsolve(K.tocsc(), b)


def cg(apply, b, tol, maxiter=100000, x0=None):
    """Plain CG.  Returns (x, iterations, residual-norm history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply(x)
    d = r.copy()
    rr = r @ r
    r0 = np.sqrt(rr)
    hist = [r0]
    if r0 == 0.0:
        return x, 0, hist
    k = 0
    while k < maxiter:
        q = apply(d)
        a = rr / (d @ q)
        x += a * d
        r -= a * q
        rr_new = r @ r
        k += 1
        hist.append(np.sqrt(rr_new))
        if np.sqrt(rr_new) < tol * r0:
            break
        d = r + (rr_new / rr) * d
        rr = rr_new
    return x, k, hist


def fast_diag_solve(d, p, n, alpha, b):
    """Exact solve of alpha (I_d (x) L) u = b with L = sum_e D_e."""
    M, _, S = mass_adv_stiff(n, p)
    lam, V = sla.eigh(S, M)
    m = M.shape[0]
    G = m**d
    grids = np.meshgrid(*([lam] * d), indexing="ij")
    denom = alpha * sum(grids)
    u = np.empty_like(b)
    for c in range(d):
        X = b[c * G : (c + 1) * G].reshape((m,) * d)
        for ax in range(d):  # apply V^T along every axis
            X = np.moveaxis(np.tensordot(V.T, X, axes=([1], [ax])), 0, ax)
        X = X / denom
        for ax in range(d):  # apply V along every axis
            X = np.moveaxis(np.tensordot(V, X, axes=([1], [ax])), 0, ax)
        u[c * G : (c + 1) * G] = X.ravel()
    return u
