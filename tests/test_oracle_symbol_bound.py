"""Pins of the symbol-based smoother bound (Sec. 5, Sec. 6.1).

* central_symbol, the symbol read off the rows of the central grid point of
  an assembled operator, times n^{d-2} equals the paper's f^{p,alpha,beta}
  (Sec. 5.1 for d = 2, Sec. 5.2 for d = 3; symbols.curl_div_symbol, built
  from cardinal B-splines, not from the assembled matrices).
* symbol_bound against the largest eigenvalue of diag(K)^{-1} K from a
  sparse eigensolver: the symbol describes the interior of the spectrum, so
  lambda_max is at least the bound less a few percent (the grid has not
  reached the symbol's maximum at small n) and at most 1.5 times it (the
  boundary rows put outliers above the symbol; measured up to 1.42 for 3D
  p = 3 with alpha = beta), the safety factor the solver applies.
* The V-cycle method with symbol bounds solves the system.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import assembly as asm
from oracle import method, solvers, symbols


@pytest.mark.parametrize("d,p,n,alpha,beta", [(2, 3, 16, 1.0, 0.3), (3, 2, 8, 1.0, 0.01), (2, 2, 12, 0.5, 2.0),
                                              (3, 3, 9, 1.0, 0.1), (2, 5, 14, 1.0, 1e-3), (3, 1, 8, 2.0, 0.5)])
def test_central_symbol_is_the_papers_symbol(d, p, n, alpha, beta):
    K = asm.curl_div_matrix(d, p, n, alpha, beta)
    m = n + p - 2
    rng = np.random.default_rng(5)
    th = [rng.uniform(-np.pi, np.pi, 64) for _ in range(d)]
    F = symbols.central_symbol(K, d, (m,) * d, th)
    f = symbols.curl_div_symbol(p, alpha, beta, th)
    assert np.abs(F * n ** (d - 2) - f).max() <= 1e-13 * np.abs(f).max()


def _lambda_max(K):
    Dm = sp.diags(1.0 / np.sqrt(K.diagonal()))
    return spla.eigsh(Dm @ K @ Dm, k=1, which="LA", return_eigenvectors=False, tol=1e-10)[0]


@pytest.mark.parametrize("d,p,n,beta", [(2, 1, 32, 0.1), (2, 2, 32, 0.1), (2, 3, 32, 0.01), (2, 4, 32, 0.1),
                                        (2, 6, 32, 1.0), (2, 3, 48, 1e-4), (3, 1, 10, 0.1), (3, 2, 10, 0.1),
                                        (3, 3, 12, 1e-3), (3, 3, 12, 1.0), (3, 4, 9, 0.1)])
def test_symbol_bound_brackets_the_spectrum(d, p, n, beta):
    K = asm.curl_div_matrix(d, p, n, 1.0, beta).tocsr()
    m = n + p - 2
    sb = symbols.symbol_bound(K, d, (m,) * d, method.symbol_samples(d))
    lam = _lambda_max(K)
    assert 0.95 * sb <= lam <= 1.5 * sb, (sb, lam, lam / sb)


@pytest.mark.parametrize("d,p,n,beta", [(2, 3, 32, 0.05), (3, 2, 16, 0.1)])
def test_vcycle_with_symbol_bounds_solves(d, p, n, beta):
    m = method.Method(d, p, n, 1.0, beta, coarse_max_dofs=300, bounds="symbol")
    assert any(L.hi == 1.5 * L.lam for L in m.levels[:-1])
    b = np.random.default_rng(6).uniform(-1, 1, m.K.shape[0])
    x, it, _ = m.solve(b, 1e-10, maxiter=500)
    xd = solvers.solve_direct(asm.curl_div_matrix(d, p, n, 1.0, beta), b)
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)
    _, it_l, _ = method.Method(d, p, n, 1.0, beta, coarse_max_dofs=300).solve(b, 1e-10, maxiter=500)
    print(f"{d}D p={p} n={n}: {it} iterations with symbol bounds, {it_l} with Lanczos")
    assert it <= 2 * it_l
