"""Pins of the oracle's solver steps (Sec. 6.1) against closed forms and brute force."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import assembly as asm
from oracle import method
from oracle import mim
from oracle import solvers


def _rand(n, seed):
    return np.random.default_rng(seed).uniform(-1, 1, n)


def test_chebyshev_error_polynomial():
    # nu Chebyshev steps from x0 with b = 0 map e0 to p_nu(D^{-1}K) e0 with
    # p_nu(t) = T_nu((theta - t)/delta) / T_nu(theta/delta)
    meth = method.Method(2, 2, 8, 1.0, 0.3, coarse_max_dofs=50)
    L = meth.levels[0]
    K, D = L.K.toarray(), L.D
    for nu in (1, 2, 3, 5):
        E = np.column_stack([method.chebyshev(L, e, np.zeros(K.shape[0]), nu)
                             for e in np.eye(K.shape[0])[:: max(1, K.shape[0] // 40)]])
        Dh = np.sqrt(D)
        w, V = np.linalg.eigh(K / Dh[:, None] / Dh[None, :])
        theta, delta = 0.5 * (L.hi + L.lo), 0.5 * (L.hi - L.lo)
        pw = np.polynomial.chebyshev.chebval((theta - w) / delta, [0] * nu + [1]) / \
            np.polynomial.chebyshev.chebval(theta / delta, [0] * nu + [1])
        Pmat = (V * pw) @ V.T
        Pfull = Pmat * (1 / Dh)[:, None] * Dh[None, :]  # p(D^{-1}K) = D^{-1/2} p(.) D^{1/2}
        cols = np.arange(K.shape[0])[:: max(1, K.shape[0] // 40)]
        np.testing.assert_allclose(E, Pfull[:, cols], atol=1e-12)


def test_power_estimate_is_rayleigh_lower_bound():
    meth = method.Method(2, 3, 16, 1.0, 0.1, coarse_max_dofs=100)
    for L in meth.levels[:-1]:
        K = L.K.toarray()
        lmax = sla.eigh(K, np.diag(L.D), eigvals_only=True)[-1]
        assert L.lam <= lmax * (1 + 1e-12)
        assert L.lam >= 0.8 * lmax


def test_gmres_matches_bruteforce_krylov_minimization():
    meth = method.Method(2, 3, 10, 1.0, 0.05, coarse_max_dofs=50)
    K = meth.K.toarray()
    r = _rand(K.shape[0], 2)
    for s in (1, 2, 3, 4):
        e = method.gmres_T(meth.K, meth.Tsolve, r, s)
        # minimize ||r - K T^{-1} W c|| over the Krylov space of K T^{-1} directly
        Tinv = np.linalg.inv(meth.T.toarray())
        KT = K @ Tinv
        W = np.column_stack([np.linalg.matrix_power(KT, j) @ r for j in range(s)])
        c = np.linalg.lstsq(KT @ W, r, rcond=None)[0]
        e_ref = Tinv @ (W @ c)
        np.testing.assert_allclose(e, e_ref, atol=1e-9 * np.abs(e_ref).max())


def test_fcg_with_identity_preconditioner_is_cg():
    K = asm.curl_div_matrix(2, 2, 8, 1.0, 0.2)
    b = _rand(K.shape[0], 9)
    meth = method.Method(2, 2, 8, 1.0, 0.2, coarse_max_dofs=50)
    meth.vcycle = lambda r, l=0: r.copy()
    x1, it1, h1 = meth.solve(b, 1e-10)
    x2, it2, h2 = solvers.cg(lambda v: K @ v, b, 1e-10)
    assert it1 == it2
    np.testing.assert_allclose(h1, h2, rtol=1e-8)


def test_single_level_vcycle_is_exact_solve():
    meth = method.Method(2, 2, 6, 1.0, 0.1, coarse_max_dofs=10**6)
    assert len(meth.levels) == 1
    b = _rand(meth.K.shape[0], 4)
    np.testing.assert_allclose(meth.vcycle(b), solvers.solve_direct(meth.K, b), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("d,p,n,beta", [(2, 2, 16, 1.0), (2, 3, 16, 0.1), (3, 2, 8, 0.1), (3, 3, 4, 0.01)])
@pytest.mark.parametrize("transfer", ["knot", "paper"])
def test_solution_matches_direct_solve(d, p, n, beta, transfer):
    meth = method.Method(d, p, n, 1.0, beta, transfer=transfer, coarse_max_dofs=60)
    assert len(meth.levels) >= 2
    b = _rand(meth.K.shape[0], 7)
    x, it, hist = meth.solve(b, 1e-12)
    xd = solvers.solve_direct(meth.K, b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    assert it < 60


def test_iterations_flat_in_n_and_growing_as_beta_falls():
    # qualitative behaviour reported in Sec. 6.2
    counts = {}
    for beta in (0.1, 0.01):
        for n in (16, 32, 64):
            meth = method.Method(2, 2, n, 1.0, beta, coarse_max_dofs=100)
            b = _rand(meth.K.shape[0], n)
            counts[(beta, n)] = meth.solve(b, 1e-7)[1]
    for beta in (0.1, 0.01):
        row = [counts[(beta, n)] for n in (16, 32, 64)]
        assert max(row) - min(row) <= 3, row
    assert all(counts[(0.01, n)] > counts[(0.1, n)] for n in (16, 32, 64))


def test_paper_mim_converges_and_is_flat():
    its = []
    for n in (15, 31):
        K = asm.curl_div_matrix(2, 2, n, 1.0, 0.1)
        b = _rand(K.shape[0], 1)
        x, it = mim.PaperMIM(2, 2, n, 1.0, 0.1, "P_MIM", K=K).solve(b)
        assert np.linalg.norm(b - K @ x) < 1e-7 * np.linalg.norm(b)
        its.append(it)
    assert abs(its[0] - its[1]) <= 3
