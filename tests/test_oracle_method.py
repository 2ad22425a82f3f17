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


def _power_rayleigh(L, iters):
    # Rayleigh quotient of the pencil (K, D) at (D^{-1} K)^iters v0
    v = method.start_vector(L.d, L.m)
    for _ in range(iters):
        v = (L.K @ v) / L.D
        v /= np.linalg.norm(v)
    return (v @ (L.K @ v)) / (v @ (L.D * v))


@pytest.mark.parametrize("d,p,n,beta", [(2, 3, 16, 0.1), (2, 1, 20, 0.3), (3, 2, 6, 0.05)])
def test_lanczos_estimate_bounded_by_krylov_optimality(d, p, n, beta):
    # The largest Ritz value maximises the Rayleigh quotient over the Krylov
    # space K_k(D^{-1} K, v0), which holds the power iterate after k-1 steps:
    # power estimate <= Ritz value <= largest pencil eigenvalue.
    meth = method.Method(d, p, n, 1.0, beta, coarse_max_dofs=10**6)
    L = meth.levels[0]
    lmax = sla.eigh(L.K.toarray(), np.diag(L.D), eigvals_only=True)[-1]
    prev = 0.0
    for k in (1, 2, 5, 10, 20):
        th = method.lanczos_estimate(L, k)
        assert th <= lmax * (1 + 1e-12)
        assert th >= _power_rayleigh(L, k - 1) * (1 - 1e-12), k
        assert th >= prev * (1 - 1e-12), k
        prev = th
    # one step: the Rayleigh quotient of v0 itself
    v0 = method.start_vector(d, L.m)
    assert abs(method.lanczos_estimate(L, 1) - (v0 @ (L.K @ v0)) / (v0 @ (L.D * v0))) <= 1e-13 * lmax
    # a full Krylov space reaches the largest eigenvalue the start vector sees
    assert method.lanczos_estimate(L, 60) >= 0.999 * lmax


def test_lanczos_restarts_when_the_start_vector_spans_an_invariant_subspace():
    # 3D p=2 n=4, level 1: the symmetric start vector spans a two-dimensional
    # invariant subspace of D^{-1} K (the recurrence breaks down at its second
    # step) whose Ritz values stay well below the top of the spectrum; the
    # restart from the fixed vector still finds it
    meth = method.Method(3, 2, 4, 1.0, 0.1, coarse_max_dofs=1)
    L = meth.levels[1]
    v = method.start_vector(L.d, L.m)
    q = v / np.sqrt(v @ (L.D * v))
    qprev, b = np.zeros_like(q), 0.0
    alpha, beta = [], []
    for _ in range(2):
        Kq = L.K @ q
        a = q @ Kq
        w = Kq / L.D - a * q - b * qprev
        b = np.sqrt(w @ (L.D * w))
        alpha.append(a)
        beta.append(b)
        qprev, q = q, w / b
    assert beta[0] > method.LANCZOS_BREAKDOWN * abs(alpha[0])
    assert beta[1] <= method.LANCZOS_BREAKDOWN * abs(alpha[1])
    lmax = sla.eigh(L.K.toarray(), np.diag(L.D), eigvals_only=True)[-1]
    sub = sla.eigvalsh_tridiagonal(np.array(alpha), np.array(beta[:1]))[-1]
    assert sub < 0.9 * lmax
    assert 0.999 * lmax <= L.lam <= lmax * (1 + 1e-12)


def test_lanczos_estimate_on_levels_is_close_to_lambda_max():
    meth = method.Method(2, 3, 16, 1.0, 0.1, coarse_max_dofs=100)
    for L in meth.levels[:-1]:
        lmax = sla.eigh(L.K.toarray(), np.diag(L.D), eigvals_only=True)[-1]
        assert 0.95 * lmax <= L.lam <= lmax * (1 + 1e-12)


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


def _vcycle_matrix(meth):
    N = meth.K.shape[0]
    return np.column_stack([meth.vcycle(e) for e in np.eye(N)])


def test_coarse_degree_keeps_vcycle_symmetric_positive_definite():
    # With Chebyshev post-smoothing everywhere, the same polynomial before and
    # after each coarse correction makes the V-cycle a symmetric positive
    # definite operator whatever the per-level degrees are; a coarse degree
    # applied on one side only breaks the symmetry.  Definiteness also needs
    # every level's interval to cover its spectrum, hence converged estimates.
    kw = dict(coarse_max_dofs=40, krylov_steps=0, lanczos_steps=100)
    m1 = method.Method(2, 2, 16, 1.0, 0.1, nu=4, nu_coarse=2, **kw)
    m2 = method.Method(2, 2, 16, 1.0, 0.1, nu=4, **kw)
    assert len(m1.levels) >= 3
    assert [L.nu for L in m1.levels[:-1]] == [4] + [2] * (len(m1.levels) - 2)
    B1, B2 = _vcycle_matrix(m1), _vcycle_matrix(m2)
    assert np.abs(B1 - B1.T).max() <= 1e-12 * np.abs(B1).max()
    assert np.linalg.eigvalsh(0.5 * (B1 + B1.T)).min() > 0
    assert np.abs(B1 - B2).max() > 1e-6 * np.abs(B2).max()


def test_coarse_degree_unused_with_two_levels():
    # Two levels: the finest is the only smoothed one, the coarsest is exact.
    kw = dict(coarse_max_dofs=300)
    m1 = method.Method(2, 3, 16, 1.0, 0.1, nu=5, nu_coarse=1, **kw)
    m2 = method.Method(2, 3, 16, 1.0, 0.1, nu=5, **kw)
    assert len(m1.levels) == 2
    b = _rand(m1.K.shape[0], 12)
    np.testing.assert_array_equal(m1.vcycle(b), m2.vcycle(b))


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


@pytest.mark.parametrize("d,p,ns,beta", [(2, 3, (24, 40), 0.05), (3, 2, (8, 12, 16), 0.1), (2, 2, (32, 16), 1.0)])
def test_anisotropic_solution_matches_direct_solve(d, p, ns, beta):
    # n_l = nu_l n: every axis is coarsened at every level; the hierarchy
    # stops when an axis cannot be halved
    meth = method.Method(d, p, ns, 1.0, beta, coarse_max_dofs=300)
    assert len(meth.levels) >= 2
    for L, Lc in zip(meth.levels, meth.levels[1:]):
        assert all(nc == nl // 2 for nl, nc in zip(L.ns, Lc.ns))
        assert Lc.K.shape[0] == d * int(np.prod([nl // 2 + p - 2 for nl in L.ns]))
    b = _rand(meth.K.shape[0], 21)
    x, it, _ = meth.solve(b, 1e-12)
    xd = solvers.solve_direct(asm.curl_div_matrix(d, p, ns, 1.0, beta), b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    assert it < 60


@pytest.mark.parametrize("d,p,ns,cmax,kind", [(2, 3, (25, 25), 60, "paper"), (2, 2, (4, 64), 10, "none"),
                                              (3, 2, (7, 8, 6), 30, "paper")])
def test_odd_and_short_axes_keep_coarsening(d, p, ns, cmax, kind):
    # an odd n switches its axis to the paper's prolongator (m -> floor(m/2));
    # an axis with one point stays as it is while the others coarsen
    meth = method.Method(d, p, ns, 1.0, 0.1, coarse_max_dofs=cmax)
    C = meth.levels[-1]
    assert C.K.shape[0] <= cmax or all(m == 1 for m in C.ms)
    kinds = set()
    for L, Lc in zip(meth.levels, meth.levels[1:]):
        for l in range(d):
            m, mc, n, nc = L.ms[l], Lc.ms[l], L.ns[l], Lc.ns[l]
            if m == 1:
                seen = "none"
                assert mc == 1
            elif nc is not None:  # knot insertion
                seen = "knot"
                assert n % 2 == 0 and nc == n // 2 and mc == nc + p - 2
            else:  # the paper's prolongator
                seen = "paper"
                assert mc == m // 2
            kinds.add(seen)
    assert kind in kinds
    b = _rand(meth.K.shape[0], 23)
    x, it, _ = meth.solve(b, 1e-12)
    xd = solvers.solve_direct(asm.curl_div_matrix(d, p, ns, 1.0, 0.1), b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


@pytest.mark.parametrize("variant", ["P_WL", "MIM"])
@pytest.mark.parametrize("d,p,n,beta", [(2, 3, 16, 0.1), (3, 2, 8, 0.1)])
def test_pwl_and_mim_solutions_match_direct_solve(variant, d, p, n, beta):
    meth = method.Method(d, p, n, 1.0, beta, coarse_max_dofs=60, variant=variant)
    b = _rand(meth.K.shape[0], 25)
    x, it, hist = meth.solve(b, 1e-11, maxiter=2000)
    xd = solvers.solve_direct(asm.curl_div_matrix(d, p, n, 1.0, beta), b)
    assert hist[-1] < 1e-11 * hist[0]
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    # the outer iteration always uses the system matrix, not the cycle's D
    assert abs(meth.K - asm.curl_div_matrix(d, p, n, 1.0, beta)).max() == 0


def test_pwl_cycle_is_the_pmim_cycle_when_alpha_equals_beta():
    # alpha = beta: the off-diagonal blocks vanish (weight alpha - beta), D = A,
    # and without the Krylov post-smoother the two cycles are the same map
    kw = dict(coarse_max_dofs=60, krylov_steps=0)
    a = method.Method(2, 3, 16, 0.8, 0.8, variant="P_WL", **kw)
    b = method.Method(2, 3, 16, 0.8, 0.8, variant="P_MIM", **kw)
    r = _rand(a.K.shape[0], 26)
    np.testing.assert_allclose(a.vcycle(r), b.vcycle(r), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("d,p,n", [(2, 2, 10), (3, 2, 4)])
def test_pwl_cycle_keeps_components_apart(d, p, n):
    meth = method.Method(d, p, n, 1.0, 0.05, coarse_max_dofs=30, variant="P_WL")
    G = meth.K.shape[0] // d
    for L in meth.levels:
        Gl = L.K.shape[0] // d
        for c in range(d):
            for e in range(d):
                if c != e:
                    assert L.K[c * Gl:(c + 1) * Gl, e * Gl:(e + 1) * Gl].nnz == 0
    r = np.zeros(meth.K.shape[0])
    r[G:2 * G] = _rand(G, 27)
    z = meth.vcycle(r)
    other = np.ones(z.size, bool)
    other[G:2 * G] = False
    assert np.abs(z[other]).max() == 0 and np.abs(z[G:2 * G]).max() > 0


def test_mim_needs_more_iterations_than_pmim():
    # the same cycle, with and without Krylov acceleration
    b = _rand(2 * 17 * 17, 28)
    it_mim = method.Method(2, 3, 16, 1.0, 0.01, coarse_max_dofs=60, variant="MIM").solve(b, 1e-8)[1]
    it_pmim = method.Method(2, 3, 16, 1.0, 0.01, coarse_max_dofs=60).solve(b, 1e-8)[1]
    assert it_mim > it_pmim


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
