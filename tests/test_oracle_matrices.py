"""Pins of the 1D matrices, symbols and the Toeplitz factor T (Sec. 3.2, 6.1)."""
import numpy as np
import pytest

from oracle import matrices as mt
from oracle import symbols as sy


@pytest.mark.parametrize("p", range(1, 7))
@pytest.mark.parametrize("n", [1, 4, 17])
def test_symmetry_and_definiteness(n, p):
    if n + p - 2 < 1:
        pytest.skip("empty space")
    M, A, S = mt.mass_adv_stiff(n, p)
    m = n + p - 2
    assert M.shape == A.shape == S.shape == (m, m)
    np.testing.assert_allclose(M, M.T, atol=1e-16)
    np.testing.assert_allclose(S, S.T, atol=1e-12 * abs(S).max())
    np.testing.assert_allclose(A, -A.T, atol=1e-13)  # skew (Sec. 3.2)
    assert np.linalg.eigvalsh(M).min() > 0
    assert np.linalg.eigvalsh(S).min() > 0  # Dirichlet stiffness is SPD


@pytest.mark.parametrize("p", range(1, 7))
def test_bandwidth(p):
    M, A, S = mt.mass_adv_stiff(20, p)
    i, j = np.indices(M.shape)
    far = np.abs(i - j) > p
    for X in (M, A, S):
        assert np.all(X[far] == 0.0)


@pytest.mark.parametrize("p", range(1, 7))
def test_central_toeplitz_entries(p):
    # Sec. 3.2: central entries are cardinal-spline values; corrections are
    # confined to the first and last 2(p-1) rows (low-rank, rank <= 4p)
    n = 6 * p + 10
    M, A, S = mt.mass_adv_stiff(n, p)
    m = n + p - 2
    c = 2 * (p - 1)
    for i in range(c, m - c):
        for j in range(max(0, i - p), min(m, i + p + 1)):
            cm, ca, cs = mt.central_entries(n, p, i - j)
            assert abs(M[i, j] - cm) < 1e-15
            assert abs(A[i, j] - ca) < 1e-13
            assert abs(S[i, j] - cs) < 1e-11 * n
    for X, k in ((M, 0), (A, 1), (S, 2)):
        T = np.zeros_like(X)
        for i in range(m):
            for j in range(max(0, i - p), min(m, i + p + 1)):
                T[i, j] = mt.central_entries(n, p, i - j)[k]
        assert np.linalg.matrix_rank(X - T, tol=1e-10 * abs(X).max()) <= 4 * p


def test_p2_closed_form_rows():
    n = 20
    M, A, S = mt.mass_adv_stiff(n, 2)
    np.testing.assert_allclose(n * M[8, 6:11], np.array([1, 26, 66, 26, 1]) / 120, rtol=1e-13)
    np.testing.assert_allclose(A[8, 6:11], np.array([-1, -10, 0, 10, 1]) / 24, atol=1e-14)
    np.testing.assert_allclose(S[8, 6:11] / n, np.array([-1, -2, 6, -2, -1]) / 6, rtol=1e-12)


def test_p1_hat_functions():
    # p = 1: hat functions, M = h/6 tridiag(1,4,1), S = 1/h tridiag(-1,2,-1), A = 1/2 tridiag(-1,0,1)
    n = 7
    M, A, S = mt.mass_adv_stiff(n, 1)
    h = 1.0 / n
    m = n - 1
    E = np.eye(m, k=1) + np.eye(m, k=-1)
    np.testing.assert_allclose(M, h / 6 * (4 * np.eye(m) + E), atol=1e-15)
    np.testing.assert_allclose(S, (2 * np.eye(m) - E) / h, atol=1e-12)
    np.testing.assert_allclose(A, 0.5 * (np.eye(m, k=1) - np.eye(m, k=-1)), atol=1e-15)


@pytest.mark.parametrize("p", range(1, 7))
def test_row_sums_central(p):
    # int N_i = 1/n for central B-splines; derivatives of the constant vanish
    n = 6 * p + 10
    M, A, S = mt.mass_adv_stiff(n, p)
    sl = slice(2 * p, n + p - 2 - 2 * p)
    np.testing.assert_allclose(M.sum(1)[sl], 1.0 / n, rtol=1e-13)
    np.testing.assert_allclose(A.sum(1)[sl], 0.0, atol=1e-13)
    np.testing.assert_allclose(S.sum(1)[sl], 0.0, atol=1e-10 * n)


@pytest.mark.parametrize("p", range(1, 7))
def test_symbol_lemma(p):
    # Lemma of Sec. 3.2: m_p > 0, m_p <= m_p(0) = 1;
    # s_p = m_{p-1} (2 - 2 cos); m_p s_p >= a_p^2 with equality only at 0.
    # The printed lower bound (2/pi)^{2p} fails at theta = pi for every p
    # (m_1(pi) = 1/3 < 4/pi^2); the bound holds with exponent 2(p+1), which
    # is the reading taken here.
    th = np.linspace(-np.pi, np.pi, 4001)
    m = sy.m_sym(p, th)
    assert abs(sy.m_sym(p, 0.0) - 1.0) < 1e-14
    assert m.min() > 0 and m.max() <= 1 + 1e-14
    assert m.min() >= (2 / np.pi) ** (2 * p + 2) - 1e-14
    assert sy.m_sym(p, np.pi) < (2 / np.pi) ** (2 * p)
    np.testing.assert_allclose(sy.s_sym(p, th), sy.m_sym(p - 1, th) * (2 - 2 * np.cos(th)), atol=1e-14)
    gap = m * sy.s_sym(p, th) - sy.a_sym(p, th) ** 2
    assert gap.min() >= -1e-15
    nz = np.abs(th) >= 1.0  # the gap has a high-order zero at 0 (about 4e-14 at 0.5 for p = 6)
    assert gap[nz].min() > 0


@pytest.mark.parametrize("p", [2, 3, 4])
def test_1d_spectra_follow_symbols(p):
    # Theorem of Sec. 3.2: {nM} ~ m_p, {S/n} ~ s_p; compare sorted eigenvalues with
    # sorted symbol samples on theta_k = k pi / m, up to a few outliers
    errs = []
    for n in (40, 160):
        M, A, S = mt.mass_adv_stiff(n, p)
        m = n + p - 2
        th = np.arange(1, m + 1) * np.pi / m
        em = np.sort(np.linalg.eigvalsh(n * M))
        es = np.sort(np.linalg.eigvalsh(S / n))
        ea = np.sort(np.linalg.eigvalsh(-1j * A))
        sm, ss = np.sort(sy.m_sym(p, th)), np.sort(sy.s_sym(p, th))
        sa = np.sort(sy.a_sym(p, np.linspace(-np.pi, np.pi, m + 2)[1:-1]))
        errs.append([np.median(np.abs(em - sm)), np.median(np.abs(es - ss) / ss.max()),
                     np.median(np.abs(ea - sa)) / np.abs(sa).max()])
    errs = np.array(errs)
    assert np.all(errs[1] < 0.012)
    assert np.all(errs[1] <= errs[0] / 2 + 1e-14)  # shrinking as n grows


@pytest.mark.parametrize("p", range(1, 7))
def test_toeplitz_T(p):
    m = 3 * p + 4
    T = mt.toeplitz_T(m, p)
    np.testing.assert_allclose(T, T.T, atol=0)
    assert np.linalg.eigvalsh(T).min() > 0
    if p == 1:
        np.testing.assert_array_equal(T, np.eye(m))
    # entries equal n times the central mass entries of degree p-1 (quadrature route)
    if p >= 2:
        n = 6 * p + 10
        Mq, _, _ = mt.mass_adv_stiff(n, p - 1)
        i0 = 2 * p
        for k in range(-(p - 1), p):
            assert abs(T[i0, i0 + k] - n * Mq[i0 + 3, i0 + 3 + k]) < 1e-13
    # its symbol is m_{p-1}; eigenvalues lie inside the symbol's range
    th = np.linspace(0, np.pi, 1001)
    ev = np.linalg.eigvalsh(T)
    sym = sy.m_sym(p - 1, th)
    assert ev.min() >= sym.min() - 1e-12 and ev.max() <= sym.max() + 1e-12


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("p", range(1, 6))
def test_g_p_is_the_symbol_of_the_d_level_T(d, p):
    # g_p = prod_i m_{p-1}(theta_i) (Sec. 6.1) must be the generating function of
    # T_m(m_{p-1})^{(x) d}: its Fourier coefficients are products of the entries
    # phi_{2p-1}(p - i + j) of the 1D Toeplitz matrix
    m = 4 * p + 3
    T1 = mt.toeplitz_T(m, p)
    c = m // 2
    coef = {k: T1[c, c + k] for k in range(-(p - 1), p)}
    rng = np.random.default_rng(p + 10 * d)
    th = [rng.uniform(-np.pi, np.pi, 50) for _ in range(d)]
    ref = np.ones(50, dtype=complex)
    for t in th:
        ref = ref * sum(v * np.exp(1j * k * t) for k, v in coef.items())
    np.testing.assert_allclose(sy.g_sym(p, th), ref.real, atol=1e-14)
    assert np.abs(ref.imag).max() < 1e-14
    # the d-level T is spectrally distributed as g_p: its eigenvalues stay in the symbol's range
    ev = np.linalg.eigvalsh(T1)
    gmin, gmax = sy.m_sym(p - 1, np.pi) ** d, 1.0
    assert ev.min() ** d >= gmin - 1e-12 and ev.max() ** d <= gmax + 1e-12


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("beta", [1.0, 0.1])
def test_preconditioned_symbol_loses_the_zeros_at_pi(d, beta):
    # Sec. 6.1: f^{p,alpha,beta} has numerical zeros where some theta_i = +-pi
    # (its smallest eigenvalue there decays geometrically in p), while
    # f / g_p stays bounded away from zero there, uniformly in p
    t = np.linspace(-np.pi, np.pi, 201 if d == 2 else 41)
    if d == 2:
        th = [np.full_like(t, np.pi), t]
    else:
        T2, T3 = np.meshgrid(t, t, indexing="ij")
        th = [np.full_like(T2, np.pi), T2, T3]
    fmin, qmin = [], []
    for p in range(1, 8):
        f = sy.curl_div_symbol(p, 1.0, beta, th)
        g = sy.g_sym(p, th)
        fmin.append(np.linalg.eigvalsh(f)[..., 0].min())
        qmin.append(np.linalg.eigvalsh(f / g[..., None, None])[..., 0].min())
    for p in range(2, 7):
        assert fmin[p] < fmin[p - 1] / 4  # p -> p + 1 (list index p is degree p + 1)
    assert min(qmin) >= min(1.0, beta) * 0.999
    assert max(qmin) / min(qmin) < 1.6
