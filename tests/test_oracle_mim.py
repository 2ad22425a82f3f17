"""Pins of the paper's multi-iterative method in the oracle (Sec. 6.1, the
setting of Sec. 6.2): the PCG post-smoother of P_WL, the Gauss-Seidel sweep,
the block-diagonal cycle of P_WL, the level count, and the MIM / P_WL
columns of Tables 1-4.

What pins what:
* ``pcg_T``: s PCG steps from zero minimise the K-norm of the error over the
  s-dimensional Krylov space of T^{-1} K started at T^{-1} r (the defining
  optimality of preconditioned CG), computed here by brute force.
* the Gauss-Seidel sweep: the forward lexicographic sweep written as a loop.
* P_WL: the cycle on the block-diagonal part D (eq. diag) maps a
  single-component input to a single-component output; with alpha = beta the operator is already block diagonal
  (Sec. 4: the off-diagonal blocks carry alpha - beta), so P_WL's operators
  equal P_MIM's.
* the tables: the paper's printed MIM and P_WL counts, at a tolerance set by
  what independent readings of the paper's unstated details reach (the
  smoothing order, the ordering of the unknowns and the Gauss-Seidel variant
  are not printed): the counts of this oracle sit 0-37% above the paper's for
  MIM at p >= 2, 42-54% above at p = 1, 4-17% above for P_WL at beta = 0.1
  and 39-67% above at beta = 0.01.  The orderings the paper shows in every
  cell (P_MIM below MIM and below P_WL, every count growing as beta falls) are
  pinned exactly.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import assembly as asm
from oracle import loadvec
from oracle import method
from oracle import mim


def _rand(n, seed):
    return np.random.default_rng(seed).uniform(-1, 1, n)


@pytest.mark.parametrize("d,p,n,beta", [(2, 2, 7, 0.1), (2, 3, 6, 0.02), (3, 2, 3, 0.1)])
def test_pcg_T_minimises_the_error_energy_over_the_krylov_space(d, p, n, beta):
    K = asm.curl_div_matrix(d, p, n, 1.0, beta)
    Kd = K.toarray()
    Tm, Tsolve = method.t_operator(d, p, n + p - 2)
    Tinv = np.linalg.inv(Tm.toarray())
    r = _rand(K.shape[0], 5)
    for s in (1, 2, 3, 4):
        e = mim.pcg_T(K, Tsolve, r, s)
        # Krylov basis T^{-1} r, (T^{-1} K) T^{-1} r, ...; minimise (e - e*)^T K (e - e*)
        W = [Tinv @ r]
        for _ in range(s - 1):
            W.append(Tinv @ (Kd @ W[-1]))
        W = np.column_stack(W)
        c = np.linalg.solve(W.T @ Kd @ W, W.T @ r)
        e_ref = W @ c
        np.testing.assert_allclose(e, e_ref, atol=1e-9 * np.abs(e_ref).max())


def test_gauss_seidel_sweep_is_forward_lexicographic():
    pm = mim.PaperMIM(2, 2, 5, 1.0, 0.1, "MIM")
    A = pm.ops[0].toarray()
    b = _rand(A.shape[0], 3)
    x0 = _rand(A.shape[0], 4)
    x = x0.copy()
    for i in range(A.shape[0]):  # new values to the left of the diagonal, old ones to the right
        x[i] = (b[i] - A[i, :i] @ x[:i] - A[i, i + 1:] @ x[i + 1:]) / A[i, i]
    np.testing.assert_allclose(pm._gs(0, x0, b), x, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("d,p,n", [(2, 2, 7), (3, 2, 3)])
def test_pwl_cycle_acts_on_each_component_alone(d, p, n):
    K = asm.curl_div_matrix(d, p, n, 1.0, 0.05)
    pw = mim.PaperMIM(d, p, n, 1.0, 0.05, "P_WL", K=K)
    G = K.shape[0] // d
    # the finest operator of P_WL is the block-diagonal part of K (eq. diag)
    Kd = K.toarray()
    D = np.zeros_like(Kd)
    for c in range(d):
        D[c * G:(c + 1) * G, c * G:(c + 1) * G] = Kd[c * G:(c + 1) * G, c * G:(c + 1) * G]
    assert abs(pw.ops[0] - sp.csr_matrix(D)).max() == 0.0
    # every level stays block diagonal, so one component in gives one component
    # out (the PCG smoother's step lengths couple the components of a general
    # input, so only this structural property holds, not separability)
    r = _rand(K.shape[0], 11)
    for c in range(d):
        rc = np.zeros_like(r)
        rc[c * G:(c + 1) * G] = r[c * G:(c + 1) * G]
        zc = pw.vcycle(rc)
        other = np.ones(K.shape[0], bool)
        other[c * G:(c + 1) * G] = False
        assert np.abs(zc[other]).max() == 0.0
        assert np.abs(zc[~other]).max() > 0.0


def test_pwl_operators_equal_pmim_operators_when_alpha_equals_beta():
    a = mim.PaperMIM(2, 3, 6, 0.7, 0.7, "P_WL")
    b = mim.PaperMIM(2, 3, 6, 0.7, 0.7, "P_MIM")
    assert len(a.ops) == len(b.ops)
    for Aa, Ab in zip(a.ops, b.ops):
        assert abs(Aa - Ab).max() <= 1e-15 * abs(Ab).max()


@pytest.mark.parametrize("p,n", [(1, 16), (2, 15), (3, 14), (2, 31), (4, 13)])
def test_paper_level_count(p, n):
    # m = n + p - 2 = 2^k - 1: log2(n+p-1) levels down to m = 1 (Sec. 6.2)
    pm = mim.PaperMIM(2, p, n, 1.0, 0.1, "MIM")
    assert len(pm.ops) == int(round(np.log2(n + p - 1)))
    assert pm.ops[-1].shape[0] == 2  # one unknown per component on the coarsest level


def _table():
    import os
    rows = {}
    path = os.path.join(os.path.dirname(__file__), "golden", "iteration_tables.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        t = line.split()
        key = (int(t[1]), float(t[2]), int(t[3]), int(t[4]))
        rows[key] = {"P_WL": t[5], "P_MIM": t[6], "MIM": t[7]}
    return rows


# (d, beta, p, n): every cell with m <= 31 in 2D and m <= 7 in 3D, p <= 4
CELLS = [(2, 0.1, 1, 16), (2, 0.1, 2, 15), (2, 0.1, 3, 14), (2, 0.1, 2, 31), (2, 0.1, 3, 30), (2, 0.1, 4, 13),
         (2, 0.01, 1, 16), (2, 0.01, 2, 15), (2, 0.01, 3, 14), (2, 0.01, 2, 31), (2, 0.01, 3, 30), (2, 0.01, 4, 13),
         (3, 0.1, 1, 8), (3, 0.1, 2, 7), (3, 0.1, 3, 6), (3, 0.01, 1, 8), (3, 0.01, 2, 7), (3, 0.01, 3, 6)]


@pytest.fixture(scope="module")
def counts():
    out = {}
    for d, beta, p, n in CELLS:
        K = asm.curl_div_matrix(d, p, n, 1.0, beta)
        b = loadvec.load_vector(d, p, n, 1.0, beta)
        for v in (("P_WL", "P_MIM", "MIM") if d == 2 else ("P_MIM", "MIM")):
            x, it = mim.PaperMIM(d, p, n, 1.0, beta, v, K=K).solve(b, 1e-7, maxiter=500)
            assert np.linalg.norm(b - K @ x) < 1e-7 * np.linalg.norm(b)
            out[(d, beta, p, n, v)] = it
    return out


@pytest.mark.parametrize("cell", CELLS, ids=lambda c: "d%d-b%g-p%d-n%d" % c)
def test_mim_and_pwl_counts_against_the_tables(counts, cell):
    d, beta, p, n = cell
    paper = _table()[cell]
    ratio = counts[cell + ("MIM",)] / int(paper["MIM"])
    lo, hi = (1.0, 1.6) if p == 1 else (0.9, 1.4)
    assert lo <= ratio <= hi, (cell, counts[cell + ("MIM",)], paper["MIM"])
    if d == 2:
        ratio = counts[cell + ("P_WL",)] / int(paper["P_WL"])
        lo, hi = (1.0, 1.2) if beta == 0.1 else (1.3, 1.75)
        assert lo <= ratio <= hi, (cell, counts[cell + ("P_WL",)], paper["P_WL"])


@pytest.mark.parametrize("cell", CELLS, ids=lambda c: "d%d-b%g-p%d-n%d" % c)
def test_orderings_the_tables_show(counts, cell):
    d, beta, p, n = cell
    c = {v: counts.get(cell + (v,)) for v in ("P_WL", "P_MIM", "MIM")}
    assert c["P_MIM"] < c["MIM"]
    if d == 2:
        assert c["P_MIM"] < c["P_WL"]
    if beta == 0.01:
        for v in ("P_WL", "P_MIM", "MIM"):
            if c[v] is not None:
                assert c[v] > counts[(d, 0.1, p, n, v)]
