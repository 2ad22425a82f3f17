"""Pins of the manufactured-solution load vector and the L2 error (Sec. 6.2).

* The load vector two ways: sum-factorized projections of the weighted
  fields (load_vector) and entry by entry from the weak form with the curl
  of each test field written out (load_vector_rows); they agree to rounding.
  The CG column of Tables 1-4, reproduced in test_oracle_assembly, pins the
  load vector end to end against the paper's printed counts.
* l2_error of the zero field is ||u||, against a 200-point Gauss rule on the
  whole domain (independent of the element quadrature).
* The L2 error of the Galerkin solution converges at order p + 1 in h for
  the smooth manufactured solutions (the approximation order of degree-p
  splines).
"""
import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

from oracle import assembly as asm
from oracle import loadvec, solvers


@pytest.mark.parametrize("d,p,n", [(2, 2, 8), (2, 3, (5, 7)), (3, 2, 4), (3, 3, (3, 4, 5))])
def test_load_vector_two_ways(d, p, n):
    b = loadvec.load_vector(d, p, n, 1.0, 0.3)
    rows = list(range(0, b.size, 3)) + [b.size - 1]
    br = loadvec.load_vector_rows(d, p, n, 1.0, 0.3, rows)
    assert np.abs(br - b[rows]).max() <= 1e-14 * np.abs(b).max()


@pytest.mark.parametrize("d", [2, 3])
def test_l2_norm_of_the_solution(d):
    t, w = leggauss(120 if d == 3 else 200)
    t, w = (t + 1) / 2, w / 2
    X = np.meshgrid(*([t] * d), indexing="ij")
    W = np.prod(np.meshgrid(*([w] * d), indexing="ij"), axis=0)
    g = np.prod([x * (1 - x) for x in X], axis=0)
    u1, u2 = np.sin(2 * np.pi * g), np.cos(2 * np.pi * g) - 1
    sq = u1**2 + u2**2 + ((u1 + u2) ** 2 if d == 3 else 0)
    ref = np.sqrt(np.sum(W * sq))
    p, n = 2, 6
    assert abs(loadvec.l2_error(d, p, n, np.zeros(d * (n + p - 2) ** d)) - ref) <= 1e-12 * ref


@pytest.mark.parametrize("d,p,ns", [(2, 2, (8, 16, 32)), (2, 3, (8, 16, 32)), (3, 2, (4, 8))])
def test_galerkin_solution_converges_at_order_p_plus_1(d, p, ns):
    errs = []
    for n in ns:
        K = asm.curl_div_matrix(d, p, n, 1.0, 0.1)
        x = solvers.solve_direct(K, loadvec.load_vector(d, p, n, 1.0, 0.1))
        errs.append(loadvec.l2_error(d, p, n, x))
    for e0, e1 in zip(errs, errs[1:]):
        assert e0 / e1 >= 0.85 * 2 ** (p + 1), errs
